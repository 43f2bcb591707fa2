// matvec dispatch over the field width (instantiations live in matvec_w*.hip).
#include "ccm_internal.hpp"

namespace ccm {
namespace mv {
hipError_t launch_widths_1(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                           int64_t *, hipStream_t);
hipError_t launch_widths_2(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                           int64_t *, hipStream_t);
hipError_t launch_widths_3(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                           int64_t *, hipStream_t);
hipError_t launch_widths_4(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                           int64_t *, hipStream_t);
}  // namespace mv

hipError_t launch_matvec(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                         const void *x, int xdtype, int64_t *y, hipStream_t s) {
  if (bits <= 16) return mv::launch_widths_1(w, rows, cols, bits, sgn, x, xdtype, y, s);
  if (bits <= 32) return mv::launch_widths_2(w, rows, cols, bits, sgn, x, xdtype, y, s);
  if (bits <= 48) return mv::launch_widths_3(w, rows, cols, bits, sgn, x, xdtype, y, s);
  return mv::launch_widths_4(w, rows, cols, bits, sgn, x, xdtype, y, s);
}

}  // namespace ccm
