// matvec instantiations for field widths 49..64 (split for parallel builds).
#include "matvec_impl.hpp"

namespace ccm {
namespace mv {

hipError_t launch_widths_4(const uint32_t *w, int64_t rows, int64_t cols, int bits,
                               int sgn, const void *x, int xdtype, int64_t *y, hipStream_t s) {
  switch (bits) {
    case 49: return launch_width<49>(w, rows, cols, sgn, x, xdtype, y, s);
    case 50: return launch_width<50>(w, rows, cols, sgn, x, xdtype, y, s);
    case 51: return launch_width<51>(w, rows, cols, sgn, x, xdtype, y, s);
    case 52: return launch_width<52>(w, rows, cols, sgn, x, xdtype, y, s);
    case 53: return launch_width<53>(w, rows, cols, sgn, x, xdtype, y, s);
    case 54: return launch_width<54>(w, rows, cols, sgn, x, xdtype, y, s);
    case 55: return launch_width<55>(w, rows, cols, sgn, x, xdtype, y, s);
    case 56: return launch_width<56>(w, rows, cols, sgn, x, xdtype, y, s);
    case 57: return launch_width<57>(w, rows, cols, sgn, x, xdtype, y, s);
    case 58: return launch_width<58>(w, rows, cols, sgn, x, xdtype, y, s);
    case 59: return launch_width<59>(w, rows, cols, sgn, x, xdtype, y, s);
    case 60: return launch_width<60>(w, rows, cols, sgn, x, xdtype, y, s);
    case 61: return launch_width<61>(w, rows, cols, sgn, x, xdtype, y, s);
    case 62: return launch_width<62>(w, rows, cols, sgn, x, xdtype, y, s);
    case 63: return launch_width<63>(w, rows, cols, sgn, x, xdtype, y, s);
    case 64: return launch_width<64>(w, rows, cols, sgn, x, xdtype, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mv
}  // namespace ccm
