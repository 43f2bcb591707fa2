// y = A^T x instantiations for field widths 49..64 (split for parallel builds).
#include "matvec_t_impl.hpp"

namespace ccm {
namespace mvt {

hipError_t launch_t_widths_4(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                              const void *x, int xdtype, int64_t *y, int64_t *part,
                              uint64_t part_words, hipStream_t s) {
  switch (bits) {
    case 49: return launch_width_t<49>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 50: return launch_width_t<50>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 51: return launch_width_t<51>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 52: return launch_width_t<52>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 53: return launch_width_t<53>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 54: return launch_width_t<54>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 55: return launch_width_t<55>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 56: return launch_width_t<56>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 57: return launch_width_t<57>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 58: return launch_width_t<58>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 59: return launch_width_t<59>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 60: return launch_width_t<60>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 61: return launch_width_t<61>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 62: return launch_width_t<62>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 63: return launch_width_t<63>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 64: return launch_width_t<64>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mvt
}  // namespace ccm
