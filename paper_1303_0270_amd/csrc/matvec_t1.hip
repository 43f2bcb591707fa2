// y = A^T x instantiations for field widths 1..16 (split for parallel builds).
#include "matvec_t_impl.hpp"

namespace ccm {
namespace mvt {

hipError_t launch_t_widths_1(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                              const void *x, int xdtype, int64_t *y, int64_t *part,
                              uint64_t part_words, hipStream_t s) {
  switch (bits) {
    case 1: return launch_width_t<1>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 2: return launch_width_t<2>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 3: return launch_width_t<3>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 4: return launch_width_t<4>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 5: return launch_width_t<5>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 6: return launch_width_t<6>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 7: return launch_width_t<7>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 8: return launch_width_t<8>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 9: return launch_width_t<9>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 10: return launch_width_t<10>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 11: return launch_width_t<11>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 12: return launch_width_t<12>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 13: return launch_width_t<13>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 14: return launch_width_t<14>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 15: return launch_width_t<15>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 16: return launch_width_t<16>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mvt
}  // namespace ccm
