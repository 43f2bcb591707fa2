// y = A^T x instantiations for field widths 17..32 (split for parallel builds).
#include "matvec_t_impl.hpp"

namespace ccm {
namespace mvt {

hipError_t launch_t_widths_2(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                              const void *x, int xdtype, int64_t *y, int64_t *part,
                              uint64_t part_words, hipStream_t s) {
  switch (bits) {
    case 17: return launch_width_t<17>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 18: return launch_width_t<18>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 19: return launch_width_t<19>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 20: return launch_width_t<20>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 21: return launch_width_t<21>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 22: return launch_width_t<22>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 23: return launch_width_t<23>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 24: return launch_width_t<24>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 25: return launch_width_t<25>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 26: return launch_width_t<26>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 27: return launch_width_t<27>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 28: return launch_width_t<28>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 29: return launch_width_t<29>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 30: return launch_width_t<30>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 31: return launch_width_t<31>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 32: return launch_width_t<32>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mvt
}  // namespace ccm
