// y = A^T x instantiations for field widths 33..48 (split for parallel builds).
#include "matvec_t_impl.hpp"

namespace ccm {
namespace mvt {

hipError_t launch_t_widths_3(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                              const void *x, int xdtype, int64_t *y, int64_t *part,
                              uint64_t part_words, hipStream_t s) {
  switch (bits) {
    case 33: return launch_width_t<33>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 34: return launch_width_t<34>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 35: return launch_width_t<35>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 36: return launch_width_t<36>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 37: return launch_width_t<37>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 38: return launch_width_t<38>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 39: return launch_width_t<39>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 40: return launch_width_t<40>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 41: return launch_width_t<41>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 42: return launch_width_t<42>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 43: return launch_width_t<43>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 44: return launch_width_t<44>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 45: return launch_width_t<45>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 46: return launch_width_t<46>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 47: return launch_width_t<47>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    case 48: return launch_width_t<48>(w, rows, cols, sgn, x, xdtype, y, part, part_words, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mvt
}  // namespace ccm
