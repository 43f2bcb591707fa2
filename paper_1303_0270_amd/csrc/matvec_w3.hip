// matvec instantiations for field widths 33..48 (split for parallel builds).
#include "matvec_impl.hpp"

namespace ccm {
namespace mv {

hipError_t launch_widths_3(const uint32_t *w, int64_t rows, int64_t cols, int bits,
                               int sgn, const void *x, int xdtype, int64_t *y, hipStream_t s) {
  switch (bits) {
    case 33: return launch_width<33>(w, rows, cols, sgn, x, xdtype, y, s);
    case 34: return launch_width<34>(w, rows, cols, sgn, x, xdtype, y, s);
    case 35: return launch_width<35>(w, rows, cols, sgn, x, xdtype, y, s);
    case 36: return launch_width<36>(w, rows, cols, sgn, x, xdtype, y, s);
    case 37: return launch_width<37>(w, rows, cols, sgn, x, xdtype, y, s);
    case 38: return launch_width<38>(w, rows, cols, sgn, x, xdtype, y, s);
    case 39: return launch_width<39>(w, rows, cols, sgn, x, xdtype, y, s);
    case 40: return launch_width<40>(w, rows, cols, sgn, x, xdtype, y, s);
    case 41: return launch_width<41>(w, rows, cols, sgn, x, xdtype, y, s);
    case 42: return launch_width<42>(w, rows, cols, sgn, x, xdtype, y, s);
    case 43: return launch_width<43>(w, rows, cols, sgn, x, xdtype, y, s);
    case 44: return launch_width<44>(w, rows, cols, sgn, x, xdtype, y, s);
    case 45: return launch_width<45>(w, rows, cols, sgn, x, xdtype, y, s);
    case 46: return launch_width<46>(w, rows, cols, sgn, x, xdtype, y, s);
    case 47: return launch_width<47>(w, rows, cols, sgn, x, xdtype, y, s);
    case 48: return launch_width<48>(w, rows, cols, sgn, x, xdtype, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mv
}  // namespace ccm
