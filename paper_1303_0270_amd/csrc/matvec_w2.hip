// matvec instantiations for field widths 17..32 (split for parallel builds).
#include "matvec_impl.hpp"

namespace ccm {
namespace mv {

hipError_t launch_widths_2(const uint32_t *w, int64_t rows, int64_t cols, int bits,
                               int sgn, const void *x, int xdtype, int64_t *y, hipStream_t s) {
  switch (bits) {
    case 17: return launch_width<17>(w, rows, cols, sgn, x, xdtype, y, s);
    case 18: return launch_width<18>(w, rows, cols, sgn, x, xdtype, y, s);
    case 19: return launch_width<19>(w, rows, cols, sgn, x, xdtype, y, s);
    case 20: return launch_width<20>(w, rows, cols, sgn, x, xdtype, y, s);
    case 21: return launch_width<21>(w, rows, cols, sgn, x, xdtype, y, s);
    case 22: return launch_width<22>(w, rows, cols, sgn, x, xdtype, y, s);
    case 23: return launch_width<23>(w, rows, cols, sgn, x, xdtype, y, s);
    case 24: return launch_width<24>(w, rows, cols, sgn, x, xdtype, y, s);
    case 25: return launch_width<25>(w, rows, cols, sgn, x, xdtype, y, s);
    case 26: return launch_width<26>(w, rows, cols, sgn, x, xdtype, y, s);
    case 27: return launch_width<27>(w, rows, cols, sgn, x, xdtype, y, s);
    case 28: return launch_width<28>(w, rows, cols, sgn, x, xdtype, y, s);
    case 29: return launch_width<29>(w, rows, cols, sgn, x, xdtype, y, s);
    case 30: return launch_width<30>(w, rows, cols, sgn, x, xdtype, y, s);
    case 31: return launch_width<31>(w, rows, cols, sgn, x, xdtype, y, s);
    case 32: return launch_width<32>(w, rows, cols, sgn, x, xdtype, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mv
}  // namespace ccm
