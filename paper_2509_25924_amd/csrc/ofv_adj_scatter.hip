// Window sums of dL/dA, adjoints of the products, b, the central difference
// and the two warps of one Gauss-Newton iteration (KR 1..12; Gx, Gy, b
// recomputed or read from the store-all record).
#include "ofv_adj_tile.h"

namespace ofv {

int adj_scatter_blocks(int w, int h, int ty) { return ((w + 63) / 64) * ((h + ty - 1) / ty); }

hipError_t launch_adj_scatter(const AdjArgs& a, int kr, bool stored, int ty, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
#define OFV_ADJX_CASE(R)                                                                           \
  case R:                                                                                          \
    if (ty == 8)                                                                                   \
      return stored ? launch_adj_scatter_cfg<R, true, 8>(a, nblocks, s)                            \
                    : launch_adj_scatter_cfg<R, false, 8>(a, nblocks, s);                          \
    return stored ? launch_adj_scatter_cfg<R, true, 16>(a, nblocks, s)                             \
                  : launch_adj_scatter_cfg<R, false, 16>(a, nblocks, s);
  switch (kr) {
    OFV_ADJX_CASE(1)
    OFV_ADJX_CASE(2)
    OFV_ADJX_CASE(3)
    OFV_ADJX_CASE(4)
    OFV_ADJX_CASE(5)
    OFV_ADJX_CASE(6)
    OFV_ADJX_CASE(7)
    OFV_ADJX_CASE(8)
    OFV_ADJX_CASE(9)
    OFV_ADJX_CASE(10)
    OFV_ADJX_CASE(11)
    OFV_ADJX_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef OFV_ADJX_CASE
}

}  // namespace ofv
