// Window sums of one Gauss-Newton iteration with the adjoint of the solve, or
// the recording forward iteration of the store-all mode (KR 1..12).
#include "ofv_adj_tile.h"

namespace ofv {

int adj_sums_blocks(int w, int h, int ty) { return ((w + 63) / 64) * ((h + ty - 1) / ty); }

hipError_t launch_adj_sums(const AdjArgs& a, int kr, int epilogue, int ty, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
#define OFV_ADJS_CASE(R)                                                                              \
  case R:                                                                                             \
    if (ty == 8)                                                                                      \
      return epilogue == ADJ_RECORD ? launch_adj_sums_cfg<R, ADJ_RECORD, 8>(a, nblocks, s)            \
                                    : launch_adj_sums_cfg<R, ADJ_SOLVE, 8>(a, nblocks, s);            \
    return epilogue == ADJ_RECORD ? launch_adj_sums_cfg<R, ADJ_RECORD, 16>(a, nblocks, s)             \
                                  : launch_adj_sums_cfg<R, ADJ_SOLVE, 16>(a, nblocks, s);
  switch (kr) {
    OFV_ADJS_CASE(1)
    OFV_ADJS_CASE(2)
    OFV_ADJS_CASE(3)
    OFV_ADJS_CASE(4)
    OFV_ADJS_CASE(5)
    OFV_ADJS_CASE(6)
    OFV_ADJS_CASE(7)
    OFV_ADJS_CASE(8)
    OFV_ADJS_CASE(9)
    OFV_ADJS_CASE(10)
    OFV_ADJS_CASE(11)
    OFV_ADJS_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef OFV_ADJS_CASE
}

}  // namespace ofv
