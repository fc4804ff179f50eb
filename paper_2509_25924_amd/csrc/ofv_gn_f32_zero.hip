// Fused Gauss-Newton iteration kernels: float image storage, input flow mode FLOW_ZERO.
#include "ofv_gn_impl.h"

namespace ofv {

hipError_t launch_gn_f32_zero(const GnArgs& a, int kr, int nblocks, hipStream_t s, bool generic) {
  return launch_gn_typed<FLOW_ZERO, float>(a, kr, nblocks, s, generic);
}

}  // namespace ofv
