// Fused Gauss-Newton iteration kernels: bf16_t image storage, input flow mode FLOW_DIRECT.
#include "ofv_gn_impl.h"

namespace ofv {

hipError_t launch_gn_bf16_direct(const GnArgs& a, int kr, int nblocks, hipStream_t s, bool generic) {
  return launch_gn_typed<FLOW_DIRECT, bf16_t>(a, kr, nblocks, s, generic);
}

}  // namespace ofv
