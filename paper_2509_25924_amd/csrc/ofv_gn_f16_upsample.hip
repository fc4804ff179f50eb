// Fused Gauss-Newton iteration kernels: _Float16 image storage, input flow mode FLOW_UPSAMPLE.
#include "ofv_gn_impl.h"

namespace ofv {

hipError_t launch_gn_f16_upsample(const GnArgs& a, int kr, int nblocks, hipStream_t s, bool generic) {
  return launch_gn_typed<FLOW_UPSAMPLE, _Float16>(a, kr, nblocks, s, generic);
}

}  // namespace ofv
