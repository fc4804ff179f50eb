// Fused Gauss-Newton iteration, 2-D tile variants: bf16_t image storage, input flow mode FLOW_UPSAMPLE.
#include "ofv_gn_tile.h"

namespace ofv {

hipError_t launch_gnt_bf16_upsample(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s, bool generic) {
  return launch_gn_tile_typed<FLOW_UPSAMPLE, bf16_t>(a, kr, variant, nblocks, s, generic);
}

}  // namespace ofv
