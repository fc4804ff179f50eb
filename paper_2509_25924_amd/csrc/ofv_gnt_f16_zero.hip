// Fused Gauss-Newton iteration, 2-D tile variants: _Float16 image storage, input flow mode FLOW_ZERO.
#include "ofv_gn_tile.h"

namespace ofv {

hipError_t launch_gnt_f16_zero(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s, bool generic) {
  return launch_gn_tile_typed<FLOW_ZERO, _Float16>(a, kr, variant, nblocks, s, generic);
}

}  // namespace ofv
