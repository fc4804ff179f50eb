// Fused Gauss-Newton iteration, 2-D tile and band variants: float image storage, input flow mode FLOW_DIRECT.
#include "ofv_gn_band.h"

namespace ofv {

hipError_t launch_gnt_f32_direct(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s, bool generic) {
  if (variant == GN_BAND4 && !generic) return launch_gn_band_typed<FLOW_DIRECT, float>(a, kr, nblocks, s);
  return launch_gn_tile_typed<FLOW_DIRECT, float>(a, kr, variant, nblocks, s, generic);
}

int gn_band_per_cu_f32_direct(int kr) { return gn_band_typed_per_cu<FLOW_DIRECT, float>(kr); }

}  // namespace ofv
