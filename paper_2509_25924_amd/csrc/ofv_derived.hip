// Live derived quantities of a measured field (the cylinder-wake
// experiment of arXiv 2509.25924, section on live measurements): vorticity,
// velocity probes and the recirculation area of Eq. (RA), in one pass.
// The kernel streams the field once (the neighbour taps of the central
// differences hit the caches), writes the vorticity plane, and counts the
// recirculating pixels with one ballot per wavefront and row; workgroup
// counts meet in a 64-bit counter, and the last workgroup to finish (a
// second counter) converts the total to an area and clears both counters
// for the next call.
#include <stdint.h>

#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

__global__ __launch_bounds__(256) void derived_kernel(const DerivedArgs a) {
  __shared__ unsigned int s_cnt;
  const int tid = threadIdx.x;
  if (tid == 0) s_cnt = 0;
  // probes: the first ceil(n / 256) workgroups, one point per lane
  const int pi = blockIdx.x * 256 + tid;
  if (pi < a.n_probes) {
    const float px = a.probe_xy[2 * pi], py = a.probe_xy[2 * pi + 1];
    a.probe_uv[2 * pi] = a.su * bilinear(a.u, a.pitch, a.w, a.h, px, py);
    a.probe_uv[2 * pi + 1] = a.sv * bilinear(a.v, a.pitch, a.w, a.h, px, py);
  }
  __syncthreads();
  unsigned int cnt = 0;  // recirculating pixels seen by this lane's wavefront (lane 0 keeps it)
  if (static_cast<int>(blockIdx.x) < a.ntiles) {
    const int ntx = (a.w + kDerivedTW - 1) / kDerivedTW;
    const int x = (blockIdx.x % ntx) * kDerivedTW + (tid & 63);
    const int yb = (blockIdx.x / ntx) * kDerivedTH + (tid >> 6);
    const bool xin = x < a.w;
    // neighbours of the x-derivative, clamped into the row: central inside,
    // one-sided at the edges, the same column (difference 0) for one column
    const int xl = max(x - 1, 0), xr = min(x + 1, a.w - 1);
    const float hx = xr - xl == 2 ? 0.5f : 1.0f;
#pragma unroll
    for (int k = 0; k < kDerivedTH / 4; ++k) {
      const int y = yb + 4 * k;
      const bool in = xin && y < a.h;
      bool hit = false;
      if (in) {
        const int64_t row = static_cast<int64_t>(y) * a.pitch;
        const float* vr = a.v + row;
        const float dv = hx * (vr[xr] - vr[xl]);
        const int yl = max(y - 1, 0), yr = min(y + 1, a.h - 1);
        const float hy = yr - yl == 2 ? 0.5f : 1.0f;
        const float du = hy * (a.u[static_cast<int64_t>(yr) * a.pitch + x] - a.u[static_cast<int64_t>(yl) * a.pitch + x]);
        const bool valid = a.mask == nullptr || a.mask[static_cast<int64_t>(y) * a.mask_pitch + x] != 0;
        if (a.omega) a.omega[static_cast<int64_t>(y) * a.omega_pitch + x] = valid ? a.cx * dv - a.cy * du : 0.0f;
        const float uc = a.u[row + x];
        hit = valid && (a.sign > 0 ? uc < 0.0f : uc > 0.0f);
      }
      if (a.area) cnt += static_cast<unsigned int>(__popcll(__ballot(hit)));
    }
  }
  if (a.area == nullptr) return;
  if ((tid & 63) == 0 && cnt) atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (tid == 0) {
    if (s_cnt) atomicAdd(&a.acc[0], static_cast<unsigned long long>(s_cnt));
    __threadfence();
    const unsigned long long done = atomicAdd(&a.acc[1], 1ull);
    if (done == static_cast<unsigned long long>(gridDim.x) - 1) {
      __threadfence();
      const unsigned long long total = atomicExch(&a.acc[0], 0ull);
      *a.area = static_cast<double>(total) * a.dx * a.dz;
      atomicExch(&a.acc[1], 0ull);
    }
  }
}

hipError_t launch_derived(const DerivedArgs& a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(derived_kernel, dim3(nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ofv
