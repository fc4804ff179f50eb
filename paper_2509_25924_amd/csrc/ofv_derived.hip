// Live derived quantities of a measured field (the cylinder-wake
// experiment of arXiv 2509.25924, section on live measurements): vorticity,
// velocity probes and the recirculation area of Eq. (RA).
// derived_kernel streams the field once (the neighbour taps of the central
// differences hit the caches) with a bounded grid that strides over 64-column
// tiles (one column of kDerivedRows consecutive rows per lane), writes the
// vorticity plane, interpolates the probes, and counts the recirculating
// pixels with one ballot per wavefront and row; the wavefronts of a
// workgroup add their counts in LDS and the workgroup stores the total in its
// own slot (no global atomics, so the count is exact and deterministic and
// the launch can be replayed in a graph).  derived_area_kernel,
// one workgroup, sums the slots and writes the area.
#include <stdint.h>

#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

__global__ __launch_bounds__(256) void derived_kernel(const DerivedArgs a) {
  __shared__ unsigned int s_cnt;
  const int tid = threadIdx.x;
  if (tid == 0) s_cnt = 0;
  for (int pi = blockIdx.x * 256 + tid; pi < a.n_probes; pi += gridDim.x * 256) {
    const float px = a.probe_xy[2 * pi], py = a.probe_xy[2 * pi + 1];
    a.probe_uv[2 * pi] = a.su * bilinear(a.u, a.pitch, a.w, a.h, px, py);
    a.probe_uv[2 * pi + 1] = a.sv * bilinear(a.v, a.pitch, a.w, a.h, px, py);
  }
  __syncthreads();
  unsigned int cnt = 0;  // recirculating pixels seen by this lane's wavefront (the same in every lane)
  const int ntx = (a.w + kDerivedTW - 1) / kDerivedTW;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    // lane: one column, kDerivedRows consecutive rows of the tile; the u rows
    // above and below are carried from row to row
    const int x = (t % ntx) * kDerivedTW + (tid & 63);
    const int y0 = (t / ntx) * kDerivedTH + kDerivedRows * (tid >> 6);
    const bool xin = x < a.w;
    // neighbours of the x-derivative, clamped into the row: central inside,
    // one-sided at the edges, the same column (difference 0) for one column
    const int xl = max(x - 1, 0), xr = min(x + 1, a.w - 1);
    const float hx = xr - xl == 2 ? 0.5f : 1.0f;
    const float* uc = a.u + x;
    float u_prev = xin && y0 >= 1 && y0 - 1 < a.h ? uc[static_cast<int64_t>(y0 - 1) * a.pitch] : 0.0f;
    float u_cur = xin && y0 < a.h ? uc[static_cast<int64_t>(y0) * a.pitch] : 0.0f;
#pragma unroll
    for (int k = 0; k < kDerivedRows; ++k) {
      const int y = y0 + k;
      const bool in = xin && y < a.h;
      const float u_next = in && y + 1 < a.h ? uc[static_cast<int64_t>(y + 1) * a.pitch] : 0.0f;
      bool hit = false;
      if (in) {
        const float* vr = a.v + static_cast<int64_t>(y) * a.pitch;
        const float dv = hx * (vr[xr] - vr[xl]);
        // central inside, one-sided at the first and last row, 0 for one row
        const float du = y == 0 ? (a.h > 1 ? u_next - u_cur : 0.0f)
                                : (y == a.h - 1 ? u_cur - u_prev : 0.5f * (u_next - u_prev));
        const bool valid = a.mask == nullptr || a.mask[static_cast<int64_t>(y) * a.mask_pitch + x] != 0;
        if (a.omega) a.omega[static_cast<int64_t>(y) * a.omega_pitch + x] = valid ? a.cx * dv - a.cy * du : 0.0f;
        hit = valid && (a.sign > 0 ? u_cur < 0.0f : u_cur > 0.0f);
      }
      if (a.partial) cnt += static_cast<unsigned int>(__popcll(__ballot(hit)));
      u_prev = u_cur;
      u_cur = u_next;
    }
  }
  if (a.partial == nullptr) return;
  if ((tid & 63) == 0 && cnt) atomicAdd(&s_cnt, cnt);  // LDS
  __syncthreads();
  if (tid == 0) a.partial[blockIdx.x] = s_cnt;
}

__global__ __launch_bounds__(1024) void derived_area_kernel(const unsigned int* partial, int n, double* area,
                                                            double dx, double dz) {
  __shared__ unsigned long long s[1024];
  unsigned long long c = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < n; i += 1024) c += partial[i];
  s[threadIdx.x] = c;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *area = static_cast<double>(s[0]) * dx * dz;
}

hipError_t launch_derived(const DerivedArgs& a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(derived_kernel, dim3(nblocks), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.area == nullptr) return e;
  hipLaunchKernelGGL(derived_area_kernel, dim3(1), dim3(1024), 0, s, static_cast<const unsigned int*>(a.partial),
                     nblocks, a.area, a.dx, a.dz);
  return hipGetLastError();
}

}  // namespace ofv
