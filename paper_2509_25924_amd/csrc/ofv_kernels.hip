// Pipeline steps 1, 2 and 4 of the estimator (section "Live-Optical Flow
// Velocimetry", arXiv 2509.25924): local intensity normalisation, one REDUCE
// level of the Burt-Adelson pyramid, and flow up-sampling.  All three are
// HBM-bound stencils; each workgroup stages its input tile (plus halo) in LDS
// or reads it through the L1/L2 caches, and writes coalesced rows.
#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

// ---------------------------------------------------------------------------
// Step 1: decode + local z-score.  Tile of 64 x 16 outputs per 256 lanes;
// the (64 + 2 NR) x (16 + 2 NR) input tile is staged in LDS once and each
// lane evaluates the window mean and the second-pass variance of 4 pixels.
// ---------------------------------------------------------------------------
constexpr int kNormTW = 64;
constexpr int kNormTH = 16;

__device__ __forceinline__ float load_frame_px(const NormJob& J, int x, int y) {
  const int64_t o = static_cast<int64_t>(y) * J.in_pitch + x;
  if (J.type == 0) {
    const float v = static_cast<float>(static_cast<const uint8_t*>(J.in)[o]);
    return v / static_cast<float>((1 << J.bits) - 1);
  }
  if (J.type == 1) {
    const float v = static_cast<float>(static_cast<const uint16_t*>(J.in)[o]);
    return v / static_cast<float>((1 << J.bits) - 1);
  }
  return static_cast<const float*>(J.in)[o];
}

template <typename TS>
__global__ __launch_bounds__(256) void normalize_kernel(const NormArgs a) {
  extern __shared__ float tile[];
  const int j = find_job(a, blockIdx.x);
  const NormJob& J = a.job[j];
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (J.w + kNormTW - 1) / kNormTW;
  const int x0 = (t % ntx) * kNormTW;
  const int y0 = (t / ntx) * kNormTH;
  const int nr = a.nr;
  const int tw = kNormTW + 2 * nr;
  const int th = kNormTH + 2 * nr;
  // all loads of the tile are issued before any is stored (up to 8 per lane
  // in flight); rows and columns outside the frame read as 0 and are never used
  const int n = tw * th;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = min(i0 + 256 * k, n - 1);
      const int gx = x0 - nr + i % tw;
      const int gy = y0 - nr + i / tw;
      const bool in = gx >= 0 && gx < J.w && gy >= 0 && gy < J.h;
      v[k] = load_frame_px(J, min(max(gx, 0), J.w - 1), min(max(gy, 0), J.h - 1));
      v[k] = in ? v[k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + 256 * k < n) tile[i0 + 256 * k] = v[k];
  }
  __syncthreads();
  const int lx = threadIdx.x & 63;
  const int gx = x0 + lx;
  if (gx >= J.w) return;
  TS* out = static_cast<TS*>(J.out);
  const int xa = max(-nr, -gx);
  const int xb = min(nr, J.w - 1 - gx);
  for (int k = 0; k < 4; ++k) {
    const int ly = (threadIdx.x >> 6) + 4 * k;
    const int gy = y0 + ly;
    if (gy >= J.h) break;
    const float* centre = tile + (ly + nr) * tw + (lx + nr);
    float nv = *centre;
    if (nr > 0) {
      const int ya = max(-nr, -gy);
      const int yb = min(nr, J.h - 1 - gy);
      const float n = static_cast<float>((yb - ya + 1) * (xb - xa + 1));
      float s = 0.0f;
      for (int dy = ya; dy <= yb; ++dy) {
        float row = 0.0f;
        for (int dx = xa; dx <= xb; ++dx) row += centre[dy * tw + dx];
        s += row;
      }
      const float mu = s / n;
      float q = 0.0f;
      for (int dy = ya; dy <= yb; ++dy) {
        for (int dx = xa; dx <= xb; ++dx) {
          const float d = centre[dy * tw + dx] - mu;
          q += d * d;
        }
      }
      nv = (nv - mu) / sqrtf(q / n + a.eps);
    }
    Px<TS>::st(out + static_cast<int64_t>(gy) * J.out_pitch + gx, nv);
  }
}

hipError_t launch_normalize(const NormArgs& a, int nblocks, hipStream_t s) {
  const size_t lds = sizeof(float) * (kNormTW + 2 * a.nr) * (kNormTH + 2 * a.nr);
  switch (a.storage) {
    case ST_F32: hipLaunchKernelGGL(normalize_kernel<float>, dim3(nblocks), dim3(256), lds, s, a); break;
    case ST_F16: hipLaunchKernelGGL(normalize_kernel<_Float16>, dim3(nblocks), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL(normalize_kernel<bf16_t>, dim3(nblocks), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 2: REDUCE.  One lane per output pixel, 64 x 4 outputs per workgroup;
// the 5 x 5 binomial stencil reads through the caches (each input pixel is
// touched by at most 9 outputs, all in neighbouring lanes and rows).
// out(x, y) = scale * sum_j w_j sum_i w_i in(clamp(2x+i), clamp(2y+j)).
// ---------------------------------------------------------------------------
constexpr int kRedTW = 64;
constexpr int kRedTH = 4;

template <typename TS>
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceArgs a) {
  const int j = find_job(a, blockIdx.x);
  const ReduceJob& J = a.job[j];
  const int wn = (J.w + 1) / 2;
  const int hn = (J.h + 1) / 2;
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (wn + kRedTW - 1) / kRedTW;
  const int x = (t % ntx) * kRedTW + (threadIdx.x & 63);
  const int y = (t / ntx) * kRedTH + (threadIdx.x >> 6);
  if (x >= wn || y >= hn) return;
  const TS* in = static_cast<const TS*>(J.in);
  const float w5[5] = {1.0f / 16, 4.0f / 16, 6.0f / 16, 4.0f / 16, 1.0f / 16};
  int xs[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) xs[i] = min(max(2 * x + i - 2, 0), J.w - 1);
  float acc = 0.0f;
#pragma unroll
  for (int jj = 0; jj < 5; ++jj) {
    const int yy = min(max(2 * y + jj - 2, 0), J.h - 1);
    const TS* row = in + static_cast<int64_t>(yy) * J.in_pitch;
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) r += w5[i] * Px<TS>::ld(row + xs[i]);
    acc += w5[jj] * r;
  }
  Px<TS>::st(static_cast<TS*>(J.out) + static_cast<int64_t>(y) * J.out_pitch + x, a.scale * acc);
}

hipError_t launch_reduce(const ReduceArgs& a, int nblocks, hipStream_t s) {
  switch (a.storage) {
    case ST_F32: hipLaunchKernelGGL(reduce_kernel<float>, dim3(nblocks), dim3(256), 0, s, a); break;
    case ST_F16: hipLaunchKernelGGL(reduce_kernel<_Float16>, dim3(nblocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(reduce_kernel<bf16_t>, dim3(nblocks), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 4 (stand-alone form): V_fine(X, Y) = 2 * bilinear(V_coarse, X/2, Y/2).
// The estimator itself fuses this read into the first Gauss-Newton
// iteration of each finer level.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void upsample_kernel(const UpsampleArgs a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.w || y >= a.h) return;
  const float fx = 0.5f * static_cast<float>(x);
  const float fy = 0.5f * static_cast<float>(y);
  const int64_t o = static_cast<int64_t>(y) * a.out_pitch + x;
  a.out_u[o] = 2.0f * bilinear(a.in_u, a.in_pitch, a.cw, a.ch, fx, fy);
  a.out_v[o] = 2.0f * bilinear(a.in_v, a.in_pitch, a.cw, a.ch, fx, fy);
}

hipError_t launch_upsample(const UpsampleArgs& a, hipStream_t s) {
  dim3 grid((a.w + 63) / 64, (a.h + 3) / 4);
  hipLaunchKernelGGL(upsample_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ofv

namespace ofv {

#define OFV_DECL(ST, MD) hipError_t launch_gn_##ST##_##MD(const GnArgs& a, int kr, int nblocks, hipStream_t s);
OFV_DECL(f32, zero)
OFV_DECL(f32, direct)
OFV_DECL(f32, upsample)
OFV_DECL(f16, zero)
OFV_DECL(f16, direct)
OFV_DECL(f16, upsample)
OFV_DECL(bf16, zero)
OFV_DECL(bf16, direct)
OFV_DECL(bf16, upsample)
#undef OFV_DECL
#define OFV_DECLT(ST, MD) \
  hipError_t launch_gnt_##ST##_##MD(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s);
OFV_DECLT(f32, zero)
OFV_DECLT(f32, direct)
OFV_DECLT(f32, upsample)
OFV_DECLT(f16, zero)
OFV_DECLT(f16, direct)
OFV_DECLT(f16, upsample)
OFV_DECLT(bf16, zero)
OFV_DECLT(bf16, direct)
OFV_DECLT(bf16, upsample)
#undef OFV_DECLT

hipError_t launch_gn(const GnArgs& a, int kr, int storage, int mode, int variant, int nblocks, hipStream_t s) {
  if (variant != GN_MARCH) {
#define OFV_PICKT(ST)                                                                     \
  if (mode == FLOW_ZERO) return launch_gnt_##ST##_zero(a, kr, variant, nblocks, s);     \
  if (mode == FLOW_DIRECT) return launch_gnt_##ST##_direct(a, kr, variant, nblocks, s); \
  return launch_gnt_##ST##_upsample(a, kr, variant, nblocks, s);
    if (storage == ST_F32) { OFV_PICKT(f32) }
    if (storage == ST_F16) { OFV_PICKT(f16) }
    OFV_PICKT(bf16)
#undef OFV_PICKT
  }
#define OFV_PICK(ST)                                                    \
  if (mode == FLOW_ZERO) return launch_gn_##ST##_zero(a, kr, nblocks, s);     \
  if (mode == FLOW_DIRECT) return launch_gn_##ST##_direct(a, kr, nblocks, s); \
  return launch_gn_##ST##_upsample(a, kr, nblocks, s);
  if (storage == ST_F32) { OFV_PICK(f32) }
  if (storage == ST_F16) { OFV_PICK(f16) }
  OFV_PICK(bf16)
#undef OFV_PICK
}

}  // namespace ofv
