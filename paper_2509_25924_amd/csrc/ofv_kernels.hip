// Pipeline steps 1, 2 and 4 of the estimator (section "Live-Optical Flow
// Velocimetry", arXiv 2509.25924): local intensity normalisation, one REDUCE
// level of the Burt-Adelson pyramid, and flow up-sampling.  All three are
// HBM-bound stencils; each workgroup stages its input tile (plus halo) in LDS
// or reads it through the L1/L2 caches, and writes coalesced rows.
#include <type_traits>

#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

// ---------------------------------------------------------------------------
// Step 1: decode + local z-score.  Tile of kNormTW x kNormTH outputs per 256 lanes;
// integer frames are scaled by the float32 reciprocal of 2^B - 1 and the
// z-score uses the hardware reciprocal square root (both within a few
// float32 rounding errors of the exact quotients);
// the (kNormTW + 2 NR) x (kNormTH + 2 NR) input tile is staged in LDS once
// (frame pixels outside the frame stored as 0) and each lane evaluates
// kNormPX vertically adjacent outputs of one column.  Every normalisation kernel
// evaluates one pixel by the same sequence of float32 operations over the
// window truncated to the frame (n pixels), so that all of them agree bit
// for bit:
//   row sums left to right, S = their sum top to bottom, rn = 1 / n,
//   mu = S rn,  q = fma chain of (I - mu)^2 in row-major order,
//   N = (I - mu) rsq(q rn + eps)        (second-pass variance)
// Taps outside the frame are stored as 0 (exact in the sums) and masked by
// a 0/1 weight in the q chain (fma(0, d, q) = q).
// For NR <= 3 the lane's (kNormPX + 2 NR) x (2 NR + 1) patch is read into
// registers once and row sums are shared between its outputs.  Larger
// radii take the generic path that walks the window in LDS.
// ---------------------------------------------------------------------------

template <typename TI>
__device__ __forceinline__ float frame_value(const void* base, int64_t o, float inv_max) {
  return static_cast<float>(static_cast<const TI*>(base)[o]) * inv_max;
}
template <>
__device__ __forceinline__ float frame_value<float>(const void* base, int64_t o, float) {
  return static_cast<const float*>(base)[o];
}

// Stage a tw x th tile whose pixel (0, 0) is frame pixel (x0, y0); up to 8
// loads per lane are in flight before the first LDS store.
template <typename TI>
__device__ __forceinline__ void stage_frame_tile(const NormJob& J, float* tile, int x0, int y0, int tw, int th) {
  const int n = tw * th;
  const float inv_max = 1.0f / static_cast<float>((1 << J.bits) - 1);
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = min(i0 + 256 * k, n - 1);
      const int ty = i / tw;
      const int gx = x0 + (i - ty * tw);
      const int gy = y0 + ty;
      const bool in = static_cast<unsigned>(gx) < static_cast<unsigned>(J.w) &&
                      static_cast<unsigned>(gy) < static_cast<unsigned>(J.h);
      const int64_t o = static_cast<int64_t>(min(max(gy, 0), J.h - 1)) * J.in_pitch + min(max(gx, 0), J.w - 1);
      v[k] = in ? frame_value<TI>(J.in, o, inv_max) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + 256 * k < n) tile[i0 + 256 * k] = v[k];
  }
}

template <typename TI>
__device__ __forceinline__ float frame_ldv(PlaneView v, uint32_t i);
template <>
__device__ __forceinline__ float frame_ldv<uint8_t>(PlaneView v, uint32_t i) {
  return static_cast<float>(__builtin_amdgcn_raw_buffer_load_b8(v, static_cast<int>(i), 0, 0));
}
template <>
__device__ __forceinline__ float frame_ldv<uint16_t>(PlaneView v, uint32_t i) {
  return static_cast<float>(__builtin_amdgcn_raw_buffer_load_b16(v, static_cast<int>(i * 2u), 0, 0));
}
template <>
__device__ __forceinline__ float frame_ldv<float>(PlaneView v, uint32_t i) {
  return ld_f32(v, i);
}

// Same as stage_frame_tile for a TW x TH tile known at compile time: every
// lane issues its ceil(TW TH / 256) loads at once through a buffer view of
// the frame (32-bit offsets; frames stay below 2 GiB with pitches below 2^24).
template <typename TI, int TW, int TH>
__device__ __forceinline__ void stage_frame_tile_c(const NormJob& J, float* tile, int x0, int y0) {
  constexpr int N = TW * TH;
  constexpr int NLD = (N + 255) / 256;
  const uint32_t pitch = static_cast<uint32_t>(J.in_pitch);
  const PlaneView fv = plane_view(J.in, pitch * static_cast<uint32_t>(J.h) * static_cast<uint32_t>(sizeof(TI)));
  const float inv_max = 1.0f / static_cast<float>((1 << J.bits) - 1);
  float v[NLD];
  if (x0 >= 0 && y0 >= 0 && x0 + TW <= J.w && y0 + TH <= J.h) {
    // the whole tile lies inside the frame (block-uniform): no clamps or masks
    const uint32_t base = __umul24(static_cast<uint32_t>(y0), pitch) + static_cast<uint32_t>(x0);
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = min(static_cast<int>(threadIdx.x) + 256 * k, N - 1);
      const int ty = i / TW;
      float x = frame_ldv<TI>(fv, base + __umul24(static_cast<uint32_t>(ty), pitch) + static_cast<uint32_t>(i - ty * TW));
      if (!std::is_same<TI, float>::value) x *= inv_max;
      v[k] = x;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = min(static_cast<int>(threadIdx.x) + 256 * k, N - 1);
      const int ty = i / TW;
      const int gx = x0 + (i - ty * TW);
      const int gy = y0 + ty;
      const bool in = static_cast<unsigned>(gx) < static_cast<unsigned>(J.w) &&
                      static_cast<unsigned>(gy) < static_cast<unsigned>(J.h);
      const uint32_t o = __umul24(static_cast<uint32_t>(min(max(gy, 0), J.h - 1)), pitch) +
                         static_cast<uint32_t>(min(max(gx, 0), J.w - 1));
      float x = frame_ldv<TI>(fv, o);
      if (!std::is_same<TI, float>::value) x *= inv_max;
      v[k] = in ? x : 0.0f;
    }
  }
#pragma unroll
  for (int k = 0; k < NLD; ++k)
    if (static_cast<int>(threadIdx.x) + 256 * k < N) tile[threadIdx.x + 256 * k] = v[k];
}

template <typename TS, int NRC>
__global__ __launch_bounds__(256) void normalize_kernel(const NormArgs a) {
#pragma clang fp contract(off)
  extern __shared__ float tile[];
  const int j = find_job(a, blockIdx.x);
  const NormJob& J = a.job[j];
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (J.w + kNormTW - 1) / kNormTW;
  const int x0 = (t % ntx) * kNormTW;
  const int y0 = (t / ntx) * kNormTH;
  const int nr = NRC > 0 ? NRC : a.nr;
  const int tw = kNormTW + 2 * nr;
  const int th = kNormTH + 2 * nr;
  if (NRC > 0) {
    constexpr int TW = kNormTW + 2 * NRC, TH = kNormTH + 2 * NRC;
    if (J.type == 0) stage_frame_tile_c<uint8_t, TW, TH>(J, tile, x0 - nr, y0 - nr);
    else if (J.type == 1) stage_frame_tile_c<uint16_t, TW, TH>(J, tile, x0 - nr, y0 - nr);
    else stage_frame_tile_c<float, TW, TH>(J, tile, x0 - nr, y0 - nr);
  } else {
    if (J.type == 0) stage_frame_tile<uint8_t>(J, tile, x0 - nr, y0 - nr, tw, th);
    else if (J.type == 1) stage_frame_tile<uint16_t>(J, tile, x0 - nr, y0 - nr, tw, th);
    else stage_frame_tile<float>(J, tile, x0 - nr, y0 - nr, tw, th);
  }
  __syncthreads();
  const int lx = threadIdx.x & 63;
  const int ly0 = kNormPX * (threadIdx.x >> 6);
  const int gx = x0 + lx;
  const int gy0 = y0 + ly0;
  if (gx >= J.w || gy0 >= J.h) return;
  TS* out = static_cast<TS*>(J.out) + static_cast<int64_t>(gy0) * J.out_pitch + gx;
  if (NRC > 0) {
    constexpr int R = NRC;
    constexpr int NC = 2 * R + 1;
    constexpr int NRW = kNormPX + 2 * R;
    float pv[NRW][NC];
    float vy[NRW], vx[NC];
#pragma unroll
    for (int r = 0; r < NRW; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) pv[r][c] = tile[(ly0 + r) * tw + lx + c];
      vy[r] = static_cast<unsigned>(gy0 - R + r) < static_cast<unsigned>(J.h) ? 1.0f : 0.0f;
    }
    float ncol = 0.0f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      vx[c] = static_cast<unsigned>(gx - R + c) < static_cast<unsigned>(J.w) ? 1.0f : 0.0f;
      ncol += vx[c];
    }
    float hs[NRW];
#pragma unroll
    for (int r = 0; r < NRW; ++r) {
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc += pv[r][c];
      hs[r] = acc;
    }
    // block-uniform: every window of the tile lies inside the frame
    if (x0 >= R && y0 >= R && x0 + kNormTW + R <= J.w && y0 + kNormTH + R <= J.h) {
      constexpr float rn = 1.0f / static_cast<float>(NC * NC);
      if (R >= 2) {
        // A window's squared deviations, row by row: those from the row's own
        // mean m_r (shared by the lane's kNormPX windows) plus NC (m_r - mu)^2.
        // Every term is a square of a deviation, as in the second-pass form,
        // with NC + 1 instead of NC * NC (subtract, multiply-add) pairs per output.
        float mr[NRW], dr[NRW];
#pragma unroll
        for (int r = 0; r < NRW; ++r) {
          mr[r] = hs[r] * (1.0f / static_cast<float>(NC));
          float acc = 0.0f;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float d = pv[r][c] - mr[r];
            acc = fmaf(d, d, acc);
          }
          dr[r] = acc;
        }
#pragma unroll
        for (int k = 0; k < kNormPX; ++k) {
          float sm = 0.0f;
#pragma unroll
          for (int r = 0; r < NC; ++r) sm += hs[k + r];
          const float mu = sm * rn;
          float q1 = 0.0f, q2 = 0.0f;
#pragma unroll
          for (int r = 0; r < NC; ++r) {
            q1 += dr[k + r];
            const float d = mr[k + r] - mu;
            q2 = fmaf(d, d, q2);
          }
          const float q = fmaf(static_cast<float>(NC), q2, q1);
          Px<TS>::st(out + k * J.out_pitch, (pv[k + R][R] - mu) * __builtin_amdgcn_rsqf(fmaf(q, rn, a.eps)));
        }
        return;
      }
#pragma unroll
      for (int k = 0; k < kNormPX; ++k) {
        float sm = 0.0f;
#pragma unroll
        for (int r = 0; r < NC; ++r) sm += hs[k + r];
        const float mu = sm * rn;
        float q = 0.0f;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float d = pv[k + r][c] - mu;
            q = fmaf(d, d, q);
          }
        }
        Px<TS>::st(out + k * J.out_pitch, (pv[k + R][R] - mu) * __builtin_amdgcn_rsqf(fmaf(q, rn, a.eps)));
      }
      return;
    }
#pragma unroll
    for (int k = 0; k < kNormPX; ++k) {
      if (gy0 + k < J.h) {
        float sm = 0.0f, nrow = 0.0f;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
          sm += hs[k + r];
          nrow += vy[k + r];
        }
        const float rn = 1.0f / (nrow * ncol);
        const float mu = sm * rn;
        float q = 0.0f;
#pragma unroll
        for (int r = 0; r < NC; ++r) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float d = pv[k + r][c] - mu;
            q = fmaf(vy[k + r] * vx[c] * d, d, q);
          }
        }
        Px<TS>::st(out + k * J.out_pitch, (pv[k + R][R] - mu) * __builtin_amdgcn_rsqf(fmaf(q, rn, a.eps)));
      }
    }
    return;
  }
  const int xa = max(-nr, -gx);
  const int xb = min(nr, J.w - 1 - gx);
  for (int k = 0; k < kNormPX; ++k) {
    const int ly = ly0 + k;
    const int gy = gy0 + k;
    if (gy >= J.h) break;
    const float* centre = tile + (ly + nr) * tw + (lx + nr);
    float nv = *centre;
    if (nr > 0) {
      const int ya = max(-nr, -gy);
      const int yb = min(nr, J.h - 1 - gy);
      const float rn = 1.0f / static_cast<float>((yb - ya + 1) * (xb - xa + 1));
      float s = 0.0f;
      for (int dy = ya; dy <= yb; ++dy) {
        float row = 0.0f;
        for (int dx = xa; dx <= xb; ++dx) row += centre[dy * tw + dx];
        s += row;
      }
      const float mu = s * rn;
      float q = 0.0f;
      for (int dy = ya; dy <= yb; ++dy) {
        for (int dx = xa; dx <= xb; ++dx) {
          const float d = centre[dy * tw + dx] - mu;
          q = fmaf(d, d, q);
        }
      }
      nv = (nv - mu) * __builtin_amdgcn_rsqf(fmaf(q, rn, a.eps));
    }
    Px<TS>::st(out + k * J.out_pitch, nv);
  }
}

template <typename TS>
hipError_t launch_normalize_typed(const NormArgs& a, int nblocks, size_t lds, hipStream_t s) {
  switch (a.nr) {
    case 1: hipLaunchKernelGGL((normalize_kernel<TS, 1>), dim3(nblocks), dim3(256), lds, s, a); break;
    case 2: hipLaunchKernelGGL((normalize_kernel<TS, 2>), dim3(nblocks), dim3(256), lds, s, a); break;
    case 3: hipLaunchKernelGGL((normalize_kernel<TS, 3>), dim3(nblocks), dim3(256), lds, s, a); break;
    default: hipLaunchKernelGGL((normalize_kernel<TS, 0>), dim3(nblocks), dim3(256), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_normalize(const NormArgs& a, int nblocks, hipStream_t s) {
  const size_t lds = sizeof(float) * (kNormTW + 2 * a.nr) * (kNormTH + 2 * a.nr);
  switch (a.storage) {
    case ST_F32: return launch_normalize_typed<float>(a, nblocks, lds, s);
    case ST_F16: return launch_normalize_typed<_Float16>(a, nblocks, lds, s);
    default: return launch_normalize_typed<bf16_t>(a, nblocks, lds, s);
  }
}

// ---------------------------------------------------------------------------
// Step 2: REDUCE.  64 x 8 outputs per 256-lane workgroup (kRedTW x kRedTH):
//   out(x, y) = scale * sum_j w_j sum_i w_i in(clamp(2x+i), clamp(2y+j)),
// w = [1, 4, 6, 4, 1] / 16, i, j = -2..2.  The 131 x 19 input tile (indices
// clamped into the plane) is staged in LDS with coalesced row loads, the
// horizontal 5-tap pass writes 19 x 64 row sums to LDS and the vertical
// pass combines 5 of them per output, two outputs per lane (the input tile
// is 2.4 input rows per output row instead of 2.75 with 4-row tiles).
// ---------------------------------------------------------------------------
constexpr int kRedInW = 2 * kRedTW + 3;  // 131 input columns
constexpr int kRedInH = 2 * kRedTH + 3;  // 19 input rows

template <typename TS>
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceArgs a) {
  __shared__ float tin[kRedInH][kRedInW + 1];
  __shared__ float th[kRedInH][kRedTW + 1];
  const int j = find_job(a, blockIdx.x);
  const ReduceJob& J = a.job[j];
  const int wn = (J.w + 1) / 2;
  const int hn = (J.h + 1) / 2;
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (wn + kRedTW - 1) / kRedTW;
  const int x0 = (t % ntx) * kRedTW;
  const int y0 = (t / ntx) * kRedTH;
  const int bx = 2 * x0 - 2;
  const int by = 2 * y0 - 2;
  const TS* in = static_cast<const TS*>(J.in);
  constexpr int NIN = kRedInH * kRedInW;
  constexpr int NLD = (NIN + 255) / 256;
  float v[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = min(static_cast<int>(threadIdx.x) + 256 * k, NIN - 1);
    const int r = i / kRedInW;
    const int c = i - r * kRedInW;
    const int gx = min(max(bx + c, 0), J.w - 1);
    const int gy = min(max(by + r, 0), J.h - 1);
    v[k] = Px<TS>::ld(in + static_cast<int64_t>(gy) * J.in_pitch + gx);
  }
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NIN) {
      const int r = i / kRedInW;
      tin[r][i - r * kRedInW] = v[k];
    }
  }
  __syncthreads();
  constexpr float w0 = 1.0f / 16, w1 = 4.0f / 16, w2 = 6.0f / 16;
  for (int i = threadIdx.x; i < kRedInH * kRedTW; i += 256) {
    const int r = i / kRedTW;
    const int c = i - r * kRedTW;
    const float* p = &tin[r][2 * c];
    float acc = w0 * p[0];
    acc += w1 * p[1];
    acc += w2 * p[2];
    acc += w1 * p[3];
    acc += w0 * p[4];
    th[r][c] = acc;
  }
  __syncthreads();
  const int lx = threadIdx.x & 63;
  const int x = x0 + lx;
  if (x >= wn) return;
#pragma unroll
  for (int ly = threadIdx.x >> 6; ly < kRedTH; ly += 4) {
    const int y = y0 + ly;
    if (y < hn) {
      float acc = w0 * th[2 * ly][lx];
      acc += w1 * th[2 * ly + 1][lx];
      acc += w2 * th[2 * ly + 2][lx];
      acc += w1 * th[2 * ly + 3][lx];
      acc += w0 * th[2 * ly + 4][lx];
      Px<TS>::st(static_cast<TS*>(J.out) + static_cast<int64_t>(y) * J.out_pitch + x, a.scale * acc);
    }
  }
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
// Step 2, NLEV levels per launch.  A workgroup owns a TW x TH tile of the
// deepest level and the matching tiles of the levels above it (2x, 4x the
// size).  Level k (input k = 0) is held in LDS over a region of
// rw(k) x rh(k) pixels whose origin is 2 * origin(k + 1) - 2: exactly the
// taps that level k + 1's region reads.  A region pixel outside its level
// stands for its clamped position (replicate border), so every tap reads
// its region directly.  Each level is rounded to the storage type before
// the next one is formed, as a separate REDUCE launch would read it, so the
// levels equal level-by-level REDUCE bit for bit.
// ---------------------------------------------------------------------------
template <int NLEV, int TW, int TH>
struct RChain {
  static constexpr int rw(int k) { return k >= NLEV ? TW : 2 * rw(k + 1) + 3; }
  static constexpr int rh(int k) { return k >= NLEV ? TH : 2 * rh(k + 1) + 3; }
  static constexpr int off(int k) { return k >= NLEV ? 0 : 2 * off(k + 1) + 2; }  // owned tile within region k
  // region buffers of levels 0 .. NLEV-1 and one horizontal-pass buffer
  static constexpr int buf(int k) { return k <= 0 ? 0 : buf(k - 1) + rw(k - 1) * rh(k - 1); }
  static constexpr int tmp_size() {
    int m = 0;
    for (int k = 1; k <= NLEV; ++k) m = rh(k - 1) * rw(k) > m ? rh(k - 1) * rw(k) : m;
    return m;
  }
  static constexpr int LDS_FLOATS = buf(NLEV) + tmp_size();
};

// Level K of the chain: region K from region K - 1 (both in LDS), rounded
// to the storage type; the owned tile is stored to `out` (pitch `opitch`).
template <typename TS, int NLEV, int TW, int TH, int NT, int K>
__device__ __forceinline__ void chain_level(float* lds, const int* ox, const int* oy, const int* lw, const int* lh,
                                            void* outp, int64_t opitch) {
  using C = RChain<NLEV, TW, TH>;
  constexpr float w0 = 1.0f / 16, w1 = 4.0f / 16, w2 = 6.0f / 16;
  constexpr int sw = C::rw(K - 1), sh = C::rh(K - 1);
  constexpr int dw = C::rw(K), dh = C::rh(K);
  constexpr int own_w = TW << (NLEV - K), own_h = TH << (NLEV - K);  // owned tile at level K
  constexpr int offk = C::off(K);
  constexpr int SRC = C::buf(K - 1), DST = C::buf(K), TMP = C::buf(NLEV);
  const float* src = lds + SRC;
  float* dst = lds + DST;
  float* tmp = lds + TMP;
  __syncthreads();
  // horizontal pass: rows of region K-1, columns of region K (value at the clamped column)
  for (int i = threadIdx.x; i < sh * dw; i += NT) {
    const int r = i / dw;
    const int c = i - r * dw;
    const int q = min(max(ox[K] + c, 0), lw[K] - 1);
    const float* p = src + r * sw + (2 * q - 2 - ox[K - 1]);
    float acc = w0 * p[0];
    acc += w1 * p[1];
    acc += w2 * p[2];
    acc += w1 * p[3];
    acc += w0 * p[4];
    tmp[i] = acc;
  }
  __syncthreads();
  // vertical pass: region K, rounded to the storage type; the owned tile goes to memory
  TS* out = static_cast<TS*>(outp);
  for (int i = threadIdx.x; i < dh * dw; i += NT) {
    const int r = i / dw;
    const int c = i - r * dw;
    const int qy = min(max(oy[K] + r, 0), lh[K] - 1);
    const float* p = tmp + (2 * qy - 2 - oy[K - 1]) * dw + c;
    float acc = w0 * p[0];
    acc += w1 * p[dw];
    acc += w2 * p[2 * dw];
    acc += w1 * p[3 * dw];
    acc += w0 * p[4 * dw];
    const float v = Px<TS>::round(acc);
    if (K < NLEV) dst[i] = v;
    const int cx = c - offk, cy = r - offk;
    const int gx = ox[K] + c, gy = oy[K] + r;
    if (static_cast<unsigned>(cx) < static_cast<unsigned>(own_w) &&
        static_cast<unsigned>(cy) < static_cast<unsigned>(own_h) && gx < lw[K] && gy < lh[K])
      Px<TS>::st(out + static_cast<int64_t>(gy) * opitch + gx, v);
  }
}

// Levels 1..NLEV from region 0 in LDS; level k goes to out[k - 1].
template <typename TS, int NLEV, int TW, int TH, int NT>
__device__ __forceinline__ void chain_levels(float* lds, const int* ox, const int* oy, const int* lw, const int* lh,
                                             void* const* out, const int64_t* opitch) {
  chain_level<TS, NLEV, TW, TH, NT, 1>(lds, ox, oy, lw, lh, out[0], opitch[0]);
  if constexpr (NLEV >= 2) chain_level<TS, NLEV, TW, TH, NT, 2>(lds, ox, oy, lw, lh, out[1], opitch[1]);
  if constexpr (NLEV >= 3) chain_level<TS, NLEV, TW, TH, NT, 3>(lds, ox, oy, lw, lh, out[2], opitch[2]);
}

// Level sizes and region origins for deepest-level tile t of a w x h input.
template <int NLEV, int TW, int TH>
__device__ __forceinline__ void chain_geometry(int w, int h, int t, int* lw, int* lh, int* ox, int* oy) {
  lw[0] = w;
  lh[0] = h;
#pragma unroll
  for (int k = 1; k <= NLEV; ++k) {
    lw[k] = (lw[k - 1] + 1) / 2;
    lh[k] = (lh[k - 1] + 1) / 2;
  }
  const int ntx = (lw[NLEV] + TW - 1) / TW;
  ox[NLEV] = (t % ntx) * TW;
  oy[NLEV] = (t / ntx) * TH;
#pragma unroll
  for (int k = NLEV - 1; k >= 0; --k) {
    ox[k] = 2 * ox[k + 1] - 2;
    oy[k] = 2 * oy[k + 1] - 2;
  }
}

template <typename TS, int NLEV, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) void reduce_multi_kernel(const ReduceMArgs a) {
  using C = RChain<NLEV, TW, TH>;
  extern __shared__ float lds[];
  const ReduceMJob& J = a.job[find_job(a, blockIdx.x)];
  int lw[NLEV + 1], lh[NLEV + 1], ox[NLEV + 1], oy[NLEV + 1];
  chain_geometry<NLEV, TW, TH>(J.w, J.h, blockIdx.x - J.tile_start, lw, lh, ox, oy);
  // stage the input region (indices clamped into the input level)
  {
    constexpr int RW0 = C::rw(0);
    constexpr int N = RW0 * C::rh(0);
    constexpr int B = 8;
    const TS* in = static_cast<const TS*>(J.in);
    for (int i0 = threadIdx.x; i0 < N; i0 += B * NT) {
      float v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int i = min(i0 + u * NT, N - 1);
        const int r = i / RW0;
        const int c = i - r * RW0;
        const int gx = min(max(ox[0] + c, 0), lw[0] - 1);
        const int gy = min(max(oy[0] + r, 0), lh[0] - 1);
        v[u] = Px<TS>::ld(in + static_cast<int64_t>(gy) * J.in_pitch + gx);
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (i0 + u * NT < N) lds[i0 + u * NT] = v[u];
    }
  }
  chain_levels<TS, NLEV, TW, TH, NT>(lds, ox, oy, lw, lh, J.out, J.out_pitch);
}

template <typename TS, int NLEV, bool SMALL>
hipError_t launch_reduce_multi_typed(const ReduceMArgs& a, int nblocks, hipStream_t s) {
  constexpr int TW = reduce_multi_tw(NLEV, SMALL), TH = reduce_multi_th(NLEV, SMALL);
  constexpr int NT = reduce_multi_nt(NLEV, SMALL);
  constexpr size_t lds = sizeof(float) * RChain<NLEV, TW, TH>::LDS_FLOATS;
  auto kern = reduce_multi_kernel<TS, NLEV, TW, TH, NT>;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename TS>
hipError_t launch_reduce_multi_st(const ReduceMArgs& a, int nlev, bool small, int nblocks, hipStream_t s) {
  if (nlev == 2) return launch_reduce_multi_typed<TS, 2, false>(a, nblocks, s);
  if (nlev == 3)
    return small ? launch_reduce_multi_typed<TS, 3, true>(a, nblocks, s)
                 : launch_reduce_multi_typed<TS, 3, false>(a, nblocks, s);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_multi(const ReduceMArgs& a, int nlev, bool small, int nblocks, hipStream_t s) {
  switch (a.storage) {
    case ST_F32: return launch_reduce_multi_st<float>(a, nlev, small, nblocks, s);
    case ST_F16: return launch_reduce_multi_st<_Float16>(a, nlev, small, nblocks, s);
    default: return launch_reduce_multi_st<bf16_t>(a, nlev, small, nblocks, s);
  }
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

#define OFV_DECL(ST, MD) \
  hipError_t launch_gn_##ST##_##MD(const GnArgs& a, int kr, int nblocks, hipStream_t s, bool generic);
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
  hipError_t launch_gnt_##ST##_##MD(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s, bool generic); \
  int gn_band_per_cu_##ST##_##MD(int kr);
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

int gn_band_per_cu(int kr, int storage, int mode) {
#define OFV_OCC(ST)                                                \
  if (mode == FLOW_ZERO) return gn_band_per_cu_##ST##_zero(kr);     \
  if (mode == FLOW_DIRECT) return gn_band_per_cu_##ST##_direct(kr); \
  return gn_band_per_cu_##ST##_upsample(kr);
  if (storage == ST_F32) { OFV_OCC(f32) }
  if (storage == ST_F16) { OFV_OCC(f16) }
  OFV_OCC(bf16)
#undef OFV_OCC
}

hipError_t launch_gn(const GnArgs& a, int kr, int storage, int mode, int variant, int nblocks, hipStream_t s,
                     bool generic) {
  variant = gn_variant_for(variant, kr);
  if (variant != GN_MARCH) {
#define OFV_PICKT(ST)                                                                     \
  if (mode == FLOW_ZERO) return launch_gnt_##ST##_zero(a, kr, variant, nblocks, s, generic);     \
  if (mode == FLOW_DIRECT) return launch_gnt_##ST##_direct(a, kr, variant, nblocks, s, generic); \
  return launch_gnt_##ST##_upsample(a, kr, variant, nblocks, s, generic);
    if (storage == ST_F32) { OFV_PICKT(f32) }
    if (storage == ST_F16) { OFV_PICKT(f16) }
    OFV_PICKT(bf16)
#undef OFV_PICKT
  }
#define OFV_PICK(ST)                                                    \
  if (mode == FLOW_ZERO) return launch_gn_##ST##_zero(a, kr, nblocks, s, generic);     \
  if (mode == FLOW_DIRECT) return launch_gn_##ST##_direct(a, kr, nblocks, s, generic); \
  return launch_gn_##ST##_upsample(a, kr, nblocks, s, generic);
  if (storage == ST_F32) { OFV_PICK(f32) }
  if (storage == ST_F16) { OFV_PICK(f16) }
  OFV_PICK(bf16)
#undef OFV_PICK
}

}  // namespace ofv
