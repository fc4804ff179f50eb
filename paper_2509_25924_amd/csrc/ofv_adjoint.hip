// Point-wise pieces of the hand-written adjoint (reverse mode, float32),
// batched over the pairs of a backward call (one launch per stage, the pair in
// blockIdx.z or in a job table): the adjoint of the solve from stored window
// sums (store-all mode), the up-sampling of a level's input field and its
// transpose, the transpose of REDUCE (image pyramids and the initial-field
// restriction) and of the local z-score normalisation.  The iteration
// kernels proper (window sums, warps) are in ofv_adj_tile.h.
//
// Transposes are written as gathers: every output element collects the
// weights with which the forward's taps reach it, so no atomics are needed.
// Derivative conventions follow the forward formulas exactly: clamp passes
// the gradient where the coordinate lies inside [0, size - 1] (ends
// included), floor has zero derivative, and a tap repeated at the border
// receives both of its weights.
#include "ofv_adj_tile.h"

namespace ofv {

namespace {

constexpr int BX = 64, BY = 4;

dim3 grid3(int w, int h, int n) { return dim3((w + BX - 1) / BX, (h + BY - 1) / BY, n); }

__device__ __forceinline__ bool pix(int& x, int& y, int w, int h) {
  x = blockIdx.x * BX + (threadIdx.x & 63);
  y = blockIdx.y * BY + (threadIdx.x >> 6);
  return x < w && y < h;
}

// ---------------------------------------------------------------- solve adjoint from stored sums

__global__ __launch_bounds__(256) void k_solve_stored(const AdjArgs a) {
  const AdjJob& J = a.job[find_job(a, blockIdx.x)];
  const int nbx = (J.w + BX - 1) / BX;
  const int b = blockIdx.x - J.tile_start;
  const int x = (b % nbx) * BX + (threadIdx.x & 63);
  const int y = (b / nbx) * BY + (threadIdx.x >> 6);
  if (x >= J.w || y >= J.h) return;
  const float* r = J.st + y * J.stp + x;
  float g5[5], du, dv;
  solve_adj(r[0], r[J.sts], r[2 * J.sts], r[3 * J.sts], r[4 * J.sts], J.vu[y * J.vp + x], J.vv[y * J.vp + x],
            J.gu[y * J.gp + x], J.gv[y * J.gp + x], a.reg_rel, a.reg_abs, g5, du, dv);
  float* o = J.gA + y * J.sp + x;
#pragma unroll
  for (int q = 0; q < 5; ++q) o[q * J.ps] = g5[q];
  o[5 * J.ps] = du;
  o[6 * J.ps] = dv;
}

// ---------------------------------------------------------------- up-sampling and its transpose

// V_fine(X) = 2 bilinear(V_coarse, X / 2), the forward kernels' arithmetic.
__global__ __launch_bounds__(256) void k_upsample(const AuxArgs a) {
  const AuxJob& J = a.job[blockIdx.z];
  int x, y;
  if (!pix(x, y, J.w, J.h)) return;
  const uint32_t cp = static_cast<uint32_t>(J.ip);
  const PlaneView cu = plane_view(J.in0, cp * static_cast<uint32_t>(J.ch) * 4u);
  const PlaneView cv = plane_view(J.in1, cp * static_cast<uint32_t>(J.ch) * 4u);
  const float cwm1 = static_cast<float>(J.cw - 1), chm1 = static_cast<float>(J.ch - 1);
  const float cwm2 = static_cast<float>(J.cw - 2), chm2 = static_cast<float>(J.ch - 2);
  const uint32_t sx = J.cw > 1 ? 1u : 0u, sy = J.ch > 1 ? cp : 0u;
  const float fx = 0.5f * static_cast<float>(x), fy = 0.5f * static_cast<float>(y);
  J.out0[y * J.op + x] = 2.0f * adj_bil(cu, fx, fy, cwm1, chm1, cwm2, chm2, cp, sx, sy);
  J.out1[y * J.op + x] = 2.0f * adj_bil(cv, fx, fy, cwm1, chm1, cwm2, chm2, cp, sx, sy);
}

// weight with which fine coordinate X (sampled at X / 2, clamped) reaches coarse index i
__device__ __forceinline__ float up_weight(int X, int i, int cw) {
  const float xc = fminf(0.5f * static_cast<float>(X), static_cast<float>(cw - 1));
  const float xf = floorf(xc);
  const float f = xc - xf;
  const int i0 = static_cast<int>(xf);
  const int i1 = min(i0 + 1, cw - 1);
  return (i0 == i ? 1.0f - f : 0.0f) + (i1 == i ? f : 0.0f);
}

// coarse (i, j) <- sum over fine (X, Y) with X in [2i - 2, 2i + 2] of 2 w(X, i) w(Y, j) g(X, Y)
__global__ __launch_bounds__(256) void k_upsample_adj(const AuxArgs a) {
  const AuxJob& J = a.job[blockIdx.z];
  int i, j;
  if (!pix(i, j, J.cw, J.ch)) return;
  const int xa = max(2 * i - 2, 0), xb = min(2 * i + 2, J.w - 1);
  const int ya = max(2 * j - 2, 0), yb = min(2 * j + 2, J.h - 1);
  float su = 0.0f, sv = 0.0f;
  for (int Y = ya; Y <= yb; ++Y) {
    const float wy = up_weight(Y, j, J.ch);
    if (wy == 0.0f) continue;
    float ru = 0.0f, rv = 0.0f;
    for (int X = xa; X <= xb; ++X) {
      const float wx = up_weight(X, i, J.cw);
      ru += wx * J.in0[Y * J.ip + X];
      rv += wx * J.in1[Y * J.ip + X];
    }
    su += wy * ru;
    sv += wy * rv;
  }
  J.out0[j * J.op + i] = 2.0f * su;
  J.out1[j * J.op + i] = 2.0f * sv;
}

// ---------------------------------------------------------------- REDUCE transposed

// weight with which coarse index xc's clamped tap 2 xc + k (k = -2..2) reaches fine X
__device__ __forceinline__ float reduce_t_weight(int X, int xc, int w) {
  const float w5[5] = {1.0f / 16, 4.0f / 16, 6.0f / 16, 4.0f / 16, 1.0f / 16};
  float s = 0.0f;
#pragma unroll
  for (int i = -2; i <= 2; ++i)
    if (min(max(2 * xc + i, 0), w - 1) == X) s += w5[i + 2];
  return s;
}

// Fine index X is reached only from coarse indices X/2 - 1 .. X/2 + 1
// (rounded down; the end indices collect the taps clamped onto them too):
// their summed weights, 0 for indices outside the coarse plane.
__device__ __forceinline__ void reduce_t_taps(int X, int w, int cw, int* xc, float* wt) {
  const int c = X >> 1;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int k = c - 1 + i;
    const bool in = k >= 0 && k < cw;
    xc[i] = in ? k : 0;
    wt[i] = in ? reduce_t_weight(X, k, w) : 0.0f;
  }
}

// fine (x, y) <- scale * sum over coarse neighbours of w(x) w(y) g_coarse; in0 coarse (pitch ip), out0 fine
__global__ __launch_bounds__(256) void k_reduce_adj(const AuxArgs a) {
  const AuxJob& J = a.job[blockIdx.z];
  int x, y;
  if (!pix(x, y, J.w, J.h)) return;
  int xc[3], yc[3];
  float wx[3], wy[3];
  reduce_t_taps(x, J.w, J.cw, xc, wx);
  reduce_t_taps(y, J.h, J.ch, yc, wy);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float* row = J.in0 + yc[j] * J.ip;
    s += wy[j] * (wx[0] * row[xc[0]] + wx[1] * row[xc[1]] + wx[2] * row[xc[2]]);
  }
  s *= a.scale;
  float* dst = J.out0 + y * J.op + x;
  *dst = a.accumulate ? *dst + s : s;
}

// both planes of every job's field set to zero over w x h (pitch op)
__global__ __launch_bounds__(256) void k_zero_fields(const AuxArgs a) {
  const AuxJob& J = a.job[blockIdx.z];
  int x, y;
  if (!pix(x, y, J.w, J.h)) return;
  J.out0[y * J.op + x] = 0.0f;
  J.out1[y * J.op + x] = 0.0f;
}

__global__ __launch_bounds__(256) void k_fill(float* p, int64_t n, float v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- normalisation adjoint
// N_k = (I_k - mu_k) / sig_k, sig_k = sqrt(var_k + eps) over the truncated
// window Omega_k (symmetric: j in Omega_k iff k in Omega_j).  With
// a_k = gN_k / (n_k sig_k), c_k = gN_k (I_k - mu_k) / (n_k sig_k^3):
//   gI_j = gN_j / sig_j - sum_{k in Omega_j} a_k - I_j sum c_k + sum c_k mu_k.

__device__ __forceinline__ float frame_px(const ImageIn& f, int x, int y) {
  const int64_t o = static_cast<int64_t>(y) * f.pitch + x;
  if (f.type == 0) return static_cast<float>(static_cast<const uint8_t*>(f.data)[o]) / static_cast<float>((1 << f.bits) - 1);
  if (f.type == 1) return static_cast<float>(static_cast<const uint16_t*>(f.data)[o]) / static_cast<float>((1 << f.bits) - 1);
  return static_cast<const float*>(f.data)[o];
}

__device__ __forceinline__ float frame_scale(const ImageIn& f) {
  return f.type == 2 ? 1.0f : 1.0f / static_cast<float>((1 << f.bits) - 1);
}

// One 64 x 16 tile of frame gradients per workgroup (job = blockIdx.z), all
// in LDS: the frame over the tile + 2 NR, then for every pixel k of the tile
// + NR its window mean and deviation and a_k, c_k, c_k mu_k, their window
// sums (horizontal pass, then vertical per output), and the output.
constexpr int kNAdjTW = 64, kNAdjTH = 16;

__host__ __device__ constexpr int norm_adj_lds_floats(int nr) {
  return (kNAdjTW + 4 * nr) * (kNAdjTH + 4 * nr) + 4 * (kNAdjTW + 2 * nr) * (kNAdjTH + 2 * nr) +
         kNAdjTW * kNAdjTH + 3 * (kNAdjTH + 2 * nr) * kNAdjTW;
}

// NRC > 0: the radius as a compile-time constant (loops unrolled); 0: a.nr
template <int NRC>
__global__ __launch_bounds__(256) void k_norm_adj_tile(const NormAdjArgs a) {
  extern __shared__ float lds[];
  const NormAdjJob& J = a.job[blockIdx.z];
  const ImageIn& f = J.f;
  const int W = f.w, H = f.h, nr = NRC > 0 ? NRC : a.nr;
  const int ntx = (W + kNAdjTW - 1) / kNAdjTW;
  const int t = blockIdx.x;
  if (t >= ntx * ((H + kNAdjTH - 1) / kNAdjTH)) return;
  const int x0 = (t % ntx) * kNAdjTW, y0 = (t / ntx) * kNAdjTH;
  const int FW = kNAdjTW + 4 * nr, FH = kNAdjTH + 4 * nr;  // frame region, origin (x0 - 2 nr, y0 - 2 nr)
  const int KW = kNAdjTW + 2 * nr, KH = kNAdjTH + 2 * nr;  // window-term region, origin (x0 - nr, y0 - nr)
  float* sF = lds;
  float* sA = sF + FW * FH;          // a, c, c mu: three KW x KH planes
  float* sG = sA + 3 * KW * KH;      // dL/dN over the window-term region
  float* sSig = sG + KW * KH;        // sigma of the tile pixels
  float* sH = sSig + kNAdjTW * kNAdjTH;  // horizontal sums: three KH x 64 planes
  const int tid = threadIdx.x;
  // the frame and dL/dN; with the radius known at compile time every load of
  // the lane is issued (at a clamped address) before any is stored
  if (NRC > 0) {
    constexpr int NF = ((kNAdjTW + 4 * NRC) * (kNAdjTH + 4 * NRC) + 255) / 256;
    constexpr int NG = ((kNAdjTW + 2 * NRC) * (kNAdjTH + 2 * NRC) + 255) / 256;
    float fv[NF], gv[NG];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int e = min(tid + 256 * k, FW * FH - 1);
      const int fy = e / FW, fx = e - fy * FW;
      fv[k] = frame_px(f, min(max(x0 - 2 * nr + fx, 0), W - 1), min(max(y0 - 2 * nr + fy, 0), H - 1));
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int e = min(tid + 256 * k, KW * KH - 1);
      const int ky = e / KW, kx = e - ky * KW;
      gv[k] = J.gN[min(max(y0 - nr + ky, 0), H - 1) * J.gp + min(max(x0 - nr + kx, 0), W - 1)];
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int e = tid + 256 * k;
      if (e < FW * FH) {
        const int fy = e / FW, fx = e - fy * FW;
        const int gx = x0 - 2 * nr + fx, gy = y0 - 2 * nr + fy;
        const bool in = static_cast<unsigned>(gx) < static_cast<unsigned>(W) &&
                        static_cast<unsigned>(gy) < static_cast<unsigned>(H);
        sF[e] = in ? fv[k] : 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int e = tid + 256 * k;
      if (e < KW * KH) sG[e] = gv[k];
    }
  } else {
    for (int e = tid; e < FW * FH; e += 256) {
      const int fy = e / FW, fx = e - fy * FW;
      const int gx = x0 - 2 * nr + fx, gy = y0 - 2 * nr + fy;
      const bool in = static_cast<unsigned>(gx) < static_cast<unsigned>(W) && static_cast<unsigned>(gy) < static_cast<unsigned>(H);
      sF[e] = in ? frame_px(f, gx, gy) : 0.0f;
    }
    for (int e = tid; e < KW * KH; e += 256) {
      const int ky = e / KW, kx = e - ky * KW;
      const int gx = min(max(x0 - nr + kx, 0), W - 1), gy = min(max(y0 - nr + ky, 0), H - 1);
      sG[e] = J.gN[gy * J.gp + gx];
    }
  }
  __syncthreads();
  for (int e = tid; e < KW * KH; e += 256) {
    const int ky = e / KW, kx = e - ky * KW;
    const int gx = x0 - nr + kx, gy = y0 - nr + ky;
    float pa = 0.0f, pc = 0.0f, pcm = 0.0f;
    if (static_cast<unsigned>(gx) < static_cast<unsigned>(W) && static_cast<unsigned>(gy) < static_cast<unsigned>(H)) {
      const int xa = max(gx - nr, 0), xb = min(gx + nr, W - 1), ya = max(gy - nr, 0), yb = min(gy + nr, H - 1);
      const float n = static_cast<float>((xb - xa + 1) * (yb - ya + 1));
      float mu, q;
      if (NRC > 0) {
        // the full window, unrolled: the frame region holds 0 outside the
        // frame, and the masks keep those pixels out of the deviations
        constexpr int NC = 2 * NRC + 1;
        float v[NC][NC], mk[NC][NC];
        float sm = 0.0f;
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            v[j][i] = sF[(ky + j) * FW + kx + i];
            mk[j][i] = (static_cast<unsigned>(gx - NRC + i) < static_cast<unsigned>(W) &&
                        static_cast<unsigned>(gy - NRC + j) < static_cast<unsigned>(H)) ? 1.0f : 0.0f;
            sm += v[j][i];
          }
        mu = sm / n;
        q = 0.0f;
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            const float d = v[j][i] - mu;
            q += mk[j][i] * (d * d);
          }
      } else {
        // frame-region coordinates of (xa, ya)
        const int ox = xa - (x0 - 2 * nr), oy = ya - (y0 - 2 * nr);
        float sm = 0.0f;
        for (int j = 0; j <= yb - ya; ++j)
          for (int i = 0; i <= xb - xa; ++i) sm += sF[(oy + j) * FW + ox + i];
        mu = sm / n;
        q = 0.0f;
        for (int j = 0; j <= yb - ya; ++j)
          for (int i = 0; i <= xb - xa; ++i) {
            const float d = sF[(oy + j) * FW + ox + i] - mu;
            q += d * d;
          }
      }
      const float sg = sqrtf(q / n + a.eps);
      const float ik = sF[(ky + nr) * FW + kx + nr];
      const float g = sG[e];
      pa = g / (n * sg);
      pc = g * (ik - mu) / (n * sg * sg * sg);
      pcm = pc * mu;
      if (kx >= nr && kx < nr + kNAdjTW && ky >= nr && ky < nr + kNAdjTH) sSig[(ky - nr) * kNAdjTW + kx - nr] = sg;
    }
    sA[e] = pa;
    sA[KW * KH + e] = pc;
    sA[2 * KW * KH + e] = pcm;
  }
  __syncthreads();
  for (int e = tid; e < KH * kNAdjTW; e += 256) {
    const int r = e / kNAdjTW, c = e - r * kNAdjTW;
    for (int q = 0; q < 3; ++q) {
      const float* row = sA + q * KW * KH + r * KW + c;
      float acc = 0.0f;
      for (int i = 0; i <= 2 * nr; ++i) acc += row[i];
      sH[q * KH * kNAdjTW + e] = acc;
    }
  }
  __syncthreads();
  for (int e = tid; e < kNAdjTW * kNAdjTH; e += 256) {
    const int ty = e / kNAdjTW, tx = e - ty * kNAdjTW;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx >= W || gy >= H) continue;
    float b[3];
    for (int q = 0; q < 3; ++q) {
      const float* col = sH + q * KH * kNAdjTW + ty * kNAdjTW + tx;
      float acc = 0.0f;
      for (int j = 0; j <= 2 * nr; ++j) acc += col[j * kNAdjTW];
      b[q] = acc;
    }
    const float ij = sF[(ty + 2 * nr) * FW + tx + 2 * nr];
    const float g = sG[(ty + nr) * KW + tx + nr] / sSig[e] - b[0] - ij * b[1] + b[2];
    J.gF[gy * J.fp + gx] = g * frame_scale(f);
  }
}

// NR 0: N = I, so the frame gradient is the level-0 gradient in the frame's units
__global__ __launch_bounds__(256) void k_norm_scale(const NormAdjArgs a) {
  const NormAdjJob& J = a.job[blockIdx.z];
  int x, y;
  if (!pix(x, y, J.f.w, J.f.h)) return;
  J.gF[y * J.fp + x] = J.gN[y * J.gp + x] * frame_scale(J.f);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

int adj_point_blocks(int w, int h) { return ((w + BX - 1) / BX) * ((h + BY - 1) / BY); }

hipError_t launch_adj_solve_stored(const AdjArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve_stored, dim3(nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_upsample_batch(const AuxArgs& a, int maxw, int maxh, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upsample, grid3(maxw, maxh, a.njobs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_upsample_adj(const AuxArgs& a, int maxcw, int maxch, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_upsample_adj, grid3(maxcw, maxch, a.njobs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_fields(const AuxArgs& a, int maxw, int maxh, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_fields, grid3(maxw, maxh, a.njobs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_adj(const AuxArgs& a, int maxw, int maxh, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_adj, grid3(maxw, maxh, a.njobs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_norm_adj(const NormAdjArgs& a, int maxw, int maxh, hipStream_t s) {
  if (a.njobs <= 0) return hipSuccess;
  if (a.nr <= 0) {
    hipLaunchKernelGGL(k_norm_scale, grid3(maxw, maxh, a.njobs), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  const int tiles = ((maxw + kNAdjTW - 1) / kNAdjTW) * ((maxh + kNAdjTH - 1) / kNAdjTH);
  const size_t lds = sizeof(float) * norm_adj_lds_floats(a.nr);
  const dim3 g(tiles, 1, a.njobs);
  if (a.nr == 1) {
    hipLaunchKernelGGL(k_norm_adj_tile<1>, g, dim3(256), lds, s, a);
  } else if (a.nr == 2) {
    hipLaunchKernelGGL(k_norm_adj_tile<2>, g, dim3(256), lds, s, a);
  } else {
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(k_norm_adj_tile<0>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       static_cast<int>(sizeof(float) * norm_adj_lds_floats(kMaxNR)));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_norm_adj_tile<0>, g, dim3(256), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace ofv
