// Adjoint (reverse mode) of one symmetric Gauss-Newton iteration as two tile
// kernels: pipeline steps 3 and 5 of section "Live-Optical Flow Velocimetry",
// Eq. of_symmetric, arXiv 2509.25924.
//
// Forward of one iteration, per pixel k: W0 = P0(k - V/2), W1 = P1(k + V/2)
// (bilinear, clamped), S = (W0 + W1)/2, T = W1 - W0, G = central difference
// of S (clamped indices), b = G . V(k) - T, products p = (Gx^2, GxGy, Gy^2,
// Gx b, Gy b); per pixel m, A = the window sums of p over the truncated
// (2KR+1)^2 window; lam = reg_rel (Axx + Ayy) + reg_abs; (A + lam I) V'(m) =
// c + lam V(m).
//
// adj_sums_kernel recomputes S, T, G, b, the products and the window sums of
// a 64 x 16 tile in LDS (the same steps as the forward's tile kernel) and
// applies the adjoint of the damped solve: dL/dA (5 planes) and the direct
// gradient lam z w.r.t. V(m) (2 planes) go to HBM.  With the record epilogue
// the same kernel is the forward iteration of the store-all mode: it solves
// and also stores the sums and Gx, Gy, b of every pixel.
//
// adj_scatter_kernel takes dL/dA over the tile plus a (KR+1)-pixel halo and
// forms its window sums in LDS (a truncated box is its own transpose), then,
// over the tile plus a one-pixel ring, the adjoints of the products and of b
// (dL/dG, dL/db); per output pixel, the transposed central difference gives
// dL/dS, which with dL/dT = -dL/db gives the gradients of the two warped
// samples; their sub-pixel derivatives give dL/dV, and their tap weights
// scatter them into the image gradients with global float atomics.  A lane
// walks down a column of the tile and a wavefront spans a tile row, so the
// taps that neighbouring pixels share (the lower row of one pixel's taps is
// usually the upper row of the next pixel's, the right column of one lane's
// the left column of the next lane's) are summed in registers and across
// lanes first: about one atomic per pixel and image instead of four.  (Float
// atomics on LDS proved several times slower than this on gfx950.)
//
// Derivative conventions follow the forward formulas: clamping passes the
// gradient where the coordinate lies inside [0, size - 1] (ends included),
// floor has zero derivative, and a tap repeated at the border receives both
// of its weights.
#pragma once

#include "ofv_adj.h"
#include "ofv_gn_tile.h"

namespace ofv {

constexpr int adj_cmax(int a, int b) { return a > b ? a : b; }

// Bilinear sample of a float plane at (x, y) clamped into W x H (the forward
// kernels' arithmetic); sx / sy: the second tap's offset in x / y, 0 for a
// single-column / single-row plane.
__device__ __forceinline__ float adj_bil(PlaneView v, float x, float y, float wm1, float hm1, float wm2, float hm2,
                                         uint32_t pitch, uint32_t sx, uint32_t sy) {
  const BilTap t = bil_setup(x, y, wm1, hm1, wm2, hm2, pitch);
  return bil_combine(ld_f32(v, t.i), ld_f32(v, t.i + sx), ld_f32(v, t.i + sy), ld_f32(v, t.i + sy + sx), t.ax, t.ay);
}

// Flow and the two midpoint warps W0 = P0(k - V/2), W1 = P1(k + V/2) of N
// pixels at level coordinates (px[c], py[c]) inside the level: the flow loads
// of all N are issued first, then their 8 N image taps, then the
// combinations, so that the loads of the N pixels are in flight together.
template <int N>
__device__ __forceinline__ void warp_pixels(const int* px, const int* py, PlaneView fu, PlaneView fv, uint32_t vp,
                                            PlaneView i0, PlaneView i1, uint32_t ip, uint32_t sx, uint32_t sy,
                                            float wm1, float hm1, float wm2, float hm2, float* u, float* v,
                                            float* w0, float* w1) {
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const uint32_t o = static_cast<uint32_t>(py[c]) * vp + static_cast<uint32_t>(px[c]);
    u[c] = ld_f32(fu, o);
    v[c] = ld_f32(fv, o);
  }
  BilTap a[N], b[N];
  float t[N][8];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const float fx = static_cast<float>(px[c]), fy = static_cast<float>(py[c]);
    a[c] = bil_setup(fx - 0.5f * u[c], fy - 0.5f * v[c], wm1, hm1, wm2, hm2, ip);
    b[c] = bil_setup(fx + 0.5f * u[c], fy + 0.5f * v[c], wm1, hm1, wm2, hm2, ip);
    t[c][0] = ld_f32(i0, a[c].i);
    t[c][1] = ld_f32(i0, a[c].i + sx);
    t[c][2] = ld_f32(i0, a[c].i + sy);
    t[c][3] = ld_f32(i0, a[c].i + sy + sx);
    t[c][4] = ld_f32(i1, b[c].i);
    t[c][5] = ld_f32(i1, b[c].i + sx);
    t[c][6] = ld_f32(i1, b[c].i + sy);
    t[c][7] = ld_f32(i1, b[c].i + sy + sx);
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    w0[c] = bil_combine(t[c][0], t[c][1], t[c][2], t[c][3], a[c].ax, a[c].ay);
    w1[c] = bil_combine(t[c][4], t[c][5], t[c][6], t[c][7], b[c].ax, b[c].ay);
  }
}

// Adjoint of the damped solve x = M^-1 r, M = [[Axx + lam, Axy], [Axy, Ayy +
// lam]], r = (Axb + lam um, Ayb + lam vm), lam = reg_rel (Axx + Ayy) +
// reg_abs, for dL/dx = (gu, gv): z = M^-1 (gu, gv) (M is symmetric), dL/dM =
// -z x^T, dL/dr = z.  Writes dL/dA (five values) and the direct gradient
// w.r.t. (um, vm).  Ill-conditioned systems (4 det / trace^2 < 1e-2) are
// solved in float64 from the same float32 sums, as in the forward.
__device__ __forceinline__ void solve_adj(float sxx, float sxy, float syy, float sxb, float syb, float um, float vm,
                                          float gu, float gv, float reg_rel, float reg_abs, float* gA, float& du,
                                          float& dv) {
  const float lam = reg_rel * (sxx + syy) + reg_abs;
  const float aa = sxx + lam, dd = syy + lam;
  const float r1 = sxb + lam * um, r2 = syb + lam * vm;
  const float det = aa * dd - sxy * sxy;
  const float tr = aa + dd;
  float xu, xv, z1, z2;
  if (det >= 2.5e-3f * tr * tr) {
    float inv = __builtin_amdgcn_rcpf(det);
    inv = fmaf(inv, fmaf(-det, inv, 1.0f), inv);
    xu = (dd * r1 - sxy * r2) * inv;
    xv = (aa * r2 - sxy * r1) * inv;
    z1 = (dd * gu - sxy * gv) * inv;
    z2 = (aa * gv - sxy * gu) * inv;
  } else {
    const double a = aa, d = dd, b = sxy;
    const double dt = a * d - b * b;
    xu = static_cast<float>((d * r1 - b * r2) / dt);
    xv = static_cast<float>((a * r2 - b * r1) / dt);
    z1 = static_cast<float>((d * gu - b * gv) / dt);
    z2 = static_cast<float>((a * gv - b * gu) / dt);
  }
  const float g_aa = -z1 * xu, g_dd = -z2 * xv;
  const float g_lam = z1 * um + z2 * vm + g_aa + g_dd;
  gA[0] = g_aa + reg_rel * g_lam;
  gA[1] = -(z1 * xv + z2 * xu);
  gA[2] = g_dd + reg_rel * g_lam;
  gA[3] = z1;
  gA[4] = z2;
  du = lam * z1;
  dv = lam * z2;
}

// ---------------------------------------------------------------- window sums + solve adjoint

template <int KR, int TX, int TY>
struct AdjSumsGeom {
  static constexpr int EX = TX + 2 * KR + 2;  // S region: product region + 1 on each side
  static constexpr int EY = TY + 2 * KR + 2;
  static constexpr int LP = EX | 1;
  static constexpr int PY = TY + 2 * KR;      // product rows
  static constexpr int NE = EX * EY;
  static constexpr int PLANE = LP * EY;
  static constexpr int CP = PY | 1;           // column pitch of the transposed horizontal sums
  static constexpr int HPL = TX * CP;
  static_assert(HPL <= PLANE, "transposed sums fit in a product plane");
  static constexpr int FLOATS = 6 * PLANE;    // S, then five product planes
};

template <int KR, int TX, int TY, int SL, int SLV, int NT, int EPI>
__global__ __launch_bounds__(NT) void adj_sums_kernel(const AdjArgs a) {
  using G = AdjSumsGeom<KR, TX, TY>;
  constexpr int EX = G::EX, EY = G::EY, LP = G::LP, PY = G::PY, PL = G::PLANE, NE = G::NE, CP = G::CP;
  constexpr int HPL = G::HPL;
  constexpr int NWIN = 2 * KR + 1;
  constexpr int NSEG = TX / SL;
  constexpr int NIT = (NSEG * PY + NT - 1) / NT;
  constexpr int NA = (NE + NT - 1) / NT;
  static_assert(TX % SL == 0 && TY % SLV == 0 && TX * (TY / SLV) <= NT, "segments must tile the output");
  extern __shared__ float lds[];
  float* sS = lds;
  float* sP = lds + PL;

  const AdjJob& J = a.job[find_job(a, blockIdx.x)];
  const int W = J.w, H = J.h;
  const int ntx = (W + TX - 1) / TX;
  const int t = xcd_tile(blockIdx.x - J.tile_start, ntx * ((H + TY - 1) / TY));
  const int x0 = (t % ntx) * TX, y0 = (t / ntx) * TY;
  const int gx0 = x0 - KR - 1, gy0 = y0 - KR - 1;  // level coordinates of ext (0, 0)
  const int tid = threadIdx.x;
  const float wm1 = static_cast<float>(W - 1), hm1 = static_cast<float>(H - 1);
  const float wm2 = static_cast<float>(W - 2), hm2 = static_cast<float>(H - 2);
  const uint32_t ip = static_cast<uint32_t>(J.ip), vp = static_cast<uint32_t>(J.vp);
  const PlaneView i0 = plane_view(J.p0, ip * static_cast<uint32_t>(H) * 4u);
  const PlaneView i1 = plane_view(J.p1, ip * static_cast<uint32_t>(H) * 4u);
  const PlaneView fu = plane_view(J.vu, vp * static_cast<uint32_t>(H) * 4u);
  const PlaneView fv = plane_view(J.vv, vp * static_cast<uint32_t>(H) * 4u);
  const uint32_t sx = W > 1 ? 1u : 0u, sy = H > 1 ? ip : 0u;

  // ---- A1: flow and the two warps over the ext region, evaluated at the
  // coordinates clamped into the level (out-of-level ext pixels repeat their
  // clamped neighbour, so the central differences below reproduce the
  // clamped-index gradient); S -> LDS, T and V stay in the lane's registers.
  float kT[NA], kU[NA], kV[NA];
  {
    constexpr int CH = NA < 8 ? NA : 8;
#pragma unroll
    for (int k0 = 0; k0 < NA; k0 += CH) {
      int px[CH], py[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int e = min(tid + NT * (k0 + c), NE - 1);  // pixels past the region: a dummy, discarded
        const int ey = e / EX, ex = e - ey * EX;
        px[c] = min(max(gx0 + ex, 0), W - 1);
        py[c] = min(max(gy0 + ey, 0), H - 1);
      }
      float u[CH], v[CH], w0[CH], w1[CH];
      warp_pixels<CH>(px, py, fu, fv, vp, i0, i1, ip, sx, sy, wm1, hm1, wm2, hm2, u, v, w0, w1);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (k0 + c < NA) {
          const int e = tid + NT * (k0 + c);
          kT[k0 + c] = w1[c] - w0[c];
          kU[k0 + c] = u[c];
          kV[k0 + c] = v[c];
          if (e < NE) {
            const int ey = e / EX, ex = e - ey * EX;
            sS[ey * LP + ex] = 0.5f * (w0[c] + w1[c]);
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- A2: G, b and the five products over the product region (0 outside the level)
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    const int e = tid + NT * k;
    if (e < NE) {
      const int ey = e / EX, ex = e - ey * EX;
      if (ex >= 1 && ex < EX - 1 && ey >= 1 && ey < EY - 1) {
        const int lx = gx0 + ex, ly = gy0 + ey;
        const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                         static_cast<unsigned>(ly) < static_cast<unsigned>(H);
        const int o = ey * LP + ex;
        float gx = 0.0f, gy = 0.0f, b = 0.0f;
        if (inl) {
          gx = 0.5f * (sS[o + 1] - sS[o - 1]);
          gy = 0.5f * (sS[o + LP] - sS[o - LP]);
          b = fmaf(gx, kU[k], fmaf(gy, kV[k], -kT[k]));
        }
        sP[o] = gx * gx;
        sP[o + PL] = gx * gy;
        sP[o + 2 * PL] = gy * gy;
        sP[o + 3 * PL] = gx * b;
        sP[o + 4 * PL] = gy * b;
        if (EPI == ADJ_RECORD && inl && static_cast<unsigned>(ex - 1 - KR) < static_cast<unsigned>(TX) &&
            static_cast<unsigned>(ey - 1 - KR) < static_cast<unsigned>(TY)) {
          float* r = J.st + ly * J.stp + lx;
          r[5 * J.sts] = gx;
          r[6 * J.sts] = gy;
          r[7 * J.sts] = b;
        }
      }
    }
  }
  __syncthreads();

  // ---- B: horizontal window sums per (product row, segment of SL outputs),
  // running sums kept in registers, then written transposed over the products
  float hsum[NIT][5][SL];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * PY) {
      const int rb = (item % PY + 1) * LP + 1 + (item / PY) * SL;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float* row = sP + lds_reg(q * PL + rb);
        float ring[NWIN];
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < SL + 2 * KR; ++k) {
          const float pq = row[k];
          if (k >= NWIN) acc -= ring[k % NWIN];
          ring[k % NWIN] = pq;
          acc = k == 0 ? pq : acc + pq;
          if (k >= 2 * KR) hsum[it][q][k - 2 * KR] = acc;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * PY) {
      const int cb = (item / PY) * SL * CP + item % PY;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float* col = sP + lds_reg(q * HPL + cb);
#pragma unroll
        for (int jj = 0; jj < SL; ++jj) col[jj * CP] = hsum[it][q][jj];
      }
    }
  }
  __syncthreads();

  // ---- C: vertical window sums per (output column, segment of SLV rows), then the epilogue
  const int j = tid % TX;
  const int sg = tid / TX;
  const int gx = x0 + j;
  if (sg < TY / SLV && gx < W) {
    const int rs = sg * SLV;
    float um[SLV], vm[SLV], gu[SLV], gv[SLV];
#pragma unroll
    for (int k = 0; k < SLV; ++k) {
      const int gy = min(y0 + rs + k, H - 1);
      const uint32_t o = static_cast<uint32_t>(gy) * vp + static_cast<uint32_t>(gx);
      um[k] = ld_f32(fu, o);
      vm[k] = ld_f32(fv, o);
      if (EPI == ADJ_SOLVE) {
        gu[k] = J.gu[gy * J.gp + gx];
        gv[k] = J.gv[gy * J.gp + gx];
      }
    }
    const float* col[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) col[q] = sP + lds_reg(q * HPL + j * CP + rs);
    float ring[5][NWIN];
    float acc[5];
#pragma unroll
    for (int k = 0; k < SLV + 2 * KR; ++k) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float hq = col[q][k];
        if (k >= NWIN) acc[q] -= ring[q][k % NWIN];
        ring[q][k % NWIN] = hq;
        acc[q] = k == 0 ? hq : acc[q] + hq;
      }
      if (k >= 2 * KR) {
        const int kk = k - 2 * KR;
        const int gy = y0 + rs + kk;
        if (gy < H) {
          if (EPI == ADJ_SOLVE) {
            float g5[5], du, dv;
            solve_adj(acc[0], acc[1], acc[2], acc[3], acc[4], um[kk], vm[kk], gu[kk], gv[kk], a.reg_rel, a.reg_abs,
                      g5, du, dv);
            float* o = J.gA + gy * J.sp + gx;
#pragma unroll
            for (int q = 0; q < 5; ++q) o[q * J.ps] = g5[q];
            o[5 * J.ps] = du;
            o[6 * J.ps] = dv;
          } else {
            float un, vn;
            solve2x2(acc[0], acc[1], acc[2], acc[3], acc[4], um[kk], vm[kk], a.reg_rel, a.reg_abs, un, vn, false,
                     a.no_fp64 != 0);
            J.ou[gy * J.op + gx] = un;
            J.ov[gy * J.op + gx] = vn;
            float* r = J.st + gy * J.stp + gx;
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q * J.sts] = acc[q];
          }
        }
      }
    }
  }
}

// TY 16 for large launches; TY 8 spreads small ones (coarse levels) over twice the workgroups
template <int KR, int EPI, int TY>
hipError_t launch_adj_sums_cfg(const AdjArgs& a, int nblocks, hipStream_t s) {
  constexpr int TX = 64;
  constexpr size_t lds = sizeof(float) * AdjSumsGeom<KR, TX, TY>::FLOATS;
  auto kern = adj_sums_kernel<KR, TX, TY, 8, TY == 16 ? 4 : 2, 256, EPI>;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- box of dL/dA + products, b, warps adjoint

template <int KR, int TX, int TY, int SL, int SLV, bool STORED>
struct AdjScatGeom {
  static constexpr int RWV = TX + 2, RHV = TY + 2;           // the tile plus a one-pixel ring ("ring region")
  static constexpr int RW = (RWV + SL - 1) / SL * SL;        // ... padded to whole segments
  static constexpr int RH = (RHV + SLV - 1) / SLV * SLV;
  static constexpr int QW = RW + 2 * KR, QY = RH + 2 * KR;   // dL/dA region
  static constexpr int QL = QW | 1;
  static constexpr int CPH = QY | 1;                         // column pitch of the transposed horizontal sums
  static constexpr int QS = adj_cmax(QL * QY, RW * CPH);     // plane stride of the dL/dA (then sums) planes
  static constexpr int SW = TX + 4, SH = TY + 4, SP = SW | 1;  // S region: the ring region + 1
  static constexpr int R1L = RWV | 1;                        // pitch of the ring planes
  static constexpr int R1S = R1L * RHV;
  static constexpr int S_OFF = 5 * QS;
  static constexpr int R_OFF = S_OFF + (STORED ? 0 : SP * SH);
  static constexpr int FLOATS = R_OFF + 5 * R1S;
};

// One bilinear sample of p at (x, y) with the forward's clamping, for its
// adjoint: the four tap positions and weights, and the derivatives of the
// sample w.r.t. x and y.
struct WarpTap {
  int ix0, ix1, iy0, iy1;
  float fx, fy;
  bool inx, iny;
  float p00, p01, p10, p11;  // the four taps (loads in flight until first used)
};

__device__ __forceinline__ WarpTap warp_tap(const float* __restrict__ p, int ip, int W, int H, float x, float y) {
  WarpTap t;
  t.inx = x >= 0.0f && x <= static_cast<float>(W - 1);
  t.iny = y >= 0.0f && y <= static_cast<float>(H - 1);
  const float xc = fminf(fmaxf(x, 0.0f), static_cast<float>(W - 1));
  const float yc = fminf(fmaxf(y, 0.0f), static_cast<float>(H - 1));
  const float xf = floorf(xc), yf = floorf(yc);
  t.fx = xc - xf;
  t.fy = yc - yf;
  t.ix0 = static_cast<int>(xf);
  t.iy0 = static_cast<int>(yf);
  t.ix1 = min(t.ix0 + 1, W - 1);
  t.iy1 = min(t.iy0 + 1, H - 1);
  t.p00 = p[t.iy0 * ip + t.ix0];
  t.p01 = p[t.iy0 * ip + t.ix1];
  t.p10 = p[t.iy1 * ip + t.ix0];
  t.p11 = p[t.iy1 * ip + t.ix1];
  return t;
}

// derivatives of the sample w.r.t. x and y (0 where the coordinate was clamped)
__device__ __forceinline__ float warp_dx(const WarpTap& t) {
  return t.inx ? (1.0f - t.fy) * (t.p01 - t.p00) + t.fy * (t.p11 - t.p10) : 0.0f;
}
__device__ __forceinline__ float warp_dy(const WarpTap& t) {
  return t.iny ? ((1.0f - t.fx) * t.p10 + t.fx * t.p11) - ((1.0f - t.fx) * t.p00 + t.fx * t.p01) : 0.0f;
}

// Adds a at (ix0, iy) and b at (ix1, iy) of the image gradient gP with
// global float atomics, for every lane of the wavefront at once (lanes with
// on == false add nothing; every lane must call it).  Where a lane's right
// column is the left column of the next lane in the same row, the next lane
// adds both values with one atomic.
__device__ __forceinline__ void emit_row(float* gP, int ip, bool on, int iy, int ix0, int ix1, float a, float b) {
  const int lane = static_cast<int>(threadIdx.x & 63);
  if (ix1 == ix0) {  // the last column: both taps on one element
    a += b;
    b = 0.0f;
  }
  const float lb = __shfl_up(b, 1);
  const int liy = __shfl_up(iy, 1), lix1 = __shfl_up(ix1, 1), lon = __shfl_up(on ? 1 : 0, 1);
  const bool take = lane > 0 && on && lon != 0 && liy == iy && lix1 == ix0;
  const bool given = __shfl_down(take ? 1 : 0, 1) != 0 && lane < 63;
  if (on) {
    atomicAdd(gP + iy * ip + ix0, take ? a + lb : a);
    if (!given && b != 0.0f) atomicAdd(gP + iy * ip + ix1, b);
  }
}

// Taps of one image still to be added: the lower row of the previous pixel of
// the lane's column.
struct PendRow {
  bool on;
  int iy, ix0, ix1;
  float a, b;
};

// The four weighted taps g w of a sample go out: the upper row merged with
// the pending lower row of the pixel above where they coincide, then added
// across the wavefront; the lower row becomes the pending row.  A pending
// row that does not continue here is added on its own.
__device__ __forceinline__ void scatter_taps(float* gP, int ip, bool on, const WarpTap& t, float g, PendRow& p) {
  float a00 = 0.0f, a01 = 0.0f, a10 = 0.0f, a11 = 0.0f;
  if (on) {
    a00 = g * (1.0f - t.fy) * (1.0f - t.fx);
    a01 = g * (1.0f - t.fy) * t.fx;
    a10 = g * t.fy * (1.0f - t.fx);
    a11 = g * t.fy * t.fx;
  }
  const bool cont = on && p.on && p.iy == t.iy0 && p.ix0 == t.ix0;
  if (cont) {
    a00 += p.a;
    a01 += p.b;
  } else if (p.on) {
    atomicAdd(gP + p.iy * ip + p.ix0, p.a);
    if (p.ix1 != p.ix0) atomicAdd(gP + p.iy * ip + p.ix1, p.b);
    else atomicAdd(gP + p.iy * ip + p.ix0, p.b);
  }
  if (on && t.iy1 == t.iy0) {  // the last row: the lower taps are the upper ones
    a00 += a10;
    a01 += a11;
  }
  emit_row(gP, ip, on, t.iy0, t.ix0, t.ix1, a00, a01);
  p.on = on && t.iy1 != t.iy0;
  p.iy = t.iy1;
  p.ix0 = t.ix0;
  p.ix1 = t.ix1;
  p.a = a10;
  p.b = a11;
}

template <int KR, int TX, int TY, int SL, int SLV, int NT, bool STORED>
__global__ __launch_bounds__(NT) void adj_scatter_kernel(const AdjArgs a) {
  using G = AdjScatGeom<KR, TX, TY, SL, SLV, STORED>;
  constexpr int RWV = G::RWV, RHV = G::RHV, RW = G::RW, RH = G::RH, QW = G::QW, QY = G::QY, QL = G::QL;
  constexpr int CPH = G::CPH, QS = G::QS, SW = G::SW, SH = G::SH, SP = G::SP, R1L = G::R1L, R1S = G::R1S;
  constexpr int NWIN = 2 * KR + 1;
  constexpr int NSEG = RW / SL;
  constexpr int NIT = (NSEG * QY + NT - 1) / NT;   // horizontal items per lane
  constexpr int NSV = RH / SLV;
  constexpr int NIT3 = (RWV * NSV + NT - 1) / NT;  // vertical items per lane
  constexpr int NQ = (QW * QY + NT - 1) / NT;      // dL/dA elements per lane
  constexpr int NSS = (SW * SH + NT - 1) / NT;     // S pixels per lane
  constexpr int NR = (RWV * RHV + NT - 1) / NT;    // ring pixels per lane (stored record)
  constexpr int NTP = TY / (NT / 64);              // output pixels per lane: a column segment
  static_assert(TX == 64 && NT % 64 == 0 && TY % (NT / 64) == 0, "a wavefront spans a tile row");
  extern __shared__ float lds[];
  float* sQ = lds;                 // dL/dA, then its horizontal sums, then the scatter buffers
  float* sS = lds + G::S_OFF;      // S over the ring region + 1
  float* sR = lds + G::R_OFF;      // ring planes: Gx, Gy, b (then dL/db), dL/dGx, dL/dGy

  const AdjJob& J = a.job[find_job(a, blockIdx.x)];
  const int W = J.w, H = J.h;
  const int ntx = (W + TX - 1) / TX;
  const int t = xcd_tile(blockIdx.x - J.tile_start, ntx * ((H + TY - 1) / TY));
  const int x0 = (t % ntx) * TX, y0 = (t / ntx) * TY;
  const int tid = threadIdx.x;
  const int ip = J.ip, vp = J.vp;

  // ---- P1: dL/dA over the tile + (KR + 1) (0 outside the level: the window is
  // truncated); S over the ring region + 1; and the flow and direct gradient
  // of the lane's P4 pixels.  Every load is issued, at a clamped address,
  // before any is used: the flows with dL/dA, then the image taps.
  const int tx = tid & 63;
  const int ty0 = (tid >> 6) * NTP;
  const int gx4 = x0 + tx;
  const int gxc4 = min(gx4, W - 1);
  float u4[NTP], v4[NTP], d0[NTP], d1[NTP];
#pragma unroll
  for (int k = 0; k < NTP; ++k) {
    const int gyc = min(y0 + ty0 + k, H - 1);
    u4[k] = J.vu[gyc * vp + gxc4];
    v4[k] = J.vv[gyc * vp + gxc4];
    const float* gd = J.gA + 5 * J.ps + gyc * J.sp + gxc4;
    d0[k] = gd[0];
    d1[k] = gd[J.ps];
  }
  const int qx0 = x0 - 1 - KR, qy0 = y0 - 1 - KR;
  float val[NQ][5];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int e = min(tid + NT * k, QW * QY - 1);
    const int qy = e / QW, qx = e - qy * QW;
    const int lx = min(max(qx0 + qx, 0), W - 1), ly = min(max(qy0 + qy, 0), H - 1);
    const float* src = J.gA + ly * J.sp + lx;
#pragma unroll
    for (int q = 0; q < 5; ++q) val[k][q] = src[q * J.ps];
  }
  float kT[NSS], kU[NSS], kV[NSS];
  float sval[NSS];   // S of the lane's S-region pixels
  if (!STORED) {
    const float wm1 = static_cast<float>(W - 1), hm1 = static_cast<float>(H - 1);
    const float wm2 = static_cast<float>(W - 2), hm2 = static_cast<float>(H - 2);
    const uint32_t uip = static_cast<uint32_t>(ip), uvp = static_cast<uint32_t>(vp);
    const PlaneView i0 = plane_view(J.p0, uip * static_cast<uint32_t>(H) * 4u);
    const PlaneView i1 = plane_view(J.p1, uip * static_cast<uint32_t>(H) * 4u);
    const PlaneView fu = plane_view(J.vu, uvp * static_cast<uint32_t>(H) * 4u);
    const PlaneView fv = plane_view(J.vv, uvp * static_cast<uint32_t>(H) * 4u);
    const uint32_t sx = W > 1 ? 1u : 0u, sy = H > 1 ? uip : 0u;
    int px[NSS], py[NSS];
#pragma unroll
    for (int k = 0; k < NSS; ++k) {
      const int e = min(tid + NT * k, SW * SH - 1);
      const int ey = e / SW, ex = e - ey * SW;
      px[k] = min(max(x0 - 2 + ex, 0), W - 1);
      py[k] = min(max(y0 - 2 + ey, 0), H - 1);
      const uint32_t o = static_cast<uint32_t>(py[k]) * uvp + static_cast<uint32_t>(px[k]);
      kU[k] = ld_f32(fu, o);
      kV[k] = ld_f32(fv, o);
    }
    // dL/dA to LDS before the taps are issued: its registers are free for them
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int e = tid + NT * k;
      if (e < QW * QY) {
        const int qy = e / QW, qx = e - qy * QW;
        const int lx = qx0 + qx, ly = qy0 + qy;
        const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                         static_cast<unsigned>(ly) < static_cast<unsigned>(H);
#pragma unroll
        for (int q = 0; q < 5; ++q) sQ[q * QS + qy * QL + qx] = inl ? val[k][q] : 0.0f;
      }
    }
    BilTap b0[NSS], b1[NSS];
    float t[NSS][8];
#pragma unroll
    for (int k = 0; k < NSS; ++k) {
      const float fx = static_cast<float>(px[k]), fy = static_cast<float>(py[k]);
      b0[k] = bil_setup(fx - 0.5f * kU[k], fy - 0.5f * kV[k], wm1, hm1, wm2, hm2, uip);
      b1[k] = bil_setup(fx + 0.5f * kU[k], fy + 0.5f * kV[k], wm1, hm1, wm2, hm2, uip);
      t[k][0] = ld_f32(i0, b0[k].i);
      t[k][1] = ld_f32(i0, b0[k].i + sx);
      t[k][2] = ld_f32(i0, b0[k].i + sy);
      t[k][3] = ld_f32(i0, b0[k].i + sy + sx);
      t[k][4] = ld_f32(i1, b1[k].i);
      t[k][5] = ld_f32(i1, b1[k].i + sx);
      t[k][6] = ld_f32(i1, b1[k].i + sy);
      t[k][7] = ld_f32(i1, b1[k].i + sy + sx);
    }
#pragma unroll
    for (int k = 0; k < NSS; ++k) {
      const float w0 = bil_combine(t[k][0], t[k][1], t[k][2], t[k][3], b0[k].ax, b0[k].ay);
      const float w1 = bil_combine(t[k][4], t[k][5], t[k][6], t[k][7], b1[k].ax, b1[k].ay);
      kT[k] = w1 - w0;
      sval[k] = 0.5f * (w0 + w1);
    }
  } else {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int e = tid + NT * k;
      if (e < QW * QY) {
        const int qy = e / QW, qx = e - qy * QW;
        const int lx = qx0 + qx, ly = qy0 + qy;
        const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                         static_cast<unsigned>(ly) < static_cast<unsigned>(H);
#pragma unroll
        for (int q = 0; q < 5; ++q) sQ[q * QS + qy * QL + qx] = inl ? val[k][q] : 0.0f;
      }
    }
    // the stored Gx, Gy and b of the ring pixels, then the taps of the P4 pixels
    float rv[NR][3];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int e = min(tid + NT * k, RWV * RHV - 1);
      const int ry = e / RWV, rx = e - ry * RWV;
      const int lx = min(max(x0 - 1 + rx, 0), W - 1), ly = min(max(y0 - 1 + ry, 0), H - 1);
      const float* src = J.st + ly * J.stp + lx;
#pragma unroll
      for (int q = 0; q < 3; ++q) rv[k][q] = src[(5 + q) * J.sts];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int e = tid + NT * k;
      if (e < RWV * RHV) {
        const int ry = e / RWV, rx = e - ry * RWV;
        const int lx = x0 - 1 + rx, ly = y0 - 1 + ry;
        const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                         static_cast<unsigned>(ly) < static_cast<unsigned>(H);
#pragma unroll
        for (int q = 0; q < 3; ++q) sR[q * R1S + ry * R1L + rx] = inl ? rv[k][q] : 0.0f;
      }
    }
  }
  if (!STORED) {
#pragma unroll
    for (int k = 0; k < NSS; ++k) {
      const int e = tid + NT * k;
      if (e < SW * SH) {
        const int ey = e / SW, ex = e - ey * SW;
        sS[ey * SP + ex] = sval[k];
      }
    }
  }
  __syncthreads();

  // ---- P2: G and b of the ring pixels; horizontal window sums of dL/dA
  if (!STORED) {
#pragma unroll
    for (int k = 0; k < NSS; ++k) {
      const int e = tid + NT * k;
      if (e < SW * SH) {
        const int ey = e / SW, ex = e - ey * SW;
        if (ex >= 1 && ex < SW - 1 && ey >= 1 && ey < SH - 1) {
          const int lx = x0 - 2 + ex, ly = y0 - 2 + ey;
          const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                           static_cast<unsigned>(ly) < static_cast<unsigned>(H);
          const int o = ey * SP + ex;
          float gx = 0.0f, gy = 0.0f, b = 0.0f;
          if (inl) {
            gx = 0.5f * (sS[o + 1] - sS[o - 1]);
            gy = 0.5f * (sS[o + SP] - sS[o - SP]);
            b = fmaf(gx, kU[k], fmaf(gy, kV[k], -kT[k]));
          }
          const int r = (ey - 1) * R1L + (ex - 1);
          sR[r] = gx;
          sR[R1S + r] = gy;
          sR[2 * R1S + r] = b;
        }
      }
    }
  }
  float hsum[NIT][5][SL];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * QY) {
      const int rb = (item % QY) * QL + (item / QY) * SL;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float* row = sQ + lds_reg(q * QS + rb);
        float ring[NWIN];
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < SL + 2 * KR; ++k) {
          const float pq = row[k];
          if (k >= NWIN) acc -= ring[k % NWIN];
          ring[k % NWIN] = pq;
          acc = k == 0 ? pq : acc + pq;
          if (k >= 2 * KR) hsum[it][q][k - 2 * KR] = acc;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * QY) {
      const int cb = (item / QY) * SL * CPH + item % QY;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float* col = sQ + lds_reg(q * QS + cb);
#pragma unroll
        for (int jj = 0; jj < SL; ++jj) col[jj * CPH] = hsum[it][q][jj];
      }
    }
  }
  __syncthreads();

  // ---- P3: vertical window sums -> dL/dp of the ring pixels; adjoints of the products and of b
#pragma unroll
  for (int it = 0; it < NIT3; ++it) {
    const int item = tid + NT * it;
    if (item < RWV * NSV) {
      const int jc = item % RWV;
      const int rs = (item / RWV) * SLV;
      const int lx = x0 - 1 + jc;
      float um[SLV], vm[SLV];   // read at clamped coordinates: used only where the pixel is inside
      const int lxc = min(max(lx, 0), W - 1);
#pragma unroll
      for (int k = 0; k < SLV; ++k) {
        const int lyc = min(max(y0 - 1 + rs + k, 0), H - 1);
        um[k] = J.vu[lyc * vp + lxc];
        vm[k] = J.vv[lyc * vp + lxc];
      }
      const float* col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) col[q] = sQ + lds_reg(q * QS + jc * CPH + rs);
      float ring[5][NWIN];
      float acc[5];
#pragma unroll
      for (int k = 0; k < SLV + 2 * KR; ++k) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float hq = col[q][k];
          if (k >= NWIN) acc[q] -= ring[q][k % NWIN];
          ring[q][k % NWIN] = hq;
          acc[q] = k == 0 ? hq : acc[q] + hq;
        }
        if (k >= 2 * KR) {
          const int kk = k - 2 * KR;
          const int r = rs + kk;
          if (r < RHV) {
            const int ly = y0 - 1 + r;
            const bool inl = static_cast<unsigned>(lx) < static_cast<unsigned>(W) &&
                             static_cast<unsigned>(ly) < static_cast<unsigned>(H);
            const int ro = r * R1L + jc;
            float gGx = 0.0f, gGy = 0.0f, gb = 0.0f;
            if (inl) {
              const float gx = sR[ro], gy = sR[R1S + ro], b = sR[2 * R1S + ro];
              gb = gx * acc[3] + gy * acc[4];
              gGx = 2.0f * gx * acc[0] + gy * acc[1] + b * acc[3] + um[kk] * gb;
              gGy = gx * acc[1] + 2.0f * gy * acc[2] + b * acc[4] + vm[kk] * gb;
            }
            sR[2 * R1S + ro] = gb;
            sR[3 * R1S + ro] = gGx;
            sR[4 * R1S + ro] = gGy;
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- P4: per output pixel (a lane walks NTP rows of one column):
  // transposed central difference, warp adjoints, dL/dV, scatter.  The flow
  // and direct gradient came with the loads of P1; the image taps of all the
  // lane's pixels are issued before any is used.
  {
    WarpTap ta[NTP], tb[NTP];
#pragma unroll
    for (int k = 0; k < NTP; ++k) {
      const float fx = static_cast<float>(gxc4), fy = static_cast<float>(min(y0 + ty0 + k, H - 1));
      ta[k] = warp_tap(J.p0, ip, W, H, fx - 0.5f * u4[k], fy - 0.5f * v4[k]);
      tb[k] = warp_tap(J.p1, ip, W, H, fx + 0.5f * u4[k], fy + 0.5f * v4[k]);
    }

    PendRow q0{false, 0, 0, 0, 0.0f, 0.0f}, q1{false, 0, 0, 0, 0.0f, 0.0f};
    const int gx = gx4;
#pragma unroll
    for (int k = 0; k < NTP; ++k) {
      const int ty = ty0 + k;
      const int gy = y0 + ty;
      const bool on = gx < W && gy < H;
      float gw0 = 0.0f, gw1 = 0.0f;
      if (on) {
        const int ro = (ty + 1) * R1L + tx + 1;
        const float* gGx = sR + 3 * R1S;
        const float* gGy = sR + 4 * R1S;
        // S(j) enters Gx(j - 1) with +1/2 and Gx(j + 1) with -1/2, and Gx(j) itself
        // where the clamped neighbour is j (the first and last column); likewise y
        float gs = 0.5f * (gGx[ro - 1] - gGx[ro + 1] + gGy[ro - R1L] - gGy[ro + R1L]);
        if (gx == W - 1) gs += 0.5f * gGx[ro];
        if (gx == 0) gs -= 0.5f * gGx[ro];
        if (gy == H - 1) gs += 0.5f * gGy[ro];
        if (gy == 0) gs -= 0.5f * gGy[ro];
        const float gb = sR[2 * R1S + ro];
        const float gxv = sR[ro], gyv = sR[R1S + ro];
        // dL/dT = -dL/db; S = (W0 + W1)/2, T = W1 - W0
        gw0 = 0.5f * gs + gb;
        gw1 = 0.5f * gs - gb;
        J.ou[gy * J.op + gx] = d0[k] + gxv * gb - 0.5f * gw0 * warp_dx(ta[k]) + 0.5f * gw1 * warp_dx(tb[k]);
        J.ov[gy * J.op + gx] = d1[k] + gyv * gb - 0.5f * gw0 * warp_dy(ta[k]) + 0.5f * gw1 * warp_dy(tb[k]);
      }
      scatter_taps(J.gP0, ip, on, ta[k], gw0, q0);
      scatter_taps(J.gP1, ip, on, tb[k], gw1, q1);
    }
    emit_row(J.gP0, ip, q0.on, q0.iy, q0.ix0, q0.ix1, q0.a, q0.b);
    emit_row(J.gP1, ip, q1.on, q1.iy, q1.ix0, q1.ix1, q1.a, q1.b);
  }
}

template <int KR, bool STORED, int TY>
hipError_t launch_adj_scatter_cfg(const AdjArgs& a, int nblocks, hipStream_t s) {
  constexpr int TX = 64, SL = 8, SLV = TY == 16 ? 6 : 5;
  constexpr size_t lds = sizeof(float) * AdjScatGeom<KR, TX, TY, SL, SLV, STORED>::FLOATS;
  auto kern = adj_scatter_kernel<KR, TX, TY, SL, SLV, 256, STORED>;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

}  // namespace ofv
