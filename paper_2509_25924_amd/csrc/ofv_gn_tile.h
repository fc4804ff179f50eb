// Fused symmetric Gauss-Newton iteration, 2-D tile variant (pipeline steps 3
// and 5 of section "Live-Optical Flow Velocimetry", Eq. of_symmetric,
// arXiv 2509.25924).  Same arithmetic as the strip-march variant in
// ofv_gn_impl.h; a different work decomposition with far more independent
// work per lane, for levels too small to give the march enough workgroups.
//
// A 256-lane workgroup computes a TX x TY tile of the new flow in three
// phases separated by barriers:
//  A. every pixel of the tile plus a (KR+1)-pixel halo, evaluated at its
//     coordinates clamped into the level: input flow (loaded or up-sampled),
//     the two midpoint bilinear warps, S and T -> LDS.  Because out-of-level
//     halo pixels repeat their clamped neighbour exactly, the central
//     differences of phase B reproduce the clamped-index gradient with no
//     border logic;
//  B. per (product row, segment of SL output columns): Gx^2, GxGy, Gy^2, Gx b,
//     Gy b formed from LDS and summed over the horizontal window by running
//     sums whose leaving terms sit in a register ring -> LDS;
//  C. per (output column, segment of SLV output rows): running vertical
//     window sums, damped 2x2 solve, coalesced store of u' and v'.
#pragma once

#include "ofv_gn_impl.h"

namespace ofv {

template <int KR, int TX, int TY>
struct TileGeom {
  static constexpr int NWIN = 2 * KR + 1;
  static constexpr int EX = TX + 2 * KR + 2;  // S region = product region + 1 on each side
  static constexpr int EY = TY + 2 * KR + 2;
  static constexpr int LP = EX | 1;           // odd LDS pitch: row-strided lanes hit distinct banks
  static constexpr int PY = TY + 2 * KR;      // product rows
  static constexpr int NE = EX * EY;
  static constexpr int HP = TX + 1;           // pitch of the horizontal-sum planes
  static constexpr int LDS_FLOATS = 4 * LP * EY + 5 * PY * HP;
};

// Bilinear sample at (x, y) clamped into a w x h plane; taps (ix, ix + sx)
// with ix <= w - 2 (sx = 0 for single-column planes), likewise rows.
template <typename TS>
__device__ __forceinline__ float bil_clamped(const TS* __restrict__ p, int pitch, float wm1, float hm1, float wm2,
                                             float hm2, int sx, int sy, float x, float y) {
  // median-of-three clamps (a NaN coordinate ends as tap 0 via the integer conversion)
  x = __builtin_amdgcn_fmed3f(x, 0.0f, wm1);
  y = __builtin_amdgcn_fmed3f(y, 0.0f, hm1);
  const float xf = __builtin_amdgcn_fmed3f(floorf(x), 0.0f, wm2);
  const float yf = __builtin_amdgcn_fmed3f(floorf(y), 0.0f, hm2);
  const float ax = x - xf;
  const float ay = y - yf;
  const TS* r0 = p + (static_cast<int>(yf) * pitch + static_cast<int>(xf));
  const float p00 = Px<TS>::ld(r0);
  const float p01 = Px<TS>::ld(r0 + sx);
  const float p10 = Px<TS>::ld(r0 + sy);
  const float p11 = Px<TS>::ld(r0 + sy + sx);
  const float top = fmaf(ax, p01 - p00, p00);
  const float bot = fmaf(ax, p11 - p10, p10);
  return fmaf(ay, bot - top, top);
}

template <int KR, int MODE, typename TS, int TX, int TY, int SL, int SLV>
__global__ __launch_bounds__(256) void gn_tile_kernel(const GnArgs a) {
  using G = TileGeom<KR, TX, TY>;
  constexpr int NWIN = G::NWIN, EX = G::EX, LP = G::LP, PY = G::PY, HP = G::HP, NE = G::NE;
  static_assert(TX % SL == 0 && TY % SLV == 0, "segments must tile the output");
  static_assert(TX * (TY / SLV) <= 256, "phase C items");
  extern __shared__ float lds[];
  float* sS = lds;
  float* sT = sS + LP * G::EY;
  float* sU = sT + LP * G::EY;
  float* sV = sU + LP * G::EY;
  float* sH = sV + LP * G::EY;  // 5 planes of PY x HP

  const int jb = find_job(a, blockIdx.x);
  const GnJob& J = a.job[jb];
  const TS* __restrict__ p0 = static_cast<const TS*>(J.p0);
  const TS* __restrict__ p1 = static_cast<const TS*>(J.p1);
  const int ip = static_cast<int>(J.img_pitch);
  const int W = J.w;
  const int H = J.h;
  const float wm1 = static_cast<float>(W - 1), hm1 = static_cast<float>(H - 1);
  const float wm2 = static_cast<float>(W - 2), hm2 = static_cast<float>(H - 2);
  const int sx = W > 1 ? 1 : 0;
  const int sy = H > 1 ? ip : 0;
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (W + TX - 1) / TX;
  const int x0 = (t % ntx) * TX;
  const int y0 = (t / ntx) * TY;
  const int gx0 = x0 - KR - 1;  // level column of ext column 0
  const int gy0 = y0 - KR - 1;
  const int tid = threadIdx.x;

  // ---- phase A: flow, warps, S, T over the ext region (clamped coordinates)
  {
    constexpr int NA = (NE + 255) / 256;
    constexpr int CH = MODE == FLOW_UPSAMPLE ? 4 : 8;
    constexpr int DY = 256 / EX, DX = 256 % EX;
    int ey = tid / EX;
    int ex = tid - ey * EX;
    const int fpitch = static_cast<int>(J.in_pitch);
    const float cwm1 = static_cast<float>(J.cw - 1), chm1 = static_cast<float>(J.ch - 1);
    const float cwm2 = static_cast<float>(J.cw - 2), chm2 = static_cast<float>(J.ch - 2);
    const int csx = J.cw > 1 ? 1 : 0;
    const int csy = J.ch > 1 ? fpitch : 0;
#pragma unroll
    for (int k0 = 0; k0 < NA; k0 += CH) {
      float uu[CH], vv[CH];
      int gx[CH], gy[CH], oo[CH];
      FlowReq fr[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        gx[k] = min(max(gx0 + ex, 0), W - 1);
        gy[k] = min(max(gy0 + ey, 0), H - 1);
        oo[k] = ey * LP + ex;
        if (MODE == FLOW_DIRECT) {
          const int o = gy[k] * fpitch + gx[k];
          uu[k] = J.in_u[o];
          vv[k] = J.in_v[o];
        } else if (MODE == FLOW_UPSAMPLE) {
          // issue the coarse taps of all CH pixels before combining any of them
          const float fx = __builtin_amdgcn_fmed3f(0.5f * static_cast<float>(gx[k]), 0.0f, cwm1);
          const float fy = __builtin_amdgcn_fmed3f(0.5f * static_cast<float>(gy[k]), 0.0f, chm1);
          const float xf = __builtin_amdgcn_fmed3f(floorf(fx), 0.0f, cwm2);
          const float yf = __builtin_amdgcn_fmed3f(floorf(fy), 0.0f, chm2);
          fr[k].wx = fx - xf;
          fr[k].wy = fy - yf;
          const int o = static_cast<int>(yf) * fpitch + static_cast<int>(xf);
          fr[k].u00 = J.in_u[o];
          fr[k].u01 = J.in_u[o + csx];
          fr[k].u10 = J.in_u[o + csy];
          fr[k].u11 = J.in_u[o + csy + csx];
          fr[k].v00 = J.in_v[o];
          fr[k].v01 = J.in_v[o + csx];
          fr[k].v10 = J.in_v[o + csy];
          fr[k].v11 = J.in_v[o + csy + csx];
        } else {
          uu[k] = 0.0f;
          vv[k] = 0.0f;
        }
        ex += DX;
        ey += DY;
        if (ex >= EX) {
          ex -= EX;
          ++ey;
        }
      }
      if (MODE == FLOW_UPSAMPLE) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const FlowReq& r = fr[k];
          const float ut = fmaf(r.wx, r.u01 - r.u00, r.u00);
          const float ub = fmaf(r.wx, r.u11 - r.u10, r.u10);
          const float vt = fmaf(r.wx, r.v01 - r.v00, r.v00);
          const float vb = fmaf(r.wx, r.v11 - r.v10, r.v10);
          uu[k] = 2.0f * fmaf(r.wy, ub - ut, ut);
          vv[k] = 2.0f * fmaf(r.wy, vb - vt, vt);
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (k0 + k < NA && tid + 256 * (k0 + k) < NE) {
          const float fx = static_cast<float>(gx[k]);
          const float fy = static_cast<float>(gy[k]);
          const float hu = 0.5f * uu[k];
          const float hv = 0.5f * vv[k];
          const float w0 = bil_clamped(p0, ip, wm1, hm1, wm2, hm2, sx, sy, fx - hu, fy - hv);
          const float w1 = bil_clamped(p1, ip, wm1, hm1, wm2, hm2, sx, sy, fx + hu, fy + hv);
          sS[oo[k]] = 0.5f * (w0 + w1);
          sT[oo[k]] = w1 - w0;
          sU[oo[k]] = uu[k];
          sV[oo[k]] = vv[k];
        }
      }
    }
  }
  __syncthreads();

  // ---- phase B: products and horizontal window sums, item = (product row, segment)
  {
    constexpr int NSEG = TX / SL;
    constexpr int NITEM = NSEG * PY;
    for (int item = tid; item < NITEM; item += 256) {
      const int r = item % PY;  // product row r = ext row r + 1
      const int sg = item / PY;
      const int xs = sg * SL;   // first product column of the first output's window
      const bool row_in = static_cast<unsigned>(gy0 + r + 1) < static_cast<unsigned>(H);
      const int base = (r + 1) * LP + xs + 1;  // LDS index of ext (r + 1, xs + 1)
      const int gxs = gx0 + xs + 1;           // level column of that pixel
      float ring[5][NWIN];
      float acc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < SL + 2 * KR; ++k) {
        const int o = base + k;
        const bool valid = row_in && static_cast<unsigned>(gxs + k) < static_cast<unsigned>(W);
        float gx = 0.5f * (sS[o + 1] - sS[o - 1]);
        float gy = 0.5f * (sS[o + LP] - sS[o - LP]);
        gx = valid ? gx : 0.0f;
        gy = valid ? gy : 0.0f;
        const float b = fmaf(gx, sU[o], fmaf(gy, sV[o], -sT[o]));
        const float p[5] = {gx * gx, gx * gy, gy * gy, gx * b, gy * b};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          if (k >= NWIN) acc[q] -= ring[q][k % NWIN];
          ring[q][k % NWIN] = p[q];
          acc[q] += p[q];
        }
        if (k >= 2 * KR) {
          const int j = xs + k - 2 * KR;  // output column
#pragma unroll
          for (int q = 0; q < 5; ++q) sH[(q * PY + r) * HP + j] = acc[q];
        }
      }
    }
  }
  __syncthreads();

  // ---- phase C: vertical window sums, solve, store; item = (output column, segment)
  {
    constexpr int NSEGV = TY / SLV;
    const int j = tid % TX;
    const int sg = tid / TX;
    const int gx = x0 + j;
    if (sg < NSEGV && gx < W) {
      float ring[5][NWIN];
      float acc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      const int rs = sg * SLV;  // first product row of the first output's window
#pragma unroll
      for (int k = 0; k < SLV + 2 * KR; ++k) {
        const int r = rs + k;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float hq = sH[(q * PY + r) * HP + j];
          if (k >= NWIN) acc[q] -= ring[q][k % NWIN];
          ring[q][k % NWIN] = hq;
          acc[q] += hq;
        }
        if (k >= 2 * KR) {
          const int oy = rs + k - 2 * KR;  // output row within the tile
          const int gy = y0 + oy;
          if (gy < H) {
            const int o = (oy + KR + 1) * LP + (j + KR + 1);
            const float um = sU[o];
            const float vm = sV[o];
            float un, vn;
            solve2x2(acc[0], acc[1], acc[2], acc[3], acc[4], um, vm, a.reg_rel, a.reg_abs, un, vn);
            const int64_t oo = static_cast<int64_t>(gy) * J.out_pitch + gx;
            J.out_u[oo] = un;
            J.out_v[oo] = vn;
          }
        }
      }
    }
  }
}

template <int KR, int MODE, typename TS, int TX, int TY, int SL, int SLV>
hipError_t launch_gn_tile_cfg(const GnArgs& a, int nblocks, hipStream_t s) {
  constexpr size_t lds = sizeof(float) * TileGeom<KR, TX, TY>::LDS_FLOATS;
  auto kern = gn_tile_kernel<KR, MODE, TS, TX, TY, SL, SLV>;
  // dynamic LDS above 64 KiB must be enabled once per kernel (thread-safe static init)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

// variant GN_TILE_64x32: 64 x 32 outputs (segments 16 columns / 8 rows);
// variant GN_TILE_64x16: 64 x 16 outputs (segments 16 columns / 4 rows).
template <int MODE, typename TS>
hipError_t launch_gn_tile_typed(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s) {
#define OFV_GNT_CASE(R)                                                                             \
  case R:                                                                                           \
    return variant == GN_TILE_64x32 ? launch_gn_tile_cfg<R, MODE, TS, 64, 32, 16, 8>(a, nblocks, s) \
                                    : launch_gn_tile_cfg<R, MODE, TS, 64, 16, 16, 4>(a, nblocks, s);
  switch (kr) {
    OFV_GNT_CASE(1)
    OFV_GNT_CASE(2)
    OFV_GNT_CASE(3)
    OFV_GNT_CASE(4)
    OFV_GNT_CASE(5)
    OFV_GNT_CASE(6)
    OFV_GNT_CASE(7)
    OFV_GNT_CASE(8)
    OFV_GNT_CASE(9)
    OFV_GNT_CASE(10)
    OFV_GNT_CASE(11)
    OFV_GNT_CASE(12)
    default: return hipErrorInvalidValue;
  }
#undef OFV_GNT_CASE
}

}  // namespace ofv
