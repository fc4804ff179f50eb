// Fused symmetric Gauss-Newton iteration, 2-D tile variant (pipeline steps 3
// and 5 of section "Live-Optical Flow Velocimetry", Eq. of_symmetric,
// arXiv 2509.25924).  Same arithmetic as the strip-march variant in
// ofv_gn_impl.h; a different work decomposition with far more independent
// work per lane, for levels too small to give the march enough workgroups.
//
// A workgroup of NT lanes computes a TX x TY tile of the new flow in five
// steps separated by barriers, with one image plane and five product planes
// in LDS:
//  A1. every pixel of the tile plus a (KR+1)-pixel halo, evaluated at its
//      coordinates clamped into the level: input flow (loaded or
//      up-sampled) and the two midpoint bilinear warps; S -> LDS, while T
//      and the flow stay in the registers of the lane that computed them.
//      Because out-of-level halo pixels repeat their clamped neighbour
//      exactly, the central differences of A2 reproduce the clamped-index
//      gradient with no border logic;
//  A2. the same lanes, for the pixels of the product region (tile plus a
//      KR halo): Gx, Gy from S, b = G . V - T, and the five products Gx^2,
//      GxGy, Gy^2, Gx b, Gy b (0 outside the level) -> five LDS planes;
//  B.  per (product row, segment of SL output columns): horizontal window
//      sums by running sums over the product planes, kept in registers ...
//  B'. ... and written back, transposed (column-major, one plane per
//      product), over the product planes once every lane has read its inputs
//      (1024-lane tiles with LDS to spare: into a region of their own, with
//      no barrier between B and B');
//  C.  per (output column, segment of SLV output rows): running vertical
//      window sums along the contiguous columns of B', damped 2x2 solve,
//      coalesced store of u' and v'.
// Every product is formed once; only the window sums repeat work at the
// segment ends.
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
  static constexpr int PLANE = LP * EY;       // one ext-sized LDS plane
  // B' output: per product, TX columns of PY horizontal sums, odd column
  // pitch (column-strided lanes of C hit distinct banks)
  static constexpr int CP = PY | 1;
  static constexpr int HPL = TX * CP;
  static_assert(HPL <= PLANE, "transposed sums fit in the product planes");
  // the S plane and five product planes, all indexed by ext coordinates
  static constexpr int LDS_FLOATS = 6 * PLANE;
};

// 1024-lane workgroups (at most two per compute unit) whose product planes
// leave room within 80 KiB put the transposed horizontal sums in an LDS
// region of their own: B then stores them as it forms them, without the
// barrier and the register round trip of writing back over the products.
template <int KR, int TX, int TY, int NT>
struct TileLds {
  using G = TileGeom<KR, TX, TY>;
  static constexpr bool HSEP = NT == 1024 && 4 * (G::LDS_FLOATS + 5 * G::HPL) <= 81920;
  static constexpr int HOFF = HSEP ? G::LDS_FLOATS : G::PLANE;  // first float of the sums
  static constexpr int FLOATS = HSEP ? G::LDS_FLOATS + 5 * G::HPL : G::LDS_FLOATS;
};

// Bilinear sample at (x, y) clamped into a w x h plane, split into the
// address set-up and the combination of the four taps: taps (ix, ix + sx)
// x (iy, iy + sy) with ix <= w - 2 (sx = 0 for single-column planes),
// likewise rows; (ax, ay) are the weights of the second tap of each pair.
struct BilTap {
  uint32_t i;  // element index of tap (ix, iy)
  float ax, ay;
};

__device__ __forceinline__ BilTap bil_setup(float x, float y, float wm1, float hm1, float wm2, float hm2,
                                            uint32_t pitch) {
  // median-of-three clamps (a NaN coordinate ends as tap 0 via the integer conversion)
  x = __builtin_amdgcn_fmed3f(x, 0.0f, wm1);
  y = __builtin_amdgcn_fmed3f(y, 0.0f, hm1);
  const float xf = __builtin_amdgcn_fmed3f(floorf(x), 0.0f, wm2);
  const float yf = __builtin_amdgcn_fmed3f(floorf(y), 0.0f, hm2);
  BilTap t;
  t.ax = x - xf;
  t.ay = y - yf;
  // plane widths and heights are below 2^24 (checked on the host)
  t.i = __umul24(static_cast<uint32_t>(yf), pitch) + static_cast<uint32_t>(xf);
  return t;
}

__device__ __forceinline__ float bil_combine(float p00, float p01, float p10, float p11, float ax, float ay) {
  const float top = fmaf(ax, p01 - p00, p00);
  const float bot = fmaf(ax, p11 - p10, p10);
  return fmaf(ay, bot - top, top);
}

// An LDS element offset that the compiler treats as unknown.  Accesses at
// constant distances from it then keep small immediate offsets from one
// register, instead of being folded into offsets from a shared base that
// overflow the 16-bit (8-bit for paired accesses) offset fields and cost an
// address add each.  Emits no instruction.
__device__ __forceinline__ int lds_reg(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

// Workgroups are handed to the 8 XCDs of the chip in turn (workgroup i to
// XCD i mod 8), and each XCD has its own L2.  Tile l of a job of n tiles is
// renumbered so that the workgroups of one XCD take a contiguous run of
// row-major tiles: neighbours then share their halo rows and columns in one
// L2 instead of fetching them from HBM once per XCD.
__device__ __forceinline__ int xcd_tile(int l, int n) {
  const int q = n >> 3;
  return l < 8 * q ? (l & 7) * q + (l >> 3) : l;
}

// Waves per SIMD that the LDS of one NT-lane workgroup leaves room for
// (160 KiB per compute unit, NT / 256 waves of each workgroup per SIMD):
// the register budget of the kernel is sized for that occupancy.
template <int KR, int TX, int TY, int NT>
struct TileOcc {
  static constexpr int lds = 4 * TileLds<KR, TX, TY, NT>::FLOATS;
  static constexpr int fit = (163840 / lds) * (NT / 256);
  // at most 4 waves per SIMD: 128 registers per lane keep the gathers of a
  // chunk in flight without spilling
  static constexpr int value = fit < 1 ? 1 : (fit > 4 ? 4 : fit);
};

// GEN: the estimator variant is read from a.est at run time (forward-additive
// warps: P0 read at the pixel itself, P1 warped by the full V, S = the warped
// P1; increment-form update: b = -T and V' = V(m) + dV); otherwise the
// symmetric estimator's consistent update is compiled in.
template <int KR, int MODE, typename TS, int TX, int TY, int SL, int SLV, int NT, bool GEN = false>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(TileOcc<KR, TX, TY, NT>::value, TileOcc<KR, TX, TY, NT>::value)))
void gn_tile_kernel(const GnArgs a) {
  using G = TileGeom<KR, TX, TY>;
  constexpr int NWIN = G::NWIN, EX = G::EX, EY = G::EY, LP = G::LP, PY = G::PY, PL = G::PLANE, NE = G::NE;
  constexpr int CP = G::CP, HPL = G::HPL;
  constexpr bool HSEP = TileLds<KR, TX, TY, NT>::HSEP;
  constexpr int HOFF = TileLds<KR, TX, TY, NT>::HOFF;
  constexpr int NSEG = TX / SL;
  static_assert(TX % SL == 0 && TY % SLV == 0, "segments must tile the output");
  static_assert(TX * (TY / SLV) <= NT, "phase C items");
  constexpr int NIT = (NSEG * PY + NT - 1) / NT;  // phase B items per lane
  // pixels per lane in A1/A2, and how many of them have their taps in flight at once
  constexpr int NA = (NE + NT - 1) / NT;
  constexpr int REGS = 512 / TileOcc<KR, TX, TY, NT>::value;
  // registers per pixel in flight: taps and weights, more when the flow is
  // up-sampled and when 16-bit taps are unpacked (values measured without spills)
  constexpr int PER = MODE == FLOW_UPSAMPLE ? (sizeof(TS) == 2 ? 28 : 20) : (sizeof(TS) == 2 ? 15 : 10);
  constexpr int CHF = (REGS - 48 - 3 * NA) / PER;
  constexpr int CH = CHF < 1 ? 1 : (CHF > NA ? NA : CHF);
  extern __shared__ float lds[];
  const bool fa = GEN && (a.est & EST_FORWARD_ADDITIVE) != 0;
  const bool inc = GEN && (a.est & EST_INCREMENT) != 0;
  const bool no_fp64 = (a.est & EST_NO_FP64) != 0;
  float* sS = lds;           // EY x LP
  float* sP = lds + PL;      // 5 planes: products, then horizontal sums (ext coordinates)

  const int jb = find_job(a, blockIdx.x);
  const GnJob& J = a.job[jb];
  const TS* __restrict__ p0 = static_cast<const TS*>(J.p0);
  const TS* __restrict__ p1 = static_cast<const TS*>(J.p1);
  const int ip = static_cast<int>(J.img_pitch);
  const int W = J.w;
  const int H = J.h;
  const float wm1 = static_cast<float>(W - 1), hm1 = static_cast<float>(H - 1);
  const float wm2 = static_cast<float>(W - 2), hm2 = static_cast<float>(H - 2);
  const int ntx = (W + TX - 1) / TX;
  const int t = xcd_tile(blockIdx.x - J.tile_start, ntx * ((H + TY - 1) / TY));
  const int x0 = (t % ntx) * TX;
  const int y0 = (t / ntx) * TY;
  const int gx0 = x0 - KR - 1;  // level column of ext column 0
  const int gy0 = y0 - KR - 1;
  const int tid = threadIdx.x;
  const uint32_t fpitch = static_cast<uint32_t>(J.in_pitch);
  const uint32_t frows = static_cast<uint32_t>(MODE == FLOW_UPSAMPLE ? J.ch : H);
  const PlaneView vu = plane_view(J.in_u, MODE == FLOW_ZERO ? 0u : fpitch * frows * 4u);
  const PlaneView vv = plane_view(J.in_v, MODE == FLOW_ZERO ? 0u : fpitch * frows * 4u);
  const float cwm1 = static_cast<float>(J.cw - 1), chm1 = static_cast<float>(J.ch - 1);
  const float cwm2 = static_cast<float>(J.cw - 2), chm2 = static_cast<float>(J.ch - 2);
  const uint32_t csx = J.cw > 1 ? 1u : 0u;
  const uint32_t csy = J.ch > 1 ? fpitch : 0u;

  // ---- A1: flow, warps and S over the ext region; T, U, V kept per lane.
  // A lane evaluates CH ext pixels at once: the input flow of all of them
  // is loaded first, then the 8 bilinear taps of each are issued, and only
  // then are any combined, so up to 8 CH gathers are in flight per lane.
  float kT[NA], kU[NA], kV[NA];
  int kO[NA];      // LDS offset of each pixel of the lane
  // up-sampling iterations: the up-sampled flow of the tile's output rows
  // goes from A1 to C through LDS where the free space allows
  constexpr bool STAGE_UV = MODE == FLOW_UPSAMPLE && !HSEP && PL + 5 * HPL + TY * LP <= 6 * PL;
  uint32_t kF = 0; // bit 2k: pixel k is in the product region; bit 2k+1: it lies inside the level
  {
    constexpr int DY = NT / EX, DX = NT % EX;
    int ey = tid / EX;
    int ex = tid - ey * EX;
    const uint32_t uip = static_cast<uint32_t>(ip);
    const uint32_t rowb = uip * Px<TS>::bytes;  // byte offset of the second tap row
    const PlaneView v0 = plane_view(p0, uip * static_cast<uint32_t>(H) * Px<TS>::bytes);
    const PlaneView v1 = plane_view(p1, uip * static_cast<uint32_t>(H) * Px<TS>::bytes);
#pragma unroll
    for (int k0 = 0; k0 < NA; k0 += CH) {
      float uu[CH], vv2[CH], fx[CH], fy[CH];
      int oo[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int gx = min(max(gx0 + ex, 0), W - 1);
        const int gy = min(max(gy0 + ey, 0), H - 1);
        fx[k] = static_cast<float>(gx);
        fy[k] = static_cast<float>(gy);
        oo[k] = ey * LP + ex;
        if (k0 + k < NA) {
          const bool prod = static_cast<unsigned>(ex - 1) < static_cast<unsigned>(EX - 2) &&
                            static_cast<unsigned>(ey - 1) < static_cast<unsigned>(EY - 2) &&
                            tid + NT * (k0 + k) < NE;
          const bool inl = static_cast<unsigned>(gx0 + ex) < static_cast<unsigned>(W) &&
                           static_cast<unsigned>(gy0 + ey) < static_cast<unsigned>(H);
          kO[k0 + k] = oo[k];
          kF |= (prod ? 1u : 0u) << (2 * (k0 + k));
          kF |= (inl ? 2u : 0u) << (2 * (k0 + k));
        }
        if (MODE == FLOW_DIRECT) {
          const uint32_t o = __umul24(static_cast<uint32_t>(gy), fpitch) + static_cast<uint32_t>(gx);
          uu[k] = ld_f32(vu, o);
          vv2[k] = ld_f32(vv, o);
        } else {
          uu[k] = 0.0f;
          vv2[k] = 0.0f;
        }
        ex += DX;
        ey += DY;
        if (ex >= EX) {
          ex -= EX;
          ++ey;
        }
      }
      if (MODE == FLOW_UPSAMPLE) {
        // V = 2 bilinear(V_coarse, x / 2, y / 2): taps of all CH pixels first
        float cu[CH][4], cv[CH][4], wx[CH], wy[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const BilTap tp = bil_setup(0.5f * fx[k], 0.5f * fy[k], cwm1, chm1, cwm2, chm2, fpitch);
          wx[k] = tp.ax;
          wy[k] = tp.ay;
          cu[k][0] = ld_f32(vu, tp.i);
          cu[k][1] = ld_f32(vu, tp.i + csx);
          cu[k][2] = ld_f32(vu, tp.i + csy);
          cu[k][3] = ld_f32(vu, tp.i + csy + csx);
          cv[k][0] = ld_f32(vv, tp.i);
          cv[k][1] = ld_f32(vv, tp.i + csx);
          cv[k][2] = ld_f32(vv, tp.i + csy);
          cv[k][3] = ld_f32(vv, tp.i + csy + csx);
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          uu[k] = 2.0f * bil_combine(cu[k][0], cu[k][1], cu[k][2], cu[k][3], wx[k], wy[k]);
          vv2[k] = 2.0f * bil_combine(cv[k][0], cv[k][1], cv[k][2], cv[k][3], wx[k], wy[k]);
        }
      }
      float g0[CH][4], g1[CH][4], a0x[CH], a0y[CH], a1x[CH], a1y[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        // symmetric: P0 at k - V/2, P1 at k + V/2; forward-additive: P0 at k
        // (through the same interpolation, so that equal planes give T = 0
        // exactly), P1 at k + V
        const float hu = fa ? 0.0f : 0.5f * uu[k];
        const float hv = fa ? 0.0f : 0.5f * vv2[k];
        const BilTap t0 = bil_setup(fx[k] - hu, fy[k] - hv, wm1, hm1, wm2, hm2, uip);
        const BilTap t1 = bil_setup(fx[k] + (fa ? uu[k] : hu), fy[k] + (fa ? vv2[k] : hv), wm1, hm1, wm2, hm2, uip);
        a0x[k] = t0.ax;
        a0y[k] = t0.ay;
        a1x[k] = t1.ax;
        a1y[k] = t1.ay;
        // levels are at least 2 x 2 here (the host sends thinner ones to
        // the march): the taps are (i, i + 1) on rows iy and iy + 1
        Px<TS>::ld2(v0, t0.i, 0, g0[k][0], g0[k][1]);
        Px<TS>::ld2(v0, t0.i, rowb, g0[k][2], g0[k][3]);
        Px<TS>::ld2(v1, t1.i, 0, g1[k][0], g1[k][1]);
        Px<TS>::ld2(v1, t1.i, rowb, g1[k][2], g1[k][3]);
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        if (k0 + k < NA) {
          const float w0 = bil_combine(g0[k][0], g0[k][1], g0[k][2], g0[k][3], a0x[k], a0y[k]);
          const float w1 = bil_combine(g1[k][0], g1[k][1], g1[k][2], g1[k][3], a1x[k], a1y[k]);
          kT[k0 + k] = w1 - w0;
          kU[k0 + k] = uu[k];
          kV[k0 + k] = vv2[k];
          if (tid + NT * (k0 + k) < NE) sS[oo[k]] = fa ? w1 : 0.5f * (w0 + w1);
        }
      }
    }
  }
  __syncthreads();

  // ---- A2: gradients, b and the five products of the product-region pixels.
  // The S reads of up to four of the lane's pixels are issued before any is
  // used (a pixel outside the product region reads an interior dummy and
  // stores nothing), so the LDS latency is not paid once per pixel.
  {
    constexpr int C2 = 4;
#pragma unroll
    for (int k0 = 0; k0 < NA; k0 += C2) {
      float sxp[C2], sxm[C2], syp[C2], sym[C2];
#pragma unroll
      for (int k = 0; k < C2; ++k) {
        if (k0 + k < NA) {
          // the four neighbours at non-negative offsets from the one above
          const int o = (kF & (1u << (2 * (k0 + k)))) ? kO[k0 + k] : LP + 1;
          const float* n = sS + (o - LP);
          sym[k] = n[0];
          sxm[k] = n[LP - 1];
          sxp[k] = n[LP + 1];
          syp[k] = n[2 * LP];
        }
      }
#pragma unroll
      for (int k = 0; k < C2; ++k) {
        if (k0 + k < NA) {
          const bool valid = kF & (2u << (2 * (k0 + k)));
          const float gx = valid ? 0.5f * (sxp[k] - sxm[k]) : 0.0f;
          const float gy = valid ? 0.5f * (syp[k] - sym[k]) : 0.0f;
          const float b = inc ? -kT[k0 + k] : fmaf(gx, kU[k0 + k], fmaf(gy, kV[k0 + k], -kT[k0 + k]));
          if (kF & (1u << (2 * (k0 + k)))) {
            const int o = kO[k0 + k];
            sP[o] = gx * gx;
            sP[o + PL] = gx * gy;
            sP[o + 2 * PL] = gy * gy;
            sP[o + 3 * PL] = gx * b;
            sP[o + 4 * PL] = gy * b;
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- B: horizontal window sums, item = (product row, segment of SL outputs)
  float hsum[NIT][5][SL];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * PY) {
      // ext column of the first product of the first window: product column c is ext column c + 1
      const int rb = (item % PY + 1) * LP + 1 + (item / PY) * SL;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const float* row = lds + lds_reg((q + 1) * PL + rb);
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
  // ---- B': the sum of output column j of product row r goes to element
  // j CP + r of the product's transposed plane (planes HPL apart from
  // HOFF): over the product planes once every lane has read them, or at
  // once into a region of their own
  if (!HSEP) __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int item = tid + NT * it;
    if (item < NSEG * PY) {
      const int cb = (item / PY) * SL * CP + item % PY;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float* col = lds + lds_reg(HOFF + q * HPL + cb);
#pragma unroll
        for (int jj = 0; jj < SL; ++jj) col[jj * CP] = hsum[it][q][jj];
      }
    }
  }
  // The up-sampled flow of the ext pixels on the tile's output rows, as A1
  // computed it, for the damping anchor of C (instead of eight more gathers
  // per output there), at their ext offsets less KR + 1 rows: U over the S
  // plane (free after A2), V past the transposed sums (free after B).
  // Slots past the ext region lie below the output rows.
  float* const sUm = lds;
  float* const sVm = lds + PL + 5 * HPL;
  if (STAGE_UV) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int d = kO[k] - (KR + 1) * LP;
      if (static_cast<unsigned>(d) < static_cast<unsigned>(TY * LP)) {
        sUm[d] = kU[k];
        sVm[d] = kV[k];
      }
    }
  }
  __syncthreads();

  // ---- C: vertical window sums, solve, store; item = (output column, segment)
  {
    constexpr int NSEGV = TY / SLV;
    const int j = tid % TX;
    const int sg = tid / TX;
    const int gx = x0 + j;
    if (sg < NSEGV && gx < W) {
      const uint32_t obytes = static_cast<uint32_t>(J.out_pitch) * static_cast<uint32_t>(H) * 4u;
      const PlaneView wu = plane_view(J.out_u, obytes);
      const PlaneView wv = plane_view(J.out_v, obytes);
      const int rs = sg * SLV;  // first product row of the first output's window
      // flow at the outputs (the damping anchor V(m)), loaded ahead of the sums
      float um[SLV], vm[SLV];
#pragma unroll
      for (int k = 0; k < SLV; ++k) {
        const int gy = min(y0 + rs + k, H - 1);
        if (MODE == FLOW_DIRECT) {
          const uint32_t o = __umul24(static_cast<uint32_t>(gy), fpitch) + static_cast<uint32_t>(gx);
          um[k] = ld_f32(vu, o);
          vm[k] = ld_f32(vv, o);
        } else if (STAGE_UV) {
          um[k] = sUm[(rs + k) * LP + KR + 1 + j];
          vm[k] = sVm[(rs + k) * LP + KR + 1 + j];
        } else if (MODE == FLOW_UPSAMPLE) {
          const BilTap tp = bil_setup(0.5f * static_cast<float>(gx), 0.5f * static_cast<float>(gy), cwm1, chm1,
                                      cwm2, chm2, fpitch);
          um[k] = 2.0f * bil_combine(ld_f32(vu, tp.i), ld_f32(vu, tp.i + csx), ld_f32(vu, tp.i + csy),
                                     ld_f32(vu, tp.i + csy + csx), tp.ax, tp.ay);
          vm[k] = 2.0f * bil_combine(ld_f32(vv, tp.i), ld_f32(vv, tp.i + csx), ld_f32(vv, tp.i + csy),
                                     ld_f32(vv, tp.i + csy + csx), tp.ax, tp.ay);
        } else {
          um[k] = 0.0f;
          vm[k] = 0.0f;
        }
      }
      const float* col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) col[q] = lds + lds_reg(HOFF + q * HPL + j * CP + rs);
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
          const int oy = rs + k - 2 * KR;  // output row within the tile
          const int gy = y0 + oy;
          if (gy < H) {
            float un, vn;
            solve2x2(acc[0], acc[1], acc[2], acc[3], acc[4], um[k - 2 * KR], vm[k - 2 * KR], a.reg_rel, a.reg_abs,
                     un, vn, inc, no_fp64);
            const uint32_t oo =
                (__umul24(static_cast<uint32_t>(gy), static_cast<uint32_t>(J.out_pitch)) + static_cast<uint32_t>(gx)) * 4u;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(un), wu, static_cast<int>(oo), 0, kStreamPolicy);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vn), wv, static_cast<int>(oo), 0, kStreamPolicy);
          }
        }
      }
    }
  }
}

template <int KR, int MODE, typename TS, int TX, int TY, int SL, int SLV, int NT, bool GEN = false>
hipError_t launch_gn_tile_cfg(const GnArgs& a, int nblocks, hipStream_t s) {
  constexpr size_t lds = sizeof(float) * TileLds<KR, TX, TY, NT>::FLOATS;
  auto kern = gn_tile_kernel<KR, MODE, TS, TX, TY, SL, SLV, NT, GEN>;
  // dynamic LDS above 64 KiB must be enabled once per kernel (thread-safe static init)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), lds, s, a);
  return hipGetLastError();
}

// variant GN_TILE_64x32: 64 x 32 outputs, 512 lanes (segments 8 columns / 4 rows);
// variant GN_TILE_64x16: 64 x 16 outputs, 256 lanes (segments 8 columns / 4 rows);
// variant GN_TILE_32x16: 32 x 16 outputs, 256 lanes (segments 4 columns / 2 rows);
// variant GN_TILE_16x16: 16 x 16 outputs, 256 lanes (segments 4 columns / 1 row);
// variants GN_TILE_64x32W / 64x16W: the same tiles with 1024 / 512 lanes
// (segments 8 columns / 2 rows), more waves to hide latency per compute unit;
// variant GN_TILE_64x64: 64 x 64 outputs, 1024 lanes (segments 8 columns / 4
// rows), the smallest halo, one workgroup per compute unit;
// variants GN_TILE_16x16W / 32x16W: the coarse-level tiles with 1024 / 512
// lanes, so that the warps of a tile are spread over more waves per SIMD;
// variant GN_TILE_32x32W: 32 x 32 outputs, 1024 lanes (segments 4 columns /
// 2 rows), two pixels per lane in A1 for mid-size levels.
// The small tiles spread coarse levels over many compute units: there the
// launch is bound by the instruction latency of few waves, not by traffic.
// generic (estimator variants read from a.est): 16 x 16 tiles whatever the variant.
template <int MODE, typename TS>
hipError_t launch_gn_tile_typed(const GnArgs& a, int kr, int variant, int nblocks, hipStream_t s, bool generic) {
#define OFV_GNT_CASE(R)                                                                             \
  case R:                                                                                           \
    if (generic) return launch_gn_tile_cfg<R, MODE, TS, 16, 16, 4, 1, 256, true>(a, nblocks, s);     \
    switch (variant) {                                                                              \
      case GN_TILE_64x32: return launch_gn_tile_cfg<R, MODE, TS, 64, 32, 8, 4, 512>(a, nblocks, s);  \
      case GN_TILE_64x16: return launch_gn_tile_cfg<R, MODE, TS, 64, 16, 8, 4, 256>(a, nblocks, s);  \
      case GN_TILE_32x16: return launch_gn_tile_cfg<R, MODE, TS, 32, 16, 4, 2, 256>(a, nblocks, s);  \
      case GN_TILE_64x32W: return launch_gn_tile_cfg<R, MODE, TS, 64, 32, 8, 2, 1024>(a, nblocks, s); \
      case GN_TILE_64x16W: return launch_gn_tile_cfg<R, MODE, TS, 64, 16, 8, 2, 512>(a, nblocks, s);  \
      case GN_TILE_64x64: return launch_gn_tile_cfg<R, MODE, TS, 64, 64, 8, 4, 1024>(a, nblocks, s);  \
      case GN_TILE_16x16W: return launch_gn_tile_cfg<R, MODE, TS, 16, 16, 4, 1, 1024>(a, nblocks, s); \
      case GN_TILE_32x16W: return launch_gn_tile_cfg<R, MODE, TS, 32, 16, 4, 2, 512>(a, nblocks, s);  \
      case GN_TILE_32x32W: return launch_gn_tile_cfg<R, MODE, TS, 32, 32, 4, 2, 1024>(a, nblocks, s); \
      default: return launch_gn_tile_cfg<R, MODE, TS, 16, 16, 4, 1, 256>(a, nblocks, s);            \
    }
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
