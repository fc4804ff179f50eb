// Fused symmetric Gauss-Newton iteration, band-march variant (pipeline steps
// 3 and 5 of section "Live-Optical Flow Velocimetry", Eq. of_symmetric,
// arXiv 2509.25924): same arithmetic as the tile and strip-march variants,
// a decomposition whose window-sum cost does not grow with the window, for
// large levels (several Mi pixels, large KR).
//
// A 256-lane workgroup owns a strip of 256 consecutive columns (lane = ext
// column: KR + 1 halo columns on each side of TX = 254 - 2 KR output
// columns) and tile_h output rows, and marches down the product rows of its
// tile in blocks of BY rows.  Per block:
//  A1. each lane evaluates its column at the block's BY new rows: input flow
//      (loaded two blocks ahead, or up-sampled), the two midpoint bilinear
//      warps, S and T.  Lanes are consecutive columns, so every gather of a
//      wavefront touches a few cache lines.  The taps are issued one block
//      ahead, right after the previous block's products (float32 planes:
//      half of the rows there, half after its horizontal sums), and stay
//      in flight behind its window sums.  S of the block's rows -> LDS.
//  A2. Gx from the neighbouring lanes' S (LDS), Gy from the lane's own
//      rows, b = G . V - T and the five products -> BY rows of five LDS
//      planes (0 outside the level).
//  B.  horizontal window sums by running sums: one item per (product,
//      row, segment of SL outputs), 5 BY NSEG items over the 256 lanes.
//  C.  vertical window sums: each output lane keeps the sum of the last
//      2 KR horizontal sums of its column and those sums in a register ring
//      indexed by the (wavefront-uniform) row number, so the vertical pass
//      costs two additions per product and row whatever KR; damped 2x2
//      solve and store of every completed output row.
// The horizontal segment ends are the only repeated work; the vertical halo
// (2 KR + 2 rows) is paid once per tile, and the host sizes the tiles so that
// one round of resident workgroups covers the level.
#pragma once

#include <type_traits>
#include <utility>

#include "ofv_gn_tile.h"

namespace ofv {

constexpr int kBandThreads = 256;

template <int KR, int BY>
struct BandGeom {
  static constexpr int NWIN = 2 * KR + 1;
  static constexpr int TX = kBandThreads - 2 * KR - 2;  // output columns of a strip
  static constexpr int PP = kBandThreads + 1;           // odd pitch of the product and sum rows
  static constexpr int NROW = 5 * BY;                   // (product, row) pairs of a block
  static constexpr int NSEG = kBandThreads / NROW;      // segments per row: NROW * NSEG items <= 256
  static constexpr int SL = (TX + NSEG - 1) / NSEG;     // outputs per segment
  static_assert(NSEG >= 1, "block too tall for one item per (product, row, segment)");
  // LDS (floats): S rows of the block, products, horizontal sums.  A
  // segment reads SL + 2 KR products from lane seg * SL + 1 on and writes SL
  // sums from column seg * SL on, up to NSEG * SL + 2 KR + 1 <= TX + NSEG + 2 KR
  // entries into its row; the 64 floats after each region keep the last
  // row's overrun inside the allocation (overrun entries are never used).
  // ANCH (KR >= 6, where registers already hold the kernel to two
  // workgroups per compute unit): the input field of the last AR ext rows,
  // u then v per row, a ring from which the vertical pass takes the damping
  // anchor V(m) of each output row instead of reading the field again.
  static constexpr bool ANCH = KR >= 6;
  static constexpr int AR = BY + KR + 1;
  static constexpr int S_OFF = 0;
  static constexpr int P_OFF = S_OFF + BY * kBandThreads;
  static constexpr int H_OFF = P_OFF + NROW * PP + 64;
  static constexpr int A_OFF = H_OFF + NROW * PP + 64;
  static constexpr int FLOATS = A_OFF + (ANCH ? AR * 2 * kBandThreads : 0);
  static_assert(TX + NSEG + 2 * KR <= PP + 64, "segment overrun fits in the slack");
};

// The bilinear taps of the two warps of n pixels of one column (rows gy0 ..
// gy0 + n - 1, clamped into the level) for the flow (u, v) of each, issued
// by band_issue and combined into S and T by band_finish: between the two
// the loads are in flight behind other work.
template <int N>
struct BandTaps {
  float g0[N][4], g1[N][4], a0x[N], a0y[N], a1x[N], a1y[N];
  float u[N], v[N];  // the flow the warps used
};

// Rows n0 .. n1 - 1 of the n rows (gy0 + n).
template <int N, typename TS, int N0 = 0, int N1 = N>
__device__ __forceinline__ void band_issue(BandTaps<N>& q, PlaneView v0, PlaneView v1, uint32_t ip, uint32_t rowb,
                                           float fx, int gy0, int H, float wm1, float hm1, float wm2, float hm2,
                                           const float* u, const float* v, bool fa) {
#pragma unroll
  for (int n = N0; n < N1; ++n) {
    const float fy = static_cast<float>(min(max(gy0 + n, 0), H - 1));
    const float hu = fa ? 0.0f : 0.5f * u[n];
    const float hv = fa ? 0.0f : 0.5f * v[n];
    const BilTap t0 = bil_setup(fx - hu, fy - hv, wm1, hm1, wm2, hm2, ip);
    const BilTap t1 = bil_setup(fx + (fa ? u[n] : hu), fy + (fa ? v[n] : hv), wm1, hm1, wm2, hm2, ip);
    q.a0x[n] = t0.ax;
    q.a0y[n] = t0.ay;
    q.a1x[n] = t1.ax;
    q.a1y[n] = t1.ay;
    q.u[n] = u[n];
    q.v[n] = v[n];
    Px<TS>::ld2(v0, t0.i, 0, q.g0[n][0], q.g0[n][1]);
    Px<TS>::ld2(v0, t0.i, rowb, q.g0[n][2], q.g0[n][3]);
    Px<TS>::ld2(v1, t1.i, 0, q.g1[n][0], q.g1[n][1]);
    Px<TS>::ld2(v1, t1.i, rowb, q.g1[n][2], q.g1[n][3]);
  }
}

template <int N>
__device__ __forceinline__ void band_finish(const BandTaps<N>& q, bool fa, float* s, float* t) {
#pragma unroll
  for (int n = 0; n < N; ++n) {
    const float w0 = bil_combine(q.g0[n][0], q.g0[n][1], q.g0[n][2], q.g0[n][3], q.a0x[n], q.a0y[n]);
    const float w1 = bil_combine(q.g1[n][0], q.g1[n][1], q.g1[n][2], q.g1[n][3], q.a1x[n], q.a1y[n]);
    s[n] = fa ? w1 : 0.5f * (w0 + w1);
    t[n] = w1 - w0;
  }
}

// 2 bilinear(V_coarse, x / 2, y / 2) at n pixels of one column: taps of all
// n first.
template <int N>
__device__ __forceinline__ void band_upsample(PlaneView vu, PlaneView vv, uint32_t fpitch, float hx, int gy0, int H,
                                              float cwm1, float chm1, float cwm2, float chm2, uint32_t csx,
                                              uint32_t csy, float* u, float* v) {
  float cu[N][4], cv[N][4], wx[N], wy[N];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    const float hy = 0.5f * static_cast<float>(min(max(gy0 + n, 0), H - 1));
    const BilTap tp = bil_setup(hx, hy, cwm1, chm1, cwm2, chm2, fpitch);
    wx[n] = tp.ax;
    wy[n] = tp.ay;
    cu[n][0] = ld_f32(vu, tp.i);
    cu[n][1] = ld_f32(vu, tp.i + csx);
    cu[n][2] = ld_f32(vu, tp.i + csy);
    cu[n][3] = ld_f32(vu, tp.i + csy + csx);
    cv[n][0] = ld_f32(vv, tp.i);
    cv[n][1] = ld_f32(vv, tp.i + csx);
    cv[n][2] = ld_f32(vv, tp.i + csy);
    cv[n][3] = ld_f32(vv, tp.i + csy + csx);
  }
#pragma unroll
  for (int n = 0; n < N; ++n) {
    u[n] = 2.0f * bil_combine(cu[n][0], cu[n][1], cu[n][2], cu[n][3], wx[n], wy[n]);
    v[n] = 2.0f * bil_combine(cv[n][0], cv[n][1], cv[n][2], cv[n][3], wx[n], wy[n]);
  }
}

// One row of the vertical window sum of a product.  `part` holds the sum of
// the window's first 2 KR rows and the ring those 2 KR horizontal sums, the
// oldest in `slot`: the window sum is part + h, after which the oldest
// leaves part and h takes its slot.  `slot` is uniform across the
// wavefront, so the array stays in registers, indexed relative to a scalar
// base.
template <int N>
__device__ __forceinline__ float band_ring(float (&ring)[N], int slot, float& part, float h) {
  const float full = part + h;
  part = full - ring[slot];
  ring[slot] = h;
  return full;
}

// f(std::integral_constant<int, I>()) for the one I of the sequence equal to
// i (wavefront-uniform: a chain of scalar compares, one inlined copy of f
// per I).
template <typename F, int... I>
__device__ __forceinline__ void band_dispatch(int i, F&& f, std::integer_sequence<int, I...>) {
  (void)((i == I ? (f(std::integral_constant<int, I>()), true) : false) || ...);
}

// The vertical rings.  A register array indexed at run time occupies a
// register tuple, and tuples come in 1-12 and 16 registers (an 18- to
// 32-float array takes 32).  A ring of 2 KR = 16 + 4 m floats (KR 10, 12) is
// therefore split into a 16-float array indexed at run time and a 4 m-float
// tail; a block's BY = 4 rows then fall in one of the two, and the tail is
// indexed by compile-time constants (one copy of the vertical pass per
// 4-slot group of the tail).  The other windows keep one array (KR 9 and 11:
// padded to 32 registers).
// Registers per lane: the rings, the next block's taps in flight (issued
// after the block's products, `pipelined`) where they fit beside them, the
// block's rows: up to 256 (2 waves per SIMD).
template <int KR>
struct BandOcc {
  static constexpr int value = 2;
  static constexpr int NR = 2 * KR;  // ring length
  static constexpr bool split = NR > 16 && NR % 4 == 0;
  static constexpr int A = split ? 16 : NR;      // run-time indexed part
  static constexpr int B = split ? NR - 16 : 1;  // compile-time indexed tail (unused unless split)
  static constexpr bool pipelined = KR <= 10 && (KR <= 8 || split);
};

// GEN: the estimator variant is read from a.est at run time (forward-additive
// warps, increment-form update); otherwise the symmetric estimator's
// consistent update is compiled in.
template <int KR, int MODE, typename TS, int BY, bool GEN = false>
__global__ __launch_bounds__(kBandThreads) __attribute__((amdgpu_waves_per_eu(BandOcc<KR>::value)))
void gn_band_kernel(const GnArgs a) {
  using G = BandGeom<KR, BY>;
  constexpr int NWIN = G::NWIN, TX = G::TX, PP = G::PP, NROW = G::NROW, NSEG = G::NSEG, SL = G::SL;
  constexpr int NR = 2 * KR;  // vertical ring length
  extern __shared__ float lds[];
  const bool fa = GEN && (a.est & EST_FORWARD_ADDITIVE) != 0;
  const bool inc = GEN && (a.est & EST_INCREMENT) != 0;
  const bool no_fp64 = (a.est & EST_NO_FP64) != 0;

  const int jb = find_job(a, blockIdx.x);
  const GnJob& J = a.job[jb];
  const int W = J.w;
  const int H = J.h;
  const int TH = a.tile_h;
  const int ntx = (W + TX - 1) / TX;
  const int nty = (H + TH - 1) / TH;
  // strip-major tile order: consecutive tiles are vertical neighbours, and
  // the XCD renumbering gives each XCD a contiguous run of them
  const int tile = xcd_tile(blockIdx.x - J.tile_start, ntx * nty);
  const int x0 = (tile / nty) * TX;
  const int y0 = (tile % nty) * TH;
  const int tid = threadIdx.x;
  const int gxr = x0 - KR - 1 + tid;  // level column of this lane's ext column
  const int gx = min(max(gxr, 0), W - 1);
  const bool prod_lane = tid >= 1 && tid <= kBandThreads - 2 && static_cast<unsigned>(gxr) < static_cast<unsigned>(W);
  const int oc = tid - KR - 1;        // output column within the strip
  const bool out_lane = oc >= 0 && oc < TX && x0 + oc < W;
  const int rows = min(TH, H - y0);   // output rows of this tile
  const int NP = rows + 2 * KR;       // product rows
  const int nblk = (NP + BY - 1) / BY;
  const int ey0 = y0 - KR - 1;        // level row of ext row 0 (product row i sits at ext row i + 1)

  const uint32_t ip = static_cast<uint32_t>(J.img_pitch);
  const uint32_t rowb = ip * Px<TS>::bytes;
  const PlaneView v0 = plane_view(J.p0, ip * static_cast<uint32_t>(H) * Px<TS>::bytes);
  const PlaneView v1 = plane_view(J.p1, ip * static_cast<uint32_t>(H) * Px<TS>::bytes);
  const float wm1 = static_cast<float>(W - 1), hm1 = static_cast<float>(H - 1);
  const float wm2 = static_cast<float>(W - 2), hm2 = static_cast<float>(H - 2);
  const uint32_t fpitch = static_cast<uint32_t>(J.in_pitch);
  const uint32_t frows = static_cast<uint32_t>(MODE == FLOW_UPSAMPLE ? J.ch : H);
  const PlaneView vu = plane_view(J.in_u, MODE == FLOW_ZERO ? 0u : fpitch * frows * 4u);
  const PlaneView vv = plane_view(J.in_v, MODE == FLOW_ZERO ? 0u : fpitch * frows * 4u);
  const float cwm1 = static_cast<float>(J.cw - 1), chm1 = static_cast<float>(J.ch - 1);
  const float cwm2 = static_cast<float>(J.cw - 2), chm2 = static_cast<float>(J.ch - 2);
  const uint32_t csx = J.cw > 1 ? 1u : 0u;
  const uint32_t csy = J.ch > 1 ? fpitch : 0u;
  const float fx = static_cast<float>(gx);
  const float hx = 0.5f * fx;

  // Input flow of n rows of this lane's column from level row gy0 on.
  auto flow_rows = [&](auto nrows, int gy0, float* u, float* v) {
    constexpr int N = decltype(nrows)::value;
    if (MODE == FLOW_DIRECT) {
#pragma unroll
      for (int n = 0; n < N; ++n) {
        const uint32_t o = __umul24(static_cast<uint32_t>(min(max(gy0 + n, 0), H - 1)), fpitch) +
                           static_cast<uint32_t>(gx);
        u[n] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(vu, static_cast<int>(o * 4u), 0,
                                                                     kStreamPolicy));
        v[n] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(vv, static_cast<int>(o * 4u), 0,
                                                                     kStreamPolicy));
      }
    } else if (MODE == FLOW_UPSAMPLE) {
      band_upsample<N>(vu, vv, fpitch, hx, gy0, H, cwm1, chm1, cwm2, chm2, csx, csy, u, v);
    } else {
#pragma unroll
      for (int n = 0; n < N; ++n) u[n] = v[n] = 0.0f;
    }
  };

  // sR[m]: S at ext row k BY + m (m = 0 .. BY + 1); tR/uR/vR[j]: T, U, V at
  // ext row k BY + 1 + j (j = 0 .. BY), for block k
  float sR[BY + 2], tR[BY + 1], uR[BY + 1], vR[BY + 1];
  {
    float u2[2], v2[2], s2[2], t2[2];
    flow_rows(std::integral_constant<int, 2>(), ey0, u2, v2);
    BandTaps<2> q2;
    band_issue<2, TS>(q2, v0, v1, ip, rowb, fx, ey0, H, wm1, hm1, wm2, hm2, u2, v2, fa);
    band_finish<2>(q2, fa, s2, t2);
    sR[0] = s2[0];
    sR[1] = s2[1];
    tR[0] = t2[1];
    uR[0] = u2[1];
    vR[0] = v2[1];
  }
  // Pipeline (PIPE): the taps of block k + 1 are issued right after block
  // k's products and combined after its window sums, and a loaded input
  // field (FLOW_DIRECT) is read two blocks ahead.  Without PIPE (large KR,
  // whose rings leave no registers for taps in flight) a block's taps are
  // issued at its start and the field is read one block ahead.
  constexpr bool PIPE = BandOcc<KR>::pipelined;
  // float32 planes: the next block's taps go out in two halves, after A2 and after B (measured
  // at 5120 x 4096: 5 % less time at KR 5, 2 % at KR 7; with 16-bit planes, whose taps are half
  // the bytes, one burst after A2 is 2-9 % faster)
  constexpr bool SPLIT = PIPE && Px<TS>::bytes == 4;
  BandTaps<BY> taps;     // PIPE: block k + 1's taps, in flight during B and C of block k
  float fu[BY], fv[BY];  // FLOW_DIRECT: the field of the next block whose taps are not yet issued
  {
    float u[BY], v[BY];
    if (PIPE) {
      flow_rows(std::integral_constant<int, BY>(), ey0 + 2, u, v);
      band_issue<BY, TS>(taps, v0, v1, ip, rowb, fx, ey0 + 2, H, wm1, hm1, wm2, hm2, u, v, fa);
      if (MODE == FLOW_DIRECT && nblk > 1) flow_rows(std::integral_constant<int, BY>(), ey0 + 2 + BY, fu, fv);
    } else if (MODE == FLOW_DIRECT) {
      flow_rows(std::integral_constant<int, BY>(), ey0 + 2, fu, fv);
    }
  }

  using O = BandOcc<KR>;
  static_assert(!O::split || BY == 4, "split rings assume 4-row blocks");
  float rg0[O::A], rg1[O::A], rg2[O::A], rg3[O::A], rg4[O::A];  // rings (split: slots 0..15)
  float rt0[O::B], rt1[O::B], rt2[O::B], rt3[O::B], rt4[O::B];  // split: slots 16..NR-1
#pragma unroll
  for (int n = 0; n < O::A; ++n) rg0[n] = rg1[n] = rg2[n] = rg3[n] = rg4[n] = 0.0f;
#pragma unroll
  for (int n = 0; n < O::B; ++n) rt0[n] = rt1[n] = rt2[n] = rt3[n] = rt4[n] = 0.0f;
  float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, acc3 = 0.0f, acc4 = 0.0f;
  int slot = 0;  // ring slot of the block's first row

  const uint32_t obytes = static_cast<uint32_t>(J.out_pitch) * static_cast<uint32_t>(H) * 4u;
  const PlaneView wu = plane_view(J.out_u, obytes);
  const PlaneView wv = plane_view(J.out_v, obytes);

  for (int k = 0; k < nblk; ++k) {
    const int e0 = k * BY + 2;  // first ext row of this block's new rows
    // ---- A1: the block's BY new rows (ext rows e0 .. e0 + BY - 1)
    if (!PIPE) {
      float u[BY], v[BY];
      if (MODE == FLOW_DIRECT) {
#pragma unroll
        for (int n = 0; n < BY; ++n) {
          u[n] = fu[n];
          v[n] = fv[n];
        }
      } else {
        flow_rows(std::integral_constant<int, BY>(), ey0 + e0, u, v);
      }
      band_issue<BY, TS>(taps, v0, v1, ip, rowb, fx, ey0 + e0, H, wm1, hm1, wm2, hm2, u, v, fa);
    }
    {
      float s[BY], t[BY];
      band_finish<BY>(taps, fa, s, t);
#pragma unroll
      for (int n = 0; n < BY; ++n) {
        sR[2 + n] = s[n];
        tR[1 + n] = t[n];
        uR[1 + n] = taps.u[n];
        vR[1 + n] = taps.v[n];
      }
    }
    // damping anchor V(m) of the output rows this block completes.  ANCH:
    // from the LDS ring in C.  Otherwise read again from the field: PIPE, in
    // flight until C; else loaded at the start of C (fewer live registers).
    const int gm0 = y0 + k * BY - 2 * KR;  // level row of the block's first output (if any)
    float um[BY], vm[BY];
    auto load_anchors = [&]() {
#pragma unroll
      for (int j = 0; j < BY; ++j) {
        const uint32_t o = __umul24(static_cast<uint32_t>(min(max(gm0 + j, 0), H - 1)), fpitch) +
                           static_cast<uint32_t>(gx);
        um[j] = ld_f32(vu, o);
        vm[j] = ld_f32(vv, o);
      }
    };
    if (MODE == FLOW_DIRECT && PIPE && !G::ANCH) load_anchors();
    // S of ext rows k BY + 1 .. k BY + BY (the product rows' own rows) for Gx
#pragma unroll
    for (int j = 0; j < BY; ++j) lds[G::S_OFF + j * kBandThreads + tid] = sR[1 + j];
    __syncthreads();
    // ---- A2: gradients, b and the five products of product rows k BY + j
    if (G::ANCH) {
      // the field of the block's new ext rows k BY + 2 .. k BY + BY + 1 into the anchor ring.  The
      // vertical pass of block k - 1 read its anchors before the barrier above, and this block's
      // reads come after the next ones; rows k BY - KR + 1 .. k BY + BY + 1 (AR rows) are live.
#pragma unroll
      for (int j = 1; j <= BY; ++j) {
        const int slot_a = (k * BY + 1 + j) % G::AR;
        lds[G::A_OFF + slot_a * 2 * kBandThreads + tid] = uR[j];
        lds[G::A_OFF + slot_a * 2 * kBandThreads + kBandThreads + tid] = vR[j];
      }
    }
    {
      const int tl = max(tid - 1, 0);
      const int tr = min(tid + 1, kBandThreads - 1);
#pragma unroll
      for (int j = 0; j < BY; ++j) {
        const int i = k * BY + j;
        const int pr = y0 - KR + i;
        const float sl = lds[G::S_OFF + j * kBandThreads + tl];
        const float sr = lds[G::S_OFF + j * kBandThreads + tr];
        const bool valid = prod_lane && static_cast<unsigned>(pr) < static_cast<unsigned>(H) && i < NP;
        const float gxv = valid ? 0.5f * (sr - sl) : 0.0f;
        const float gyv = valid ? 0.5f * (sR[j + 2] - sR[j]) : 0.0f;
        const float b = inc ? -tR[j] : fmaf(gxv, uR[j], fmaf(gyv, vR[j], -tR[j]));
        float* p = lds + G::P_OFF + j * PP + tid;
        p[0] = gxv * gxv;
        p[BY * PP] = gxv * gyv;
        p[2 * BY * PP] = gyv * gyv;
        p[3 * BY * PP] = gxv * b;
        p[4 * BY * PP] = gyv * b;
      }
    }
    // the next block's taps, in flight behind the window sums
    if (PIPE && k + 1 < nblk) {
      float u[BY], v[BY];
      if (MODE == FLOW_DIRECT) {
#pragma unroll
        for (int n = 0; n < BY; ++n) {
          u[n] = fu[n];
          v[n] = fv[n];
        }
      } else {
        flow_rows(std::integral_constant<int, BY>(), ey0 + e0 + BY, u, v);
      }
      if (SPLIT) {
        // the first half of the rows here, the rest after B
#pragma unroll
        for (int n = 0; n < BY; ++n) {
          taps.u[n] = u[n];
          taps.v[n] = v[n];
        }
        band_issue<BY, TS, 0, BY / 2>(taps, v0, v1, ip, rowb, fx, ey0 + e0 + BY, H, wm1, hm1, wm2, hm2, u, v, fa);
      } else {
        band_issue<BY, TS>(taps, v0, v1, ip, rowb, fx, ey0 + e0 + BY, H, wm1, hm1, wm2, hm2, u, v, fa);
        if (MODE == FLOW_DIRECT && k + 2 < nblk)
          flow_rows(std::integral_constant<int, BY>(), ey0 + e0 + 2 * BY, fu, fv);
      }
    }
    // without PIPE: the next block's field, in flight behind the window sums
    if (!PIPE && MODE == FLOW_DIRECT && k + 1 < nblk)
      flow_rows(std::integral_constant<int, BY>(), ey0 + e0 + BY, fu, fv);
    __syncthreads();
    // ---- B: horizontal window sums, item = (product row r = q BY + j, segment).
    // The sums' row is a constant distance from the products' row, both off
    // one base register the compiler treats as opaque: reads keep small
    // immediate offsets, and the compiler still sees that no store overlaps a
    // read, so the running sum streams its reads ahead of its stores.
    {
      const int r = tid % NROW;
      const int seg = tid / NROW;
      if (seg < NSEG) {
        // without PIPE (large KR, registers at the limit) the sums take a base
        // register of their own: fewer address registers, stores and reads in order
        float* const row = lds + lds_reg(G::P_OFF + r * PP + seg * SL + 1);
        float* const hrow = PIPE ? row + (G::H_OFF - G::P_OFF - 1) : lds + lds_reg(G::H_OFF + r * PP + seg * SL);
        float ring[NWIN];
        float acc = 0.0f;
#pragma unroll
        for (int n = 0; n < SL + 2 * KR; ++n) {
          const float pq = row[n];
          if (n >= NWIN) acc -= ring[n % NWIN];
          ring[n % NWIN] = pq;
          acc = n == 0 ? pq : acc + pq;
          if (n >= 2 * KR) hrow[n - 2 * KR] = acc;
        }
      }
    }
    __syncthreads();
    // the second half of the next block's taps and, two blocks ahead, the field
    if (SPLIT && k + 1 < nblk) {
      band_issue<BY, TS, BY / 2, BY>(taps, v0, v1, ip, rowb, fx, ey0 + e0 + BY, H, wm1, hm1, wm2, hm2, taps.u, taps.v,
                                     fa);
      if (MODE == FLOW_DIRECT && k + 2 < nblk) flow_rows(std::integral_constant<int, BY>(), ey0 + e0 + 2 * BY, fu, fv);
    }
    // ---- C: vertical window sums, solve and store of the completed output rows
    {
      if (!G::ANCH) {
        if (MODE == FLOW_DIRECT && !PIPE) load_anchors();
        if (MODE == FLOW_UPSAMPLE && out_lane) {
          band_upsample<BY>(vu, vv, fpitch, hx, gm0, H, cwm1, chm1, cwm2, chm2, csx, csy, um, vm);
        } else if (MODE == FLOW_ZERO) {
#pragma unroll
          for (int j = 0; j < BY; ++j) um[j] = vm[j] = 0.0f;
        }
      }
      // solve and store of output row m = k BY + j - 2 KR from its window sums
      auto finish_row = [&](int j, float f0, float f1, float f2, float f3, float f4) {
        const int m = k * BY + j - 2 * KR;  // output row within the tile
        if (m >= 0 && m < rows) {
          float un, vn;
          if (G::ANCH) {
            // V(m): the field of ext row m + KR + 1 (the same value the warps of that row used)
            const int slot_a = (m + KR + 1) % G::AR;
            um[j] = MODE == FLOW_ZERO ? 0.0f : lds[G::A_OFF + slot_a * 2 * kBandThreads + tid];
            vm[j] = MODE == FLOW_ZERO ? 0.0f : lds[G::A_OFF + slot_a * 2 * kBandThreads + kBandThreads + tid];
          }
          solve2x2(f0, f1, f2, f3, f4, um[j], vm[j], a.reg_rel, a.reg_abs, un, vn, inc, no_fp64);
          const uint32_t oo = (__umul24(static_cast<uint32_t>(y0 + m), static_cast<uint32_t>(J.out_pitch)) +
                               static_cast<uint32_t>(gx)) * 4u;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(un), wu, static_cast<int>(oo), 0, kStreamPolicy);
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vn), wv, static_cast<int>(oo), 0, kStreamPolicy);
        }
      };
      const int sl0 = __builtin_amdgcn_readfirstlane(slot);
      const float* hcol = lds + lds_reg(G::H_OFF + oc);
      if (!O::split || sl0 < 16) {
#pragma unroll
        for (int j = 0; j < BY; ++j) {
          // slot of row j: split rings hold 4-row blocks in slots 4 g .. 4 g + 3
          const int sl = O::split ? sl0 + j : __builtin_amdgcn_readfirstlane((sl0 + j) % NR);
          if (out_lane) {
            float f0, f1, f2, f3, f4;  // the window sums of this row
            if (PIPE) {
              // the row's five horizontal sums of this column, read before the ring updates
              float hv[5];
#pragma unroll
              for (int q = 0; q < 5; ++q) hv[q] = hcol[(q * BY + j) * PP];
              f0 = band_ring(rg0, sl, acc0, hv[0]);
              f1 = band_ring(rg1, sl, acc1, hv[1]);
              f2 = band_ring(rg2, sl, acc2, hv[2]);
              f3 = band_ring(rg3, sl, acc3, hv[3]);
              f4 = band_ring(rg4, sl, acc4, hv[4]);
            } else {
              f0 = band_ring(rg0, sl, acc0, hcol[j * PP]);
              f1 = band_ring(rg1, sl, acc1, hcol[(BY + j) * PP]);
              f2 = band_ring(rg2, sl, acc2, hcol[(2 * BY + j) * PP]);
              f3 = band_ring(rg3, sl, acc3, hcol[(3 * BY + j) * PP]);
              f4 = band_ring(rg4, sl, acc4, hcol[(4 * BY + j) * PP]);
            }
            finish_row(j, f0, f1, f2, f3, f4);
          }
        }
      } else {
        // the block's rows are tail slots 16 + 4 g .. 16 + 4 g + 3: one copy per g
        auto tail = [&](auto gc) {
          constexpr int t0 = 4 * decltype(gc)::value;
#pragma unroll
          for (int j = 0; j < BY; ++j) {
            if (out_lane) {
              float hv[5];
#pragma unroll
              for (int q = 0; q < 5; ++q) hv[q] = hcol[(q * BY + j) * PP];
              const float f0 = band_ring(rt0, t0 + j, acc0, hv[0]);
              const float f1 = band_ring(rt1, t0 + j, acc1, hv[1]);
              const float f2 = band_ring(rt2, t0 + j, acc2, hv[2]);
              const float f3 = band_ring(rt3, t0 + j, acc3, hv[3]);
              const float f4 = band_ring(rt4, t0 + j, acc4, hv[4]);
              finish_row(j, f0, f1, f2, f3, f4);
            }
          }
        };
        band_dispatch((sl0 - 16) / 4, tail, std::make_integer_sequence<int, O::B / 4>());
      }
      slot = (sl0 + BY) % NR;
    }
    // rows carried into the next block
    sR[0] = sR[BY];
    sR[1] = sR[BY + 1];
    tR[0] = tR[BY];
    uR[0] = uR[BY];
    vR[0] = vR[BY];
  }
}

template <int KR, int MODE, typename TS, int BY, bool GEN = false>
hipError_t launch_gn_band_cfg(const GnArgs& a, int nblocks, hipStream_t s) {
  constexpr size_t lds = sizeof(float) * BandGeom<KR, BY>::FLOATS;
  auto kern = gn_band_kernel<KR, MODE, TS, BY, GEN>;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     static_cast<int>(lds));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kBandThreads), lds, s, a);
  return hipGetLastError();
}

// Workgroups of one band kernel that fit on a compute unit at once (0 on error).
template <int KR, int MODE, typename TS, int BY, bool GEN = false>
int gn_band_cfg_per_cu() {
  constexpr size_t lds = sizeof(float) * BandGeom<KR, BY>::FLOATS;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gn_band_kernel<KR, MODE, TS, BY, GEN>, kBandThreads, lds) !=
      hipSuccess)
    return 0;
  return n;
}

// Band kernels of one storage type and input-flow mode (symmetric estimator,
// consistent update), by window radius.
template <int MODE, typename TS>
hipError_t launch_gn_band_typed(const GnArgs& a, int kr, int nblocks, hipStream_t s) {
  switch (kr) {
#define OFV_GNB_CASE(R) \
  case R: return launch_gn_band_cfg<R, MODE, TS, 4>(a, nblocks, s);
    OFV_GNB_CASE(1)
    OFV_GNB_CASE(2)
    OFV_GNB_CASE(3)
    OFV_GNB_CASE(4)
    OFV_GNB_CASE(5)
    OFV_GNB_CASE(6)
    OFV_GNB_CASE(7)
    OFV_GNB_CASE(8)
    OFV_GNB_CASE(9)
    OFV_GNB_CASE(10)
    OFV_GNB_CASE(11)
    OFV_GNB_CASE(12)
#undef OFV_GNB_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int MODE, typename TS>
int gn_band_typed_per_cu(int kr) {
  switch (kr) {
#define OFV_GNB_CASE(R) \
  case R: return gn_band_cfg_per_cu<R, MODE, TS, 4>();
    OFV_GNB_CASE(1)
    OFV_GNB_CASE(2)
    OFV_GNB_CASE(3)
    OFV_GNB_CASE(4)
    OFV_GNB_CASE(5)
    OFV_GNB_CASE(6)
    OFV_GNB_CASE(7)
    OFV_GNB_CASE(8)
    OFV_GNB_CASE(9)
    OFV_GNB_CASE(10)
    OFV_GNB_CASE(11)
    OFV_GNB_CASE(12)
#undef OFV_GNB_CASE
    default: return 0;
  }
}

}  // namespace ofv
