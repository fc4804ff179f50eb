// Fused symmetric Gauss-Newton iteration (pipeline steps 3 and 5 of section
// "Live-Optical Flow Velocimetry", Eq. of_symmetric, arXiv 2509.25924).
//
// One launch performs one Jacobi iteration at one pyramid level for up to
// kMaxJobs image pairs.  Per pixel k it computes the midpoint warps
// W0 = P0(k - V/2), W1 = P1(k + V/2), S = (W0 + W1)/2, T = W1 - W0, the
// central-difference gradient G of S, b = G.V(k) - T and the five products
// Gx^2, GxGy, Gy^2, Gx b, Gy b; per pixel m it sums those products over the
// (2KR+1)^2 window truncated to the image and solves the damped 2x2 system
//   (A + lam I) V'(m) = c + lam V(m),   lam = reg_rel (Sxx + Syy) + reg_abs.
//
// Work decomposition (memory-bound stencil, no dense contraction):
//  * a 256-lane workgroup owns a strip of 256 consecutive columns: 2KR+2
//    halo columns plus TX = 254 - 2KR output columns, one column per lane;
//  * it marches down TY output rows (plus 2KR+2 halo rows).  The march is
//    software-pipelined so no global-memory latency sits on its critical
//    path: the flow of row r+3 is requested while the bilinear gathers of
//    row r+2 are in flight and row r+1's S/T are being formed (workgroup
//    barriers on gfx950 only wait for LDS, so loads stay in flight);
//  * the S row goes through LDS for the horizontal gradient; the vertical
//    gradient comes from the lane's own registers;
//  * horizontal window sums: a DPP inclusive prefix scan per wavefront
//    (six row-shift / row-broadcast steps), the prefix row through LDS, and
//    a difference of two prefixes (plus the neighbouring wavefront's total
//    where a window spans two wavefronts);
//  * vertical window sums: running sums over a ring of the last 2KR+1
//    horizontal sums held in registers (the march is unrolled by 2KR+1 so
//    every ring index is static); the damping term's V(m) comes from a
//    register ring of the same depth.
#pragma once

#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

// Cache policy of buffer accesses to data a Gauss-Newton launch touches once
// (the output field; in the band march also the input field its warps read):
// non-temporal, so those lines leave the L2 first and the image rows, which
// the bilinear rows of neighbouring pixels and tiles read again, stay.
// Measured on MI355X: 5 % less time per full-resolution launch of the 64 x 64
// tiles at 1 Mp, 7 % (float32 planes) and 5 % (bfloat16) for the band march
// at 5120 x 4096.
constexpr int kStreamPolicy = 2;


template <typename TS>
struct GnCtx {
  const TS* p0;
  const TS* p1;
  int64_t ip;
  const float* fu;
  const float* fv;
  int64_t fp;
  int w, h, cw, ch, mode;
};

// ---------------------------------------------------------------- split-phase loads
// A "request" holds loaded-but-unused values; the matching "finish" combines
// them.  Issuing a request one or two march steps before finishing it keeps
// the loads in flight behind the intervening work.

// Input flow at a pixel: DIRECT = two loads; UPSAMPLE = bilinear taps of the
// coarse field (8 loads) and the weights; ZERO = nothing.
struct FlowReq {
  float u00, u01, u10, u11, v00, v01, v10, v11;
  float wx, wy;
};

template <int MODE, typename TS>
__device__ __forceinline__ void flow_issue(const GnCtx<TS>& c, int x, int y, FlowReq& r) {
  // y is clamped into the level by the caller: every path issues a fixed
  // number of loads, so waits can be counted exactly across march steps
  if (MODE == FLOW_ZERO) {
    r.u00 = r.v00 = 0.0f;
    return;
  }
  if (MODE == FLOW_DIRECT) {
    const int64_t o = static_cast<int64_t>(y) * c.fp + x;
    r.u00 = c.fu[o];
    r.v00 = c.fv[o];
    return;
  }
  const float fx = fminf(fmaxf(0.5f * static_cast<float>(x), 0.0f), static_cast<float>(c.cw - 1));
  const float fy = fminf(fmaxf(0.5f * static_cast<float>(y), 0.0f), static_cast<float>(c.ch - 1));
  const float xf = floorf(fx);
  const float yf = floorf(fy);
  r.wx = fx - xf;
  r.wy = fy - yf;
  const int ix = static_cast<int>(xf);
  const int iy = static_cast<int>(yf);
  const int dx = ix < c.cw - 1 ? 1 : 0;
  const int64_t dy = iy < c.ch - 1 ? c.fp : 0;
  const int64_t o = static_cast<int64_t>(iy) * c.fp + ix;
  r.u00 = c.fu[o];
  r.u01 = c.fu[o + dx];
  r.u10 = c.fu[o + dy];
  r.u11 = c.fu[o + dy + dx];
  r.v00 = c.fv[o];
  r.v01 = c.fv[o + dx];
  r.v10 = c.fv[o + dy];
  r.v11 = c.fv[o + dy + dx];
}

__device__ __forceinline__ float lerp4(float p00, float p01, float p10, float p11, float ax, float ay) {
  const float top = p00 + ax * (p01 - p00);
  const float bot = p10 + ax * (p11 - p10);
  return top + ay * (bot - top);
}

template <int MODE>
__device__ __forceinline__ void flow_finish(const FlowReq& r, bool valid, float& u, float& v) {
  if (MODE == FLOW_UPSAMPLE) {
    u = 2.0f * lerp4(r.u00, r.u01, r.u10, r.u11, r.wx, r.wy);
    v = 2.0f * lerp4(r.v00, r.v01, r.v10, r.v11, r.wx, r.wy);
  } else {
    u = r.u00;
    v = r.v00;
  }
  u = valid ? u : 0.0f;
  v = valid ? v : 0.0f;
}

// Midpoint warps of both images at (x, y) for flow (u, v): 8 taps and the
// four interpolation weights.
struct WarpReq {
  float a00, a01, a10, a11, b00, b01, b10, b11;
  float ax0, ay0, ax1, ay1;
};

template <typename TS>
__device__ __forceinline__ void tap4(const TS* p, int64_t pitch, int w, int h, float x, float y, float& q00,
                                     float& q01, float& q10, float& q11, float& ax, float& ay) {
  x = fminf(fmaxf(x, 0.0f), static_cast<float>(w - 1));
  y = fminf(fmaxf(y, 0.0f), static_cast<float>(h - 1));
  const float xf = floorf(x);
  const float yf = floorf(y);
  ax = x - xf;
  ay = y - yf;
  const int ix = static_cast<int>(xf);
  const int iy = static_cast<int>(yf);
  const int dx = ix < w - 1 ? 1 : 0;
  const int64_t dy = iy < h - 1 ? pitch : 0;
  const TS* r0 = p + static_cast<int64_t>(iy) * pitch + ix;
  q00 = Px<TS>::ld(r0);
  q01 = Px<TS>::ld(r0 + dx);
  q10 = Px<TS>::ld(r0 + dy);
  q11 = Px<TS>::ld(r0 + dy + dx);
}

// Symmetric warps of Eq. (of_symmetric): P0 at k - V/2 and P1 at k + V/2,
// S the mean of the two.  fa (the forward-additive estimator): P0 at k
// itself (integer position: the interpolation weights are exactly 0) and
// P1 at k + V, S the warped P1.
template <typename TS>
__device__ __forceinline__ void warp_issue(const GnCtx<TS>& c, int x, int y, float u, float v, WarpReq& g, bool fa) {
  const float fx = static_cast<float>(x);
  const float fy = static_cast<float>(y);
  const float hu = fa ? 0.0f : 0.5f * u;
  const float hv = fa ? 0.0f : 0.5f * v;
  tap4(c.p0, c.ip, c.w, c.h, fx - hu, fy - hv, g.a00, g.a01, g.a10, g.a11, g.ax0, g.ay0);
  tap4(c.p1, c.ip, c.w, c.h, fx + (fa ? u : hu), fy + (fa ? v : hv), g.b00, g.b01, g.b10, g.b11, g.ax1, g.ay1);
}

__device__ __forceinline__ void warp_finish(const WarpReq& g, bool valid, float& s, float& t, bool fa) {
  const float w0 = lerp4(g.a00, g.a01, g.a10, g.a11, g.ax0, g.ay0);
  const float w1 = lerp4(g.b00, g.b01, g.b10, g.b11, g.ax1, g.ay1);
  s = valid ? (fa ? w1 : 0.5f * (w0 + w1)) : 0.0f;
  t = valid ? w1 - w0 : 0.0f;
}

// ---------------------------------------------------------------- wavefront prefix scan (DPP)
// Inclusive prefix sum over the 64 lanes of a wavefront: Hillis-Steele
// shifts of 1, 2, 4, 8 lanes within each 16-lane row (zeros shifted in), then
// the row totals are carried across rows with the row-broadcast controls.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true);
  return x + __int_as_float(y);
}

__device__ __forceinline__ float wave_prefix(float x) {
  x = dpp_shift_add<0x111, 0xf>(x);  // row_shr:1
  x = dpp_shift_add<0x112, 0xf>(x);  // row_shr:2
  x = dpp_shift_add<0x114, 0xf>(x);  // row_shr:4
  x = dpp_shift_add<0x118, 0xf>(x);  // row_shr:8
  x = dpp_shift_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_shift_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// GEN: the estimator variant is read from a.est at run time (forward-additive
// warps, increment-form update); otherwise the symmetric estimator's
// consistent update is compiled in.
template <int KR, int MODE, typename TS, bool GEN = false>
__global__ __launch_bounds__(kGnThreads) void gn_kernel(const GnArgs a) {
  constexpr int NWIN = 2 * KR + 1;
  constexpr int TX = kGnThreads - 2 * KR - 2;
  __shared__ float s_row[2][kGnThreads];
  __shared__ float p_row[2][5][kGnThreads];

  const bool fwd = GEN && (a.est & EST_FORWARD_ADDITIVE) != 0;
  const bool inc = GEN && (a.est & EST_INCREMENT) != 0;
  const bool no_fp64 = (a.est & EST_NO_FP64) != 0;
  const int jb = find_job(a, blockIdx.x);
  const GnJob& J = a.job[jb];
  GnCtx<TS> c;
  c.p0 = static_cast<const TS*>(J.p0);
  c.p1 = static_cast<const TS*>(J.p1);
  c.ip = J.img_pitch;
  c.fu = J.in_u;
  c.fv = J.in_v;
  c.fp = J.in_pitch;
  c.w = J.w;
  c.h = J.h;
  c.cw = J.cw;
  c.ch = J.ch;
  c.mode = MODE;
  const int W = J.w;
  const int H = J.h;
  const int t = blockIdx.x - J.tile_start;
  const int ntx = (W + TX - 1) / TX;
  const int x0 = (t % ntx) * TX;
  const int y0 = (t / ntx) * a.tile_h;
  const int tid = threadIdx.x;
  const int col = x0 - KR - 1 + tid;
  const bool col_in = col >= 0 && col < W;
  const int cc = min(max(col, 0), W - 1);
  const bool out_lane = tid >= KR + 1 && tid < KR + 1 + TX && col_in;
  const bool prod_lane = tid >= 1 && tid < kGnThreads - 1 && col_in;
  const int tl = max(tid - 1, 0);
  const int tr = min(tid + 1, kGnThreads - 1);
  const bool has_left = col - 1 >= 0;
  const bool has_right = col + 1 < W;
  // horizontal window of output lane tid: prefix(ia) - prefix(ib) (+ total of wave(ib))
  const int ia = min(tid + KR, kGnThreads - 1);
  const int ib = max(tid - KR - 1, 0);
  const bool cross = (ia >> 6) != (ib >> 6);
  const int itot = (ib & ~63) + 63;
  auto row_ok = [&](int r) { return r >= 0 && r < H; };
  auto rc = [&](int r) { return min(max(r, 0), H - 1); };

  // ---- prologue: S of rows y0-KR-1 and y0-KR, flow of rows up to y0-KR+2
  const int r0 = y0 - KR - 1;
  float s_m, s_0, t_0, u_0, v_0;
  float u_1, v_1, u_2, v_2;
  WarpReq g1;      // gathers of row pr+1, in flight
  FlowReq f2, f3;  // flows of rows pr+2 and pr+3, in flight
  {
    FlowReq fa, fb, fc;
    flow_issue<MODE>(c, cc, rc(r0), fa);
    flow_issue<MODE>(c, cc, rc(r0 + 1), fb);
    flow_issue<MODE>(c, cc, rc(r0 + 2), fc);
    flow_issue<MODE>(c, cc, rc(r0 + 3), f2);
    float ua, va;
    flow_finish<MODE>(fa, row_ok(r0), ua, va);
    flow_finish<MODE>(fb, row_ok(r0 + 1), u_0, v_0);
    flow_finish<MODE>(fc, row_ok(r0 + 2), u_1, v_1);
    WarpReq ga, gb;
    warp_issue(c, cc, rc(r0), ua, va, ga, fwd);
    warp_issue(c, cc, rc(r0 + 1), u_0, v_0, gb, fwd);
    warp_issue(c, cc, rc(r0 + 2), u_1, v_1, g1, fwd);
    flow_issue<MODE>(c, cc, rc(r0 + 4), f3);
    float tdummy;
    warp_finish(ga, row_ok(r0), s_m, tdummy, fwd);
    warp_finish(gb, row_ok(r0 + 1), s_0, t_0, fwd);
  }
  s_row[0][tid] = s_0;
  __syncthreads();

  float ring[5][NWIN];
  float ru[NWIN], rv[NWIN];
  float acc[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    acc[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < NWIN; ++k) ring[q][k] = 0.0f;
  }
#pragma unroll
  for (int k = 0; k < NWIN; ++k) ru[k] = rv[k] = 0.0f;

  const int nprod = a.tile_h + 2 * KR;
  for (int base = 0; base < nprod; base += NWIN) {
#pragma unroll
    for (int k = 0; k < NWIN; ++k) {
      const int i = base + k;
      if (i < nprod) {
        const int pr = y0 - KR + i;  // product row of this step
        const int slot = i & 1;
        // pipeline: S/T of row pr+1 (gathers issued last step); gathers of
        // row pr+2 (flow requested two steps ago); flow of row pr+4.
        float s_p, t_p;
        warp_finish(g1, row_ok(pr + 1), s_p, t_p, fwd);
        flow_finish<MODE>(f2, row_ok(pr + 2), u_2, v_2);
        warp_issue(c, cc, rc(pr + 2), u_2, v_2, g1, fwd);
        f2 = f3;
        flow_issue<MODE>(c, cc, rc(pr + 4), f3);
        // gradient of S at (col, pr), indices clamped to the level
        const float sl = has_left ? s_row[slot][tl] : s_0;
        const float sr = has_right ? s_row[slot][tr] : s_0;
        const float su = pr - 1 >= 0 ? s_m : s_0;
        const float sd = pr + 1 < H ? s_p : s_0;
        const float gx = 0.5f * (sr - sl);
        const float gy = 0.5f * (sd - su);
        const float b = inc ? -t_0 : fmaf(gx, u_0, fmaf(gy, v_0, -t_0));
        const bool valid = prod_lane && row_ok(pr);
        float pq[5];
        pq[0] = valid ? gx * gx : 0.0f;
        pq[1] = valid ? gx * gy : 0.0f;
        pq[2] = valid ? gy * gy : 0.0f;
        pq[3] = valid ? gx * b : 0.0f;
        pq[4] = valid ? gy * b : 0.0f;
        s_row[slot ^ 1][tid] = s_p;
#pragma unroll
        for (int q = 0; q < 5; ++q) p_row[slot][q][tid] = wave_prefix(pq[q]);
        ru[k] = u_0;
        rv[k] = v_0;
        __syncthreads();
        // horizontal window sums from the prefix row (meaningful on output lanes)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float* prow = p_row[slot][q];
          float hsum = prow[ia] - prow[ib];
          if (cross) hsum += prow[itot];
          hsum = out_lane ? hsum : 0.0f;
          ring[q][k] = hsum;
          acc[q] += hsum;
        }
        if (i >= 2 * KR) {
          const int orow = pr - KR;
          if (out_lane && orow < H) {
            // V(m) of the output row entered the ring KR steps ago
            const float um = ru[(k + KR + 1) % NWIN];
            const float vm = rv[(k + KR + 1) % NWIN];
            float un, vn;
            solve2x2(acc[0], acc[1], acc[2], acc[3], acc[4], um, vm, a.reg_rel, a.reg_abs, un, vn, inc, no_fp64);
            const int64_t o = static_cast<int64_t>(orow) * J.out_pitch + col;
            __builtin_nontemporal_store(un, J.out_u + o);
            __builtin_nontemporal_store(vn, J.out_v + o);
          }
          // the row leaving the window next step sits in slot (i - 2KR) mod NWIN
#pragma unroll
          for (int q = 0; q < 5; ++q) acc[q] -= ring[q][(k + 1) % NWIN];
        }
        s_m = s_0;
        s_0 = s_p;
        t_0 = t_p;
        u_0 = u_1;
        v_0 = v_1;
        u_1 = u_2;
        v_1 = v_2;
      }
    }
  }
}

template <int MODE, typename TS>
hipError_t launch_gn_typed(const GnArgs& a, int kr, int nblocks, hipStream_t s, bool generic) {
  const dim3 grid(nblocks);
  const dim3 block(kGnThreads);
  switch (kr) {
#define OFV_GN_CASE(R)                                                                   \
  case R:                                                                                \
    if (generic) hipLaunchKernelGGL((gn_kernel<R, MODE, TS, true>), grid, block, 0, s, a); \
    else hipLaunchKernelGGL((gn_kernel<R, MODE, TS, false>), grid, block, 0, s, a);       \
    break;
    OFV_GN_CASE(1)
    OFV_GN_CASE(2)
    OFV_GN_CASE(3)
    OFV_GN_CASE(4)
    OFV_GN_CASE(5)
    OFV_GN_CASE(6)
    OFV_GN_CASE(7)
    OFV_GN_CASE(8)
    OFV_GN_CASE(9)
    OFV_GN_CASE(10)
    OFV_GN_CASE(11)
    OFV_GN_CASE(12)
#undef OFV_GN_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ofv
