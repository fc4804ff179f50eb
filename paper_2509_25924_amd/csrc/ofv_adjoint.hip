// Hand-written adjoint of the estimator (reverse mode, float32).
//
// Forward (section "Live-Optical Flow Velocimetry", Eq. of_symmetric): per
// pixel k, W0 = P0(k - V/2), W1 = P1(k + V/2) (bilinear, clamped), S = (W0 +
// W1)/2, T = W1 - W0, G = central difference of S (clamped), b = G.V(k) - T,
// products p = (Gx^2, GxGy, Gy^2, Gx b, Gy b); per pixel m, sums A = Box(p)
// over the truncated (2KR+1)^2 window; lam = reg_rel (Sxx + Syy) + reg_abs;
// (A + lam I) V'(m) = c + lam V(m).  The backward of one iteration recomputes
// S, T, G, b and the sums from the saved input field V and then applies, in
// reverse order, the adjoints of the solve, the window sums (a truncated box
// is its own transpose), the products, b, the central difference, and the two
// bilinear warps (gathers become float atomic scatter-adds into the image
// gradients; the sub-pixel weights give the flow gradient).  Also here: the
// adjoints of up-sampling, REDUCE (and the initial-flow restriction) and the
// local z-score normalisation.
//
// Derivative conventions follow the forward formulas exactly: clamp passes
// the gradient where the coordinate lies inside [0, size - 1] (ends
// included), floor has zero derivative, and a tap repeated at the border
// receives both of its weights.
#include "ofv_internal.h"
#include "ofv_px.h"

namespace ofv {

namespace {

constexpr int BX = 64, BY = 4;

dim3 grid2(int w, int h) { return dim3((w + BX - 1) / BX, (h + BY - 1) / BY); }

__device__ __forceinline__ bool pix(int& x, int& y, int w, int h) {
  x = blockIdx.x * BX + (threadIdx.x & 63);
  y = blockIdx.y * BY + (threadIdx.x >> 6);
  return x < w && y < h;
}

// Bilinear sample with the forward's clamping; also returns the partial
// derivatives w.r.t. the (unclamped) coordinates and the four tap weights.
struct Bil {
  float val, dx, dy;
  int o00, o01, o10, o11;
  float w00, w01, w10, w11;
};

__device__ __forceinline__ Bil bil_fwd(const float* p, int pitch, int w, int h, float x, float y) {
  Bil r;
  const bool inx = x >= 0.0f && x <= static_cast<float>(w - 1);
  const bool iny = y >= 0.0f && y <= static_cast<float>(h - 1);
  const float xc = fminf(fmaxf(x, 0.0f), static_cast<float>(w - 1));
  const float yc = fminf(fmaxf(y, 0.0f), static_cast<float>(h - 1));
  const float xf = floorf(xc), yf = floorf(yc);
  const float fx = xc - xf, fy = yc - yf;
  const int ix0 = static_cast<int>(xf), iy0 = static_cast<int>(yf);
  const int ix1 = min(ix0 + 1, w - 1), iy1 = min(iy0 + 1, h - 1);
  r.o00 = iy0 * pitch + ix0;
  r.o01 = iy0 * pitch + ix1;
  r.o10 = iy1 * pitch + ix0;
  r.o11 = iy1 * pitch + ix1;
  const float p00 = p[r.o00], p01 = p[r.o01], p10 = p[r.o10], p11 = p[r.o11];
  r.w00 = (1.0f - fy) * (1.0f - fx);
  r.w01 = (1.0f - fy) * fx;
  r.w10 = fy * (1.0f - fx);
  r.w11 = fy * fx;
  r.val = (1.0f - fy) * ((1.0f - fx) * p00 + fx * p01) + fy * ((1.0f - fx) * p10 + fx * p11);
  r.dx = inx ? (1.0f - fy) * (p01 - p00) + fy * (p11 - p10) : 0.0f;
  r.dy = iny ? ((1.0f - fx) * p10 + fx * p11) - ((1.0f - fx) * p00 + fx * p01) : 0.0f;
  return r;
}

// ---------------------------------------------------------------- forward recompute of one iteration

__global__ __launch_bounds__(256) void k_terms(const AdjLevel a) {
  int x, y;
  if (!pix(x, y, a.w, a.h)) return;
  const int ov = y * a.vp + x;
  const float u = a.vu[ov], v = a.vv[ov];
  const Bil b0 = bil_fwd(a.p0, a.ip, a.w, a.h, x - 0.5f * u, y - 0.5f * v);
  const Bil b1 = bil_fwd(a.p1, a.ip, a.w, a.h, x + 0.5f * u, y + 0.5f * v);
  const int o = y * a.sp + x;
  a.S[o] = 0.5f * (b0.val + b1.val);
  a.T[o] = b1.val - b0.val;
}

__global__ __launch_bounds__(256) void k_products(const AdjLevel a) {
  int x, y;
  if (!pix(x, y, a.w, a.h)) return;
  const int o = y * a.sp + x;
  const float* S = a.S;
  const float gx = 0.5f * (S[y * a.sp + min(x + 1, a.w - 1)] - S[y * a.sp + max(x - 1, 0)]);
  const float gy = 0.5f * (S[min(y + 1, a.h - 1) * a.sp + x] - S[max(y - 1, 0) * a.sp + x]);
  const int ov = y * a.vp + x;
  const float b = gx * a.vu[ov] + gy * a.vv[ov] - a.T[o];
  a.GX[o] = gx;
  a.GY[o] = gy;
  a.B[o] = b;
  a.A[0][o] = gx * gx;
  a.A[1][o] = gx * gy;
  a.A[2][o] = gy * gy;
  a.A[3][o] = gx * b;
  a.A[4][o] = gy * b;
}

// truncated box sums of radius r over up to 5 planes: horizontal pass then vertical pass
struct PlaneList {
  const float* in[5];
  float* out[5];
};

__global__ __launch_bounds__(256) void k_box_h5(const PlaneList l, int n, int w, int h, int pitch, int r) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  const int x0 = max(x - r, 0), x1 = min(x + r, w - 1);
  for (int q = 0; q < n; ++q) {
    const float* row = l.in[q] + y * pitch;
    float s = 0.0f;
    for (int i = x0; i <= x1; ++i) s += row[i];
    l.out[q][y * pitch + x] = s;
  }
}

__global__ __launch_bounds__(256) void k_box_v5(const PlaneList l, int n, int w, int h, int pitch, int r) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  const int y0 = max(y - r, 0), y1 = min(y + r, h - 1);
  for (int q = 0; q < n; ++q) {
    float s = 0.0f;
    for (int j = y0; j <= y1; ++j) s += l.in[q][j * pitch + x];
    l.out[q][y * pitch + x] = s;
  }
}

// ---------------------------------------------------------------- adjoints

// solve: x = M^-1 rhs with M = [[Sxx+lam, Sxy], [Sxy, Syy+lam]], rhs = (Sxb + lam u, Syb + lam v)
__global__ __launch_bounds__(256) void k_solve_adj(const AdjLevel a) {
  int x, y;
  if (!pix(x, y, a.w, a.h)) return;
  const int o = y * a.sp + x;
  const int ov = y * a.vp + x;
  const float sxx = a.A[0][o], sxy = a.A[1][o], syy = a.A[2][o], sxb = a.A[3][o], syb = a.A[4][o];
  const float um = a.vu[ov], vm = a.vv[ov];
  const float lam = a.reg_rel * (sxx + syy) + a.reg_abs;
  const float aa = sxx + lam, dd = syy + lam;
  const float det = aa * dd - sxy * sxy;
  const float r1 = sxb + lam * um, r2 = syb + lam * vm;
  const float xu = (dd * r1 - sxy * r2) / det;
  const float xv = (aa * r2 - sxy * r1) / det;
  const float gu = a.gu[y * a.gp + x], gv = a.gv[y * a.gp + x];
  const float z1 = (dd * gu - sxy * gv) / det;   // dL/drhs = M^-T g
  const float z2 = (aa * gv - sxy * gu) / det;
  const float g_aa = -z1 * xu, g_dd = -z2 * xv, g_sxy = -(z1 * xv + z2 * xu);
  const float g_lam = z1 * um + z2 * vm + g_aa + g_dd;
  a.gA[0][o] = g_aa + a.reg_rel * g_lam;
  a.gA[1][o] = g_sxy;
  a.gA[2][o] = g_dd + a.reg_rel * g_lam;
  a.gA[3][o] = z1;
  a.gA[4][o] = z2;
  a.gVu[o] = lam * z1;
  a.gVv[o] = lam * z2;
}

// products and b: gp = Box(gA) is in gA (after the box pass)
__global__ __launch_bounds__(256) void k_prod_adj(const AdjLevel a) {
  int x, y;
  if (!pix(x, y, a.w, a.h)) return;
  const int o = y * a.sp + x;
  const int ov = y * a.vp + x;
  const float gx = a.GX[o], gy = a.GY[o], b = a.B[o];
  const float g0 = a.gA[0][o], g1 = a.gA[1][o], g2 = a.gA[2][o], g3 = a.gA[3][o], g4 = a.gA[4][o];
  const float gb = gx * g3 + gy * g4;
  a.gGx[o] = 2.0f * gx * g0 + gy * g1 + b * g3 + a.vu[ov] * gb;
  a.gGy[o] = gx * g1 + 2.0f * gy * g2 + b * g4 + a.vv[ov] * gb;
  a.gT[o] = -gb;
  a.gVu[o] += gx * gb;
  a.gVv[o] += gy * gb;
}

// central difference transposed, S and T -> W0, W1, bilinear warps transposed
__global__ __launch_bounds__(256) void k_warp_adj(const AdjLevel a) {
  int x, y;
  if (!pix(x, y, a.w, a.h)) return;
  const int sp = a.sp;
  const int w = a.w, h = a.h;
  // gS(j) = sum over k whose clamped +1 neighbour is j of gG(k)/2 minus those whose clamped -1 neighbour is j
  float gs = 0.0f;
  if (x - 1 >= 0) gs += 0.5f * a.gGx[y * sp + x - 1];
  if (x == w - 1) gs += 0.5f * a.gGx[y * sp + x];
  if (x + 1 <= w - 1) gs -= 0.5f * a.gGx[y * sp + x + 1];
  if (x == 0) gs -= 0.5f * a.gGx[y * sp + x];
  if (y - 1 >= 0) gs += 0.5f * a.gGy[(y - 1) * sp + x];
  if (y == h - 1) gs += 0.5f * a.gGy[y * sp + x];
  if (y + 1 <= h - 1) gs -= 0.5f * a.gGy[(y + 1) * sp + x];
  if (y == 0) gs -= 0.5f * a.gGy[y * sp + x];
  const int o = y * sp + x;
  const float gt = a.gT[o];
  const float gw0 = 0.5f * gs - gt;
  const float gw1 = 0.5f * gs + gt;
  const int ov = y * a.vp + x;
  const float u = a.vu[ov], v = a.vv[ov];
  const Bil b0 = bil_fwd(a.p0, a.ip, w, h, x - 0.5f * u, y - 0.5f * v);
  const Bil b1 = bil_fwd(a.p1, a.ip, w, h, x + 0.5f * u, y + 0.5f * v);
  atomicAdd(a.gP0 + b0.o00, gw0 * b0.w00);
  atomicAdd(a.gP0 + b0.o01, gw0 * b0.w01);
  atomicAdd(a.gP0 + b0.o10, gw0 * b0.w10);
  atomicAdd(a.gP0 + b0.o11, gw0 * b0.w11);
  atomicAdd(a.gP1 + b1.o00, gw1 * b1.w00);
  atomicAdd(a.gP1 + b1.o01, gw1 * b1.w01);
  atomicAdd(a.gP1 + b1.o10, gw1 * b1.w10);
  atomicAdd(a.gP1 + b1.o11, gw1 * b1.w11);
  const int oo = y * a.op + x;
  a.ou[oo] = a.gVu[o] - 0.5f * gw0 * b0.dx + 0.5f * gw1 * b1.dx;
  a.ov[oo] = a.gVv[o] - 0.5f * gw0 * b0.dy + 0.5f * gw1 * b1.dy;
}

// V_fine(X) = 2 bilinear(V_coarse, X / 2): scatter 2 w g into the coarse gradient
__global__ __launch_bounds__(256) void k_upsample_adj(const float* gfu, const float* gfv, int w, int h, int fp,
                                                      float* gcu, float* gcv, int cw, int ch, int cp) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  const float gu = 2.0f * gfu[y * fp + x], gv = 2.0f * gfv[y * fp + x];
  const float xc = fminf(0.5f * x, static_cast<float>(cw - 1));
  const float yc = fminf(0.5f * y, static_cast<float>(ch - 1));
  const float xf = floorf(xc), yf = floorf(yc);
  const float fx = xc - xf, fy = yc - yf;
  const int ix0 = static_cast<int>(xf), iy0 = static_cast<int>(yf);
  const int ix1 = min(ix0 + 1, cw - 1), iy1 = min(iy0 + 1, ch - 1);
  const float w00 = (1.0f - fy) * (1.0f - fx), w01 = (1.0f - fy) * fx, w10 = fy * (1.0f - fx), w11 = fy * fx;
  atomicAdd(gcu + iy0 * cp + ix0, gu * w00);
  atomicAdd(gcu + iy0 * cp + ix1, gu * w01);
  atomicAdd(gcu + iy1 * cp + ix0, gu * w10);
  atomicAdd(gcu + iy1 * cp + ix1, gu * w11);
  atomicAdd(gcv + iy0 * cp + ix0, gv * w00);
  atomicAdd(gcv + iy0 * cp + ix1, gv * w01);
  atomicAdd(gcv + iy1 * cp + ix0, gv * w10);
  atomicAdd(gcv + iy1 * cp + ix1, gv * w11);
}

// REDUCE transposed, as a gather: fine pixel X collects w_i from every coarse
// x whose clamped tap 2x + i lands on X.
__device__ __forceinline__ float reduce_t_weight(int X, int xc, int w) {
  const float w5[5] = {1.0f / 16, 4.0f / 16, 6.0f / 16, 4.0f / 16, 1.0f / 16};
  float s = 0.0f;
#pragma unroll
  for (int i = -2; i <= 2; ++i)
    if (min(max(2 * xc + i, 0), w - 1) == X) s += w5[i + 2];
  return s;
}

__global__ __launch_bounds__(256) void k_reduce_adj(const float* gc, int cw, int ch, int cp, float* gf, int w, int h,
                                                    int fp, float scale, int accumulate) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  // coarse neighbours that can reach (x, y): |2 xc - x| <= 2 (plus the clamped border taps)
  const int xa = max((x - 2) / 2 - 1, 0), xb = min((x + 2) / 2 + 1, cw - 1);
  const int ya = max((y - 2) / 2 - 1, 0), yb = min((y + 2) / 2 + 1, ch - 1);
  float s = 0.0f;
  for (int j = ya; j <= yb; ++j) {
    const float wy = reduce_t_weight(y, j, h);
    if (wy == 0.0f) continue;
    float row = 0.0f;
    for (int i = xa; i <= xb; ++i) {
      const float wx = reduce_t_weight(x, i, w);
      row += wx * gc[j * cp + i];
    }
    s += wy * row;
  }
  s *= scale;
  float* dst = gf + y * fp + x;
  *dst = accumulate ? *dst + s : s;
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

__global__ __launch_bounds__(256) void k_norm_terms(const ImageIn f, int nr, float eps, const float* gN, int gp,
                                                    float* I, float* sig, float* pa, float* pc, float* pcm, int sp) {
  int x, y;
  if (!pix(x, y, f.w, f.h)) return;
  const int xa = max(x - nr, 0), xb = min(x + nr, f.w - 1), ya = max(y - nr, 0), yb = min(y + nr, f.h - 1);
  const float n = static_cast<float>((xb - xa + 1) * (yb - ya + 1));
  float s = 0.0f;
  for (int j = ya; j <= yb; ++j)
    for (int i = xa; i <= xb; ++i) s += frame_px(f, i, j);
  const float mu = s / n;
  float q = 0.0f;
  for (int j = ya; j <= yb; ++j)
    for (int i = xa; i <= xb; ++i) {
      const float d = frame_px(f, i, j) - mu;
      q += d * d;
    }
  const float sg = sqrtf(q / n + eps);
  const float ik = frame_px(f, x, y);
  const float g = gN[y * gp + x];
  const int o = y * sp + x;
  I[o] = ik;
  sig[o] = sg;
  pa[o] = g / (n * sg);
  const float c = g * (ik - mu) / (n * sg * sg * sg);
  pc[o] = c;
  pcm[o] = c * mu;
}

__global__ __launch_bounds__(256) void k_norm_out(int w, int h, const float* gN, int gp, const float* I,
                                                  const float* sig, const float* ba, const float* bc,
                                                  const float* bcm, int sp, float scale, float* gF, int fp) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  const int o = y * sp + x;
  const float g = gN[y * gp + x] / sig[o] - ba[o] - I[o] * bc[o] + bcm[o];
  gF[y * fp + x] = g * scale;
}

__global__ __launch_bounds__(256) void k_scale_copy(const float* in, int ip, float* out, int op, int w, int h,
                                                    float scale) {
  int x, y;
  if (!pix(x, y, w, h)) return;
  out[y * op + x] = in[y * ip + x] * scale;
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

static hipError_t box5(float* const* planes, float* const* tmp, int n, int w, int h, int pitch, int r, hipStream_t s) {
  PlaneList a{}, b{};
  for (int q = 0; q < n; ++q) {
    a.in[q] = planes[q];
    a.out[q] = tmp[q];
    b.in[q] = tmp[q];
    b.out[q] = planes[q];
  }
  hipLaunchKernelGGL(k_box_h5, grid2(w, h), dim3(256), 0, s, a, n, w, h, pitch, r);
  hipLaunchKernelGGL(k_box_v5, grid2(w, h), dim3(256), 0, s, b, n, w, h, pitch, r);
  return hipGetLastError();
}

hipError_t launch_adj_iteration(const AdjLevel& a, hipStream_t s) {
  const dim3 g = grid2(a.w, a.h);
  hipLaunchKernelGGL(k_terms, g, dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_products, g, dim3(256), 0, s, a);
  hipError_t e = box5(a.A, a.tmp, 5, a.w, a.h, a.sp, a.kr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_adj, g, dim3(256), 0, s, a);
  e = box5(a.gA, a.tmp, 5, a.w, a.h, a.sp, a.kr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prod_adj, g, dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_warp_adj, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_upsample_adj(const float* gfu, const float* gfv, int w, int h, int fp, float* gcu, float* gcv, int cw,
                               int ch, int cp, hipStream_t s) {
  hipLaunchKernelGGL(k_upsample_adj, grid2(w, h), dim3(256), 0, s, gfu, gfv, w, h, fp, gcu, gcv, cw, ch, cp);
  return hipGetLastError();
}

hipError_t launch_reduce_adj(const float* gc, int cw, int ch, int cp, float* gf, int w, int h, int fp, float scale,
                             int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_adj, grid2(w, h), dim3(256), 0, s, gc, cw, ch, cp, gf, w, h, fp, scale, accumulate);
  return hipGetLastError();
}

hipError_t launch_norm_adj(const ImageIn& f, int nr, float eps, const float* gN, int gp, float* const* scratch, int sp,
                           float* gF, int fp, hipStream_t s) {
  const float scale = f.type == 2 ? 1.0f : 1.0f / static_cast<float>((1 << f.bits) - 1);
  if (nr <= 0) {
    hipLaunchKernelGGL(k_scale_copy, grid2(f.w, f.h), dim3(256), 0, s, gN, gp, gF, fp, f.w, f.h, scale);
    return hipGetLastError();
  }
  float* I = scratch[0];
  float* sig = scratch[1];
  float* planes[3] = {scratch[2], scratch[3], scratch[4]};
  float* tmp[3] = {scratch[5], scratch[6], scratch[7]};
  hipLaunchKernelGGL(k_norm_terms, grid2(f.w, f.h), dim3(256), 0, s, f, nr, eps, gN, gp, I, sig, planes[0], planes[1],
                     planes[2], sp);
  hipError_t e = box5(planes, tmp, 3, f.w, f.h, sp, nr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norm_out, grid2(f.w, f.h), dim3(256), 0, s, f.w, f.h, gN, gp, I, sig, planes[0], planes[1],
                     planes[2], sp, scale, gF, fp);
  return hipGetLastError();
}

}  // namespace ofv
