// Storage element types of the image planes and their float32 conversions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ofv {

struct bf16_t {
  uint16_t bits;
};

// Raw buffer view of one plane: the base and size sit in scalar registers
// and every access is a 32-bit byte offset from the base; an access at or
// beyond `bytes` reads 0 instead of touching memory (gfx9 raw-buffer
// descriptor: stride 0, 32-bit data format).  Planes stay below 2 GiB.
using PlaneView = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ PlaneView plane_view(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}

__device__ __forceinline__ float ld_f32(PlaneView v, uint32_t i) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(v, static_cast<int>(i * 4u), 0, 0));
}

template <typename T>
struct Px;

template <>
struct Px<float> {
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ float round(float v) { return v; }
  static __device__ __forceinline__ float ldv(PlaneView v, uint32_t i) { return ld_f32(v, i); }
  // element i + j of the plane, j a byte offset uniform across the wavefront
  static __device__ __forceinline__ float ldvs(PlaneView v, uint32_t i, uint32_t jb) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(v, static_cast<int>(i * 4u), static_cast<int>(jb), 0));
  }
  static constexpr uint32_t bytes = 4;
  // elements i and i + 1 (j a uniform byte offset)
  static __device__ __forceinline__ void ld2(PlaneView v, uint32_t i, uint32_t jb, float& a, float& b) {
    a = ldvs(v, i, jb);
    b = ldvs(v, i + 1, jb);
  }
  static __device__ __forceinline__ void st(float* p, float v) { *p = v; }
};

// float32 -> float16, round to nearest even, from a value the compiler treats
// as opaque: the conversion always takes the float32-rounded result, never
// a multiply-add fused with it into one rounding (v_fma_mix), which the
// compiler would otherwise do at some call sites and not at others, so that
// kernels computing the same sums could store different halves.
__device__ __forceinline__ _Float16 to_half(float v) {
  asm volatile("" : "+v"(v));
  return static_cast<_Float16>(v);
}

template <>
struct Px<_Float16> {
  static __device__ __forceinline__ float ld(const _Float16* p) { return static_cast<float>(*p); }
  static __device__ __forceinline__ float round(float v) { return static_cast<float>(to_half(v)); }
  static __device__ __forceinline__ float ldv(PlaneView v, uint32_t i) { return ldvs(v, i, 0); }
  static __device__ __forceinline__ float ldvs(PlaneView v, uint32_t i, uint32_t jb) {
    const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(v, static_cast<int>(i * 2u), static_cast<int>(jb), 0);
    return static_cast<float>(__builtin_bit_cast(_Float16, b));
  }
  static constexpr uint32_t bytes = 2;
  // elements i and i + 1 in one 32-bit load (2-byte aligned: buffer accesses
  // need no natural alignment on gfx9)
  static __device__ __forceinline__ void ld2(PlaneView v, uint32_t i, uint32_t jb, float& a, float& b) {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(v, static_cast<int>(i * 2u), static_cast<int>(jb), 0);
    a = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffffu)));
    b = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16)));
  }
  static __device__ __forceinline__ void st(_Float16* p, float v) { *p = to_half(v); }
};

// bfloat16 = the upper half of an IEEE binary32; conversion from float rounds
// to nearest, ties to even, and keeps NaNs quiet.
template <>
struct Px<bf16_t> {
  static __device__ __forceinline__ float ld(const bf16_t* p) {
    return __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
  }
  static __device__ __forceinline__ float round(float v) {
    bf16_t b;
    st(&b, v);
    return ld(&b);
  }
  static __device__ __forceinline__ float ldv(PlaneView v, uint32_t i) { return ldvs(v, i, 0); }
  static __device__ __forceinline__ float ldvs(PlaneView v, uint32_t i, uint32_t jb) {
    const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(v, static_cast<int>(i * 2u), static_cast<int>(jb), 0);
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
  }
  static constexpr uint32_t bytes = 2;
  // elements i and i + 1 in one 32-bit load (2-byte aligned: buffer accesses
  // need no natural alignment on gfx9)
  static __device__ __forceinline__ void ld2(PlaneView v, uint32_t i, uint32_t jb, float& a, float& b) {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(v, static_cast<int>(i * 2u), static_cast<int>(jb), 0);
    a = __uint_as_float(w << 16);
    b = __uint_as_float(w & 0xffff0000u);
  }
  static __device__ __forceinline__ void st(bf16_t* p, float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) {
      p->bits = static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
      return;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    p->bits = static_cast<uint16_t>(u >> 16);
  }
};

// Bilinear sample of a plane at (x, y); coordinates are clamped to
// [0, w-1] x [0, h-1] first, so every address stays inside the plane (NaN
// coordinates clamp to 0).
template <typename T>
__device__ __forceinline__ float bilinear(const T* __restrict__ p, int64_t pitch, int w, int h, float x,
                                          float y) {
  x = fminf(fmaxf(x, 0.0f), static_cast<float>(w - 1));
  y = fminf(fmaxf(y, 0.0f), static_cast<float>(h - 1));
  const float xf = floorf(x);
  const float yf = floorf(y);
  const float ax = x - xf;
  const float ay = y - yf;
  const int ix = static_cast<int>(xf);
  const int iy = static_cast<int>(yf);
  const int dx = ix < w - 1 ? 1 : 0;
  const int64_t dy = iy < h - 1 ? pitch : 0;
  const T* r0 = p + static_cast<int64_t>(iy) * pitch + ix;
  const float p00 = Px<T>::ld(r0);
  const float p01 = Px<T>::ld(r0 + dx);
  const float p10 = Px<T>::ld(r0 + dy);
  const float p11 = Px<T>::ld(r0 + dy + dx);
  const float top = p00 + ax * (p01 - p00);
  const float bot = p10 + ax * (p11 - p10);
  return top + ay * (bot - top);
}

// Damped 2x2 solve of one Gauss-Newton step (Eq. of_symmetric linearised):
//   (A + lam I) V' = c + lam V(m),  lam = reg_rel (Sxx + Syy) + reg_abs,
// by Cramer's rule in float32 (one reciprocal of the determinant).  Where
// the system is ill-conditioned
// (q = 4 det / trace^2 < 1e-2) the float32 determinant has lost leading
// digits to cancellation; there the determinant and the solution are
// recomputed in float64 from the same float32 sums (products of two floats
// are exact in double, so det is then exact up to one rounding), unless
// `no_fp64` switches that fallback off.
// inc (the increment form of the update): (A + lam I) dV = c with c the sums
// of G (-T), and V' = V(m) + dV.
__device__ __forceinline__ void solve2x2(float sxx, float sxy, float syy, float sxb, float syb, float um, float vm,
                                         float reg_rel, float reg_abs, float& u, float& v, bool inc = false,
                                         bool no_fp64 = false) {
  const float lam = reg_rel * (sxx + syy) + reg_abs;
  const float aa = sxx + lam;
  const float dd = syy + lam;
  const float r1 = inc ? sxb : sxb + lam * um;
  const float r2 = inc ? syb : syb + lam * vm;
  const float det = aa * dd - sxy * sxy;
  const float tr = aa + dd;
  if (det >= 2.5e-3f * tr * tr || no_fp64) {
    // hardware reciprocal (1 ulp) refined by one Newton step
    float inv = __builtin_amdgcn_rcpf(det);
    inv = fmaf(inv, fmaf(-det, inv, 1.0f), inv);
    u = (dd * r1 - sxy * r2) * inv;
    v = (aa * r2 - sxy * r1) * inv;
  } else {
    const double a = aa, d = dd, b = sxy, x1 = r1, x2 = r2;
    const double dt = a * d - b * b;
    u = static_cast<float>((d * x1 - b * x2) / dt);
    v = static_cast<float>((a * x2 - b * x1) / dt);
  }
  if (inc) {
    u += um;
    v += vm;
  }
}

// Workgroup -> job lookup: jobs are laid out consecutively in the 1-D grid.
template <typename Args>
__device__ __forceinline__ int find_job(const Args& a, int block) {
  int j = 0;
  while (j + 1 < a.njobs && block >= a.job[j + 1].tile_start) ++j;
  return j;
}

}  // namespace ofv
