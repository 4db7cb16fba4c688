// dm_fft.hpp -- register-resident DFT building blocks for gfx950 (wave64).
//
// A length-F transform (F = 16 * B) is computed as F = 16 x B:
//   n = B*n1 + n2,  k = k1 + 16*k2,
//   X[k1 + 16 k2] = sum_{n2} W_B^{n2 k2} * W_F^{n2 k1} * sum_{n1} x[B n1 + n2] W_16^{n1 k1}
// so a thread that owns the 16 samples x[B*n1 + n2] (fixed n2) does a 16-point
// DFT in registers, multiplies by the twiddle W_F^{n2 k1}, and after an
// exchange through LDS a thread that owns all n2 for fixed k1 finishes with a
// B-point DFT.  The inverse runs the same steps mirrored, so data returns to
// the thread and register it started from.  DIR = -1 is the forward kernel
// exp(-2 pi i nk/F), DIR = +1 the (unnormalised) inverse.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmk {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// multiply by i*DIR  (DIR=-1: -i, DIR=+1: +i)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
  if constexpr (DIR < 0) return make_float2(a.y, -a.x);
  else return make_float2(-a.y, a.x);
}

// cos(2 pi m / 16) and sin(2 pi m / 16), m = 0..15
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// a * exp(DIR * 2 pi i m / 16) with compile-time m; exact for m multiple of 4
template <int DIR, int M>
__device__ __forceinline__ float2 tw16(float2 a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return mul_i<DIR>(a);
  else if constexpr (m == 8) return make_float2(-a.x, -a.y);
  else if constexpr (m == 12) return mul_i<-DIR>(a);
  else {
    const float c = kCos16[m];
    const float s = DIR * kSin16[m];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 8-point DFT, natural order in and out: 2 x 4 split.
template <int DIR>
__device__ __forceinline__ void dft8(float2 (&a)[8]) {
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  o1 = tw16<DIR, 2>(o1);
  o2 = tw16<DIR, 4>(o2);
  o3 = tw16<DIR, 6>(o3);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

template <int DIR, int N2, int K1>
__device__ __forceinline__ void tw16_apply(float2 (&y)[16]) {
  y[N2 * 4 + K1] = tw16<DIR, N2 * K1>(y[N2 * 4 + K1]);
}

// 16-point DFT, natural order in and out: 4 x 4 split.
template <int DIR>
__device__ __forceinline__ void dft16(float2 (&a)[16]) {
  float2 y[16];
  // stage 1: 4-point DFTs over n1 for each n2 (x[4 n1 + n2])
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 b0 = a[n2], b1 = a[4 + n2], b2 = a[8 + n2], b3 = a[12 + n2];
    dft4<DIR>(b0, b1, b2, b3);
    y[n2 * 4 + 0] = b0; y[n2 * 4 + 1] = b1; y[n2 * 4 + 2] = b2; y[n2 * 4 + 3] = b3;
  }
  // twiddles W16^{n2 k1}
  tw16_apply<DIR, 1, 1>(y); tw16_apply<DIR, 1, 2>(y); tw16_apply<DIR, 1, 3>(y);
  tw16_apply<DIR, 2, 1>(y); tw16_apply<DIR, 2, 2>(y); tw16_apply<DIR, 2, 3>(y);
  tw16_apply<DIR, 3, 1>(y); tw16_apply<DIR, 3, 2>(y); tw16_apply<DIR, 3, 3>(y);
  // stage 2: 4-point DFTs over n2 for each k1 -> X[k1 + 4 k2]
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 b0 = y[k1], b1 = y[4 + k1], b2 = y[8 + k1], b3 = y[12 + k1];
    dft4<DIR>(b0, b1, b2, b3);
    a[k1] = b0; a[k1 + 4] = b1; a[k1 + 8] = b2; a[k1 + 12] = b3;
  }
}

// B-point DFT of a[0..B-1] in natural order, B in {1, 2, 4, 8, 16}
template <int DIR, int B>
__device__ __forceinline__ void dftB(float2* a) {
  if constexpr (B == 1) {
  } else if constexpr (B == 2) {
    dft2<DIR>(a[0], a[1]);
  } else if constexpr (B == 4) {
    dft4<DIR>(a[0], a[1], a[2], a[3]);
  } else if constexpr (B == 8) {
    float2 t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = a[i];
    dft8<DIR>(t);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = t[i];
  } else {
    static_assert(B == 16, "B must be 1, 2, 4, 8 or 16");
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = a[i];
    dft16<DIR>(t);
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = t[i];
  }
}

// ---------------------------------------------------------------------------
// raw buffer access: a per-lane byte offset in one VGPR plus a wave-uniform
// byte offset (SGPR), so unrolled row loops do not materialise one 64-bit
// address per row.  Out-of-range offsets read 0 and drop stores.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ float2 bload2(rsrc_t r, int voff, int soff) {
  u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ float bload1(rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore2(rsrc_t r, float2 x, int voff, int soff) {
  u32x2 v = {__float_as_uint(x.x), __float_as_uint(x.y)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}
// the same with the non-temporal cache hint (streamed data that should not
// displace the probe and object from L2)
__device__ __forceinline__ float2 bload2_nt(rsrc_t r, int voff, int soff) {
  u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ void bstore2_nt(rsrc_t r, float2 x, int voff, int soff) {
  u32x2 v = {__float_as_uint(x.x), __float_as_uint(x.y)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 2);
}

// A value every lane of the wave holds alike (a view index, a position, an
// object width read from memory), moved to an SGPR so that buffer offsets
// built from it are scalar; without it the compiler cannot prove uniformity
// of values loaded through pointers it cannot show read-only, and wraps
// each buffer access that takes it as its scalar offset in a readfirstlane
// loop.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Index arrays that no kernel writes (view positions, the view order, the
// tile lists) are read through constant-address-space pointers: where the
// index is uniform in a wave the load goes through the scalar cache instead
// of the vector memory path.
typedef const __attribute__((address_space(4))) int* kidx_t;
__device__ __forceinline__ kidx_t kidx(const int* p) { return (kidx_t)p; }

// Index that is the same for every lane of a wave when F >= 64 (a wave's 64
// lanes then share t / F); keeping it in an SGPR makes its table loads scalar.
template <int F>
__device__ __forceinline__ int wave_uniform_div(int t) {
  if constexpr (F >= 64) return __builtin_amdgcn_readfirstlane(t / F);
  else return t / F;
}

// twiddle table: tw[m] = exp(-2 pi i m / F), m in [0, F); inverse uses conj
template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int m, float2 a) {
  float2 w = tw[m];
  if constexpr (DIR > 0) w.y = -w.y;
  return cmul(a, w);
}

}  // namespace dmk
