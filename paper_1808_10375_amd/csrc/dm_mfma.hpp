// dm_mfma.hpp -- the BF16x3 precision form of the view update for F = 128:
// the 2-D DFT as dense complex matrix products with the DFT matrix W on the
// matrix cores (v_mfma_f32_16x16x32_bf16), every real product split into
// hi*hi + hi*lo + lo*hi of bfloat16 pieces with float32 accumulation.  The
// modulus scale, error norms and updates stay float32.
//
// Three kernels around the spectrum buffer T [N][M][F][F]:
//   (1) k_mf_rows_fwd  T = Z W            Z = 2 P O - psi      (Eqs. 2-3)
//   (2) k_mf_cols      U = W T, modulus projection (definition of F_c),
//                      V = conj(W) U' / F^2, written back over T
//   (3) k_mf_rows_inv  Z' = V conj(W), psi' = psi + beta (Z' - P O), the
//                      per-view object numerator and eps_psi partials
// All three keep the split W (real/imaginary x hi/lo, 128 KB) in LDS and are
// persistent: each block loads W once and walks its share of the work.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (one wave, 64 lanes):
//   A (16 x 32):  lane l holds row l%16, k = 8*(l/16) + e, e = 0..7
//   B (32 x 16):  lane l holds col l%16, k = 8*(l/16) + e
//   C (16 x 16):  lane l holds col l%16, rows 4*(l/16) + r, r = 0..3
// W is stored in B-fragment order, Wf[mat][ks][nt][lane] (16 bytes each),
// mat = 0..3 for Re hi, Re lo, Im hi, Im lo; because W is symmetric the
// same fragment also serves as the A operand of row tile nt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dm_kernels.hpp"

namespace dmk {

typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mf_f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfF = 128;                    // frame edge of this form
constexpr int kMfKs = kMfF / 32;             // k steps of 32
constexpr int kMfNt = kMfF / 16;             // 16-wide tiles
constexpr int kMfFrag = kMfKs * kMfNt * 64;  // uint4 per matrix
constexpr int kMfWords = 4 * kMfFrag;        // uint4 of the whole table (128 KB)
constexpr int kMfMaxModes = 8;

// float -> bfloat16 bits, round to nearest even (the conversion gfx950 does
// in hardware, two values per v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t mf_bf16_rne(float f) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)f);
}

// split 8 floats into packed bfloat16 hi and lo pieces (lo = bf16(x - hi))
__device__ __forceinline__ void mf_split8(const float (&x)[8], uint4& hi, uint4& lo) {
  uint32_t h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    h[e] = mf_bf16_rne(x[e]);
    l[e] = mf_bf16_rne(x[e] - __uint_as_float(h[e] << 16));
  }
  hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                  h[6] | (h[7] << 16));
  lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16),
                  l[6] | (l[7] << 16));
}

__device__ __forceinline__ uint4 mf_neg(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u,
                    v.w ^ 0x80008000u);
}

__device__ __forceinline__ mf_f32x4 mf_mma(uint4 a, uint4 b, mf_f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mf_bf16x8, a),
                                                 __builtin_bit_cast(mf_bf16x8, b), c, 0, 0, 0);
}

// c += a * b with the three-term split (a, b given as hi/lo pieces)
__device__ __forceinline__ mf_f32x4 mf_mma3(uint4 ah, uint4 al, uint4 bh, uint4 bl,
                                            mf_f32x4 c) {
  c = mf_mma(ah, bh, c);
  c = mf_mma(ah, bl, c);
  c = mf_mma(al, bh, c);
  return c;
}

// A operand of a complex product, split: re, im and -im pieces
struct MfA {
  uint4 rh, rl, ih, il;
};

__device__ __forceinline__ MfA mf_split_complex(const float2 (&z)[8]) {
  float re[8], im[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) { re[e] = z[e].x; im[e] = z[e].y; }
  MfA a;
  mf_split8(re, a.rh, a.rl);
  mf_split8(im, a.ih, a.il);
  return a;
}

// W fragment (ks, nt) of matrix `mat` from LDS
__device__ __forceinline__ uint4 mf_w(const uint4* wl, int mat, int ks, int nt, int lane) {
  return wl[((mat * kMfKs + ks) * kMfNt + nt) * 64 + lane];
}

// acc_re += Ar Wr - Ai Wi ; acc_im += Ar Wi + Ai Wr   (product with W)
// acc_re += Ar Wr + Ai Wi ; acc_im += Ai Wr - Ar Wi   (product with conj W)
template <bool CONJ>
__device__ __forceinline__ void mf_cmma(const MfA& a, uint4 wrh, uint4 wrl, uint4 wih, uint4 wil,
                                        mf_f32x4& re, mf_f32x4& im) {
  if constexpr (!CONJ) {
    re = mf_mma3(a.rh, a.rl, wrh, wrl, re);
    re = mf_mma3(mf_neg(a.ih), mf_neg(a.il), wih, wil, re);
    im = mf_mma3(a.rh, a.rl, wih, wil, im);
    im = mf_mma3(a.ih, a.il, wrh, wrl, im);
  } else {
    re = mf_mma3(a.rh, a.rl, wrh, wrl, re);
    re = mf_mma3(a.ih, a.il, wih, wil, re);
    im = mf_mma3(a.ih, a.il, wrh, wrl, im);
    im = mf_mma3(mf_neg(a.rh), mf_neg(a.rl), wih, wil, im);
  }
}

__device__ __forceinline__ void mf_load_w(uint4* wl, const uint4* __restrict__ wf) {
  for (int i = threadIdx.x; i < kMfWords; i += blockDim.x) wl[i] = wf[i];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// (1) row transform: T[r][c] = sum_k Z[r][k] W[k][c] for one (view, mode)
// frame per iteration of the block loop; eight waves (two per SIMD), wave w
// owns rows 16w .. 16w+15.
// ---------------------------------------------------------------------------
constexpr int kMfRowsThreads = 512;

__global__ __launch_bounds__(kMfRowsThreads) void k_mf_rows_fwd(const ScanDev* __restrict__ scans,
                                                                const int2* __restrict__ vmap,
                                                                int total_views, int M,
                                                                const uint4* __restrict__ wf) {
  extern __shared__ uint4 wl[];
  mf_load_w(wl, wf);
  constexpr int F = kMfF, FF = F * F;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int total = total_views * M;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int2 vm = vmap[item / M];
    const int m = item % M;
    const ScanDev& sc = scans[vm.x];
    const int j = uni(vm.y);
    const int W = uni(sc.W);
    const int y0 = uni(kidx(sc.pos)[2 * j]), x0 = uni(kidx(sc.pos)[2 * j + 1]);
    const float2* __restrict__ psi = sc.psi + ((size_t)j * M + m) * FF;
    const float2* __restrict__ P = sc.P + (size_t)m * FF;
    const float2* __restrict__ O = sc.O + (size_t)y0 * W + x0;
    float2* __restrict__ T = sc.tspec + ((size_t)j * M + m) * FF;
    mf_f32x4 re[kMfNt], im[kMfNt];
#pragma unroll
    for (int nt = 0; nt < kMfNt; ++nt) {
      re[nt] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
      im[nt] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int row = 16 * wave + (lane & 15);
    // the raw loads of k step ks + 1 go out before the products of step ks
    float2 pv[8], ov[8], sv[8];
    auto load_step = [&](int ks) {
      const int k0 = 32 * ks + 8 * (lane >> 4);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        pv[e] = P[row * F + k0 + e];
        ov[e] = O[(size_t)row * W + k0 + e];
        sv[e] = psi[row * F + k0 + e];
      }
    };
    load_step(0);
#pragma unroll
    for (int ks = 0; ks < kMfKs; ++ks) {
      float2 z[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float2 phi = cmul(pv[e], ov[e]);
        z[e] = make_float2(2.f * phi.x - sv[e].x, 2.f * phi.y - sv[e].y);
      }
      const MfA a = mf_split_complex(z);
      if (ks + 1 < kMfKs) {
        load_step(ks + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int nt = 0; nt < kMfNt; ++nt)
        mf_cmma<false>(a, mf_w(wl, 0, ks, nt, lane), mf_w(wl, 1, ks, nt, lane),
                       mf_w(wl, 2, ks, nt, lane), mf_w(wl, 3, ks, nt, lane), re[nt], im[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < kMfNt; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int orow = 16 * wave + 4 * (lane >> 4) + r;
        T[orow * F + 16 * nt + (lane & 15)] = make_float2(re[nt][r], im[nt][r]);
      }
  }
}

// ---------------------------------------------------------------------------
// (2) column transform, modulus projection and inverse column transform for
// 16 columns n0 .. n0+15 of every mode of one view, in place in T.  Eight
// waves (two per SIMD, so one's memory waits overlap the other's products);
// wave w owns output tile w (rows a = 16 w .. 16 w + 15 of U^T, V^T).
//   U^T[n][a] = sum_k T[k][n] W[k][a]
//   U' = U * sqrt(I / sum_m |U_m|^2) / F^2
//   V^T[n][a'] = sum_a U'^T[n][a] conj(W)[a][a']   (A operand via LDS)
// ---------------------------------------------------------------------------
constexpr int kMfColsThreads = 512;

__global__ __launch_bounds__(kMfColsThreads) void k_mf_cols(const ScanDev* __restrict__ scans,
                                                            const int2* __restrict__ vmap,
                                                            int total_views, int M,
                                                            const uint4* __restrict__ wf) {
  extern __shared__ uint4 wl[];
  mf_load_w(wl, wf);
  // U' of one mode in A-fragment order: [mat][ks][lane] uint4, mat = re hi,
  // re lo, im hi, im lo; two buffers, used by alternate modes, so that one
  // barrier per mode suffices (a wave writes mode m + 1's fragments only
  // after every wave has passed mode m's barrier, i.e. finished reading the
  // buffer of mode m - 1)
  uint16_t* const ua2 = reinterpret_cast<uint16_t*>(wl + kMfWords);
  constexpr int F = kMfF, FF = F * F;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = wave;  // this wave's 16 columns of the transform output
  const int total = total_views * kMfNt;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int2 vm = vmap[item / kMfNt];
    const int n0 = 16 * (item % kMfNt);
    const ScanDev& sc = scans[vm.x];
    const int j = uni(vm.y);
    float2* __restrict__ T = sc.tspec + (size_t)j * M * FF;
    const float* __restrict__ I = sc.I + (size_t)j * FF;
    mf_f32x4 ure[kMfMaxModes], uim[kMfMaxModes];
#pragma unroll
    for (int m = 0; m < kMfMaxModes; ++m) {
      if (m < M) {
        const float2* __restrict__ Tm = T + (size_t)m * FF;
        ure[m] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
        uim[m] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
        // all of this mode's column loads first: one memory latency per mode
        float2 zall[kMfKs][8];
#pragma unroll
        for (int ks = 0; ks < kMfKs; ++ks)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            zall[ks][e] = Tm[(32 * ks + 8 * (lane >> 4) + e) * F + n0 + (lane & 15)];
#pragma unroll
        for (int ks = 0; ks < kMfKs; ++ks) {
          const MfA a = mf_split_complex(zall[ks]);
          mf_cmma<false>(a, mf_w(wl, 0, ks, nt, lane), mf_w(wl, 1, ks, nt, lane),
                         mf_w(wl, 2, ks, nt, lane), mf_w(wl, 3, ks, nt, lane), ure[m], uim[m]);
        }
      }
    }
    // modulus projection: lane holds a = 16 w + lane%16 and n = 4 (lane/16) + r
    const float inv_ff = 1.0f / (float)FF;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = 0.f;
#pragma unroll
      for (int m = 0; m < kMfMaxModes; ++m)
        if (m < M) s += ure[m][r] * ure[m][r] + uim[m][r] * uim[m][r];
      const int a = 16 * wave + (lane & 15);
      const int n = 4 * (lane >> 4) + r;
      const float iv = fmaxf(I[a * F + n0 + n], 0.f);
      const float g = (s > FLT_MIN) ? sqrtf(iv / s) * inv_ff : 0.f;
#pragma unroll
      for (int m = 0; m < kMfMaxModes; ++m)
        if (m < M) { ure[m][r] *= g; uim[m][r] *= g; }
    }
    // inverse column transform, one mode at a time through LDS
#pragma unroll
    for (int m = 0; m < kMfMaxModes; ++m) {
      if (m < M) {
        uint16_t* const ua = ua2 + (m & 1) * (4 * kMfKs * 512);
        // element (n, a) of U'^T goes to A fragment ks = a/32, lane
        // n + 16 ((a%32)/8), slot a%8; here a = 16 w + lane%16, so
        // a/32 = w/2 and (a%32)/8 = 2 (w%2) + (lane%16)/8
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = 4 * (lane >> 4) + r;
          const int l2 = n + 16 * (2 * (wave & 1) + ((lane & 15) >> 3));
          const int slot = (((wave >> 1) * 64 + l2) * 8) + (lane & 7);
          const float vr = ure[m][r], vi = uim[m][r];
          const uint32_t rh = mf_bf16_rne(vr), ih = mf_bf16_rne(vi);
          const uint32_t rl = mf_bf16_rne(vr - __uint_as_float(rh << 16));
          const uint32_t il = mf_bf16_rne(vi - __uint_as_float(ih << 16));
          ua[0 * kMfKs * 512 + slot] = (uint16_t)rh;
          ua[1 * kMfKs * 512 + slot] = (uint16_t)rl;
          ua[2 * kMfKs * 512 + slot] = (uint16_t)ih;
          ua[3 * kMfKs * 512 + slot] = (uint16_t)il;
        }
        __syncthreads();
        const uint4* uq = reinterpret_cast<const uint4*>(ua);
        mf_f32x4 vre = mf_f32x4{0.f, 0.f, 0.f, 0.f}, vim = mf_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kMfKs; ++ks) {
          MfA a;
          a.rh = uq[(0 * kMfKs + ks) * 64 + lane];
          a.rl = uq[(1 * kMfKs + ks) * 64 + lane];
          a.ih = uq[(2 * kMfKs + ks) * 64 + lane];
          a.il = uq[(3 * kMfKs + ks) * 64 + lane];
          mf_cmma<true>(a, mf_w(wl, 0, ks, nt, lane), mf_w(wl, 1, ks, nt, lane),
                        mf_w(wl, 2, ks, nt, lane), mf_w(wl, 3, ks, nt, lane), vre, vim);
        }
        // V^T[n][a'] -> T[a'][n0 + n]; lane holds a' = 16 w + lane%16,
        // n = 4 (lane/16) + r
        float2* __restrict__ Tm = T + (size_t)m * FF;
        const int ap = 16 * wave + (lane & 15);
        float4* dst = reinterpret_cast<float4*>(Tm + ap * F + n0 + 4 * (lane >> 4));
        dst[0] = make_float4(vre[0], vim[0], vre[1], vim[1]);
        dst[1] = make_float4(vre[2], vim[2], vre[3], vim[3]);
      }
    }
    __syncthreads();  // the LDS fragments are rewritten by the next item
  }
}

// ---------------------------------------------------------------------------
// (3) inverse row transform and the view update for all rows and modes of
// one view; eight waves (two per SIMD), wave w owns rows 16w .. 16w+15.  The
// view's eps_psi partials go to part 2j (part 2j + 1 is left at zero).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMfRowsThreads) void k_mf_rows_inv(const ScanDev* __restrict__ scans,
                                                     const int2* __restrict__ vmap,
                                                     int total_views, int M,
                                                     const uint4* __restrict__ wf) {
  extern __shared__ uint4 wl[];
  mf_load_w(wl, wf);
  __shared__ float red[2 * (kMfRowsThreads / 64)];
  constexpr int F = kMfF, FF = F * F;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int total = total_views;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int2 vm = vmap[item];
    const ScanDev& sc = scans[vm.x];
    const int j = uni(vm.y);
    const int W = uni(sc.W);
    const float beta = sc.beta;
    const int y0 = uni(kidx(sc.pos)[2 * j]), x0 = uni(kidx(sc.pos)[2 * j + 1]);
    const float2* __restrict__ O = sc.O + (size_t)y0 * W + x0;
    const int rbase = 16 * wave;
    float2 oacc[kMfNt][4];
#pragma unroll
    for (int nt = 0; nt < kMfNt; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) oacc[nt][r] = make_float2(0.f, 0.f);
    float e_d = 0.f, e_n = 0.f;
    for (int m = 0; m < M; ++m) {
      const float2* __restrict__ V = sc.tspec + ((size_t)j * M + m) * FF;
      float2* __restrict__ psi = sc.psi + ((size_t)j * M + m) * FF;
      const float2* __restrict__ P = sc.P + (size_t)m * FF;
      mf_f32x4 re[kMfNt], im[kMfNt];
#pragma unroll
      for (int nt = 0; nt < kMfNt; ++nt) {
        re[nt] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
        im[nt] = mf_f32x4{0.f, 0.f, 0.f, 0.f};
      }
      for (int ks = 0; ks < kMfKs; ++ks) {
        float2 z[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = V[(rbase + (lane & 15)) * F + 32 * ks + 8 * (lane >> 4) + e];
        const MfA a = mf_split_complex(z);
#pragma unroll
        for (int nt = 0; nt < kMfNt; ++nt)
          mf_cmma<true>(a, mf_w(wl, 0, ks, nt, lane), mf_w(wl, 1, ks, nt, lane),
                        mf_w(wl, 2, ks, nt, lane), mf_w(wl, 3, ks, nt, lane), re[nt], im[nt]);
      }
      // the psi' stores may alias later loads as far as the compiler knows:
      // each tile's loads are issued before its stores
#pragma unroll
      for (int nt = 0; nt < kMfNt; ++nt) {
        const int col = 16 * nt + (lane & 15);
        float2 pr[4], ov[4], pv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rbase + 4 * (lane >> 4) + r;
          pr[r] = P[row * F + col];
          ov[r] = O[(size_t)row * W + col];
          pv[r] = psi[row * F + col];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rbase + 4 * (lane >> 4) + r;
          const float2 phi = cmul(pr[r], ov[r]);
          const float2 d = make_float2(beta * (re[nt][r] - phi.x), beta * (im[nt][r] - phi.y));
          const float2 pn = cadd(pv[r], d);
          psi[row * F + col] = pn;
          e_d += cabs2(d);
          e_n += cabs2(pn);
          oacc[nt][r] = cadd(oacc[nt][r], cmulc(pr[r], pn));
        }
      }
    }
    float2* __restrict__ oj = sc.opart + (size_t)j * FF;
#pragma unroll
    for (int nt = 0; nt < kMfNt; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        oj[(rbase + 4 * (lane >> 4) + r) * F + 16 * nt + (lane & 15)] = oacc[nt][r];
    block_sum2<kMfRowsThreads>(e_d, e_n, red);
    if (threadIdx.x == 0) {
      sc.err_psi[4 * j] = e_d;
      sc.err_psi[4 * j + 1] = e_n;
      sc.err_psi[4 * j + 2] = 0.f;
      sc.err_psi[4 * j + 3] = 0.f;
    }
    __syncthreads();  // red is reused by the next item
  }
}

}  // namespace dmk
