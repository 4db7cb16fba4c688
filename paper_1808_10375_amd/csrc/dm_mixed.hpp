// dm_mixed.hpp -- the view update (Eq. 3 with F_c, Section II) for frames
// whose edge is not a power of two: F = R * Q with R a power of two and Q
// odd (188 = 4 * 47, 200 = 8 * 25, the frame sizes the paper's own
// measurements use).  Three kernels around the spectrum buffer, as for F =
// 256: row DFTs, then column DFTs with the mode sum and modulus scale and the
// inverse column DFTs, then inverse row DFTs with the update.
//
// One length-F line is transformed by Q threads with one level of the
// Cooley-Tukey split n = Q n1 + n2, k = k1 + R k2:
//   X[k1 + R k2] = sum_{n2} W_Q^{n2 k2} W_F^{n2 k1} sum_{n1} x[Q n1 + n2] W_R^{n1 k1}
// Thread n2 holds x[Q n1 + n2] (n1 < R) in registers, does the R-point DFT
// there, applies W_F^{n2 k1} and writes its R values to the line's LDS rows;
// thread q then forms the Q-point DFT for k2 = q directly, X[k1 + R q] for
// all k1, reading every row once (each row read is shared by the line's Q
// lanes).  The inverse runs the mirror image, so every value returns to the
// thread and register it came from, and no step needs a reordering.
// Q-point twiddles W_Q^{(n q) mod Q} come from a table in LDS every eighth
// step and by one complex product with W_Q^q in between.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>

#include "dm_kernels.hpp"

namespace dmk {

template <int F>
struct MixCfg;
template <>
struct MixCfg<188> {
  static constexpr int R = 4, Q = 47;
};
template <>
struct MixCfg<200> {
  static constexpr int R = 8, Q = 25;
};

template <int F>
struct MixRows {
  static constexpr int R = MixCfg<F>::R, Q = MixCfg<F>::Q;
  static constexpr int RB = 256 / Q;                  // rows per block
  static constexpr int NT = (RB * Q + 63) / 64 * 64;  // whole waves
  static constexpr int NBLK = (F + RB - 1) / RB;      // row blocks per frame
  static constexpr int LS = Q * R + 2;                // LDS line stride (complex)
};

// LDS tables: twl[m] = W_F^m = exp(-2 pi i m / F), m < F; twq[m] = W_Q^m.
template <int F>
__device__ __forceinline__ void mix_load_tables(const float2* __restrict__ tw, float2* twl,
                                                float2* twq, int t, int nt) {
  constexpr int R = MixCfg<F>::R, Q = MixCfg<F>::Q;
  for (int i = t; i < F; i += nt) twl[i] = tw[i];
  for (int i = t; i < Q; i += nt) twq[i] = tw[R * i];
}

// a[k1] *= W_F^{DIR n k1}
template <int F, int DIR>
__device__ __forceinline__ void mix_twiddle(float2 (&a)[MixCfg<F>::R], const float2* twl, int n) {
  constexpr int R = MixCfg<F>::R;
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) {
    float2 w = twl[n * k1];
    if constexpr (DIR > 0) w.y = -w.y;
    a[k1] = cmul(a[k1], w);
  }
}

// a[k1] = sum_{n < Q} line[n * R + k1] W_Q^{DIR n q}
template <int F, int DIR>
__device__ __forceinline__ void mix_qdft(float2 (&a)[MixCfg<F>::R], const float2* line,
                                         const float2* twq, int q) {
  constexpr int R = MixCfg<F>::R, Q = MixCfg<F>::Q;
  float2 acc[R];
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) acc[k1] = make_float2(0.f, 0.f);
  float2 step = twq[q];
  if constexpr (DIR > 0) step.y = -step.y;
  int idx = 0;  // (n * q) mod Q at the start of each group of eight
#pragma unroll 1
  for (int n0 = 0; n0 < Q; n0 += 8) {
    float2 w = twq[idx];
    if constexpr (DIR > 0) w.y = -w.y;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int n = n0 + s;
      if (n < Q) {
        const float4* row = reinterpret_cast<const float4*>(line + n * R);
#pragma unroll
        for (int h = 0; h < R / 2; ++h) {
          const float4 v = row[h];
          acc[2 * h].x += v.x * w.x - v.y * w.y;
          acc[2 * h].y += v.x * w.y + v.y * w.x;
          acc[2 * h + 1].x += v.z * w.x - v.w * w.y;
          acc[2 * h + 1].y += v.z * w.y + v.w * w.x;
        }
        w = cmul(w, step);
      }
    }
    idx += 8 * q;
    idx %= Q;
  }
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) a[k1] = acc[k1];
}

// R values of a line row to LDS as 16-byte stores
template <int R>
__device__ __forceinline__ void mix_store_row(float2* dst, const float2 (&a)[R]) {
  float4* d = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int h = 0; h < R / 2; ++h)
    d[h] = make_float4(a[2 * h].x, a[2 * h].y, a[2 * h + 1].x, a[2 * h + 1].y);
}

// (1) Z = 2 P O - psi and the DFT along rows; RB rows of one view-mode per
// block, Q threads per row.
template <int F>
__global__ __launch_bounds__(MixRows<F>::NT) void k_mix_rows_fwd(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap,
    const float2* __restrict__ tw, int M) {
  using C = MixRows<F>;
  constexpr int R = C::R, Q = C::Q, RB = C::RB, LS = C::LS, FF = F * F;
  __shared__ __align__(16) float2 xb[RB * LS];
  __shared__ float2 twl[F];
  __shared__ float2 twq[Q];
  const int t = threadIdx.x;
  const int2 vm = vmap[blockIdx.x / M];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y), m = blockIdx.x % M;
  const int jm = j * M + m;
  const int rl = t / Q, n2 = t % Q;
  const int row = blockIdx.y * RB + rl;
  const bool active = rl < RB && row < F;
  mix_load_tables<F>(tw, twl, twq, t, C::NT);
  float2 a[R] = {};
  if (active) {
    const int W = uni(sc.W);
    const int y0 = uni(sc.pos[2 * j]), x0 = uni(sc.pos[2 * j + 1]);
    const float2* __restrict__ pm = sc.psi + (size_t)jm * FF + (size_t)row * F;
    const float2* __restrict__ Pm = sc.P + (size_t)m * FF + (size_t)row * F;
    const float2* __restrict__ Or = sc.O + (size_t)(y0 + row) * W + x0;
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      const int v = Q * n1 + n2;
      const float2 phi = cmul(Pm[v], Or[v]);
      const float2 ps = pm[v];
      a[n1] = make_float2(2.f * phi.x - ps.x, 2.f * phi.y - ps.y);
    }
  }
  __syncthreads();  // tables
  if (active) {
    dftB<-1, R>(a);
    mix_twiddle<F, -1>(a, twl, n2);
    mix_store_row<R>(xb + rl * LS + n2 * R, a);
  }
  __syncthreads();
  if (active) {
    mix_qdft<F, -1>(a, xb + rl * LS, twq, n2);
    float2* __restrict__ Tr = sc.tspec + (size_t)jm * FF + (size_t)row * F + R * n2;
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) Tr[k1] = a[k1];
  }
}

// (2) DFT along CB columns of every mode of one view, the mode sum, the
// modulus scale and the inverse DFT along the columns, in place in the
// spectrum buffer.  Thread (c, n2, m) with c fastest; dynamic LDS: CB * M
// exchange lines, then the mode powers s [M][CB][F] and the scale g [CB][F].
template <int F>
__global__ __launch_bounds__(1024) void k_mix_cols(const ScanDev* __restrict__ scans,
                                                   const int2* __restrict__ vmap,
                                                   const float2* __restrict__ tw, int M, int CB) {
  constexpr int R = MixCfg<F>::R, Q = MixCfg<F>::Q, LS = MixRows<F>::LS, FF = F * F;
  extern __shared__ __align__(16) float2 dyn[];
  __shared__ float2 twl[F];
  __shared__ float2 twq[Q];
  const int t = threadIdx.x;
  const int nblk = (F + CB - 1) / CB;
  const int slot = xcd_group_slot(blockIdx.x, gridDim.x);
  const int2 vm = vmap[slot / nblk];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const int col0 = (slot % nblk) * CB;
  const int c = t % CB;
  const int rest = t / CB;
  const int n2 = rest % Q;
  const int m = rest / Q;
  const bool active = m < M && col0 + c < F;
  const int line = m * CB + c;
  float2* xl = dyn + (size_t)line * LS;
  float* s = reinterpret_cast<float*>(dyn + (size_t)CB * M * LS);
  float* g = s + (size_t)M * CB * F;
  float2* __restrict__ Tm = sc.tspec + ((size_t)j * M + m) * FF + col0 + c;
  mix_load_tables<F>(tw, twl, twq, t, blockDim.x);
  float2 a[R] = {};
  if (active) {
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) a[n1] = Tm[(size_t)(Q * n1 + n2) * F];
  }
  __syncthreads();
  if (active) {
    dftB<-1, R>(a);
    mix_twiddle<F, -1>(a, twl, n2);
    mix_store_row<R>(xl + n2 * R, a);
  }
  __syncthreads();
  if (active) {
    mix_qdft<F, -1>(a, xl, twq, n2);  // a[k1] = spectrum at row k1 + R n2
    float* sl = s + (size_t)line * F + R * n2;
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) sl[k1] = cabs2(a[k1]);
  }
  __syncthreads();
  // one thread per pixel of the block's columns: sum over modes, scale
  // sqrt(I / S) / F^2 (0 where S vanishes); pixels in column-major order
  const float* __restrict__ Ij = sc.I + (size_t)j * FF + col0;
  const float inv_ff = 1.0f / (float)FF;
  for (int p = t; p < CB * F; p += blockDim.x) {
    const int cc = p / F, kk = p - cc * F;
    if (col0 + cc >= F) continue;
    float sum = 0.f;
    for (int mm = 0; mm < M; ++mm) sum += s[(size_t)(mm * CB + cc) * F + kk];
    const float iv = fmaxf(Ij[(size_t)kk * F + cc], 0.f);
    g[cc * F + kk] = (sum > FLT_MIN) ? sqrtf(iv / sum) * inv_ff : 0.f;
  }
  __syncthreads();
  if (active) {
    const float* gl = g + c * F + R * n2;
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) a[k1] = cscale(a[k1], gl[k1]);
    // the forward reads of this line finished before the barriers above
    mix_store_row<R>(xl + n2 * R, a);
  }
  __syncthreads();
  if (active) {
    mix_qdft<F, 1>(a, xl, twq, n2);
    mix_twiddle<F, 1>(a, twl, n2);
    dftB<1, R>(a);
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) Tm[(size_t)(Q * n1 + n2) * F] = a[n1];
  }
}

// (3) inverse DFT along rows, psi' = psi + beta (Z' - P O), the view's
// object numerator sum_m conj(P_m) psi'_m and the eps_psi partial sums; all
// modes of RB rows per block.
template <int F>
__global__ __launch_bounds__(MixRows<F>::NT) void k_mix_rows_inv(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap,
    const float2* __restrict__ tw, int M) {
  using C = MixRows<F>;
  constexpr int R = C::R, Q = C::Q, RB = C::RB, LS = C::LS, NT = C::NT, FF = F * F;
  __shared__ __align__(16) float2 xb[RB * LS];
  __shared__ float2 twl[F];
  __shared__ float2 twq[Q];
  __shared__ float red[2 * (NT / 64)];
  const int t = threadIdx.x;
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const int rl = t / Q, n2 = t % Q;
  const int row = blockIdx.y * RB + rl;
  const bool active = rl < RB && row < F;
  const int W = uni(sc.W);
  const float beta = sc.beta;
  const int y0 = uni(sc.pos[2 * j]), x0 = uni(sc.pos[2 * j + 1]);
  const float2* __restrict__ Or = sc.O + (size_t)(y0 + row) * W + x0;
  mix_load_tables<F>(tw, twl, twq, t, NT);
  float2 oacc[R];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) oacc[n1] = make_float2(0.f, 0.f);
  float e_d = 0.f, e_n = 0.f;
  for (int m = 0; m < M; ++m) {
    const size_t base = ((size_t)j * M + m) * FF + (size_t)row * F;
    float2 a[R] = {};
    if (active) {
      const float2* __restrict__ Tr = sc.tspec + base + R * n2;
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) a[k1] = Tr[k1];
    }
    __syncthreads();  // the previous mode's reads of xb (and the tables)
    if (active) mix_store_row<R>(xb + rl * LS + n2 * R, a);
    __syncthreads();
    if (active) {
      mix_qdft<F, 1>(a, xb + rl * LS, twq, n2);
      mix_twiddle<F, 1>(a, twl, n2);
      dftB<1, R>(a);  // a[n1] = Z' at column Q n1 + n2
      float2* __restrict__ pm = sc.psi + base;
      const float2* __restrict__ Pm = sc.P + (size_t)m * FF + (size_t)row * F;
      float2 pr[R], ov[R], pv[R];
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) {
        const int v = Q * n1 + n2;
        pr[n1] = Pm[v];
        ov[n1] = Or[v];
        pv[n1] = pm[v];
      }
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) {
        const float2 phi = cmul(pr[n1], ov[n1]);
        const float2 d = make_float2(beta * (a[n1].x - phi.x), beta * (a[n1].y - phi.y));
        const float2 pn = cadd(pv[n1], d);
        pm[Q * n1 + n2] = pn;
        e_d += cabs2(d);
        e_n += cabs2(pn);
        oacc[n1] = cadd(oacc[n1], cmulc(pr[n1], pn));
      }
    }
  }
  if (active) {
    float2* __restrict__ oj = sc.opart + (size_t)j * FF + (size_t)row * F;
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) oj[Q * n1 + n2] = oacc[n1];
  }
  block_sum2<NT>(e_d, e_n, red);
  if (t == 0) {
    const int part = j * gridDim.y + blockIdx.y;
    sc.err_psi[2 * part] = e_d;
    sc.err_psi[2 * part + 1] = e_n;
  }
}

}  // namespace dmk
