// dm_mixed.hpp -- the view update (Eq. 3 with F_c, Section II) for frames
// whose edge is not a power of two: F = R * Q with R a power of two and Q
// odd (188 = 4 * 47, 200 = 8 * 25, the frame sizes the paper's own
// measurements use).  Three kernels around the spectrum buffer, as for F =
// 256: row DFTs, then column DFTs with the mode sum and modulus scale and the
// inverse column DFTs, then inverse row DFTs with the update.
//
// One length-F line is transformed with one level of the Cooley-Tukey split
// n = Q n1 + n2, k = k1 + R k2:
//   X[k1 + R k2] = sum_{n2} W_Q^{n2 k2} W_F^{n2 k1} sum_{n1} x[Q n1 + n2] W_R^{n1 k1}
// by Q + 1 threads.  Thread n2 < Q holds x[Q n1 + n2] (n1 < R) in registers,
// does the R-point DFT there, applies W_F^{n2 k1} and writes its R values to
// row n2 of the line's LDS buffer.  The Q-point DFTs over the rows use the
// symmetry of W_Q for odd Q: with u_n = y_n + y_{Q-n} and v_n = y_n - y_{Q-n}
// (formed in place, 1 <= n <= (Q-1)/2) and c_n + i s_n = W_Q^{n p},
//   Y_p     = y_0 + sum_n c_n u_n + i sum_n s_n v_n,
//   Y_{Q-p} = y_0 + sum_n c_n u_n - i sum_n s_n v_n,
// so thread t forms the two real-weighted sums for p = t / 2 over half of the
// k1 range (half t % 2) and gets both outputs: a quarter of the products of
// the direct sum, and each LDS row read serves two outputs.  The inverse runs
// the same steps with conjugate twiddles and one more exchange, so values
// return to the thread and register they came from.  Q-point twiddles come
// from a table in LDS every eighth step and by one complex product with
// W_Q^p in between.
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
struct Mix {
  static constexpr int R = MixCfg<F>::R, Q = MixCfg<F>::Q;
  static constexpr int QT = Q + 1;         // threads per line
  static constexpr int H = R / 2;         // k1 values per pair thread
  static constexpr int NP = (Q - 1) / 2;  // symmetric pairs of rows
  static constexpr int LS = Q * R + 2;    // LDS line stride (complex)
  static constexpr int RB = 256 / QT;     // rows per block of the row kernels
  static constexpr int NT = (RB * QT + 63) / 64 * 64;  // whole waves
  static constexpr int NBLK = (F + RB - 1) / RB;      // row blocks per frame
};

// LDS tables: twl[m] = W_F^m = exp(-2 pi i m / F), m < F; twq[m] = W_Q^m.
template <int F>
__device__ __forceinline__ void mix_load_tables(const float2* __restrict__ tw, float2* twl,
                                                float2* twq, int t, int nt) {
  constexpr int R = Mix<F>::R, Q = Mix<F>::Q;
  for (int i = t; i < F; i += nt) twl[i] = tw[i];
  for (int i = t; i < Q; i += nt) twq[i] = tw[R * i];
}

// Thread n < Q of a line: R-point DFT of its registers, twiddle W_F^{DIR n k1},
// row n of the line buffer.
template <int F, int DIR>
__device__ __forceinline__ void mix_first(float2 (&a)[Mix<F>::R], float2* line,
                                          const float2* twl, int n) {
  constexpr int R = Mix<F>::R;
  dftB<DIR, R>(a);
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) {
    float2 w = twl[n * k1];
    if constexpr (DIR > 0) w.y = -w.y;
    a[k1] = cmul(a[k1], w);
  }
  float4* d = reinterpret_cast<float4*>(line + n * R);
#pragma unroll
  for (int h = 0; h < R / 2; ++h)
    d[h] = make_float4(a[2 * h].x, a[2 * h].y, a[2 * h + 1].x, a[2 * h + 1].y);
}

// Rows n and Q - n (1 <= n <= (Q-1)/2, thread n of the line) become their
// sum and difference, in place.
template <int F>
__device__ __forceinline__ void mix_uv(float2* line, int n) {
  constexpr int R = Mix<F>::R, NP = Mix<F>::NP, Q = Mix<F>::Q;
  if (n < 1 || n > NP) return;
  float4* a = reinterpret_cast<float4*>(line + n * R);
  float4* b = reinterpret_cast<float4*>(line + (Q - n) * R);
#pragma unroll
  for (int h = 0; h < R / 2; ++h) {
    const float4 x = a[h], y = b[h];
    a[h] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
    b[h] = make_float4(x.x - y.x, x.y - y.y, x.z - y.z, x.w - y.w);
  }
}

// Positions (k1 + R k2) of a thread's pair outputs: lo = Y_p, hi = Y_{Q-p},
// H consecutive values each; p = 0 has no hi.
template <int F>
__device__ __forceinline__ void mix_pair_pos(int t, int& ilo, int& ihi) {
  constexpr int R = Mix<F>::R, Q = Mix<F>::Q, H = Mix<F>::H;
  const int p = t >> 1, h = t & 1;
  ilo = h * H + R * p;
  ihi = p > 0 ? h * H + R * (Q - p) : -1;
}

// Q-point DFTs over the rows (after mix_uv), thread t of the line:
// lo[k] = Y_p[k1], hi[k] = Y_{Q-p}[k1] with p = t / 2, k1 = (t % 2) H + k.
template <int F, int DIR>
__device__ __forceinline__ void mix_pairs(float2 (&lo)[Mix<F>::H], float2 (&hi)[Mix<F>::H],
                                          const float2* line, const float2* twq, int t) {
  constexpr int R = Mix<F>::R, Q = Mix<F>::Q, H = Mix<F>::H, NP = Mix<F>::NP;
  const int p = t >> 1, h = t & 1;
  float2 su[H], sv[H];
#pragma unroll
  for (int k = 0; k < H; ++k) { su[k] = make_float2(0.f, 0.f); sv[k] = make_float2(0.f, 0.f); }
  float2 step = twq[p];
  if constexpr (DIR > 0) step.y = -step.y;
  int idx = p;  // (n p) mod Q at the start of each group of eight
#pragma unroll 1
  for (int n0 = 1; n0 <= NP; n0 += 8) {
    float2 w = twq[idx];
    if constexpr (DIR > 0) w.y = -w.y;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int n = n0 + s;
      if (n <= NP) {
        const float2* u = line + n * R + h * H;
        const float2* v = line + (Q - n) * R + h * H;
        float2 uu[H], vv[H];
#pragma unroll
        for (int k = 0; k < H; k += 2) {
          const float4 a = *reinterpret_cast<const float4*>(u + k);
          const float4 b = *reinterpret_cast<const float4*>(v + k);
          uu[k] = make_float2(a.x, a.y); uu[k + 1] = make_float2(a.z, a.w);
          vv[k] = make_float2(b.x, b.y); vv[k + 1] = make_float2(b.z, b.w);
        }
#pragma unroll
        for (int k = 0; k < H; ++k) {
          su[k].x += w.x * uu[k].x; su[k].y += w.x * uu[k].y;
          sv[k].x += w.y * vv[k].x; sv[k].y += w.y * vv[k].y;
        }
        w = cmul(w, step);
      }
    }
    idx += 8 * p;
    idx %= Q;
  }
  const float2* y0 = line + h * H;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float2 a = make_float2(y0[k].x + su[k].x, y0[k].y + su[k].y);
    lo[k] = make_float2(a.x - sv[k].y, a.y + sv[k].x);
    hi[k] = make_float2(a.x + sv[k].y, a.y - sv[k].x);
  }
}

// a thread's pair values to their rows of the line buffer
template <int F>
__device__ __forceinline__ void mix_put_pairs(float2* line, const float2 (&lo)[Mix<F>::H],
                                              const float2 (&hi)[Mix<F>::H], int t) {
  constexpr int H = Mix<F>::H;
  int ilo, ihi;
  mix_pair_pos<F>(t, ilo, ihi);
#pragma unroll
  for (int k = 0; k < H; k += 2) {
    *reinterpret_cast<float4*>(line + ilo + k) =
        make_float4(lo[k].x, lo[k].y, lo[k + 1].x, lo[k + 1].y);
    if (ihi >= 0)
      *reinterpret_cast<float4*>(line + ihi + k) =
          make_float4(hi[k].x, hi[k].y, hi[k + 1].x, hi[k + 1].y);
  }
}

// Thread n < Q after the inverse Q-point DFTs are back in the rows: row n,
// twiddle W_F^{-n k1}, inverse R-point DFT; a[n1] = x[Q n1 + n].
template <int F>
__device__ __forceinline__ void mix_last_inv(float2 (&a)[Mix<F>::R], const float2* line,
                                             const float2* twl, int n) {
  constexpr int R = Mix<F>::R;
  const float4* r = reinterpret_cast<const float4*>(line + n * R);
#pragma unroll
  for (int h = 0; h < R / 2; ++h) {
    const float4 v = r[h];
    a[2 * h] = make_float2(v.x, v.y);
    a[2 * h + 1] = make_float2(v.z, v.w);
  }
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) {
    float2 w = twl[n * k1];
    w.y = -w.y;
    a[k1] = cmul(a[k1], w);
  }
  dftB<1, R>(a);
}

// Inverse line transform of the rows already in `line` (row k2 holds
// X[k1 + R k2]); the caller synchronised after writing them.  Thread n < Q
// of the line ends with a[n1] = x[Q n1 + n] (unnormalised).  Four barriers.
template <int F>
__device__ __forceinline__ void mix_inverse(float2 (&a)[Mix<F>::R], float2* line,
                                            const float2* twl, const float2* twq, int t,
                                            bool active) {
  constexpr int H = Mix<F>::H, Q = Mix<F>::Q;
  if (active) mix_uv<F>(line, t);
  __syncthreads();
  float2 lo[H], hi[H];
  if (active) mix_pairs<F, 1>(lo, hi, line, twq, t);
  __syncthreads();
  if (active) mix_put_pairs<F>(line, lo, hi, t);
  __syncthreads();
  if (active && t < Q) mix_last_inv<F>(a, line, twl, t);
}

// (1) Z = 2 P O - psi and the DFT along rows; RB rows of every mode of one
// view per block, Q + 1 threads per row, mode after mode with the next
// mode's psi in flight (the tables are loaded once per block).
template <int F>
__global__ __launch_bounds__(Mix<F>::NT) void k_mix_rows_fwd(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap,
    const float2* __restrict__ tw, int M) {
  using C = Mix<F>;
  constexpr int R = C::R, Q = C::Q, QT = C::QT, H = C::H, RB = C::RB, LS = C::LS, FF = F * F;
  __shared__ __align__(16) float2 xb[RB * LS];
  __shared__ float2 twl[F];
  __shared__ float2 twq[Q];
  const int t = threadIdx.x;
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const int rl = t / QT, tl = t % QT;
  const int row = blockIdx.y * RB + rl;
  const bool active = rl < RB && row < F;
  const bool owner = active && tl < Q;
  float2* line = xb + rl * LS;
  mix_load_tables<F>(tw, twl, twq, t, C::NT);
  const int W = uni(sc.W);
  const int y0 = uni(kidx(sc.pos)[2 * j]), x0 = uni(kidx(sc.pos)[2 * j + 1]);
  const float2* __restrict__ p0 = sc.psi + (size_t)j * M * FF + (size_t)row * F;
  const float2* __restrict__ Or = sc.O + (size_t)(y0 + row) * W + x0;
  // at R = 4 the object row values are held across the modes (188^2 x 4
  // modes: 27.9 -> 27.6 ms for the view update); at R = 8 holding them
  // costs a wave per SIMD and was slower
  constexpr bool kHoldO = R <= 4;
  float2 psn[R], ov[R];
  if (owner) {
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      psn[n1] = p0[Q * n1 + tl];
      if constexpr (kHoldO) ov[n1] = Or[Q * n1 + tl];
    }
  }
  for (int m = 0; m < M; ++m) {
    const int jm = j * M + m;
    float2 a[R] = {};
    if (owner) {
      const float2* __restrict__ Pm = sc.P + (size_t)m * FF + (size_t)row * F;
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) {
        const int v = Q * n1 + tl;
        const float2 phi = cmul(Pm[v], kHoldO ? ov[n1] : Or[v]);
        a[n1] = make_float2(2.f * phi.x - psn[n1].x, 2.f * phi.y - psn[n1].y);
      }
      if (m + 1 < M) {
        const float2* __restrict__ pq = p0 + (size_t)(m + 1) * FF;
#pragma unroll
        for (int n1 = 0; n1 < R; ++n1) psn[n1] = pq[Q * n1 + tl];
      }
    }
    __syncthreads();  // tables; the previous mode's reads of the lines are done
    if (owner) mix_first<F, -1>(a, line, twl, tl);
    __syncthreads();
    if (active) mix_uv<F>(line, tl);
    __syncthreads();
    if (active) {
      float2 lo[H], hi[H];
      mix_pairs<F, -1>(lo, hi, line, twq, tl);
      int ilo, ihi;
      mix_pair_pos<F>(tl, ilo, ihi);
      float2* __restrict__ Tr = sc.tspec + (size_t)jm * FF + (size_t)row * F;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        Tr[ilo + k] = lo[k];
        if (ihi >= 0) Tr[ihi + k] = hi[k];
      }
    }
  }
}

// Slot (view * nblk + column block) of block b when every column block of a
// view runs on one XCD: the dispatcher sends block b to XCD b % 8, so XCD x
// takes the views v = x, x + 8, ... whole, one after the other.  A row of an
// F = 188 or 200 frame is not a multiple of 128 bytes, so column strips of
// one view share cache lines across their edges; on one XCD those lines are
// fetched into its L2 once.  Bijective on whole groups of 8 views; the
// remaining blocks keep their index.
__device__ __forceinline__ int xcd_view_slot(int b, int n, int nblk) {
  const int full = (n / (8 * nblk)) * (8 * nblk);
  if (b >= full) return b;
  const int x = b & 7, i = b >> 3;
  return (8 * (i / nblk) + x) * nblk + i % nblk;
}

// (2) DFT along CB columns of every mode of one view, the mode sum, the
// modulus scale and the inverse DFT along the columns, in place in the
// spectrum buffer.  Thread (c, tl, m) with c fastest.  All LDS is dynamic,
// so the line buffers start at offset 0 and their 16-byte accesses are
// aligned: CB * M line buffers, the mode powers s [M][CB][F], the scale g
// [CB][F], then the twiddle tables (F + Q complex).
template <int F>
__global__ __launch_bounds__(1024) void k_mix_cols(const ScanDev* __restrict__ scans,
                                                   const int2* __restrict__ vmap,
                                                   const float2* __restrict__ tw, int M, int CB,
                                                   int direct) {
  using C = Mix<F>;
  constexpr int R = C::R, Q = C::Q, QT = C::QT, H = C::H, LS = C::LS, FF = F * F;
  extern __shared__ __align__(16) float2 dyn[];
  const int t = threadIdx.x;
  const int nblk = (F + CB - 1) / CB;
  const int slot = xcd_view_slot(blockIdx.x, gridDim.x, nblk);
  const int2 vm = vmap[slot / nblk];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const int col0 = (slot % nblk) * CB;
  const int c = t % CB;
  const int rest = t / CB;
  const int tl = rest % QT;
  const int m = rest / QT;
  const bool active = m < M && col0 + c < F;
  const int line_id = m * CB + c;
  float2* line = dyn + (size_t)line_id * LS;
  float* s = reinterpret_cast<float*>(dyn + (size_t)CB * M * LS);
  float* g = s + (size_t)M * CB * F;
  float2* twl = reinterpret_cast<float2*>(g + (size_t)CB * F);  // F even: 8-byte aligned
  float2* twq = twl + F;
  float2* __restrict__ Tm = sc.tspec + ((size_t)j * M + m) * FF + col0 + c;
  mix_load_tables<F>(tw, twl, twq, t, blockDim.x);
  float2 a[R] = {};
  if (active && tl < Q) {
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) a[n1] = Tm[(size_t)(Q * n1 + tl) * F];
  }
  __syncthreads();
  if (active && tl < Q) mix_first<F, -1>(a, line, twl, tl);
  __syncthreads();
  if (active) mix_uv<F>(line, tl);
  __syncthreads();
  float2 lo[H], hi[H];
  int ilo, ihi;
  mix_pair_pos<F>(tl, ilo, ihi);
  if (active) {
    mix_pairs<F, -1>(lo, hi, line, twq, tl);  // spectrum at rows ilo + k, ihi + k
    float* sl = s + (size_t)line_id * F;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      sl[ilo + k] = cabs2(lo[k]);
      if (ihi >= 0) sl[ihi + k] = cabs2(hi[k]);
    }
  }
  __syncthreads();
  // one thread per pixel of the block's columns: sum over modes, scale
  // sqrt(I / S) / F^2 (0 where S vanishes), or beta times that less 1/F^2
  // for the update without psi; pixels in column-major order
  const float* __restrict__ Ij = sc.I + (size_t)j * FF + col0;
  const float inv_ff = 1.0f / (float)FF;
  const float beta = sc.beta;
  for (int p = t; p < CB * F; p += blockDim.x) {
    const int cc = p / F, kk = p - cc * F;
    if (col0 + cc >= F) continue;
    float sum = 0.f;
    for (int mm = 0; mm < M; ++mm) sum += s[(size_t)(mm * CB + cc) * F + kk];
    const float iv = fmaxf(Ij[(size_t)kk * F + cc], 0.f);
    const float gg = (sum > FLT_MIN) ? sqrtf(iv / sum) * inv_ff : 0.f;
    g[cc * F + kk] = direct ? beta * gg - inv_ff : gg;
  }
  __syncthreads();
  if (active) {
    const float* gl = g + c * F;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      lo[k] = cscale(lo[k], gl[ilo + k]);
      if (ihi >= 0) hi[k] = cscale(hi[k], gl[ihi + k]);
    }
    // the forward reads of this line ended before the barriers above
    mix_put_pairs<F>(line, lo, hi, tl);
  }
  __syncthreads();
  mix_inverse<F>(a, line, twl, twq, tl, active);
  if (active && tl < Q) {
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) Tm[(size_t)(Q * n1 + tl) * F] = a[n1];
  }
}

// (3) inverse DFT along rows, psi' = psi + beta (Z' - P O), the view's
// object numerator sum_m conj(P_m) psi'_m and the eps_psi partial sums; all
// modes of RB rows per block.  The line buffers alternate between modes, so
// a mode's spectrum rows go from global memory straight into the buffer the
// previous mode did not use (its last readers passed the barriers of that
// mode).  DIRECT: the column kernel scaled the spectra by beta g - 1/F^2, the
// inverse is beta Z' - Z, and psi' = (2 - beta) P O + that (Eq. 3 with
// psi = 2 P O - Z): psi is not read and the eps_psi partials are zero.
template <int F, bool DIRECT>
__device__ __forceinline__ void mix_rows_inv(const ScanDev* __restrict__ scans,
                                             const int2* __restrict__ vmap,
                                             const float2* __restrict__ tw, int M) {
  using C = Mix<F>;
  constexpr int R = C::R, Q = C::Q, QT = C::QT, RB = C::RB, LS = C::LS, NT = C::NT, FF = F * F;
  __shared__ __align__(16) float2 xb[2 * RB * LS];
  __shared__ float2 twl[F];
  __shared__ float2 twq[Q];
  __shared__ float red[2 * (NT / 64)];
  const int t = threadIdx.x;
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const int rl = t / QT, tl = t % QT;
  const int row = blockIdx.y * RB + rl;
  const bool active = rl < RB && row < F;
  const bool owner = active && tl < Q;  // holds pixels Q n1 + tl of the row
  const int W = uni(sc.W);
  const float beta = sc.beta;
  const int y0 = uni(kidx(sc.pos)[2 * j]), x0 = uni(kidx(sc.pos)[2 * j + 1]);
  const float2* __restrict__ Or = sc.O + (size_t)(y0 + row) * W + x0;
  mix_load_tables<F>(tw, twl, twq, t, NT);
  float2 oacc[R];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) oacc[n1] = make_float2(0.f, 0.f);
  float e_d = 0.f, e_n = 0.f;
  for (int m = 0; m < M; ++m) {
    const size_t base = ((size_t)j * M + m) * FF + (size_t)row * F;
    float2* line = xb + (m & 1) * (RB * LS) + rl * LS;
    if (owner) {
      const float4* __restrict__ Tr = reinterpret_cast<const float4*>(sc.tspec + base + R * tl);
      float4* d = reinterpret_cast<float4*>(line + R * tl);
#pragma unroll
      for (int h = 0; h < R / 2; ++h) d[h] = Tr[h];
    }
    // the update's operands go out before the transform
    float2* __restrict__ pm = sc.psi + base;
    float2 pr[R], ov[R], pv[R];
    if (owner) {
      const float2* __restrict__ Pm = sc.P + (size_t)m * FF + (size_t)row * F;
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) {
        const int v = Q * n1 + tl;
        pr[n1] = Pm[v];
        ov[n1] = Or[v];
        if constexpr (!DIRECT) pv[n1] = pm[v];
      }
    }
    __syncthreads();  // the rows (and, in the first mode, the tables)
    float2 a[R] = {};
    mix_inverse<F>(a, line, twl, twq, tl, active);  // a[n1] = Z' at column Q n1 + tl
    if (owner) {
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) {
        const float2 phi = cmul(pr[n1], ov[n1]);
        float2 pn;
        if constexpr (DIRECT) {
          pn = make_float2((2.f - beta) * phi.x + a[n1].x, (2.f - beta) * phi.y + a[n1].y);
        } else {
          const float2 d = make_float2(beta * (a[n1].x - phi.x), beta * (a[n1].y - phi.y));
          pn = cadd(pv[n1], d);
          e_d += cabs2(d);
        }
        pm[Q * n1 + tl] = pn;
        e_n += cabs2(pn);
        oacc[n1] = cadd(oacc[n1], cmulc(pr[n1], pn));
      }
    }
  }
  if (owner) {
    float2* __restrict__ oj = sc.opart + (size_t)j * FF + (size_t)row * F;
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) oj[Q * n1 + tl] = oacc[n1];
  }
  block_sum2<NT>(e_d, e_n, red);
  if (t == 0) {
    const int part = j * gridDim.y + blockIdx.y;
    sc.err_psi[2 * part] = e_d;
    sc.err_psi[2 * part + 1] = e_n;
  }
}

template <int F>
__global__ __launch_bounds__(Mix<F>::NT) void k_mix_rows_inv(const ScanDev* __restrict__ scans,
                                                             const int2* __restrict__ vmap,
                                                             const float2* __restrict__ tw,
                                                             int M) {
  mix_rows_inv<F, false>(scans, vmap, tw, M);
}

template <int F>
__global__ __launch_bounds__(Mix<F>::NT) void k_mix_rows_inv_direct(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap,
    const float2* __restrict__ tw, int M) {
  mix_rows_inv<F, true>(scans, vmap, tw, M);
}

}  // namespace dmk
