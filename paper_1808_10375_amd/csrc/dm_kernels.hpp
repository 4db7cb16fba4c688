// dm_kernels.hpp -- gfx950 kernels of one multi-mode difference-map iteration
// (Section II of arXiv:1808.10375: Eq. 3 view update with the constrained
// transform F_c, Eq. 5 object update, Eq. 4 probe update, Eq. 6 errors).
//
// Layouts: psi [N][M][F][F], P [M][F][F], O [H][W] (complex64 as float2),
// I [N][F][F] float, pos [N][2] int (y, x top-left).
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "dm_fft.hpp"

namespace dmk {

// Device copy of the public dm_errors record (same size and field order).
struct DevErrors {
  int32_t iter;
  float eps_psi, eps_obj, eps_probe;
  float eps_mode[16];
};

constexpr int kRing = 4096;

// Device-side description of one scan of a batch: its buffers in the
// workspace and its sizes.  Kernels look a scan up once per workgroup.
struct ScanDev {
  float2* psi;            // [N][M][F][F]
  const float* I;         // [N][F][F] (caller's)
  float2* P;              // [M][F][F]
  float2* O;              // [L][H][W] (L object modes; 1 on every path but
                          // the three-kernel one)
  const int* pos;         // [N][2]
  const int* order;       // [N] views in spatial order
  float2* opart;          // [N][L][F][F] per-view object numerators
  float* gscr;            // [N][F][F] per-view modulus scale (fused path)
  float2* tspec;          // [N][L M][F][F] spectrum buffer (three-kernel path)
  float* D;               // [F][F] mode power
  float2* num_part;       // [Cmax][M][F][F]
  float* den_part;        // [Cmax][F][F]
  float* err_psi;         // [n_psi_parts][2]
  float* err_obj;         // [ntiles_max][2]
  float* err_probe;       // [n_pblk][M][2]
  const int* tile_ptr;    // [ntiles + 1]
  const int* tile_views;  // [nnz]
  int* counter;           // iteration counter of this scan
  DevErrors* ring;        // [kRing]
  int N, H, W, tiles_x, ntiles, C, chunk, n_psi_parts;
  float beta;
  int L;                  // object modes; views hold the pairs (k, l) of
                          // Eqs. 1-5 at mode index l * M + k
};

// ---------------------------------------------------------------------------
// block reduction of two floats (fixed order: lanes, then waves in order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int NT>
__device__ __forceinline__ void block_sum2(float& a, float& b, float* red) {
  constexpr int NW = (NT + 63) / 64;
  if constexpr (NT < 64) {
    // fewer lanes than a wave: plain LDS sum in thread order
    __shared__ float tmp[2 * 64];
    __syncthreads();
    tmp[2 * threadIdx.x] = a;
    tmp[2 * threadIdx.x + 1] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
      float sa = 0.f, sb = 0.f;
      for (int i = 0; i < NT; ++i) { sa += tmp[2 * i]; sb += tmp[2 * i + 1]; }
      a = sa; b = sb;
    }
    return;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float sa = 0.f, sb = 0.f;
    for (int i = 0; i < NW; ++i) { sa += red[2 * i]; sb += red[2 * i + 1]; }
    a = sa; b = sb;
  }
}

// runtime block size version
__device__ __forceinline__ void block_sum2_rt(float& a, float& b, float* red) {
  const int nw = (blockDim.x + 63) >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float sa = 0.f, sb = 0.f;
    for (int i = 0; i < nw; ++i) { sa += red[2 * i]; sb += red[2 * i + 1]; }
    a = sa; b = sb;
  }
}

// ---------------------------------------------------------------------------
// 2-D transform of one F x F frame held by F*F/16 "virtual threads" of 16
// values each; a real thread runs V of them (virtual thread t + v*NT, NT =
// F*F/(16 V)), so every LDS exchange moves all V between one pair of barriers.
// Virtual thread vt = g*F + c.  Spatial layout: a[u1] = x[B*u1 + g][c].
// Spectral layout:  a[i*B + l2] = X[c][(g + B*i) + 16*l2].
// buf: LDS, F rows of LD = F + 1 float2 (one padding column).
// ---------------------------------------------------------------------------
template <int F, int DIR, int V = 1>
struct Frame2D {
  static constexpr int B = F / 16;
  static constexpr int NI = 16 / B;  // k1 values per thread after the exchange
  static constexpr int LD = F + 1;
  static constexpr int GS = B / V;   // g step between a thread's virtual threads

  // forward: spatial -> spectral; g is the first virtual thread's row group
  __device__ __forceinline__ static void fwd(float2 (&a)[V][16], float2* buf,
                                             const float2* __restrict__ tw, int c, int g0) {
    static_assert(DIR < 0, "fwd is the forward transform");
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int g = g0 + v * GS;
      dft16<-1>(a[v]);
      if constexpr (B > 1) {
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) a[v][k1] = twiddle<-1>(tw, g * k1, a[v][k1]);
      }
      if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (B > 1) {
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) buf[(k1 * B + g0 + v * GS) * LD + c] = a[v][k1];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int q = 0; q < B; ++q) a[v][i * B + q] = buf[((g + B * i) * B + q) * LD + c];
#pragma unroll
        for (int i = 0; i < NI; ++i) dftB<-1, B>(&a[v][i * B]);
        if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
    // transpose to rows: Xc[(g + B i) + 16 k2][c] -> row c of the buffer
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int g = g0 + v * GS;
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) buf[((g + B * i) + 16 * k2) * LD + c] = a[v][i * B + k2];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int g = g0 + v * GS;
#pragma unroll
      for (int v1 = 0; v1 < 16; ++v1) a[v][v1] = buf[c * LD + B * v1 + g];
      // rows: 16-point over v1
      dft16<-1>(a[v]);
      if constexpr (B > 1) {
#pragma unroll
        for (int l1 = 1; l1 < 16; ++l1) a[v][l1] = twiddle<-1>(tw, g * l1, a[v][l1]);
      }
      if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (B > 1) {
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int l1 = 0; l1 < 16; ++l1) buf[c * LD + l1 * B + g0 + v * GS] = a[v][l1];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int q = 0; q < B; ++q) a[v][i * B + q] = buf[c * LD + (g + B * i) * B + q];
#pragma unroll
        for (int i = 0; i < NI; ++i) dftB<-1, B>(&a[v][i * B]);
        if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // inverse (unnormalised): spectral -> spatial, exact mirror of fwd
  __device__ __forceinline__ static void inv(float2 (&a)[V][16], float2* buf,
                                             const float2* __restrict__ tw, int c, int g0) {
    static_assert(DIR > 0, "inv is the inverse transform");
    if constexpr (B > 1) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
#pragma unroll
        for (int i = 0; i < NI; ++i) dftB<1, B>(&a[v][i * B]);
        if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int q = 0; q < B; ++q) buf[c * LD + (g + B * i) * B + q] = a[v][i * B + q];
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int l1 = 0; l1 < 16; ++l1) a[v][l1] = buf[c * LD + l1 * B + g];
#pragma unroll
        for (int l1 = 1; l1 < 16; ++l1) a[v][l1] = twiddle<1>(tw, g * l1, a[v][l1]);
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      dft16<1>(a[v]);
      if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int v1 = 0; v1 < 16; ++v1) buf[c * LD + B * v1 + g0 + v * GS] = a[v][v1];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int g = g0 + v * GS;
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) a[v][i * B + k2] = buf[((g + B * i) + 16 * k2) * LD + c];
    }
    if constexpr (B > 1) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
#pragma unroll
        for (int i = 0; i < NI; ++i) dftB<1, B>(&a[v][i * B]);
        if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int q = 0; q < B; ++q) buf[((g + B * i) * B + q) * LD + c] = a[v][i * B + q];
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) a[v][k1] = buf[(k1 * B + g) * LD + c];
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) a[v][k1] = twiddle<1>(tw, g * k1, a[v][k1]);
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      dft16<1>(a[v]);
      if constexpr (V > 1) __builtin_amdgcn_sched_barrier(0);
    }
  }
};

// ---------------------------------------------------------------------------
// Fused view update for F <= 128 (Eq. 3 with F_c): one workgroup per view.
//   pass 1: for every mode, Z = 2 P O - psi, 2-D DFT, accumulate the mode sum
//           S = sum_k |Z~_k|^2 in registers (every thread owns the same
//           spectral pixels for every mode);
//   scale:  g = sqrt(I / S) / F^2 (0 where S == 0) for the thread's pixels,
//           parked in a per-view scratch in thread-major order (coalesced,
//           private to this workgroup, re-read from L2 once per mode);
//   pass 2: modes in reverse order (the last one's spectrum is still in
//           registers; the others are recomputed), Z~ * g, inverse DFT -> Z',
//           psi' = psi + beta (Z' - P O), with psi held in registers (F < 128)
//           or read once more (F = 128, whose register budget is spent).  The object numerator of
//           the view, sum_k conj(P_k) psi'_k, accumulates in registers and is
//           written once; so are the two partial sums of eps_psi.
// Workgroup b takes view order[slot(b)]: consecutive workgroups go to
// different XCDs, so each XCD walks its own spatially compact run of views
// and keeps its part of the object in its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_slot(int b, int nblocks) {
  // b -> (b % 8) * ceil(n / 8) + b / 8, clamped for the ragged last group
  const int per = (nblocks + 7) >> 3;
  const int x = b & 7, k = b >> 3;
  const int full = nblocks - (per - 1) * 8;  // XCD groups that get `per` items
  return (x < full) ? x * per + k : full * per + (x - full) * (per - 1) + k;
}

// Workgroup b runs on XCD b mod 8.  Map the blocks so that each XCD takes
// runs of four consecutive tiles: a view's numerator rows rarely start on a
// cache-line boundary, so neighbouring tiles share lines, which then come
// from the same L2.  Blocks past the last multiple of 32 map to themselves.
__device__ __forceinline__ int xcd_group_slot(int b, int n) {
  const int full = n & ~31;
  if (b >= full) return b;
  const int x = b & 7, k = b >> 3;
  return ((k >> 2) * 8 + x) * 4 + (k & 3);
}

// One view's intensities I (F x F floats) into LDS rows padded to F + 1,
// for NT threads: each thread's loads (up to 16 at a time) are issued before
// any of them is written, so a view waits on one memory latency instead of
// one per element; the barrier that frees the LDS the rows alias waits
// while the first loads are in flight.
template <int F, int NT>
__device__ __forceinline__ void stage_padded_rows(float* bI, const float* Ij, int t) {
  constexpr int FF = F * F, K = FF / NT, KB = K < 16 ? K : 16;
  static_assert(FF % NT == 0 && K % KB == 0, "whole batches per thread");
  const rsrc_t r = make_rsrc(Ij, (uint32_t)(FF * 4));
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += KB) {
    float v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) v[k] = bload1(r, t * 4, (k0 + k) * NT * 4);
    if (k0 == 0) __syncthreads();
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int e = t + (k0 + k) * NT;
      bI[(e / F) * (F + 1) + (e % F)] = v[k];
    }
  }
  __syncthreads();
}

template <int F, int V>
__global__ __launch_bounds__(F * F / (16 * V)) void k_fourier_fused(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap, int total,
    const float2* __restrict__ tw, int M) {
  constexpr int B = F / 16;
  constexpr int NT = F * B / V;  // threads; each runs V virtual threads
  constexpr int GS = B / V;      // row-group step between a thread's virtual threads
  constexpr int LD = F + 1;
  constexpr int FF = F * F;
  __shared__ float2 buf[F * LD];
  __shared__ float red[2 * ((NT + 63) / 64)];
  __shared__ float2 twl[F];  // twiddles read from LDS, not held in SGPRs

  const int t = threadIdx.x;
  for (int i = t; i < F; i += NT) twl[i] = tw[i];
  __syncthreads();  // the twiddles are read by every wave
  const int2 vm = vmap[xcd_slot(blockIdx.x, total)];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  float2* __restrict__ psi = sc.psi;
  const float* __restrict__ I = sc.I;
  const float2* __restrict__ P = sc.P;
  const float2* __restrict__ O = sc.O;
  const kidx_t pos = kidx(sc.pos);
  float2* __restrict__ opart = sc.opart;
  float* __restrict__ gscr = sc.gscr;
  float* __restrict__ err_psi = sc.err_psi;
  const int H = uni(sc.H), W = uni(sc.W);
  const float beta = sc.beta;
  const int c = t % F;
  const int g0 = wave_uniform_div<F>(t);
  const int y0 = uni(pos[2 * j]), x0 = uni(pos[2 * j + 1]);
  // buffers: this view's modes, the probe, the object, this view's scale
  const rsrc_t rpsi = make_rsrc(psi + (size_t)j * M * FF, (uint32_t)(M * FF * 8));
  const rsrc_t rP = make_rsrc(P, (uint32_t)(M * FF * 8));
  const rsrc_t rO = make_rsrc(O, (uint32_t)((size_t)H * W * 8));
  const rsrc_t rg = make_rsrc(gscr + (size_t)j * FF, (uint32_t)(FF * 4));
  // per-lane byte offsets of the first virtual thread (row g0, column c);
  // the other virtual threads and rows differ by wave-uniform offsets
  const int vF = (g0 * F + c) * 8;
  const int vO = (g0 * W + c) * 8;
  const int sO = (y0 * W + x0) * 8;
  const int vG = t * 4;
  // byte offset of row B*u1 + v*GS relative to the first virtual thread's row
  auto rowF = [&](int v, int u1) { return (B * u1 + v * GS) * F * 8; };
  auto rowO = [&](int v, int u1) { return (B * u1 + v * GS) * W * 8; };

  // The view is held in registers through both transforms when they fit
  // (F < 128 with one virtual thread, or F = 128 with two virtual threads per
  // 256-VGPR thread); otherwise it is read once more in the epilogue.
  constexpr bool kHold = (F < 128);
  float2 a[V][16];
  float2 hold[kHold ? V : 1][kHold ? 16 : 1];
  {
    float S[V][16];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < 16; ++r) S[v][r] = 0.f;

    // ---- pass 1: mode sum of |DFT(2 phi - psi)|^2
    for (int m = 0; m < M; ++m) {
      const int sm = m * FF * 8;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u1 = 0; u1 < 16; ++u1) {
          const float2 ps = bload2(rpsi, vF, sm + rowF(v, u1));
          const float2 phi =
              cmul(bload2(rP, vF, sm + rowF(v, u1)), bload2(rO, vO, sO + rowO(v, u1)));
          a[v][u1] = make_float2(2.f * phi.x - ps.x, 2.f * phi.y - ps.y);
          if constexpr (kHold) hold[kHold ? v : 0][kHold ? u1 : 0] = ps;
          if ((u1 & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
      Frame2D<F, -1, V>::fwd(a, buf, twl, c, g0);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int r = 0; r < 16; ++r) S[v][r] += cabs2(a[v][r]);
    }

    // ---- modulus scale: stage I through LDS (padded rows), form g, park it
    float* bI = reinterpret_cast<float*>(buf);
    stage_padded_rows<F, NT>(bI, I + (size_t)j * FF, t);
    const float inv_ff = 1.0f / (float)FF;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int g = g0 + v * GS;
#pragma unroll
      for (int i = 0; i < 16 / B; ++i)
#pragma unroll
        for (int l2 = 0; l2 < B; ++l2) {
          const int r = i * B + l2;
          const int l = (g + B * i) + 16 * l2;
          const float iv = fmaxf(bI[c * (F + 1) + l], 0.f);
          const float sv = S[v][r];
          S[v][r] = (sv > FLT_MIN) ? sqrtf(iv / sv) * inv_ff : 0.f;
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(S[v][r]), rg, vG,
                                              (v * 16 + r) * NT * 4, 0);
  }

  // ---- pass 2: projected spectra back to views, modes in reverse order
  float2 oacc[V][16];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int r = 0; r < 16; ++r) oacc[v][r] = make_float2(0.f, 0.f);
  float e_d = 0.f, e_n = 0.f;

  for (int m = M - 1; m >= 0; --m) {
    const int sm = m * FF * 8;
    if (m != M - 1) {
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int u1 = 0; u1 < 16; ++u1) {
          const float2 ps = bload2(rpsi, vF, sm + rowF(v, u1));
          const float2 phi =
              cmul(bload2(rP, vF, sm + rowF(v, u1)), bload2(rO, vO, sO + rowO(v, u1)));
          a[v][u1] = make_float2(2.f * phi.x - ps.x, 2.f * phi.y - ps.y);
          if constexpr (kHold) hold[kHold ? v : 0][kHold ? u1 : 0] = ps;
          if ((u1 & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
      Frame2D<F, -1, V>::fwd(a, buf, twl, c, g0);
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        a[v][r] = cscale(a[v][r], bload1(rg, vG, (v * 16 + r) * NT * 4));
    Frame2D<F, 1, V>::inv(a, buf, twl, c, g0);
    // the psi' stores may alias later loads as far as the compiler knows:
    // each batch issues its loads before any of its stores
    constexpr int KB = 4;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int b = 0; b < 16; b += KB) {
        float2 pr[KB], ov[KB], pv[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          pr[k] = bload2(rP, vF, sm + rowF(v, b + k));
          ov[k] = bload2(rO, vO, sO + rowO(v, b + k));
          pv[k] = kHold ? hold[kHold ? v : 0][kHold ? b + k : 0]
                        : bload2(rpsi, vF, sm + rowF(v, b + k));
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int u1 = b + k;
          const float2 phi = cmul(pr[k], ov[k]);
          const float2 d =
              make_float2(beta * (a[v][u1].x - phi.x), beta * (a[v][u1].y - phi.y));
          const float2 pn = cadd(pv[k], d);
          bstore2(rpsi, pn, vF, sm + rowF(v, u1));
          e_d += cabs2(d);
          e_n += cabs2(pn);
          oacc[v][u1] = cadd(oacc[v][u1], cmulc(pr[k], pn));
        }
      }
  }

  const rsrc_t ropart = make_rsrc(opart + (size_t)j * FF, (uint32_t)(FF * 8));
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int u1 = 0; u1 < 16; ++u1) bstore2(ropart, oacc[v][u1], vF, rowF(v, u1));

  block_sum2<NT>(e_d, e_n, red);
  if (t == 0) {
    err_psi[2 * j] = e_d;
    err_psi[2 * j + 1] = e_n;
  }
}

// ---------------------------------------------------------------------------
// Streamed view update (F <= 128): a persistent grid of one workgroup per
// compute unit; workgroup b owns a slot of scratch (the spectra of every
// mode of the view in hand, thread-major so each thread reads back exactly
// what it wrote) and walks views b, b + G, ... of the XCD-interleaved order.
//   pass 1  per mode: Z = 2 P O - psi, forward DFT, mode sum S += |Z~|^2,
//           Z~ -> scratch
//   scale   g = sqrt(I / S) / F^2 (definition of F_c)
//   pass 2  per mode, last mode first (in the merged form with V = 1 the
//           last spectrum never leaves the registers): Z~ from scratch,
//           times g, inverse DFT; with MERGE the view update
//           psi' = psi + beta (Z' - P O) (Eq. 3) and the object numerator
//           sum_k conj(P_k) psi'_k follow at once, otherwise Z' goes back to
//           scratch and
//   pass 3  per mode: Z' from scratch, the view update and the numerator
//           (no transform runs while the numerator is live)
// Every mode is transformed twice (no recomputation); psi is written once
// and read once or twice, with the non-temporal hint (NT) so the probe and
// the object stay in L2 (the merged form with the eps_psi partials reads
// psi through the caches in pass 1 and streams the slot instead).
// The merged form without PSI_ERR never reads psi in pass 2: since
// psi = 2 P O - Z and the transforms are linear,
//   psi' = psi + beta (Z' - P O) = (2 - beta) P O + F^-1[(beta g - 1/F^2) Z~]
// (the unnormalised inverse of the spectrum scaled by beta g - 1/F^2 is
// beta Z' - Z), so one inverse transform gives psi' directly.  What it
// cannot give is psi' - psi, so the eps_psi partial sums are left at zero;
// with PSI_ERR the update reads psi again and forms them.
// A thread runs V virtual threads of the transform (F*F/(16 V) threads).
// With V = 1 (128 registers a thread) the merged form parks the scale to
// make room for the numerator: the rows that fit beside the exchange buffer
// in LDS, the rest in the slot; with V = 2 (256 registers) the scale and the
// numerator both stay in registers.
// ---------------------------------------------------------------------------
template <int F, int V, bool NT_HINT, bool MERGE, bool PSI_ERR = true>
__global__ __launch_bounds__(F * F / (16 * V)) void k_fourier_stream(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap, int total,
    const float2* __restrict__ tw, int M, float2* __restrict__ vscr) {
  constexpr int B = F / 16;
  constexpr int NT = F * B / V;  // threads
  constexpr int GS = B / V;      // row-group step between a thread's virtual threads
  constexpr int LD = F + 1;
  constexpr int FF = F * F;
  constexpr bool kPark = MERGE && V == 1;
  constexpr bool kDirect = MERGE && !PSI_ERR;  // psi' without reading psi
  constexpr bool kKeep = kPark;  // keeps the last spectrum in registers
  // scale rows parked in LDS: as many as fit in 160 KB beside the rest
  constexpr int kLdsFixed = F * LD * 8 + 2 * ((NT + 63) / 64) * 4 + 256;
  constexpr int kLdsRows = !kPark ? 0
                           : ((163840 - kLdsFixed) / (NT * 4) < 16 ? (163840 - kLdsFixed) / (NT * 4)
                                                                   : 16);
  __shared__ float2 buf[F * LD];
  __shared__ float red[2 * ((NT + 63) / 64)];
  __shared__ float gl[kLdsRows > 0 ? kLdsRows * NT : 1];

  // twiddles come straight from the global table: their index is
  // wave-uniform for F >= 64, so they are scalar loads
  const int t = threadIdx.x;
  const int c = t % F;
  const int g0 = wave_uniform_div<F>(t);
  // slot: the spectra [M][V][16][NT] complex, then the modulus scale [16][NT]
  const size_t slot_words = (size_t)M * FF * 2 + FF;
  float* const slot = reinterpret_cast<float*>(vscr) + (size_t)blockIdx.x * slot_words;
  const rsrc_t rs = make_rsrc(slot, (uint32_t)(slot_words * 4));
  const int sG = M * FF * 8;  // byte offset of the scale in the slot
  const int vS = t * 8;
  auto rowS = [&](int m, int v, int r) { return ((m * V + v) * 16 + r) * NT * 8; };

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int2 vm = vmap[xcd_slot(item, total)];
    const ScanDev& sc = scans[vm.x];
    const int j = uni(vm.y);
    const int H = uni(sc.H), W = uni(sc.W);
    const float beta = sc.beta;
    const int y0 = uni(kidx(sc.pos)[2 * j]), x0 = uni(kidx(sc.pos)[2 * j + 1]);
    const rsrc_t rpsi = make_rsrc(sc.psi + (size_t)j * M * FF, (uint32_t)(M * FF * 8));
    const rsrc_t rP = make_rsrc(sc.P, (uint32_t)(M * FF * 8));
    const rsrc_t rO = make_rsrc(sc.O, (uint32_t)((size_t)H * W * 8));
    // per-lane offsets of the first virtual thread (row g0, column c); rows
    // of the other virtual threads differ by wave-uniform offsets
    const int vF = (g0 * F + c) * 8;
    const int vO = (g0 * W + c) * 8;
    const int sO = (y0 * W + x0) * 8;
    auto rowF = [&](int v, int u1) { return (B * u1 + v * GS) * F * 8; };
    auto rowO = [&](int v, int u1) { return (B * u1 + v * GS) * W * 8; };
    auto ld_psi = [&](int off) { return NT_HINT ? bload2_nt(rpsi, vF, off) : bload2(rpsi, vF, off); };
    // merged form with the eps_psi partials (the update re-reads psi right
    // after each inverse transform): pass 1 reads psi through the caches,
    // so that the re-read often hits in the memory-side cache, and the
    // slot's spectra are streamed with the hint instead (measured: 2.07 ms
    // against 2.22 ms at 2500 x 5 x 128^2; the other forms were slower so)
    constexpr bool kReRead = NT_HINT && MERGE && PSI_ERR;
    auto ld_psi1 = [&](int off) {
      return (NT_HINT && !kReRead) ? bload2_nt(rpsi, vF, off) : bload2(rpsi, vF, off);
    };
    auto st_slot = [&](float2 x, int off) {
      if (kReRead) bstore2_nt(rs, x, vS, off);
      else bstore2(rs, x, vS, off);
    };
    auto ld_slot = [&](int off) { return kReRead ? bload2_nt(rs, vS, off) : bload2(rs, vS, off); };

    float2 a[V][16];
    float S[V][16];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < 16; ++r) S[v][r] = 0.f;
    // ---- pass 1: all of the mode's psi first, into the transform registers
    // (one memory latency per mode instead of two: 1.95 -> 1.88 ms at 2500 x
    // 5 x 128^2), then the cached probe and object in two batches
    for (int m = 0; m < M; ++m) {
      const int sm = m * FF * 8;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int r = 0; r < 16; ++r) a[v][r] = ld_psi1(sm + rowF(v, r));
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int b = 0; b < 16; b += 8) {
          float2 pp[8], oo[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            pp[k] = bload2(rP, vF, sm + rowF(v, b + k));
            oo[k] = bload2(rO, vO, sO + rowO(v, b + k));
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const float2 phi = cmul(pp[k], oo[k]);
            a[v][b + k] = make_float2(2.f * phi.x - a[v][b + k].x, 2.f * phi.y - a[v][b + k].y);
          }
        }
      Frame2D<F, -1, V>::fwd(a, buf, tw, c, g0);
      // merged form: the last mode's spectrum stays in registers for pass 2
      const bool keep = kKeep && (m == M - 1);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          S[v][r] += cabs2(a[v][r]);
          if (!keep) st_slot(a[v][r], rowS(m, v, r));
        }
    }
    // ---- modulus scale from I staged through LDS (padded rows)
    {
      float* bI = reinterpret_cast<float*>(buf);
      stage_padded_rows<F, NT>(bI, sc.I + (size_t)j * FF, t);
      const float inv_ff = 1.0f / (float)FF;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int g = g0 + v * GS;
#pragma unroll
        for (int i = 0; i < 16 / B; ++i)
#pragma unroll
          for (int l2 = 0; l2 < B; ++l2) {
            const int r = i * B + l2;
            const int l = (g + B * i) + 16 * l2;
            const float iv = fmaxf(bI[c * (F + 1) + l], 0.f);
            const float sv = S[v][r];
            // hardware reciprocal and square root (1 ulp each) instead of the
            // correctly rounded division and root: branch-free, and the
            // scale is within 3 ulp of sqrt(I / S) / F^2
            const float q = iv * __builtin_amdgcn_rcpf(fmaxf(sv, FLT_MIN));
            const float g = (sv > FLT_MIN) ? __builtin_amdgcn_sqrtf(q) * inv_ff : 0.f;
            S[v][r] = kDirect ? beta * g - inv_ff : g;
          }
      }
      __syncthreads();  // bI aliases the exchange buffer
    }
    float2 oacc[V][16];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < 16; ++r) oacc[v][r] = make_float2(0.f, 0.f);
    float e_d = 0.f, e_n = 0.f;
    // The stores of psi' may alias later loads as far as the compiler knows,
    // so no load is moved above a store: every batch issues all of its loads
    // first, then computes and stores.
    constexpr int KB = 4;  // elements per batch
    // view update of mode m from Z' (zp(v, u) gives element u of virtual thread v)
    auto update = [&](int m, auto zp_of) {
      const int sm = m * FF * 8;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int b = 0; b < 16; b += KB) {
          float2 zp[KB], pr[KB], ov[KB], ps[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            zp[k] = zp_of(v, b + k);
            pr[k] = bload2(rP, vF, sm + rowF(v, b + k));
            ov[k] = bload2(rO, vO, sO + rowO(v, b + k));
            ps[k] = ld_psi(sm + rowF(v, b + k));
          }
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            const float2 phi = cmul(pr[k], ov[k]);
            const float2 d = make_float2(beta * (zp[k].x - phi.x), beta * (zp[k].y - phi.y));
            const float2 pn = cadd(ps[k], d);
            if (NT_HINT) bstore2_nt(rpsi, pn, vF, sm + rowF(v, b + k));
            else bstore2(rpsi, pn, vF, sm + rowF(v, b + k));
            e_d += cabs2(d);
            e_n += cabs2(pn);
            oacc[v][b + k] = cadd(oacc[v][b + k], cmulc(pr[k], pn));
          }
        }
    };
    // psi' = (2 - beta) P O + W of mode m from W = beta Z' - Z (wp(v, u))
    auto update_direct = [&](int m, auto wp_of) {
      const int sm = m * FF * 8;
      const float c2 = 2.f - beta;
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int b = 0; b < 16; b += KB) {
          float2 pr[KB], ov[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            pr[k] = bload2(rP, vF, sm + rowF(v, b + k));
            ov[k] = bload2(rO, vO, sO + rowO(v, b + k));
          }
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            const float2 phi = cmul(pr[k], ov[k]);
            const float2 w = wp_of(v, b + k);
            const float2 pn = make_float2(c2 * phi.x + w.x, c2 * phi.y + w.y);
            if (NT_HINT) bstore2_nt(rpsi, pn, vF, sm + rowF(v, b + k));
            else bstore2(rpsi, pn, vF, sm + rowF(v, b + k));
            e_n += cabs2(pn);
            oacc[v][b + k] = cadd(oacc[v][b + k], cmulc(pr[k], pn));
          }
        }
    };
    // ---- pass 2: scaled spectra back to the spatial domain
    if constexpr (kPark) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r < kLdsRows) gl[r * NT + t] = S[0][r];
        else
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(S[0][r]), rs, t * 4,
                                                sG + r * NT * 4, 0);
      }
    }
    for (int m = M - 1; m >= 0; --m) {
      if (!kKeep || m != M - 1) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int r = 0; r < 16; ++r) a[v][r] = ld_slot(rowS(m, v, r));
      }
      if constexpr (kPark) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          a[0][r] = cscale(a[0][r], r < kLdsRows ? gl[r * NT + t]
                                                 : bload1(rs, t * 4, sG + r * NT * 4));
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int r = 0; r < 16; ++r) a[v][r] = cscale(a[v][r], S[v][r]);
      }
      Frame2D<F, 1, V>::inv(a, buf, tw, c, g0);
      if constexpr (kDirect) {
        update_direct(m, [&](int v, int u) { return a[v][u]; });
      } else if constexpr (MERGE) {
        update(m, [&](int v, int u) { return a[v][u]; });
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int r = 0; r < 16; ++r) st_slot(a[v][r], rowS(m, v, r));
      }
    }
    // ---- pass 3: view update and the object numerator
    if constexpr (!MERGE) {
      for (int m = 0; m < M; ++m)
        update(m, [&](int v, int u) { return ld_slot(rowS(m, v, u)); });
    }
    const rsrc_t ropart = make_rsrc(sc.opart + (size_t)j * FF, (uint32_t)(FF * 8));
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int u1 = 0; u1 < 16; ++u1) {
        if (NT_HINT) bstore2_nt(ropart, oacc[v][u1], vF, rowF(v, u1));
        else bstore2(ropart, oacc[v][u1], vF, rowF(v, u1));
      }
    block_sum2<NT>(e_d, e_n, red);
    if (t == 0) {
      sc.err_psi[2 * j] = e_d;
      sc.err_psi[2 * j + 1] = e_n;
    }
    __syncthreads();  // red and buf are reused by the next view
  }
}

// ---------------------------------------------------------------------------
// Multi-pass view update (any F = 16 B, used for F = 256): three kernels
// around a spectrum buffer T [N][M][F][F] held k-major: after the DFT along
// rows, element (row u, frequency l) of a frame sits at T[l][u], so every
// line the column kernel transforms is contiguous; the row kernels transpose
// their RB x F tiles through LDS and touch T along rows (RB consecutive
// values of one line per run).
// ---------------------------------------------------------------------------
// Loads and stores with the non-temporal hint.  The power-of-two
// three-kernel path streams psi and the spectrum buffer through them and
// the probe sums read psi' through them, so that the probe, the object and
// the intensities stay in the caches (at 10000 x 8 x 256^2 the view update
// takes 62.3 ms with the hints and 65.4 ms without; the probe sums 6.05
// against 6.78 ms).  The mixed-radix kernels read the buffer along columns,
// where neighbouring lanes share cache lines that the hint would give up:
// their view update took 52 ms with it, against 28 ms.
typedef float ntf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ntl2(const float2* p) {
  const ntf2 v = __builtin_nontemporal_load(reinterpret_cast<const ntf2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void nts2(float2 x, float2* p) {
  ntf2 v = {x.x, x.y};
  __builtin_nontemporal_store(v, reinterpret_cast<ntf2*>(p));
}
// rows per block of the row kernels: up to 256 threads, B threads per row
template <int F>
struct RowCfg {
  static constexpr int B = F / 16;
  static constexpr int RB = (256 / B < F) ? 256 / B : F;
  static constexpr int NT = RB * B;
};

// LDS layout of the 16 x B exchange of one line (row or column) in the
// multi-pass kernels: element (k1, n2) at k1 * (B + 1) + n2.  Writes by k1
// (lanes along n2) are consecutive; reads by n2 (lanes along k1) step B + 1
// complex values, which spreads them over the banks.  Lines are XL_ROW (row
// kernels: rows of a 16-lane group land on disjoint banks) or XL_COL (column
// kernel, whose lanes run over 8 columns first) complex values apart.
template <int F>
struct XCfg {
  static constexpr int B = F / 16;
  static constexpr int XS = B + 1;
  static constexpr int XL_ROW = 16 * (B + 1) + 8;
  static constexpr int XL_COL = 16 * (B + 1) + 2;
};

// (1) Z = 2 P O - psi and the DFT along rows: RB rows of every frame of one
// view per block, frame after frame, the next frame's psi rows loaded while
// the current one is transformed (at 10000 x 8 x 256^2: 66.1 ms for the view
// update against 68.8 ms with one block per frame).  The object rows are
// loaded once per object mode and held across its probe modes (both row
// kernels: 62.0 -> 60.6 ms).  M is the number of
// probe modes; with L object modes a view holds L M frames, frame c = l M + k
// being the pair of probe mode k and object mode l.
template <int F>
__global__ __launch_bounds__(256) void k_rows_fwd(
    const ScanDev* __restrict__ scans, const int2* __restrict__ vmap,
    const float2* __restrict__ tw, int M) {
  constexpr int B = F / 16, RB = RowCfg<F>::RB, FF = F * F, NI = 16 / B;
  constexpr int XS = XCfg<F>::XS, LD = XCfg<F>::XL_ROW;
  __shared__ float2 buf[RB * LD];
  const int t = threadIdx.x;
  const int MT = M * scans[0].L;
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  const float2* __restrict__ psi = sc.psi;
  const float2* __restrict__ P = sc.P;
  const float2* __restrict__ O = sc.O;
  const kidx_t pos = kidx(sc.pos);
  float2* __restrict__ T = sc.tspec;
  const int W = uni(sc.W);
  const int rl = t / B, n2 = t % B;
  const int row = blockIdx.y * RB + rl;
  const int y0 = uni(pos[2 * j]), x0 = uni(pos[2 * j + 1]);
  const float2* __restrict__ p0 = psi + (size_t)j * MT * FF + (size_t)row * F;
  constexpr int LT = F + 1;
  static_assert(LT <= LD, "the tile fits the exchange buffer");
  const int r = t % RB, kg = t / RB;
  float2 pn[16], ov[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) pn[n1] = ntl2(&p0[B * n1 + n2]);
  for (int mc = 0; mc < MT; ++mc) {
    const int m = mc % M, l = mc / M;
    const int jm = j * MT + mc;
    const float2* __restrict__ Pm = P + (size_t)m * FF + (size_t)row * F;
    if (m == 0) {
      const float2* __restrict__ Or =
          O + (size_t)l * uni(sc.H) * W + (size_t)(y0 + row) * W + x0;
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) ov[n1] = Or[B * n1 + n2];
    }
    float2 a[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const int v = B * n1 + n2;
      const float2 phi = cmul(Pm[v], ov[n1]);
      a[n1] = make_float2(2.f * phi.x - pn[n1].x, 2.f * phi.y - pn[n1].y);
    }
    if (mc + 1 < MT) {
      const float2* __restrict__ pq = p0 + (size_t)(mc + 1) * FF;
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) pn[n1] = ntl2(&pq[B * n1 + n2]);
    }
    dft16<-1>(a);
    __syncthreads();  // the previous mode's reads of buf are done
    if constexpr (B > 1) {
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) a[k1] = twiddle<-1>(tw, n2 * k1, a[k1]);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) buf[rl * LD + k1 * XS + n2] = a[k1];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int q = 0; q < B; ++q) a[i * B + q] = buf[rl * LD + (n2 + B * i) * XS + q];
#pragma unroll
      for (int i = 0; i < NI; ++i) dftB<-1, B>(&a[i * B]);
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) buf[rl * LT + (n2 + B * i) + 16 * k2] = a[i * B + k2];
    __syncthreads();
    float2* __restrict__ Tt = T + (size_t)jm * FF + (size_t)blockIdx.y * RB + r;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int l2 = kg + B * q;
      nts2(buf[r * LT + l2], &Tt[(size_t)l2 * F]);
    }
  }
}

// (2) DFT along columns for CB columns of every mode of one view, the mode
// sum, the modulus scale, and the inverse DFT along columns, in place in T.
// Block = CB * B * M threads, B consecutive threads per line (each line a
// contiguous run of the k-major buffer); dynamic LDS: CB * M lines of XL_COL
// complex.  One-dimensional grid of views x (F / CB) column blocks, mapped
// so that each XCD takes runs of four neighbouring column blocks of one
// view (their reads of I share cache lines).
template <int F>
__global__ __launch_bounds__(1024) void k_cols(const ScanDev* __restrict__ scans,
                                               const int2* __restrict__ vmap,
                                               const float2* __restrict__ tw, int M, int CB,
                                               int direct) {
  constexpr int B = F / 16, FF = F * F, NI = 16 / B;
  constexpr int XS = XCfg<F>::XS, LD = XCfg<F>::XL_COL;
  extern __shared__ float2 dyn[];
  const int t = threadIdx.x;
  const int nblk = F / CB;
  const int slot = xcd_group_slot(blockIdx.x, gridDim.x);
  const int2 vm = vmap[slot / nblk];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  float2* __restrict__ T = sc.tspec;
  const float* __restrict__ I = sc.I;
  const int col0 = (slot % nblk) * CB;
  const int n2 = t % B;
  const int c = (t / B) % CB;
  const int m = t / (B * CB);
  const int line = m * CB + c;
  float2* __restrict__ Tm = T + ((size_t)j * M + m) * FF + (size_t)(col0 + c) * F;
  // the first KI of this thread's intensities (of the pixels whose scale it
  // forms below) go out before the transform, which hides their latency
  constexpr int KI = 4;
  const float* __restrict__ Ij = I + (size_t)j * FF + col0;
  float ivp[KI];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int p = t + i * (int)blockDim.x;
    const int cc = p / F, kk = p - cc * F;
    ivp[i] = (p < CB * F) ? Ij[(size_t)kk * F + cc] : 0.f;
  }
  float2 a[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) a[n1] = ntl2(&Tm[B * n1 + n2]);
  dft16<-1>(a);
  if constexpr (B > 1) {
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) a[k1] = twiddle<-1>(tw, n2 * k1, a[k1]);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) dyn[line * LD + k1 * XS + n2] = a[k1];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int q = 0; q < B; ++q) a[i * B + q] = dyn[line * LD + (n2 + B * i) * XS + q];
#pragma unroll
    for (int i = 0; i < NI; ++i) dftB<-1, B>(&a[i * B]);
  }
  // mode sum and scale through LDS (aliasing the exchange buffer): |Z~|^2
  // of every mode -> s; each thread then forms the scale of CB * F / NT
  // pixels from the M partial values and I (column-major pixel order, so a
  // wave reads consecutive LDS words and consecutive rows of I), writes it to
  // g, and reads back the scale of its own 16 pixels.  Rows of s and g are
  // padded to F + 4 words: the 8 columns x 4 row offsets a half-wave touches
  // fall in distinct banks.
  constexpr int LS = F + 4;
  float* s = reinterpret_cast<float*>(dyn);
  float* gsh = s + (size_t)M * CB * LS;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) s[line * LS + (n2 + B * i) + 16 * k2] = cabs2(a[i * B + k2]);
  __syncthreads();
  const float inv_ff = 1.0f / (float)FF;
  // g = sqrt(I / S) / F^2, or beta g - 1/F^2 for the update without psi
  const float beta = sc.beta;
  auto scale = [&](float iv, float sum) {
    const float g = (sum > FLT_MIN) ? sqrtf(iv / sum) * inv_ff : 0.f;
    return direct ? beta * g - inv_ff : g;
  };
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int p = t + i * (int)blockDim.x;
    if (p < CB * F) {
      const int cc = p / F, kk = p - cc * F;
      float sum = 0.f;
      for (int mm = 0; mm < M; ++mm) sum += s[(mm * CB + cc) * LS + kk];
      gsh[cc * LS + kk] = scale(fmaxf(ivp[i], 0.f), sum);
    }
  }
  for (int p = t + KI * (int)blockDim.x; p < CB * F; p += blockDim.x) {
    const int cc = p / F, kk = p - cc * F;
    float sum = 0.f;
    for (int mm = 0; mm < M; ++mm) sum += s[(mm * CB + cc) * LS + kk];
    gsh[cc * LS + kk] = scale(fmaxf(Ij[(size_t)kk * F + cc], 0.f), sum);
  }
  __syncthreads();
  float gs[16];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) gs[i * B + k2] = gsh[c * LS + (n2 + B * i) + 16 * k2];
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = cscale(a[r], gs[r]);
  __syncthreads();
  if constexpr (B > 1) {
#pragma unroll
    for (int i = 0; i < NI; ++i) dftB<1, B>(&a[i * B]);
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int q = 0; q < B; ++q) dyn[line * LD + (n2 + B * i) * XS + q] = a[i * B + q];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) a[k1] = dyn[line * LD + k1 * XS + n2];
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) a[k1] = twiddle<1>(tw, n2 * k1, a[k1]);
  }
  dft16<1>(a);
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) nts2(a[n1], &Tm[B * n1 + n2]);
}

// (3) inverse DFT along rows, psi' = psi + beta (Z' - P O), object numerator
// of the view and eps_psi partial sums; all modes of RB rows per block.  With
// L object modes the frames run l-major (c = l M + k) and the numerator of
// object mode l, sum_k conj(P_k) psi'_{(k,l)}, is written after its M
// frames.  DIRECT: the column kernel scaled the spectra by beta g - 1/F^2,
// so the inverse is beta Z' - Z and psi' = (2 - beta) P O + that (Eq. 3 with
// psi = 2 P O - Z): psi is not read and the eps_psi partials are zero.
template <int F, bool DIRECT>
__device__ __forceinline__ void rows_inv(const ScanDev* __restrict__ scans,
                                         const int2* __restrict__ vmap,
                                         const float2* __restrict__ tw, int M) {
  constexpr int B = F / 16, RB = RowCfg<F>::RB, FF = F * F, NI = 16 / B;
  constexpr int XS = XCfg<F>::XS, LD = XCfg<F>::XL_ROW;
  constexpr int NT = RowCfg<F>::NT;
  constexpr int LT = F + 1;  // row stride of the transposed tile in buf
  static_assert(LT <= LD, "the tile fits the exchange buffer");
  __shared__ float2 buf[RB * LD];
  __shared__ float red[2 * ((NT + 63) / 64)];
  const int t = threadIdx.x;
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = uni(vm.y);
  float2* __restrict__ psi = sc.psi;
  const float2* __restrict__ P = sc.P;
  const float2* __restrict__ O = sc.O;
  const kidx_t pos = kidx(sc.pos);
  const float2* __restrict__ T = sc.tspec;
  float2* __restrict__ opart = sc.opart;
  float* __restrict__ err_psi = sc.err_psi;
  const int W = uni(sc.W);
  const float beta = sc.beta;
  const int rl = t / B, n2 = t % B;
  const int row = blockIdx.y * RB + rl;
  const int y0 = uni(pos[2 * j]), x0 = uni(pos[2 * j + 1]);
  const int L = uni(sc.L), MT = M * L;
  const size_t HW = (size_t)uni(sc.H) * W;
  float2 oacc[16], ovh[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) oacc[r] = make_float2(0.f, 0.f);
  float e_d = 0.f, e_n = 0.f;
  for (int mc = 0; mc < MT; ++mc) {
    const int m = mc % M, l = mc / M;
    if (m == 0) {
      const float2* __restrict__ Or = O + (size_t)l * HW + (size_t)(y0 + row) * W + x0;
#pragma unroll
      for (int r = 0; r < 16; ++r) ovh[r] = Or[B * r + n2];
    }
    const size_t base = ((size_t)j * MT + mc) * FF + (size_t)row * F;
    // the block's RB x F tile, read along the k-major lines (thread (r, kg)
    // loads T[l][row0 + r] for l = kg + B s) and transposed through LDS
    {
      const int r = t % RB, kg = t / RB;
      const float2* __restrict__ Tt =
          T + ((size_t)j * MT + mc) * FF + (size_t)blockIdx.y * RB + r;
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = ntl2(&Tt[(size_t)(kg + B * q) * F]);
      __syncthreads();  // the previous mode's reads of buf are done
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[r * LT + kg + B * q] = v[q];
      __syncthreads();
    }
    float2* __restrict__ pm = psi + base;
    // the first half of this frame's psi rows go out before the transform,
    // the second half before the first half's stores (66.2 -> 65.5 ms for
    // the view update at 10000 x 8 x 256^2)
    float2 psn[8];
    if constexpr (!DIRECT) {
#pragma unroll
      for (int k = 0; k < 8; ++k) psn[k] = ntl2(&pm[B * k + n2]);
    }
    float2 a[16];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) a[i * B + k2] = buf[rl * LT + (n2 + B * i) + 16 * k2];
    if constexpr (B > 1) {
#pragma unroll
      for (int i = 0; i < NI; ++i) dftB<1, B>(&a[i * B]);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int q = 0; q < B; ++q) buf[rl * LD + (n2 + B * i) * XS + q] = a[i * B + q];
      __syncthreads();
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) a[k1] = buf[rl * LD + k1 * XS + n2];
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) a[k1] = twiddle<1>(tw, n2 * k1, a[k1]);
    }
    dft16<1>(a);
    const float2* __restrict__ Pm = P + (size_t)m * FF + (size_t)row * F;
    // loads of a batch before its stores (the compiler may not move a load
    // above a store it cannot show to be elsewhere)
#pragma unroll
    for (int b = 0; b < 16; b += 8) {
      float2 pr[8], ov[8], pv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int v = B * (b + k) + n2;
        pr[k] = Pm[v];
        ov[k] = ovh[b + k];
        if constexpr (!DIRECT) pv[k] = psn[k];
      }
      if constexpr (!DIRECT) {
        if (b == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k) psn[k] = ntl2(&pm[B * (8 + k) + n2]);
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int n1 = b + k;
        const int v = B * n1 + n2;
        const float2 phi = cmul(pr[k], ov[k]);
        float2 pn;
        if constexpr (DIRECT) {
          pn = make_float2((2.f - beta) * phi.x + a[n1].x, (2.f - beta) * phi.y + a[n1].y);
        } else {
          const float2 d = make_float2(beta * (a[n1].x - phi.x), beta * (a[n1].y - phi.y));
          pn = cadd(pv[k], d);
          e_d += cabs2(d);
        }
        nts2(pn, &pm[v]);
        e_n += cabs2(pn);
        oacc[n1] = cadd(oacc[n1], cmulc(pr[k], pn));
      }
    }
    if (m == M - 1) {
      float2* __restrict__ oj = opart + ((size_t)j * L + l) * FF + (size_t)row * F;
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) {
        oj[B * n1 + n2] = oacc[n1];
        oacc[n1] = make_float2(0.f, 0.f);
      }
    }
  }
  block_sum2<NT>(e_d, e_n, red);
  if (t == 0) {
    const int part = j * gridDim.y + blockIdx.y;
    err_psi[2 * part] = e_d;
    err_psi[2 * part + 1] = e_n;
  }
}

template <int F>
__global__ __launch_bounds__(256) void k_rows_inv(const ScanDev* __restrict__ scans,
                                                  const int2* __restrict__ vmap,
                                                  const float2* __restrict__ tw, int M) {
  rows_inv<F, false>(scans, vmap, tw, M);
}

template <int F>
__global__ __launch_bounds__(256) void k_rows_inv_direct(const ScanDev* __restrict__ scans,
                                                         const int2* __restrict__ vmap,
                                                         const float2* __restrict__ tw, int M) {
  rows_inv<F, true>(scans, vmap, tw, M);
}

// ---------------------------------------------------------------------------
// Object update (Eq. 5) as an atomics-free gather: one block per T x T object
// tile walks the list of views whose window meets the tile and sums their
// per-view numerators sum_k conj(P_k) psi'_k and the mode power
// D = sum_k |P_k|^2 (the normaliser, in double).  The block has G groups of
// 256 threads; group q takes the views e = q, q + G, ... of the tile's list
// (ascending), U at a time (8 for 16 x 16 tiles, 2 for 32 x 32), so G * U
// views are in flight; the G partial
// sums of each pixel are then added in group order through LDS.  The order of
// every sum is fixed, so results are bitwise reproducible.  blockIdx.y is the
// object mode l (numerators opart[j][l], object O_l; the normaliser is the
// same for every l).
// ---------------------------------------------------------------------------
template <int T, int G>
__global__ __launch_bounds__(256 * G) void k_object(const ScanDev* __restrict__ scans,
                                                    const int2* __restrict__ tmap, int F) {
  constexpr int PPT = T * T / 256;  // pixels per thread
  constexpr int RSTEP = 256 / T;    // rows between a thread's pixels
  __shared__ float red[2 * ((256 * G + 63) / 64)];
  __shared__ float2 pnum[G > 1 ? (G - 1) : 1][T * T];
  __shared__ double pden[G > 1 ? (G - 1) : 1][T * T];
  const int q = uni(threadIdx.x >> 8);  // group (uniform in a wave)
  const int t = threadIdx.x & 255;  // pixel lane within the group
  const int2 tm = tmap[xcd_group_slot(blockIdx.x, gridDim.x)];
  const ScanDev& sc = scans[tm.x];
  const int tile = tm.y;
  const int L = uni(sc.L), l = blockIdx.y;
  const float2* __restrict__ opart = sc.opart;
  const float* __restrict__ D = sc.D;
  float2* __restrict__ O = sc.O + (size_t)l * uni(sc.H) * uni(sc.W);
  // every index here is uniform in a wave: scalar loads
  const kidx_t pos = kidx(sc.pos);
  const kidx_t tile_ptr = kidx(sc.tile_ptr);
  const kidx_t tile_views = kidx(sc.tile_views);
  float* __restrict__ err_obj = sc.err_obj;
  const int H = uni(sc.H), W = uni(sc.W), tiles_x = uni(sc.tiles_x);
  const int ty = tile / tiles_x, tx = tile % tiles_x;
  const int col = t % T, row0 = t / T;
  const int cx = tx * T + col;
  const int ry = ty * T + row0;
  float2 num[PPT];
  double den[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) { num[k] = make_float2(0.f, 0.f); den[k] = 0.0; }
  const int e0 = tile_ptr[tile], e1 = tile_ptr[tile + 1];
  const size_t FF = (size_t)F * F;
  constexpr int U = (8 / PPT > 2) ? 8 / PPT : 2;  // views per group in flight
  int e = e0 + q;
  for (; e + (U - 1) * G < e1; e += U * G) {
    float2 vv[U][PPT];
    float dd[U][PPT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int jv = tile_views[e + u * G];
      const int yj = pos[2 * jv], xj = pos[2 * jv + 1];
      const int v = cx - xj;
      const float2* __restrict__ oj = opart + ((size_t)jv * L + l) * FF;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int uu = ry + RSTEP * k - yj;
        const bool in = ((unsigned)v < (unsigned)F) && ((unsigned)uu < (unsigned)F);
        vv[u][k] = in ? oj[(size_t)uu * F + v] : make_float2(0.f, 0.f);
        dd[u][k] = in ? D[uu * F + v] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        num[k] = cadd(num[k], vv[u][k]);
        den[k] += (double)dd[u][k];
      }
  }
  for (; e < e1; e += G) {
    const int jv = tile_views[e];
    const int yj = pos[2 * jv], xj = pos[2 * jv + 1];
    const int v = cx - xj;
    const float2* __restrict__ oj = opart + ((size_t)jv * L + l) * FF;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int uu = ry + RSTEP * k - yj;
      if (((unsigned)v < (unsigned)F) && ((unsigned)uu < (unsigned)F)) {
        num[k] = cadd(num[k], oj[(size_t)uu * F + v]);
        den[k] += (double)D[uu * F + v];
      }
    }
  }
  if constexpr (G > 1) {
    if (q > 0) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        pnum[q - 1][t + 256 * k] = num[k];
        pden[q - 1][t + 256 * k] = den[k];
      }
    }
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int g = 0; g < G - 1; ++g)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          num[k] = cadd(num[k], pnum[g][t + 256 * k]);
          den[k] += pden[g][t + 256 * k];
        }
    }
  }
  float e_d = 0.f, e_n = 0.f;
  if (q == 0) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int r = ry + RSTEP * k;
      if (r < H && cx < W && den[k] > 0.0) {
        const float inv = (float)(1.0 / den[k]);
        const float2 on = make_float2(num[k].x * inv, num[k].y * inv);
        const float2 oo = O[(size_t)r * W + cx];
        e_d += cabs2(csub(on, oo));
        e_n += cabs2(on);
        O[(size_t)r * W + cx] = on;
      }
    }
  }
  block_sum2<256 * G>(e_d, e_n, red);
  if (threadIdx.x == 0) {
    const int part = l * uni(sc.ntiles) + tile;
    err_obj[2 * part] = e_d;
    err_obj[2 * part + 1] = e_n;
  }
}

// ---------------------------------------------------------------------------
// Probe update (Eq. 4), stage 1: per chunk of views (consecutive in the
// spatial view order) and block of 256 probe pixels,
// sum_j conj(O'[win_j]) psi'_{j,k} for every mode and sum_j |O'[win_j]|^2.
// Modes in groups of 8 held in registers; four views' loads in flight.  With
// L object modes both sums also run over l (views' frames l M + k), the
// object modes in order inside each view.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_probe_partial(const ScanDev* __restrict__ scans,
                                                       const int2* __restrict__ cmap, int M,
                                                       int F) {
  const int FF = F * F;
  const int pix = blockIdx.x * 256 + threadIdx.x;
  const int2 cm = cmap[blockIdx.y];
  const ScanDev& sc = scans[cm.x];
  const int cidx = cm.y;
  const float2* __restrict__ psi = sc.psi;
  const float2* __restrict__ O = sc.O;
  const kidx_t pos = kidx(sc.pos);
  const kidx_t order = kidx(sc.order);
  float2* __restrict__ num_part = sc.num_part;
  float* __restrict__ den_part = sc.den_part;
  const int N = sc.N, W = sc.W, chunk = sc.chunk;
  const int L = sc.L, MT = M * L;
  const size_t HW = (size_t)sc.H * W;
  if (pix >= FF) return;  // F * F need not fill the last block (no barriers here)
  const int j0 = cidx * chunk;
  const int j1 = min(N, j0 + chunk);
  const int u = pix / F, v = pix % F;
  for (int mg = 0; mg < M; mg += 8) {
    float2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = make_float2(0.f, 0.f);
    float den = 0.f;
    // kVU views per step, all of their loads issued before their use
    constexpr int kVU = 4;
    int i = j0;
    // one object mode: views kVU at a time; then (and with object modes
    // throughout) view by view
    for (; L == 1 && i + kVU <= j1; i += kVU) {
      float2 o[kVU], w[kVU][8];
#pragma unroll
      for (int k = 0; k < kVU; ++k) {
        const int jv = order[i + k];
        const int yj = pos[2 * jv], xj = pos[2 * jv + 1];
        o[k] = O[(size_t)(yj + u) * W + xj + v];
        const float2* __restrict__ pj = psi + ((size_t)jv * M + mg) * FF + pix;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          w[k][q] = (mg + q < M) ? ntl2(&pj[(size_t)q * FF]) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int k = 0; k < kVU; ++k) {
        den += cabs2(o[k]);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = cadd(acc[q], cmulc(o[k], w[k][q]));
      }
    }
    for (; i < j1; ++i) {
      const int jv = order[i];
      const int yj = pos[2 * jv], xj = pos[2 * jv + 1];
      for (int l = 0; l < L; ++l) {
        const float2 o = O[(size_t)l * HW + (size_t)(yj + u) * W + xj + v];
        den += cabs2(o);
        const float2* __restrict__ pj = psi + ((size_t)jv * MT + l * M + mg) * FF + pix;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (mg + q < M) acc[q] = cadd(acc[q], cmulc(o, ntl2(&pj[(size_t)q * FF])));
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (mg + q < M) num_part[((size_t)cidx * M + mg + q) * FF + pix] = acc[q];
    if (mg == 0) den_part[(size_t)cidx * FF + pix] = den;
  }
}

// Probe update, stage 2: fixed-order sum over chunks, division (zero
// denominators keep the old value), per-mode eps_P partials and the mode
// power D = sum_k |P'_k|^2 used by the next object update.
__global__ __launch_bounds__(256) void k_probe_final(const ScanDev* __restrict__ scans, int M,
                                                     int FF) {
  __shared__ float red[8];
  const ScanDev& sc = scans[blockIdx.y];
  const float2* __restrict__ num_part = sc.num_part;
  const float* __restrict__ den_part = sc.den_part;
  float2* __restrict__ P = sc.P;
  float* __restrict__ D = sc.D;
  float* __restrict__ err_probe = sc.err_probe;
  const int C = sc.C;
  // pixels past F * F (frames whose F * F is not a multiple of 256) read
  // pixel 0 and store nothing; they stay for the block sums' barriers
  const bool in = blockIdx.x * 256 + threadIdx.x < FF;
  const int pix = in ? blockIdx.x * 256 + threadIdx.x : 0;
  // chunk partials are added in chunk order; loads go out in batches of 8
  float den = 0.f;
  int cc = 0;
  for (; cc + 8 <= C; cc += 8) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = den_part[(size_t)(cc + k) * FF + pix];
#pragma unroll
    for (int k = 0; k < 8; ++k) den += v[k];
  }
  for (; cc < C; ++cc) den += den_part[(size_t)cc * FF + pix];
  float dsum = 0.f;
  for (int m = 0; m < M; ++m) {
    float2 num = make_float2(0.f, 0.f);
    int c2 = 0;
    for (; c2 + 8 <= C; c2 += 8) {
      float2 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = num_part[((size_t)(c2 + k) * M + m) * FF + pix];
#pragma unroll
      for (int k = 0; k < 8; ++k) num = cadd(num, v[k]);
    }
    for (; c2 < C; ++c2) num = cadd(num, num_part[((size_t)c2 * M + m) * FF + pix]);
    const float2 po = P[(size_t)m * FF + pix];
    float2 pn = po;
    if (den > 0.f) {
      const float inv = 1.0f / den;
      pn = make_float2(num.x * inv, num.y * inv);
    }
    if (in) P[(size_t)m * FF + pix] = pn;
    float e_d = in ? cabs2(csub(pn, po)) : 0.f, e_n = in ? cabs2(pn) : 0.f;
    dsum += e_n;
    block_sum2<256>(e_d, e_n, red);
    if (threadIdx.x == 0) {
      err_probe[((size_t)blockIdx.x * M + m) * 2] = e_d;
      err_probe[((size_t)blockIdx.x * M + m) * 2 + 1] = e_n;
    }
  }
  if (in) D[pix] = dsum;
}

// ---------------------------------------------------------------------------
// Error norms (Eq. 6): fixed-order FP64 sums of the partials, written to the
// ring slot of this iteration; the device iteration counter advances.
// ---------------------------------------------------------------------------
__device__ double block_sum_d(double x, double* red) {
  const int t = threadIdx.x;
  red[t] = x;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// sqrt(d / n) of two sums of squares; 0/0 is 0, d/0 infinite, and a NaN in
// either sum stays NaN (so a diverged iteration is never reported as 0)
__device__ __forceinline__ float rel_norm(double d, double n) {
  if (isnan(d) || isnan(n)) return NAN;
  return (n > 0) ? (float)sqrt(d / n) : (d > 0 ? INFINITY : 0.f);
}

// psi_valid = 0: this iteration's view kernel formed no eps_psi partials;
// eps_psi is then reported as NaN and not taken for divergence.
__global__ __launch_bounds__(256) void k_errors(const ScanDev* __restrict__ scans, int n_pblk,
                                                int M, int* __restrict__ flags, int psi_valid) {
  __shared__ double red[256];
  const ScanDev& sc = scans[blockIdx.x];
  const float* __restrict__ err_psi = sc.err_psi;
  const float* __restrict__ err_obj = sc.err_obj;
  const float* __restrict__ err_probe = sc.err_probe;
  int* __restrict__ counter = sc.counter;
  DevErrors* __restrict__ ring = sc.ring;
  const int n_psi = sc.n_psi_parts, n_obj = sc.ntiles * sc.L;
  const int t = threadIdx.x;
  double v[4];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int i = t; i < n_psi; i += 256) { s0 += err_psi[2 * i]; s1 += err_psi[2 * i + 1]; }
  for (int i = t; i < n_obj; i += 256) { s2 += err_obj[2 * i]; s3 += err_obj[2 * i + 1]; }
  v[0] = block_sum_d(s0, red);
  v[1] = block_sum_d(s1, red);
  v[2] = block_sum_d(s2, red);
  v[3] = block_sum_d(s3, red);
  double pd_tot = 0, pn_tot = 0;
  float modes[16];
  for (int m = 0; m < M; ++m) {
    double a = 0, b = 0;
    for (int i = t; i < n_pblk; i += 256) {
      a += err_probe[((size_t)i * M + m) * 2];
      b += err_probe[((size_t)i * M + m) * 2 + 1];
    }
    a = block_sum_d(a, red);
    b = block_sum_d(b, red);
    pd_tot += a;
    pn_tot += b;
    modes[m] = rel_norm(a, b);
  }
  if (t == 0) {
    const int it = *counter;
    DevErrors e;
    e.iter = it + 1;
    e.eps_psi = !psi_valid ? NAN : rel_norm(v[0], v[1]);
    e.eps_obj = rel_norm(v[2], v[3]);
    e.eps_probe = rel_norm(pd_tot, pn_tot);
    bool bad = (psi_valid && !isfinite(e.eps_psi)) || !isfinite(e.eps_obj) ||
               !isfinite(e.eps_probe);
    for (int m = 0; m < 16; ++m) {
      e.eps_mode[m] = (m < M) ? modes[m] : 0.f;
      if (m < M && !isfinite(modes[m])) bad = true;
    }
    ring[it % kRing] = e;
    *counter = it + 1;
    if (bad) atomicOr(flags + 1 + blockIdx.x, 1);
  }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------
// psi_{j,(k,l)} = P_k * O_l[window_j]; one block per (view, frame), frame
// c = l M + k of the L M frames of a view (L object modes, O [L][H][W])
__global__ __launch_bounds__(256) void k_init_psi(float2* __restrict__ psi,
                                                  const float2* __restrict__ P,
                                                  const float2* __restrict__ O,
                                                  const int* __restrict__ pos, int M, int F,
                                                  int W, int L, int H) {
  const int jm = blockIdx.x;
  const int MT = M * L;
  const int j = jm / MT, c = jm % MT;
  const int m = c % M, l = c / M;
  const int FF = F * F;
  const int y0 = uni(pos[2 * j]), x0 = uni(pos[2 * j + 1]);
  const float2* __restrict__ Ol = O + (size_t)l * H * W;
  for (int p = threadIdx.x; p < FF; p += blockDim.x) {
    const int u = p / F, v = p % F;
    psi[(size_t)jm * FF + p] = cmul(P[(size_t)m * FF + p], Ol[(size_t)(y0 + u) * W + x0 + v]);
  }
}

// D = sum_k |P_k|^2
__global__ __launch_bounds__(256) void k_mode_power(const float2* __restrict__ P,
                                                    float* __restrict__ D, int M, int FF) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= FF) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += cabs2(P[(size_t)m * FF + p]);
  D[p] = s;
}

// flags |= 2 if any intensity is NaN or Inf
__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ I, size_t n,
                                                      int* __restrict__ flags) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(I[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 2);
}

// small fills (used instead of memset so the sequence stays graph-safe)
__global__ void k_fill_int(int* __restrict__ p, int n, int val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// Warm start: per-view object numerators of the exit waves psi_{j,k} =
// P_k * patch_j, i.e. sum_k conj(P_k) P_k patch_j = D * patch_j, so that the
// object gather (Eq. 5) stitches the patches with the weights D.
__global__ __launch_bounds__(256) void k_warm_opart(float2* __restrict__ opart,
                                                    const float* __restrict__ D,
                                                    const float2* __restrict__ patches, int N,
                                                    int FF) {
  const size_t total = (size_t)N * FF;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const float d = D[e % FF];
    const float2 q = patches[e];
    opart[e] = make_float2(d * q.x, d * q.y);
  }
}

}  // namespace dmk
