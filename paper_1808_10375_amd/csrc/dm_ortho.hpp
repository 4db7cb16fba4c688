// dm_ortho.hpp -- orthogonal probe modes.  The multi-mode model of Section II
// (Eq. 1) sums the intensities of the modes, so any unitary mix of the modes
// describes the same measurement; the paper leaves the modes free and cites
// the mixed-state treatment, whose natural representative is the set of
// eigenmodes of the overlap (Gram) matrix
//   G[k][l] = sum_r conj(P_k(r)) P_l(r)   (M x M, Hermitian, PSD).
// With G = V diag(lam) V^H (lam descending) the new modes are
//   Q_a = sum_k V[k][a] P_k,  so  sum_r conj(Q_a) Q_b = lam_a delta_ab,
// and the views get the same mix, psi'_{j,a} = sum_k V[k][a] psi_{j,k}, so the
// iteration continues from an equivalent state (the mode sum of F_c and the
// updates of Eqs. 4-5 are unchanged by a unitary mix of the modes).  Each
// column of V is given a fixed phase: its entry of largest modulus (the first
// such) is made real and positive.
//
// Three kernels, all in FP64 arithmetic on the FP32 data:
//   k_gram_partial  G's upper triangle, per chunk of pixels (fixed order)
//   k_ortho_eig     chunk sums, cyclic Jacobi eigen-decomposition of G in one
//                   wave, eigenvalues sorted descending, phases fixed
//   k_mix_modes     P and every view mixed by V in place
// Scratch (device memory the caller or the library provides), in double2:
//   [kOrthoChunks][pairs] partial sums, then V [16][16], then lam [16].
#pragma once
#include <hip/hip_runtime.h>

#include "dm_kernels.hpp"

namespace dmk {

constexpr int kOrthoMaxModes = 16;
constexpr int kOrthoChunks = 16;
constexpr int kOrthoMaxPairs = kOrthoMaxModes * (kOrthoMaxModes + 1) / 2;
constexpr size_t kOrthoPartWords = (size_t)kOrthoChunks * kOrthoMaxPairs;  // double2 each
constexpr size_t kOrthoVWord = kOrthoPartWords;
constexpr size_t kOrthoLamWord = kOrthoVWord + kOrthoMaxModes * kOrthoMaxModes;
constexpr size_t kOrthoScratchBytes = (kOrthoLamWord + kOrthoMaxModes) * sizeof(double2);

// pair index -> (k, l), k <= l, row-major over the upper triangle
__device__ __forceinline__ void ortho_pair(int pair, int M, int& k, int& l) {
  k = 0;
  while (pair >= M - k) {
    pair -= M - k;
    ++k;
  }
  l = k + pair;
}

// grid (pairs, kOrthoChunks), 256 threads: sum_r conj(P_k) P_l over one
// chunk of the F^2 pixels, in FP64, fixed order (threads, then a tree)
__global__ __launch_bounds__(256) void k_gram_partial(const float2* __restrict__ P, int M, int FF,
                                                      double2* __restrict__ scratch) {
  __shared__ double red[256];
  int k, l;
  ortho_pair(blockIdx.x, M, k, l);
  const int len = (FF + kOrthoChunks - 1) / kOrthoChunks;
  const int r0 = blockIdx.y * len, r1 = min(FF, r0 + len);
  const float2* __restrict__ Pk = P + (size_t)k * FF;
  const float2* __restrict__ Pl = P + (size_t)l * FF;
  double re = 0.0, im = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += 256) {
    const float2 a = Pk[r], b = Pl[r];
    re += (double)a.x * b.x + (double)a.y * b.y;
    im += (double)a.x * b.y - (double)a.y * b.x;
  }
  re = block_sum_d(re, red);
  im = block_sum_d(im, red);
  if (threadIdx.x == 0) {
    const int npairs = M * (M + 1) / 2;
    scratch[(size_t)blockIdx.y * npairs + blockIdx.x] = make_double2(re, im);
  }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

// One wave.  Lane k works on row/column k of the M x M matrices in LDS.
// Cyclic Jacobi: for every pair (p, q) with A[p][q] = r w (r = |A[p][q]|,
// |w| = 1), column q is multiplied by conj(w) and row q by w, which makes
// A[p][q] = r real; then the real rotation [[c, s], [-s, c]] on columns and
// rows p, q with cot(2 theta) = (A[q][q] - A[p][p]) / (2 r) zeroes it.  V
// accumulates the same column operations.  Sweeps stop when the squared
// off-diagonal norm is below 1e-30 of the squared norm of A (or after 40).
__global__ __launch_bounds__(64) void k_ortho_eig(int M, double2* __restrict__ scratch,
                                                  double* __restrict__ lam_out) {
  __shared__ double2 A[kOrthoMaxModes][kOrthoMaxModes + 1];
  __shared__ double2 V[kOrthoMaxModes][kOrthoMaxModes + 1];
  __shared__ double rot[3];  // c, s, skip
  __shared__ double2 wsh;
  __shared__ int done;
  __shared__ int idx[kOrthoMaxModes];
  const int t = threadIdx.x;
  const int npairs = M * (M + 1) / 2;
  for (int pair = t; pair < npairs; pair += 64) {
    double re = 0.0, im = 0.0;
    for (int ch = 0; ch < kOrthoChunks; ++ch) {
      const double2 v = scratch[(size_t)ch * npairs + pair];
      re += v.x;
      im += v.y;
    }
    int k, l;
    ortho_pair(pair, M, k, l);
    if (k == l) {
      A[k][k] = make_double2(re, 0.0);
    } else {
      A[k][l] = make_double2(re, im);
      A[l][k] = make_double2(re, -im);
    }
  }
  if (t < M)
    for (int l = 0; l < M; ++l) V[t][l] = make_double2(t == l ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();
    if (t == 0) {
      double off = 0.0, tot = 0.0;
      for (int k = 0; k < M; ++k)
        for (int l = 0; l < M; ++l) {
          const double a2 = A[k][l].x * A[k][l].x + A[k][l].y * A[k][l].y;
          tot += a2;
          if (k != l) off += a2;
        }
      done = (off <= 1e-30 * tot) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int p = 0; p < M - 1; ++p)
      for (int q = p + 1; q < M; ++q) {
        __syncthreads();  // every lane has read the previous rotation
        if (t == 0) {
          const double2 apq = A[p][q];
          const double r = sqrt(apq.x * apq.x + apq.y * apq.y);
          if (r == 0.0) {
            rot[2] = 1.0;
          } else {
            const double th = (A[q][q].x - A[p][p].x) / (2.0 * r);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(tt * tt + 1.0);
            rot[0] = c;
            rot[1] = tt * c;
            rot[2] = 0.0;
            wsh = make_double2(apq.x / r, apq.y / r);
          }
        }
        __syncthreads();
        if (rot[2] != 0.0) continue;  // uniform across the wave
        const double c = rot[0], s = rot[1];
        const double2 w = wsh, wc = zconj(w);
        // phase: column q times conj(w), then row q times w
        if (t < M) {
          A[t][q] = zmul(A[t][q], wc);
          V[t][q] = zmul(V[t][q], wc);
        }
        __syncthreads();
        if (t < M) A[q][t] = zmul(A[q][t], w);
        __syncthreads();
        // rotation of columns p, q (A and V), then of rows p, q (A)
        if (t < M) {
          const double2 akp = A[t][p], akq = A[t][q];
          A[t][p] = make_double2(c * akp.x - s * akq.x, c * akp.y - s * akq.y);
          A[t][q] = make_double2(s * akp.x + c * akq.x, s * akp.y + c * akq.y);
          const double2 vkp = V[t][p], vkq = V[t][q];
          V[t][p] = make_double2(c * vkp.x - s * vkq.x, c * vkp.y - s * vkq.y);
          V[t][q] = make_double2(s * vkp.x + c * vkq.x, s * vkp.y + c * vkq.y);
        }
        __syncthreads();
        if (t < M) {
          const double2 apk = A[p][t], aqk = A[q][t];
          A[p][t] = make_double2(c * apk.x - s * aqk.x, c * apk.y - s * aqk.y);
          A[q][t] = make_double2(s * apk.x + c * aqk.x, s * apk.y + c * aqk.y);
        }
        __syncthreads();
        if (t == 0) {
          A[p][q] = make_double2(0.0, 0.0);
          A[q][p] = make_double2(0.0, 0.0);
          A[p][p].y = 0.0;
          A[q][q].y = 0.0;
        }
        __syncthreads();
      }
  }
  // eigenvalues descending (stable insertion sort of the indices), then the
  // phase of every eigenvector column
  if (t == 0) {
    for (int a = 0; a < M; ++a) idx[a] = a;
    for (int a = 1; a < M; ++a) {
      const int x = idx[a];
      int b = a - 1;
      while (b >= 0 && A[idx[b]][idx[b]].x < A[x][x].x) {
        idx[b + 1] = idx[b];
        --b;
      }
      idx[b + 1] = x;
    }
  }
  __syncthreads();
  double2* __restrict__ Vout = scratch + kOrthoVWord;
  double2* __restrict__ lam = scratch + kOrthoLamWord;
  if (t < M) {
    const int col = idx[t];
    int kmax = 0;
    double best = -1.0;
    for (int k = 0; k < M; ++k) {
      const double m2 = V[k][col].x * V[k][col].x + V[k][col].y * V[k][col].y;
      if (m2 > best) {
        best = m2;
        kmax = k;
      }
    }
    const double2 v = V[kmax][col];
    const double mag = sqrt(best);
    const double2 ph = make_double2(v.x / mag, -v.y / mag);  // conj(v) / |v|
    for (int k = 0; k < M; ++k) Vout[k * kOrthoMaxModes + t] = zmul(V[k][col], ph);
    lam[t] = make_double2(A[col][col].x, 0.0);
    if (lam_out) lam_out[t] = A[col][col].x;
  }
}

// grid (ceil(F^2 / 256), any): sets s = blockIdx.y, blockIdx.y + gridDim.y,
// ... up to n_views; set s < n_views mixes the M modes of view s of psi, set
// n_views mixes the probe; x_a <- sum_k V[k][a] x_k per pixel (FP64 sums,
// rounded to FP32 once).
__global__ __launch_bounds__(256) void k_mix_modes(float2* __restrict__ psi, float2* __restrict__ P,
                                                   int n_views, int M, int FF,
                                                   const double2* __restrict__ scratch) {
  __shared__ double2 Vs[kOrthoMaxModes * kOrthoMaxModes];
  const double2* __restrict__ Vg = scratch + kOrthoVWord;
  for (int e = threadIdx.x; e < kOrthoMaxModes * kOrthoMaxModes; e += 256) Vs[e] = Vg[e];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= FF) return;
  for (int s = blockIdx.y; s <= n_views; s += gridDim.y) {
    float2* __restrict__ base = (s < n_views) ? psi + (size_t)s * M * FF : P;
    float2 x[kOrthoMaxModes];
#pragma unroll
    for (int k = 0; k < kOrthoMaxModes; ++k)
      if (k < M) x[k] = base[(size_t)k * FF + p];
#pragma unroll
    for (int a = 0; a < kOrthoMaxModes; ++a) {
      if (a >= M) break;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int k = 0; k < kOrthoMaxModes; ++k) {
        if (k >= M) break;
        const double2 v = Vs[k * kOrthoMaxModes + a];
        re += v.x * x[k].x - v.y * x[k].y;
        im += v.x * x[k].y + v.y * x[k].x;
      }
      base[(size_t)a * FF + p] = make_float2((float)re, (float)im);
    }
  }
}

}  // namespace dmk
