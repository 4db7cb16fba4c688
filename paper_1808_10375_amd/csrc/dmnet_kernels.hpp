// dmnet_kernels.hpp -- gfx950 kernels of the warm-start encoder-decoder:
// direct 3x3 / 1x1 convolutions (bfloat16-stored weights, float32
// accumulation) forward and data-gradient, weight/bias gradients by
// fixed-order block reductions (no atomics), pooling, upsampling, ReLU mask,
// MSE, Adam, input preprocessing and patch upsampling.  Activations are NCHW
// float32 with a per-sample stride, so a tensor can be a channel slice of a
// concatenation buffer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmn {

__device__ __forceinline__ float bf16_bits_to_f(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

// round to nearest bfloat16, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f_to_bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// Convolution, forward (TRANS = false) or data gradient (TRANS = true).
//   forward:  y[n][o][p] = b[o] + sum_c sum_t w[o][c][t] x[n][c][p + off_t]
//   gradient: y[n][c][p] = sum_o sum_t w[o][c][K*K-1-t] x[n][o][p + off_t]
//             (x is then the gradient of the forward output)
// w has shape [w_cout][w_cin][K][K].  One thread per output pixel, COB
// output channels per block row; weights are wave-uniform loads.
// grid (ceil(H*W / blockDim), ceil(yc / COB), n)
// ---------------------------------------------------------------------------
template <int K, int COB, bool TRANS, bool FP32W>
__global__ __launch_bounds__(256) void k_conv(const float* __restrict__ x, int xc, int H, int W,
                                              long x_ns, const uint16_t* __restrict__ wb,
                                              const float* __restrict__ wf,
                                              const float* __restrict__ bias, int w_cin,
                                              float* __restrict__ y, int yc, long y_ns,
                                              int relu) {
  constexpr int KK = K * K;
  const int HW = H * W;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  const int i = p / W, j = p % W;
  const int o0 = blockIdx.y * COB;
  const int n = blockIdx.z;
  const float* __restrict__ xn = x + (long)n * x_ns;
  float acc[COB];
#pragma unroll
  for (int o = 0; o < COB; ++o) acc[o] = (!TRANS && bias && o0 + o < yc) ? bias[o0 + o] : 0.f;
  for (int c = 0; c < xc; ++c) {
    float xv[KK];
#pragma unroll
    for (int t = 0; t < KK; ++t) {
      const int ii = i + t / K - K / 2, jj = j + t % K - K / 2;
      xv[t] = ((unsigned)ii < (unsigned)H && (unsigned)jj < (unsigned)W)
                  ? xn[(long)c * HW + ii * W + jj]
                  : 0.f;
    }
#pragma unroll
    for (int o = 0; o < COB; ++o) {
      if (o0 + o < yc) {
#pragma unroll
        for (int t = 0; t < KK; ++t) {
          const long wi = TRANS ? ((long)c * w_cin + (o0 + o)) * KK + (KK - 1 - t)
                                : ((long)(o0 + o) * w_cin + c) * KK + t;
          const float wv = FP32W ? wf[wi] : bf16_bits_to_f(wb[wi]);
          acc[o] += wv * xv[t];
        }
      }
    }
  }
  float* __restrict__ yn = y + (long)n * y_ns;
#pragma unroll
  for (int o = 0; o < COB; ++o)
    if (o0 + o < yc) yn[(long)(o0 + o) * HW + p] = relu ? fmaxf(acc[o], 0.f) : acc[o];
}

// ---------------------------------------------------------------------------
// Weight and bias gradient of a convolution over one chunk of positions:
//   dwp[z][o][c][t] = sum_{(n, p) in chunk z} dz[n][o][p] x[n][c][p + off_t]
//   dbp[z][o]       = sum_{(n, p) in chunk z} dz[n][o][p]   (block row 0 only)
// (positions n * H*W + p in chunks of `chunk`); the chunk partials are then
// added in chunk order (k_sum_chunks).  One block per (o, group of CIB input
// channels, chunk); each thread sums a strided subset of the chunk's
// positions, then the block adds the per-thread sums in thread order.
// grid (zc, ceil(xc / CIB), n_chunks), 256 threads.
// ---------------------------------------------------------------------------
template <int K, int CIB>
__global__ __launch_bounds__(256) void k_conv_wgrad(const float* __restrict__ x, int xc, int H,
                                                    int W, long x_ns, const float* __restrict__ dz,
                                                    long z_ns, int n_samples, int chunk,
                                                    float* __restrict__ dwp,
                                                    float* __restrict__ dbp) {
  constexpr int KK = K * K;
  constexpr int NV = CIB * KK + 1;
  __shared__ float red[NV][257];
  const int HW = H * W;
  const int zc = gridDim.x;
  const int o = blockIdx.x;
  const int c0 = blockIdx.y * CIB;
  const int z = blockIdx.z;
  const int t = threadIdx.x;
  float acc[CIB * KK];
  float accb = 0.f;
#pragma unroll
  for (int q = 0; q < CIB * KK; ++q) acc[q] = 0.f;
  const int total = n_samples * HW;
  const int p0 = z * chunk, p1 = min(total, p0 + chunk);
  for (int pos = p0 + t; pos < p1; pos += 256) {
    const int n = pos / HW, p = pos % HW;
    const int i = p / W, j = p % W;
    const float g = dz[(long)n * z_ns + (long)o * HW + p];
    accb += g;
    const float* __restrict__ xn = x + (long)n * x_ns;
#pragma unroll
    for (int ci = 0; ci < CIB; ++ci) {
      if (c0 + ci < xc) {
#pragma unroll
        for (int tt = 0; tt < KK; ++tt) {
          const int ii = i + tt / K - K / 2, jj = j + tt % K - K / 2;
          if ((unsigned)ii < (unsigned)H && (unsigned)jj < (unsigned)W)
            acc[ci * KK + tt] += g * xn[(long)(c0 + ci) * HW + ii * W + jj];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CIB * KK; ++q) red[q][t] = acc[q];
  red[NV - 1][t] = accb;
  __syncthreads();
  for (int q = t; q < NV; q += 256) {
    float s = 0.f;
    for (int k = 0; k < 256; ++k) s += red[q][k];
    if (q == NV - 1) {
      if (dbp && blockIdx.y == 0) dbp[(long)z * zc + o] = s;
    } else {
      const int ci = q / KK, tt = q % KK;
      if (c0 + ci < xc) dwp[(((long)z * zc + o) * xc + c0 + ci) * KK + tt] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// 3x3 convolutions on the matrix cores (v_mfma_f32_16x16x32_bf16): implicit
// GEMMs with bfloat16 operands and float32 accumulation.  Pixels of all
// samples form one index P = sample * H*W + p.  Operand layout (one wave):
// A (16 x 32): lane l holds row l%16, k = 8*(l/16) + e; B (32 x 16): lane l
// holds column l%16, k = 8*(l/16) + e; C: lane l holds column l%16, rows
// 4*(l/16) + r.
// ---------------------------------------------------------------------------
typedef __bf16 nb_bf16x8 __attribute__((ext_vector_type(8)));
typedef float nb_f32x4 __attribute__((ext_vector_type(4)));
typedef short nb_s16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ nb_f32x4 nb_mma(nb_s16x8 a, nb_s16x8 b, nb_f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(nb_bf16x8, a),
                                                 __builtin_bit_cast(nb_bf16x8, b), c, 0, 0, 0);
}

// value of the 3x3 im2col matrix at (k = c*9 + t, pixel P), zero outside
__device__ __forceinline__ float im2col3(const float* __restrict__ x, long x_ns, int xc, int H,
                                         int W, int sample, int i, int j, int k, int K) {
  if (k >= K) return 0.f;
  const int c = k / 9, t = k - 9 * c;
  const int ii = i + t / 3 - 1, jj = j + t % 3 - 1;
  if ((unsigned)ii >= (unsigned)H || (unsigned)jj >= (unsigned)W) return 0.f;
  return x[(long)sample * x_ns + ((long)c * H + ii) * W + jj];
}

// y[o][P] = b[o] + sum_k A[o][k] im2col(x)[k][P]  (K = xc * 9), optional ReLU.
// A: bfloat16 [yc][xc * 9].  With A = the flipped, transposed weights and
// x = the output gradient this is the data gradient.
// Block: 4 waves; tile 32 output channels x 256 pixels (64 per wave).
// grid (ceil(n H W / 256), ceil(yc / 32))
__global__ __launch_bounds__(256) void k_conv3_mfma(const float* __restrict__ x, int xc, int H,
                                                    int W, long x_ns, int n,
                                                    const uint16_t* __restrict__ A,
                                                    const float* __restrict__ bias,
                                                    float* __restrict__ y, int yc, long y_ns,
                                                    int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HW = H * W, NP = n * HW, K = xc * 9;
  const int o0 = blockIdx.y * 32;
  const int pw = blockIdx.x * 256 + wave * 64;  // first pixel of this wave
  // the four pixels this lane feeds to the B operands
  int smp[4], pi[4], pj[4];
  bool pok[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int P = pw + 16 * ct + (lane & 15);
    pok[ct] = P < NP;
    const int Pc = pok[ct] ? P : 0;
    smp[ct] = Pc / HW;
    const int p = Pc - smp[ct] * HW;
    pi[ct] = p / W;
    pj[ct] = p - pi[ct] * W;
  }
  nb_f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int kb = k0 + 8 * (lane >> 4);
    nb_s16x8 a[2], b[4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int o = o0 + 16 * rt + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        a[rt][e] = (o < yc && kb + e < K) ? (short)A[(long)o * K + kb + e] : (short)0;
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float v = pok[ct] ? im2col3(x, x_ns, xc, H, W, smp[ct], pi[ct], pj[ct], kb + e, K)
                                : 0.f;
        b[ct][e] = (short)f_to_bf16_bits(v);
      }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_mma(a[rt], b[ct], acc[rt][ct]);
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    if (!pok[ct]) continue;
    const int p = pi[ct] * W + pj[ct];
    float* __restrict__ yn = y + (long)smp[ct] * y_ns;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + 16 * rt + 4 * (lane >> 4) + r;
        if (o < yc) {
          float v = acc[rt][ct][r] + (bias ? bias[o] : 0.f);
          yn[(long)o * HW + p] = relu ? fmaxf(v, 0.f) : v;
        }
      }
  }
}

// x (float32 [n][C][H*W], sample stride x_ns) -> bfloat16 channel-last
// xs[n][H*W][C] (round to nearest even), C a multiple of 8.  One thread per
// (8 channels, pixel), pixels fastest: the reads of a wave are consecutive
// pixels of one channel, each write is 16 bytes.
__global__ void k_to_cl_bf16(const float* __restrict__ x, int C, int HW, long x_ns, int n,
                             uint16_t* __restrict__ xs) {
  const long np = (long)n * HW;
  const long total = np * (C / 8);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long P = e % np;
    const int c8 = (int)(e / np);
    const int smp = (int)(P / HW), p = (int)(P - (long)smp * HW);
    const float* __restrict__ src = x + (long)smp * x_ns + (long)(c8 * 8) * HW + p;
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = (uint32_t)f_to_bf16_bits(src[(long)(2 * q) * HW]) |
             ((uint32_t)f_to_bf16_bits(src[(long)(2 * q + 1) * HW]) << 16);
    *reinterpret_cast<uint4*>(xs + P * C + c8 * 8) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// y[o][P] = b[o] + sum_{t, c} A2[o][t][c] xs[P + off_t][c] over the 3 x 3 taps t
// (zero padding), optional ReLU: the same convolution as k_conv3_mfma with
// a channel-last bfloat16 input xs[n][H][W][xc] (xc a multiple of 32) and
// tap-major weights A2 [yc][9][xc].  K = 9 xc runs in steps of 32 that are
// one tap and 32 channels, so each lane's 8 values of an operand fragment
// are 8 consecutive channels: one 16-byte load.  With A2 the flipped,
// transposed weights and xs the output gradient this is the data gradient.
// Block: 4 waves; tile 32 output channels x 256 pixels (64 per wave).
// grid (ceil(n H W / 256), ceil(yc / 32))
__global__ __launch_bounds__(256) void k_conv3_mfma_cl(const uint16_t* __restrict__ xs, int xc,
                                                       int H, int W, int n,
                                                       const uint16_t* __restrict__ A2,
                                                       const float* __restrict__ bias,
                                                       float* __restrict__ y, int yc, long y_ns,
                                                       int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HW = H * W, NP = n * HW, K = xc * 9;
  const int o0 = blockIdx.y * 32;
  const int pw = blockIdx.x * 256 + wave * 64;
  int smp[4], pi[4], pj[4];
  bool pok[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int P = pw + 16 * ct + (lane & 15);
    pok[ct] = P < NP;
    const int Pc = pok[ct] ? P : 0;
    smp[ct] = Pc / HW;
    const int p = Pc - smp[ct] * HW;
    pi[ct] = p / W;
    pj[ct] = p - pi[ct] * W;
  }
  const int q8 = 8 * (lane >> 4);
  const nb_s16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  nb_f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int t = k0 / xc;
    const int c = k0 - t * xc + q8;
    const int dy = t / 3 - 1, dx = t - 3 * (t / 3) - 1;
    nb_s16x8 a[2], b[4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int o = o0 + 16 * rt + (lane & 15);
      a[rt] = (o < yc) ? *reinterpret_cast<const nb_s16x8*>(A2 + (long)o * K + k0 + q8) : zero8;
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int ii = pi[ct] + dy, jj = pj[ct] + dx;
      const bool ok = pok[ct] && (unsigned)ii < (unsigned)H && (unsigned)jj < (unsigned)W;
      b[ct] = ok ? *reinterpret_cast<const nb_s16x8*>(
                       xs + (((long)smp[ct] * H + ii) * W + jj) * xc + c)
                 : zero8;
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_mma(a[rt], b[ct], acc[rt][ct]);
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    if (!pok[ct]) continue;
    const int p = pi[ct] * W + pj[ct];
    float* __restrict__ yn = y + (long)smp[ct] * y_ns;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + 16 * rt + 4 * (lane >> 4) + r;
        if (o < yc) {
          float v = acc[rt][ct][r] + (bias ? bias[o] : 0.f);
          yn[(long)o * HW + p] = relu ? fmaxf(v, 0.f) : v;
        }
      }
  }
}

// bfloat16 copies for the weight gradient (round to nearest even):
//   xs3[d][n][C][H][W] = x[n][C][i][j + d - 1] (0 outside), d = 0, 1, 2
// the input shifted by each column offset of the 3 x 3 taps, so that 8
// consecutive output pixels of a row read 8 consecutive, 16-byte aligned
// values for every tap; x float32 [n][C][H*W], sample stride x_ns.
__global__ void k_to_bf16_shift3(const float* __restrict__ x, int C, int H, int W, long x_ns,
                                 int n, uint16_t* __restrict__ xs3) {
  const long per = (long)n * C * H * W;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < per;
       e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e % W);
    const long r = e / W;  // (s * C + c) * H + i
    const int i = (int)(r % H);
    const long sc = r / H;
    const int c = (int)(sc % C), smp = (int)(sc / C);
    const float* __restrict__ row = x + (long)smp * x_ns + ((long)c * H + i) * W;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int jj = j + d - 1;
      xs3[(long)d * per + e] = ((unsigned)jj < (unsigned)W) ? f_to_bf16_bits(row[jj]) : 0;
    }
  }
}

// dz float32 [n][C][HW] (sample stride z_ns) -> bfloat16 [n][C][HW]
__global__ void k_to_bf16_nchw(const float* __restrict__ dz, int C, int HW, long z_ns, int n,
                               uint16_t* __restrict__ out) {
  const long per = (long)C * HW, total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int smp = (int)(e / per);
    out[e] = f_to_bf16_bits(dz[(long)smp * z_ns + (e - (long)smp * per)]);
  }
}

// Weight gradient of a 3x3 convolution over one chunk of pixels from the
// bfloat16 copies above (same sums as k_conv3_wgrad_mfma):
//   part[chunk][o][k] = sum_{P in chunk} dz[o][P] im2col(x)[k][P],  k = c*9 + t
// A fragment: 8 consecutive pixels of one output channel of dzb; B fragment:
// 8 consecutive pixels of one (c, t) from the shifted copy of its column
// offset, rows outside the image read as zero.  W must be a multiple of 8
// and chunk a multiple of 32.  Block: 4 waves; tile 32 o x 256 k.
// grid (ceil(K / 256), ceil(zc / 32), n_chunks)
__global__ __launch_bounds__(256) void k_conv3_wgrad_mfma_s(
    const uint16_t* __restrict__ xs3, int xc, int H, int W, const uint16_t* __restrict__ dzb,
    int zc, int n, int chunk, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HW = H * W, NP = n * HW, K = xc * 9;
  const long per = (long)n * xc * HW;  // one shifted copy
  const int o0 = blockIdx.y * 32;
  const int kw = blockIdx.x * 256 + wave * 64;
  const int P0 = blockIdx.z * chunk, P1 = min(NP, P0 + chunk);
  const nb_s16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  // the (channel, tap) of each of this lane's four B columns
  int bc[4], bdy[4];
  long bbase[4];
  bool bok[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int k = kw + 16 * ct + (lane & 15);
    bok[ct] = k < K;
    const int kc = bok[ct] ? k : 0;
    bc[ct] = kc / 9;
    const int t = kc - 9 * bc[ct];
    bdy[ct] = t / 3 - 1;
    bbase[ct] = (long)(t - 3 * (t / 3)) * per;  // shifted copy of the tap's column offset
  }
  nb_f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int Ps = P0; Ps < P1; Ps += 32) {
    const int Pb = Ps + 8 * (lane >> 4);  // 8 consecutive pixels of one row
    const bool in = Pb < P1;
    const int smp = in ? Pb / HW : 0;
    const int p = in ? Pb - smp * HW : 0;
    const int i = p / W, j = p - (p / W) * W;
    nb_s16x8 a[2], b[4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int o = o0 + 16 * rt + (lane & 15);
      a[rt] = (in && o < zc)
                  ? *reinterpret_cast<const nb_s16x8*>(dzb + ((long)smp * zc + o) * HW + p)
                  : zero8;
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int ii = i + bdy[ct];
      const bool ok = in && bok[ct] && (unsigned)ii < (unsigned)H;
      b[ct] = ok ? *reinterpret_cast<const nb_s16x8*>(
                       xs3 + bbase[ct] + (((long)smp * xc + bc[ct]) * H + ii) * W + j)
                 : zero8;
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_mma(a[rt], b[ct], acc[rt][ct]);
  }
  float* __restrict__ pc = part + (long)blockIdx.z * zc * K;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int k = kw + 16 * ct + (lane & 15);
      if (k >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + 16 * rt + 4 * (lane >> 4) + r;
        if (o < zc) pc[(long)o * K + k] = acc[rt][ct][r];
      }
    }
}

// Tap-major copies of the bfloat16 3 x 3 weights w[o][c][t] (yc x xc):
// wK[o][t][c] = w[o][c][t] (forward) and wTK[c][8 - t][o] = w[o][c][t]
// (data gradient: flipped, transposed)
__global__ void k_tapmajor3(const uint16_t* __restrict__ w, int yc, int xc,
                            uint16_t* __restrict__ wK, uint16_t* __restrict__ wTK) {
  const long total = (long)yc * xc * 9;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int t = (int)(e % 9);
    const long oc = e / 9;
    const int c = (int)(oc % xc), o = (int)(oc / xc);
    wK[((long)o * 9 + t) * xc + c] = w[e];
    wTK[((long)c * 9 + (8 - t)) * yc + o] = w[e];
  }
}

// Weight gradient of a 3x3 convolution over one chunk of pixels:
//   part[chunk][o][k] = sum_{P in chunk} dz[o][P] im2col(x)[k][P]
// GEMM rows o (zc), columns k (xc * 9), reduction over P in steps of 32.
// H*W must be a multiple of 8 (8 consecutive pixels stay in one sample).
// Block: 4 waves; tile 32 o x 256 k (64 per wave).
// grid (ceil(K / 256), ceil(zc / 32), n_chunks)
__global__ __launch_bounds__(256) void k_conv3_wgrad_mfma(
    const float* __restrict__ x, int xc, int H, int W, long x_ns, const float* __restrict__ dz,
    int zc, long z_ns, int n, int chunk, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HW = H * W, NP = n * HW, K = xc * 9;
  const int o0 = blockIdx.y * 32;
  const int kw = blockIdx.x * 256 + wave * 64;
  const int P0 = blockIdx.z * chunk, P1 = min(NP, P0 + chunk);
  nb_f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int Ps = P0; Ps < P1; Ps += 32) {
    const int Pb = Ps + 8 * (lane >> 4);  // 8 consecutive pixels of one sample
    const bool in = Pb < P1;
    const int sample = in ? Pb / HW : 0;
    const int p = in ? Pb - sample * HW : 0;
    nb_s16x8 a[2], b[4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int o = o0 + 16 * rt + (lane & 15);
      const float* __restrict__ src = dz + (long)sample * z_ns + (long)o * HW + p;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        a[rt][e] = (short)f_to_bf16_bits((in && o < zc && Pb + e < P1) ? src[e] : 0.f);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int k = kw + 16 * ct + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float v = 0.f;
        if (in && Pb + e < P1) {
          const int pe = p + e;
          const int i = pe / W, j = pe - (pe / W) * W;
          v = im2col3(x, x_ns, xc, H, W, sample, i, j, k, K);
        }
        b[ct][e] = (short)f_to_bf16_bits(v);
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = nb_mma(a[rt], b[ct], acc[rt][ct]);
  }
  float* __restrict__ pc = part + (long)blockIdx.z * zc * K;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int k = kw + 16 * ct + (lane & 15);
      if (k >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + 16 * rt + 4 * (lane >> 4) + r;
        if (o < zc) pc[(long)o * K + k] = acc[rt][ct][r];
      }
    }
}

// dw[e] = sum over chunks of part[chunk][e], in chunk order (loads issued
// eight chunks at a time)
__global__ void k_sum_chunks(const float* __restrict__ part, int n_chunks, long count,
                             float* __restrict__ dw) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    int c = 0;
    for (; c + 8 <= n_chunks; c += 8) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[(long)(c + q) * count + e];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; c < n_chunks; ++c) s += part[(long)c * count + e];
    dw[e] = s;
  }
}

// dbp[z][o] = sum over the positions of chunk z of dz[o] (positions
// n * H*W + p in chunks of `chunk`); one block per (o, chunk), the 256
// per-thread sums added in thread order.  grid (zc, n_chunks)
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ dz, long z_ns,
                                                   int HW, int n, int chunk,
                                                   float* __restrict__ dbp) {
  __shared__ float red[256];
  const int o = blockIdx.x, z = blockIdx.y;
  const int p0 = z * chunk, p1 = min(n * HW, p0 + chunk);
  float s = 0.f;
  for (int P = p0 + threadIdx.x; P < p1; P += 256) {
    const int sample = P / HW, p = P - sample * HW;
    s += dz[(long)sample * z_ns + (long)o * HW + p];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int i = 0; i < 256; ++i) t += red[i];
    dbp[(long)z * gridDim.x + o] = t;
  }
}

// wT[c][o][8 - t] = w[o][c][t]: the weights of the data gradient as a GEMM
// operand [xc][yc * 9]
__global__ void k_flip_transpose3(const uint16_t* __restrict__ w, int yc, int xc,
                                  uint16_t* __restrict__ wT) {
  const long total = (long)yc * xc * 9;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int t = (int)(e % 9);
    const long oc = e / 9;
    const int c = (int)(oc % xc), o = (int)(oc / xc);
    wT[((long)c * yc + o) * 9 + (8 - t)] = w[e];
  }
}

// ---------------------------------------------------------------------------
// elementwise pieces; grid-stride loops over n * C * H * W
// ---------------------------------------------------------------------------
// dst = 2x2 average of src (C channels, src H x W)
__global__ void k_avgpool2(const float* __restrict__ src, long s_ns, float* __restrict__ dst,
                           long d_ns, int C, int H, int W, int n) {
  const int Ho = H / 2, Wo = W / 2;
  const long per = (long)C * Ho * Wo, total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / per);
    const long r = e % per;
    const int c = (int)(r / (Ho * Wo)), q = (int)(r % (Ho * Wo));
    const int i = q / Wo, j = q % Wo;
    const float* s = src + nn * s_ns + (long)c * H * W + (2 * i) * W + 2 * j;
    dst[nn * d_ns + (long)c * Ho * Wo + q] = 0.25f * (s[0] + s[1] + s[W] + s[W + 1]);
  }
}

// dst (H x W) += gradient of the 2x2 average pooling whose output gradient is
// g (H/2 x W/2)
__global__ void k_avgpool2_bwd_add(const float* __restrict__ g, long g_ns,
                                   float* __restrict__ dst, long d_ns, int C, int H, int W,
                                   int n) {
  const long per = (long)C * H * W, total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / per);
    const long r = e % per;
    const int c = (int)(r / (H * W)), q = (int)(r % (H * W));
    const int i = q / W, j = q % W;
    dst[nn * d_ns + r] += 0.25f * g[nn * g_ns + (long)c * (H / 2) * (W / 2) + (i / 2) * (W / 2) + j / 2];
  }
}

// dst (2H x 2W) = nearest upsampling of src (H x W)
__global__ void k_upsample2(const float* __restrict__ src, long s_ns, float* __restrict__ dst,
                            long d_ns, int C, int H, int W, int n) {
  const int Ho = 2 * H, Wo = 2 * W;
  const long per = (long)C * Ho * Wo, total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / per);
    const long r = e % per;
    const int c = (int)(r / (Ho * Wo)), q = (int)(r % (Ho * Wo));
    const int i = q / Wo, j = q % Wo;
    dst[nn * d_ns + r] = src[nn * s_ns + (long)c * H * W + (i / 2) * W + j / 2];
  }
}

// dst (H x W) = gradient of nearest upsampling: sum of the 4 children of g
__global__ void k_upsample2_bwd(const float* __restrict__ g, long g_ns, float* __restrict__ dst,
                                long d_ns, int C, int H, int W, int n) {
  const long per = (long)C * H * W, total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / per);
    const long r = e % per;
    const int c = (int)(r / (H * W)), q = (int)(r % (H * W));
    const int i = q / W, j = q % W;
    const float* s = g + nn * g_ns + (long)c * 4 * H * W + (2 * i) * (2 * W) + 2 * j;
    dst[nn * d_ns + r] = s[0] + s[1] + s[2 * W] + s[2 * W + 1];
  }
}

// g *= (act > 0)
__global__ void k_relu_mask(float* __restrict__ g, long g_ns, const float* __restrict__ act,
                            long a_ns, long per, int n) {
  const long total = per * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / per);
    const long r = e % per;
    if (!(act[nn * a_ns + r] > 0.f)) g[nn * g_ns + r] = 0.f;
  }
}

// dy = 2 (y - t) / denom over the count outputs of each sample, and the
// per-sample sums of (y - t)^2 in partial[] (denom: number of outputs the
// loss averages over); grid: one block per sample
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, long y_ns,
                                             const float* __restrict__ t, long t_ns, long count,
                                             float denom, float* __restrict__ dy, long dy_ns,
                                             float* __restrict__ partial) {
  // one block per sample: sample k's outputs at y + k y_ns (count values)
  __shared__ float red[256];
  const int smp = blockIdx.x;
  const float* __restrict__ ys = y + (long)smp * y_ns;
  const float* __restrict__ ts = t + (long)smp * t_ns;
  float* __restrict__ ds = dy + (long)smp * dy_ns;
  float s = 0.f;
  const float k = 2.0f / denom;
  for (long e = threadIdx.x; e < count; e += 256) {
    const float d = ys[e] - ts[e];
    s += d * d;
    ds[e] = k * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[smp] = red[0];
}

__global__ void k_sum_partials(const float* __restrict__ partial, int n, long count,
                               float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    out[0] = (float)(s / (double)count);
  }
}

// Adam with bias-corrected moments; refresh the bfloat16 copy
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ wb, long n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float mh = me / c1, vh = ve / c2;
    const float pe = p[e] - lr * mh / (sqrtf(vh) + eps);
    p[e] = pe;
    wb[e] = f_to_bf16_bits(pe);
  }
}

__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ wb, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    wb[e] = f_to_bf16_bits(p[e]);
}

__global__ void k_fill(float* __restrict__ p, long n, float v) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    p[e] = v;
}

// x[n][0][i][j] = log1p(sum of the 2x2 block of max(I, 0)) / 10
__global__ void k_preprocess(const float* __restrict__ I, int F, int n, float* __restrict__ x) {
  const int S = F / 2;
  const long total = (long)n * S * S;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / (S * S));
    const int q = (int)(e % (S * S));
    // zero frequency (pixel 0, 0 of the frame) to the centre of the input
    const int i = (q / S + S / 2) % S, j = (q % S + S / 2) % S;
    const float* b = I + (long)nn * F * F + (2 * i) * F + 2 * j;
    const float s = fmaxf(b[0], 0.f) + fmaxf(b[1], 0.f) + fmaxf(b[F], 0.f) + fmaxf(b[F + 1], 0.f);
    x[e] = log1pf(s) * 0.1f;
  }
}

// complex patch [2S][2S] by bilinear 2x upsampling of y [2][S][S]
__global__ void k_patches(const float* __restrict__ y, int S, int n, float2* __restrict__ out) {
  const int P = 2 * S;
  const long total = (long)n * P * P;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int nn = (int)(e / (P * P));
    const int q = (int)(e % (P * P));
    const int u = q / P, v = q % P;
    const float sy = fminf(fmaxf(0.5f * u - 0.25f, 0.f), (float)(S - 1));
    const float sx = fminf(fmaxf(0.5f * v - 0.25f, 0.f), (float)(S - 1));
    const int i0 = (int)sy, j0 = (int)sx;
    const int i1 = min(i0 + 1, S - 1), j1 = min(j0 + 1, S - 1);
    const float fy = sy - i0, fx = sx - j0;
    float r[2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const float* c = y + ((long)nn * 2 + ch) * S * S;
      const float a = c[i0 * S + j0] * (1.f - fx) + c[i0 * S + j1] * fx;
      const float b = c[i1 * S + j0] * (1.f - fx) + c[i1 * S + j1] * fx;
      r[ch] = a * (1.f - fy) + b * fy;
    }
    out[e] = make_float2(r[0], r[1]);
  }
}

}  // namespace dmn
