// dmnet_api.hip -- host side of the warm-start network (include/dmnet.h):
// workspace carving, the forward / backward layer sequence and Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dmnet.h"
#include "dmnet_kernels.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Conv {
  int cin, cout, k, level;
  size_t w_off, b_off;  // offsets (in floats) into the parameter vector
};

// pixels per block of the matrix-core weight gradient (a multiple of 32)
constexpr int kWgradChunk = 1024;
constexpr int kVGradChunk = 1024;  // positions per partial of the vector-unit gradients

struct Shape {
  std::vector<Conv> convs;  // parameter order
  std::vector<int> ch;      // C_l
  size_t n_params = 0;
};

bool valid(const dmnet_desc* d) {
  if (!d || d->batch < 1 || d->base_ch < 1 || d->levels < 2 || d->levels > 6 ||
      d->size < 4 || d->reserved != 0 || (d->flags & ~DMNET_FLAG_FP32_WEIGHTS))
    return false;
  if (d->size % (1 << (d->levels - 1))) return false;
  if (!(d->lr > 0.f) || !(d->beta1 >= 0.f && d->beta1 < 1.f) ||
      !(d->beta2 >= 0.f && d->beta2 < 1.f) || !(d->eps > 0.f))
    return false;
  return true;
}

Shape make_shape(const dmnet_desc& d) {
  Shape s;
  const int L = d.levels;
  for (int l = 0; l < L; ++l) s.ch.push_back(d.base_ch << l);
  auto add = [&](int cin, int cout, int k, int level) {
    Conv c{cin, cout, k, level, s.n_params, 0};
    s.n_params += (size_t)cin * cout * k * k;
    c.b_off = s.n_params;
    s.n_params += cout;
    s.convs.push_back(c);
  };
  int prev = 1;
  for (int l = 0; l < L; ++l) {
    add(prev, s.ch[l], 3, l);
    add(s.ch[l], s.ch[l], 3, l);
    prev = s.ch[l];
  }
  for (int l = L - 2; l >= 0; --l) {
    add(s.ch[l + 1] + s.ch[l], s.ch[l], 3, l);
    add(s.ch[l], s.ch[l], 3, l);
  }
  add(s.ch[0], 2, 1, 0);
  return s;
}

// Activation buffers per level (floats per sample)
struct ActLayout {
  std::vector<size_t> enc_mid, enc_out, pool, cat, dec_mid, dec_out;  // offsets
  size_t bott, y, total;  // floats per sample for one copy of the activations
};

ActLayout act_layout(const dmnet_desc& d, const Shape& s) {
  ActLayout a;
  const int L = d.levels;
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off += n;
    return o;
  };
  for (int l = 0; l < L; ++l) {
    const size_t S = (size_t)(d.size >> l), HW = S * S;
    a.enc_mid.push_back(take(s.ch[l] * HW));
    if (l < L - 1) {
      a.cat.push_back(take((size_t)(s.ch[l + 1] + s.ch[l]) * HW));
      a.enc_out.push_back(a.cat.back() + (size_t)s.ch[l + 1] * HW);  // skip slice
      a.pool.push_back(take(s.ch[l] * HW / 4));
      a.dec_mid.push_back(take(s.ch[l] * HW));
      a.dec_out.push_back(take(s.ch[l] * HW));
    }
  }
  a.bott = take((size_t)s.ch[L - 1] * (d.size >> (L - 1)) * (d.size >> (L - 1)));
  a.enc_out.push_back(a.bott);
  a.y = take((size_t)2 * d.size * d.size);
  a.total = off;
  return a;
}

struct NetLayout {
  size_t params, wb, wbT, wbK, wTK, grads, m, v, acts, grad_acts, xcl, wgb, wpart, partial,
      loss, total;
};

// chunks of the matrix-core weight gradient of conv c at n samples
int wgrad_chunks(const dmnet_desc& d, const Conv& c, int n) {
  const long hw = (long)(d.size >> c.level) * (d.size >> c.level);
  return (int)((n * hw + kWgradChunk - 1) / kWgradChunk);
}

// chunks of the vector-unit weight and bias gradients of conv c at n samples
int vgrad_chunks(const dmnet_desc& d, const Conv& c, int n) {
  const long hw = (long)(d.size >> c.level) * (d.size >> c.level);
  return (int)((n * hw + kVGradChunk - 1) / kVGradChunk);
}

constexpr int kMseBlocks = 256;

NetLayout net_layout(const dmnet_desc& d, const Shape& s, const ActLayout& a) {
  NetLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.params = take(s.n_params * 4);
  L.wb = take(s.n_params * 2);
  L.wbT = take(s.n_params * 2);  // flipped, transposed 3x3 weights (data gradient)
  L.wbK = take(s.n_params * 2);  // tap-major 3x3 weights [o][t][c]
  L.wTK = take(s.n_params * 2);  // tap-major flipped, transposed [c][t][o]
  L.grads = take(s.n_params * 4);
  L.m = take(s.n_params * 4);
  L.v = take(s.n_params * 4);
  L.acts = take(a.total * 4 * d.batch);
  L.grad_acts = take(a.total * 4 * d.batch);
  // channel-last bfloat16 copy of a 3x3 convolution's input (or output
  // gradient), one convolution at a time
  size_t xcl = 8;
  for (const Conv& c : s.convs)
    if (c.k == 3) {
      const size_t hw = (size_t)(d.size >> c.level) * (d.size >> c.level);
      xcl = std::max(xcl, (size_t)d.batch * hw * std::max(c.cin, c.cout));
    }
  L.xcl = take(xcl * 2);
  // bfloat16 copies for a 3x3 weight gradient: the input shifted by each
  // column offset (3 copies) and the output gradient
  size_t wgb = 8;
  for (const Conv& c : s.convs)
    if (c.k == 3) {
      const size_t hw = (size_t)(d.size >> c.level) * (d.size >> c.level);
      wgb = std::max(wgb, (size_t)d.batch * hw * (3 * (size_t)c.cin + c.cout));
    }
  L.wgb = take(wgb * 2);
  // chunk partials of the weight and bias gradients (one conv at a time)
  size_t wpart = 1;
  for (const Conv& c : s.convs) {
    if (c.k == 3)
      wpart = std::max(wpart, (size_t)wgrad_chunks(d, c, d.batch) * c.cout * c.cin * 9);
    wpart = std::max(wpart, (size_t)vgrad_chunks(d, c, d.batch) * c.cout *
                                (1 + (size_t)c.cin * c.k * c.k));
  }
  L.wpart = take(wpart * 4);
  L.partial = take(kMseBlocks * 4);
  L.loss = take(4);
  L.total = off;
  return L;
}

}  // namespace

struct dmnet {
  dmnet_desc d;
  Shape s;
  ActLayout a;
  NetLayout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  long step = 0;
  bool failed = false;
  std::string err;
  float* f(size_t off) { return reinterpret_cast<float*>(ws + off); }
  float* params() { return f(L.params); }
  uint16_t* wb() { return reinterpret_cast<uint16_t*>(ws + L.wb); }
  uint16_t* wbT() { return reinterpret_cast<uint16_t*>(ws + L.wbT); }
  uint16_t* wbK() { return reinterpret_cast<uint16_t*>(ws + L.wbK); }
  uint16_t* wTK() { return reinterpret_cast<uint16_t*>(ws + L.wTK); }
  uint16_t* xcl() { return reinterpret_cast<uint16_t*>(ws + L.xcl); }
  uint16_t* wgb() { return reinterpret_cast<uint16_t*>(ws + L.wgb); }
  bool mfma() const { return !(d.flags & DMNET_FLAG_FP32_WEIGHTS); }
  float* grads() { return f(L.grads); }
  float* act(size_t o) { return f(L.acts) + o; }     // per-sample stride a.total
  float* gact(size_t o) { return f(L.grad_acts) + o; }
};

namespace {

dm_status fail(dmnet* n, hipError_t e, const char* where) {
  n->failed = true;
  n->err = std::string(where) + ": " + hipGetErrorString(e);
  return DM_E_HIP;
}

#define NET_LAUNCHED(net, name)                           \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return fail((net), e_, name);   \
  } while (0)

#define NET_HIP(net, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return fail((net), e_, #call);    \
  } while (0)

#define NET_TRY(expr)           \
  do {                          \
    dm_status s_ = (expr);      \
    if (s_ != DM_OK) return s_; \
  } while (0)

dm_status check(dmnet* n, int count) {
  if (!n) return DM_E_ARG;
  if (n->failed) return DM_E_STATE;
  if (count < 1 || count > n->d.batch) {
    n->err = "sample count out of range";
    return DM_E_ARG;
  }
  return DM_OK;
}

unsigned grid_for(long n) { return (unsigned)std::min<long>((n + 255) / 256, 8192); }

// the flipped, transposed bfloat16 weights of every 3x3 convolution, the A
// operand of the matrix-core data gradient; redone whenever the weights change
dm_status refresh_transposed(dmnet* net) {
  if (!net->mfma()) return DM_OK;
  for (const Conv& c : net->s.convs) {
    if (c.k != 3) continue;
    const long cnt = (long)c.cout * c.cin * 9;
    hipLaunchKernelGGL(dmn::k_flip_transpose3, dim3(grid_for(cnt)), dim3(256), 0, net->stream,
                       net->wb() + c.w_off, c.cout, c.cin, net->wbT() + c.w_off);
    hipLaunchKernelGGL(dmn::k_tapmajor3, dim3(grid_for(cnt)), dim3(256), 0, net->stream,
                       net->wb() + c.w_off, c.cout, c.cin, net->wbK() + c.w_off,
                       net->wTK() + c.w_off);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    net->failed = true;
    net->err = std::string("k_flip_transpose3: ") + hipGetErrorString(e);
    return DM_E_HIP;
  }
  return DM_OK;
}

// y = conv(x) (+ ReLU); x, y are per-sample-strided tensors
dm_status conv_fwd(dmnet* net, const Conv& c, const float* x, long x_ns, float* y, long y_ns,
                   int H, int W, int n, bool relu) {
  const bool fp32w = net->d.flags & DMNET_FLAG_FP32_WEIGHTS;
  const float* wf = net->params() + c.w_off;
  const uint16_t* wb = net->wb() + c.w_off;
  const float* b = net->params() + c.b_off;
  const int HW = H * W;
  if (net->mfma() && c.k == 3) {
    dim3 g((unsigned)(((long)n * HW + 255) / 256), (c.cout + 31) / 32);
    if (c.cin % 32 == 0 && c.w_off % 8 == 0) {
      // channel-last bfloat16 copy of the input, then 16-byte operand loads
      // (the weight rows start 16-byte aligned)
      const long cnt = (long)n * HW * (c.cin / 8);
      hipLaunchKernelGGL(dmn::k_to_cl_bf16, dim3(grid_for(cnt)), dim3(256), 0, net->stream, x,
                         c.cin, HW, x_ns, n, net->xcl());
      NET_LAUNCHED(net, "k_to_cl_bf16");
      hipLaunchKernelGGL(dmn::k_conv3_mfma_cl, g, dim3(256), 0, net->stream, net->xcl(), c.cin,
                         H, W, n, net->wbK() + c.w_off, b, y, c.cout, y_ns, relu ? 1 : 0);
      NET_LAUNCHED(net, "k_conv3_mfma_cl");
      return DM_OK;
    }
    hipLaunchKernelGGL(dmn::k_conv3_mfma, g, dim3(256), 0, net->stream, x, c.cin, H, W, x_ns, n,
                       wb, b, y, c.cout, y_ns, relu ? 1 : 0);
    NET_LAUNCHED(net, "k_conv3_mfma");
    return DM_OK;
  }
  const int bs = std::min(256, HW);
  constexpr int COB = 8;
  dim3 grid((HW + bs - 1) / bs, (c.cout + COB - 1) / COB, n);
  if (c.k == 3) {
    if (fp32w)
      hipLaunchKernelGGL((dmn::k_conv<3, COB, false, true>), grid, dim3(bs), 0, net->stream, x,
                         c.cin, H, W, x_ns, wb, wf, b, c.cin, y, c.cout, y_ns, relu ? 1 : 0);
    else
      hipLaunchKernelGGL((dmn::k_conv<3, COB, false, false>), grid, dim3(bs), 0, net->stream,
                         x, c.cin, H, W, x_ns, wb, wf, b, c.cin, y, c.cout, y_ns, relu ? 1 : 0);
  } else {
    if (fp32w)
      hipLaunchKernelGGL((dmn::k_conv<1, COB, false, true>), grid, dim3(bs), 0, net->stream, x,
                         c.cin, H, W, x_ns, wb, wf, b, c.cin, y, c.cout, y_ns, relu ? 1 : 0);
    else
      hipLaunchKernelGGL((dmn::k_conv<1, COB, false, false>), grid, dim3(bs), 0, net->stream,
                         x, c.cin, H, W, x_ns, wb, wf, b, c.cin, y, c.cout, y_ns, relu ? 1 : 0);
  }
  NET_LAUNCHED(net, "k_conv forward");
  return DM_OK;
}

// dz is the gradient at the conv output (already masked by the ReLU);
// writes dW, db into the gradient vector and, if dx, the input gradient
dm_status conv_bwd(dmnet* net, const Conv& c, const float* x, long x_ns, const float* dz,
                   long z_ns, float* dx, long dx_ns, int H, int W, int n) {
  const bool fp32w = net->d.flags & DMNET_FLAG_FP32_WEIGHTS;
  const float* wf = net->params() + c.w_off;
  const uint16_t* wb = net->wb() + c.w_off;
  float* dw = net->grads() + c.w_off;
  float* db = net->grads() + c.b_off;
  if (net->mfma() && c.k == 3 && (H * W) % 8 == 0) {
    const int K = c.cin * 9;
    const int nch = wgrad_chunks(net->d, c, n);
    float* part = net->f(net->L.wpart);
    const dim3 wg((K + 255) / 256, (c.cout + 31) / 32, nch);
    if (W % 8 == 0) {
      // bfloat16 copies: x shifted by each column offset, and dz
      uint16_t* xs3 = net->wgb();
      uint16_t* dzb = xs3 + (size_t)3 * n * c.cin * H * W;
      hipLaunchKernelGGL(dmn::k_to_bf16_shift3, dim3(grid_for((long)n * c.cin * H * W)),
                         dim3(256), 0, net->stream, x, c.cin, H, W, x_ns, n, xs3);
      NET_LAUNCHED(net, "k_to_bf16_shift3");
      hipLaunchKernelGGL(dmn::k_to_bf16_nchw, dim3(grid_for((long)n * c.cout * H * W)),
                         dim3(256), 0, net->stream, dz, c.cout, H * W, z_ns, n, dzb);
      NET_LAUNCHED(net, "k_to_bf16_nchw");
      hipLaunchKernelGGL(dmn::k_conv3_wgrad_mfma_s, wg, dim3(256), 0, net->stream, xs3, c.cin,
                         H, W, dzb, c.cout, n, kWgradChunk, part);
      NET_LAUNCHED(net, "k_conv3_wgrad_mfma_s");
    } else {
      hipLaunchKernelGGL(dmn::k_conv3_wgrad_mfma, wg, dim3(256), 0, net->stream, x, c.cin, H,
                         W, x_ns, dz, c.cout, z_ns, n, kWgradChunk, part);
      NET_LAUNCHED(net, "k_conv3_wgrad_mfma");
    }
    const long cnt = (long)c.cout * K;
    hipLaunchKernelGGL(dmn::k_sum_chunks, dim3(grid_for(cnt)), dim3(256), 0, net->stream, part,
                       nch, cnt, dw);
    NET_LAUNCHED(net, "k_sum_chunks");
    const int bch = vgrad_chunks(net->d, c, n);
    hipLaunchKernelGGL(dmn::k_bias_grad, dim3(c.cout, bch), dim3(256), 0, net->stream, dz,
                       z_ns, H * W, n, kVGradChunk, part);
    NET_LAUNCHED(net, "k_bias_grad");
    hipLaunchKernelGGL(dmn::k_sum_chunks, dim3(grid_for(c.cout)), dim3(256), 0, net->stream,
                       part, bch, (long)c.cout, db);
    NET_LAUNCHED(net, "k_sum_chunks (bias)");
    if (dx) {
      dim3 g((unsigned)(((long)n * H * W + 255) / 256), (c.cin + 31) / 32);
      if (c.cout % 32 == 0 && c.w_off % 8 == 0) {
        const long cnt = (long)n * H * W * (c.cout / 8);
        hipLaunchKernelGGL(dmn::k_to_cl_bf16, dim3(grid_for(cnt)), dim3(256), 0, net->stream,
                           dz, c.cout, H * W, z_ns, n, net->xcl());
        NET_LAUNCHED(net, "k_to_cl_bf16 (output gradient)");
        hipLaunchKernelGGL(dmn::k_conv3_mfma_cl, g, dim3(256), 0, net->stream, net->xcl(),
                           c.cout, H, W, n, net->wTK() + c.w_off, nullptr, dx, c.cin, dx_ns, 0);
        NET_LAUNCHED(net, "k_conv3_mfma_cl (data gradient)");
      } else {
        hipLaunchKernelGGL(dmn::k_conv3_mfma, g, dim3(256), 0, net->stream, dz, c.cout, H, W,
                           z_ns, n, net->wbT() + c.w_off, nullptr, dx, c.cin, dx_ns, 0);
        NET_LAUNCHED(net, "k_conv3_mfma (data gradient)");
      }
    }
    return DM_OK;
  }
  {
    const int vch = vgrad_chunks(net->d, c, n);
    float* part = net->f(net->L.wpart);
    const long nw = (long)c.cout * c.cin * c.k * c.k;
    float* bpart = part + (size_t)vch * nw;  // bias partials after the weight partials
    if (c.k == 3) {
      constexpr int CIB = 4;
      hipLaunchKernelGGL((dmn::k_conv_wgrad<3, CIB>), dim3(c.cout, (c.cin + CIB - 1) / CIB, vch),
                         dim3(256), 0, net->stream, x, c.cin, H, W, x_ns, dz, z_ns, n,
                         kVGradChunk, part, bpart);
    } else {
      constexpr int CIB = 16;
      hipLaunchKernelGGL((dmn::k_conv_wgrad<1, CIB>), dim3(c.cout, (c.cin + CIB - 1) / CIB, vch),
                         dim3(256), 0, net->stream, x, c.cin, H, W, x_ns, dz, z_ns, n,
                         kVGradChunk, part, bpart);
    }
    NET_LAUNCHED(net, "k_conv_wgrad");
    hipLaunchKernelGGL(dmn::k_sum_chunks, dim3(grid_for(nw)), dim3(256), 0, net->stream, part,
                       vch, nw, dw);
    NET_LAUNCHED(net, "k_sum_chunks (weights)");
    hipLaunchKernelGGL(dmn::k_sum_chunks, dim3(grid_for(c.cout)), dim3(256), 0, net->stream,
                       bpart, vch, (long)c.cout, db);
    NET_LAUNCHED(net, "k_sum_chunks (bias)");
  }
  if (dx) {
    const int HW = H * W;
    const int bs = std::min(256, HW);
    constexpr int COB = 8;
    dim3 grid((HW + bs - 1) / bs, (c.cin + COB - 1) / COB, n);
    if (c.k == 3) {
      if (fp32w)
        hipLaunchKernelGGL((dmn::k_conv<3, COB, true, true>), grid, dim3(bs), 0, net->stream, dz,
                           c.cout, H, W, z_ns, wb, wf, nullptr, c.cin, dx, c.cin, dx_ns, 0);
      else
        hipLaunchKernelGGL((dmn::k_conv<3, COB, true, false>), grid, dim3(bs), 0, net->stream,
                           dz, c.cout, H, W, z_ns, wb, wf, nullptr, c.cin, dx, c.cin, dx_ns, 0);
    } else {
      if (fp32w)
        hipLaunchKernelGGL((dmn::k_conv<1, COB, true, true>), grid, dim3(bs), 0, net->stream, dz,
                           c.cout, H, W, z_ns, wb, wf, nullptr, c.cin, dx, c.cin, dx_ns, 0);
      else
        hipLaunchKernelGGL((dmn::k_conv<1, COB, true, false>), grid, dim3(bs), 0, net->stream,
                           dz, c.cout, H, W, z_ns, wb, wf, nullptr, c.cin, dx, c.cin, dx_ns, 0);
    }
    NET_LAUNCHED(net, "k_conv data gradient");
  }
  return DM_OK;
}

dm_status relu_mask(dmnet* net, float* g, const float* act, long ns, long per, int n) {
  hipLaunchKernelGGL(dmn::k_relu_mask, dim3(grid_for(per * n)), dim3(256), 0, net->stream, g, ns,
                     act, ns, per, n);
  NET_LAUNCHED(net, "k_relu_mask");
  return DM_OK;
}

// forward pass; output into y (per-sample stride y_ns)
dm_status forward(dmnet* net, const float* x, int n, float* y, long y_ns) {
  const dmnet_desc& d = net->d;
  const Shape& s = net->s;
  const ActLayout& a = net->a;
  const long T = (long)a.total;
  const int L = d.levels;
  int ci = 0;
  const float* in = x;
  long in_ns = (long)d.size * d.size;
  for (int l = 0; l < L; ++l) {
    const int S = d.size >> l;
    NET_TRY(conv_fwd(net, s.convs[ci++], in, in_ns, net->act(a.enc_mid[l]), T, S, S, n, true));
    NET_TRY(conv_fwd(net, s.convs[ci++], net->act(a.enc_mid[l]), T, net->act(a.enc_out[l]), T, S,
                     S, n, true));
    if (l < L - 1) {
      const long tot = (long)s.ch[l] * (S / 2) * (S / 2) * n;
      hipLaunchKernelGGL(dmn::k_avgpool2, dim3(grid_for(tot)), dim3(256), 0, net->stream,
                         net->act(a.enc_out[l]), T, net->act(a.pool[l]), T, s.ch[l], S, S, n);
      NET_LAUNCHED(net, "k_avgpool2");
      in = net->act(a.pool[l]);
      in_ns = T;
    }
  }
  const float* h = net->act(a.bott);
  for (int l = L - 2; l >= 0; --l) {
    const int S = d.size >> l;
    const long tot = (long)s.ch[l + 1] * S * S * n;
    hipLaunchKernelGGL(dmn::k_upsample2, dim3(grid_for(tot)), dim3(256), 0, net->stream, h, T,
                       net->act(a.cat[l]), T, s.ch[l + 1], S / 2, S / 2, n);
    NET_LAUNCHED(net, "k_upsample2");
    NET_TRY(conv_fwd(net, s.convs[ci++], net->act(a.cat[l]), T, net->act(a.dec_mid[l]), T, S, S,
                     n, true));
    NET_TRY(conv_fwd(net, s.convs[ci++], net->act(a.dec_mid[l]), T, net->act(a.dec_out[l]), T, S,
                     S, n, true));
    h = net->act(a.dec_out[l]);
  }
  NET_TRY(conv_fwd(net, s.convs[ci++], h, T, y, y_ns, d.size, d.size, n, false));
  return DM_OK;
}

// backward pass from dy (gradient at the output, per-sample stride T)
dm_status backward(dmnet* net, const float* x, int n, float* dy) {
  const dmnet_desc& d = net->d;
  const Shape& s = net->s;
  const ActLayout& a = net->a;
  const long T = (long)a.total;
  const int L = d.levels;
  int ci = (int)s.convs.size() - 1;
  // head
  NET_TRY(conv_bwd(net, s.convs[ci--], net->act(a.dec_out[0]), T, dy, T, net->gact(a.dec_out[0]),
                   T, d.size, d.size, n));
  // decoder, l = 0 .. L-2 (reverse of the forward order)
  for (int l = 0; l <= L - 2; ++l) {
    const int S = d.size >> l;
    const long per = (long)s.ch[l] * S * S;
    NET_TRY(relu_mask(net, net->gact(a.dec_out[l]), net->act(a.dec_out[l]), T, per, n));
    NET_TRY(conv_bwd(net, s.convs[ci--], net->act(a.dec_mid[l]), T, net->gact(a.dec_out[l]), T,
                     net->gact(a.dec_mid[l]), T, S, S, n));
    NET_TRY(relu_mask(net, net->gact(a.dec_mid[l]), net->act(a.dec_mid[l]), T, per, n));
    NET_TRY(conv_bwd(net, s.convs[ci--], net->act(a.cat[l]), T, net->gact(a.dec_mid[l]), T,
                     net->gact(a.cat[l]), T, S, S, n));
    // gradient of the upsampled part goes to the next-deeper output
    float* dh = (l + 1 <= L - 2) ? net->gact(a.dec_out[l + 1]) : net->gact(a.bott);
    const long tot = (long)s.ch[l + 1] * (S / 2) * (S / 2) * n;
    hipLaunchKernelGGL(dmn::k_upsample2_bwd, dim3(grid_for(tot)), dim3(256), 0, net->stream,
                       net->gact(a.cat[l]), T, dh, T, s.ch[l + 1], S / 2, S / 2, n);
    NET_LAUNCHED(net, "k_upsample2_bwd");
  }
  // encoder, l = L-1 .. 0
  for (int l = L - 1; l >= 0; --l) {
    const int S = d.size >> l;
    const long per = (long)s.ch[l] * S * S;
    float* g_out = net->gact(a.enc_out[l]);  // skip slice of the concat gradient, or bottleneck
    if (l < L - 1) {
      hipLaunchKernelGGL(dmn::k_avgpool2_bwd_add, dim3(grid_for(per * n)), dim3(256), 0,
                         net->stream, net->gact(a.pool[l]), T, g_out, T, s.ch[l], S, S, n);
      NET_LAUNCHED(net, "k_avgpool2_bwd_add");
    }
    NET_TRY(relu_mask(net, g_out, net->act(a.enc_out[l]), T, per, n));
    NET_TRY(conv_bwd(net, s.convs[ci--], net->act(a.enc_mid[l]), T, g_out, T,
                     net->gact(a.enc_mid[l]), T, S, S, n));
    NET_TRY(relu_mask(net, net->gact(a.enc_mid[l]), net->act(a.enc_mid[l]), T, per, n));
    const float* in = (l == 0) ? x : net->act(a.pool[l - 1]);
    const long in_ns = (l == 0) ? (long)d.size * d.size : T;
    float* g_in = (l == 0) ? nullptr : net->gact(a.pool[l - 1]);
    NET_TRY(conv_bwd(net, s.convs[ci--], in, in_ns, net->gact(a.enc_mid[l]), T, g_in, T, S, S,
                     n));
  }
  return DM_OK;
}

// forward, loss and backward; grads land in net->grads()
dm_status loss_and_grad(dmnet* net, const float* x, const float* target, int n) {
  const ActLayout& a = net->a;
  const long T = (long)a.total;
  const long per = 2L * net->d.size * net->d.size;
  NET_TRY(forward(net, x, n, net->act(a.y), T));
  // the outputs of the n samples sit T floats apart: one block per sample,
  // each leaving its sum of squares in partial[k]; the loss averages over
  // all n * per outputs
  hipLaunchKernelGGL(dmn::k_mse, dim3(n), dim3(256), 0, net->stream, net->act(a.y), T, target,
                     per, per, (float)(per * n), net->gact(a.y), T, net->f(net->L.partial));
  NET_LAUNCHED(net, "k_mse");
  return DM_OK;
}

}  // namespace

extern "C" {

size_t dmnet_n_params(const dmnet_desc* d) {
  if (!valid(d)) return 0;
  return make_shape(*d).n_params;
}

size_t dmnet_workspace_bytes(const dmnet_desc* d) {
  if (!valid(d)) return 0;
  Shape s = make_shape(*d);
  ActLayout a = act_layout(*d, s);
  return net_layout(*d, s, a).total;
}

dm_status dmnet_create(dmnet** out, const dmnet_desc* d, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!out) return DM_E_ARG;
  *out = nullptr;
  if (!valid(d) || !ws) return DM_E_ARG;
  if (d->batch > 256) return DM_E_UNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return DM_E_ARG;
  dmnet* n = new (std::nothrow) dmnet();
  if (!n) return DM_E_ARG;
  n->d = *d;
  n->s = make_shape(*d);
  n->a = act_layout(*d, n->s);
  n->L = net_layout(*d, n->s, n->a);
  if (ws_bytes < n->L.total) {
    delete n;
    return DM_E_WORKSPACE;
  }
  n->ws = reinterpret_cast<char*>(ws);
  n->stream = reinterpret_cast<hipStream_t>(stream);
  const long P = (long)n->s.n_params;
  hipLaunchKernelGGL(dmn::k_fill, dim3(grid_for(P)), dim3(256), 0, n->stream, n->params(), P,
                     0.f);
  hipLaunchKernelGGL(dmn::k_fill, dim3(grid_for(P)), dim3(256), 0, n->stream, n->f(n->L.m), P,
                     0.f);
  hipLaunchKernelGGL(dmn::k_fill, dim3(grid_for(P)), dim3(256), 0, n->stream, n->f(n->L.v), P,
                     0.f);
  hipLaunchKernelGGL(dmn::k_to_bf16, dim3(grid_for(P)), dim3(256), 0, n->stream, n->params(),
                     n->wb(), P);
  if (hipGetLastError() != hipSuccess || refresh_transposed(n) != DM_OK) {
    delete n;
    return DM_E_HIP;
  }
  *out = n;
  return DM_OK;
}

dm_status dmnet_set_params(dmnet* n, const float* p) {
  if (!n || !p) return DM_E_ARG;
  if (n->failed) return DM_E_STATE;
  const long P = (long)n->s.n_params;
  NET_HIP(n, hipMemcpyAsync(n->params(), p, P * 4, hipMemcpyDeviceToDevice, n->stream));
  hipLaunchKernelGGL(dmn::k_to_bf16, dim3(grid_for(P)), dim3(256), 0, n->stream, n->params(),
                     n->wb(), P);
  NET_LAUNCHED(n, "k_to_bf16");
  NET_TRY(refresh_transposed(n));
  hipLaunchKernelGGL(dmn::k_fill, dim3(grid_for(P)), dim3(256), 0, n->stream, n->f(n->L.m), P,
                     0.f);
  hipLaunchKernelGGL(dmn::k_fill, dim3(grid_for(P)), dim3(256), 0, n->stream, n->f(n->L.v), P,
                     0.f);
  NET_LAUNCHED(n, "k_fill");
  n->step = 0;
  return DM_OK;
}

dm_status dmnet_get_params(dmnet* n, float* p) {
  if (!n || !p) return DM_E_ARG;
  if (n->failed) return DM_E_STATE;
  NET_HIP(n, hipMemcpyAsync(p, n->params(), n->s.n_params * 4, hipMemcpyDeviceToDevice,
                            n->stream));
  return DM_OK;
}

dm_status dmnet_forward(dmnet* n, const float* x, float* y, int32_t count) {
  NET_TRY(check(n, count));
  if (!x || !y) return DM_E_ARG;
  return forward(n, x, count, y, 2L * n->d.size * n->d.size);
}

dm_status dmnet_loss_grad(dmnet* n, const float* x, const float* target, int32_t count,
                          float* grads_out, float* loss_host) {
  NET_TRY(check(n, count));
  if (!x || !target) return DM_E_ARG;
  NET_TRY(loss_and_grad(n, x, target, count));
  NET_TRY(backward(n, x, count, n->gact(n->a.y)));
  // loss: mean of the squared errors over every output of the batch
  hipLaunchKernelGGL(dmn::k_sum_partials, dim3(1), dim3(64), 0, n->stream, n->f(n->L.partial),
                     count, 2L * n->d.size * n->d.size * count, n->f(n->L.loss));
  NET_LAUNCHED(n, "k_sum_partials");
  if (grads_out)
    NET_HIP(n, hipMemcpyAsync(grads_out, n->grads(), n->s.n_params * 4, hipMemcpyDeviceToDevice,
                              n->stream));
  if (loss_host) {
    float l = 0.f;
    NET_HIP(n, hipMemcpyAsync(&l, n->f(n->L.loss), 4, hipMemcpyDeviceToHost, n->stream));
    NET_HIP(n, hipStreamSynchronize(n->stream));
    *loss_host = l;
  }
  return DM_OK;
}

dm_status dmnet_train_step(dmnet* n, const float* x, const float* target, int32_t count,
                           float* loss_host) {
  NET_TRY(dmnet_loss_grad(n, x, target, count, nullptr, loss_host));
  n->step++;
  const long P = (long)n->s.n_params;
  const float c1 = (float)(1.0 - std::pow((double)n->d.beta1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow((double)n->d.beta2, (double)n->step));
  hipLaunchKernelGGL(dmn::k_adam, dim3(grid_for(P)), dim3(256), 0, n->stream, n->params(),
                     n->f(n->L.m), n->f(n->L.v), n->grads(), n->wb(), P, n->d.lr, n->d.beta1,
                     n->d.beta2, n->d.eps, c1, c2);
  NET_LAUNCHED(n, "k_adam");
  return refresh_transposed(n);
}

dm_status dmnet_preprocess(dmnet* n, const float* I, int32_t count, int32_t frame, float* x) {
  if (!n || !I || !x || count < 1) return DM_E_ARG;
  if (n->failed) return DM_E_STATE;
  if (frame != 2 * n->d.size) {
    n->err = "frame must be twice the network size";
    return DM_E_ARG;
  }
  const long tot = (long)count * n->d.size * n->d.size;
  hipLaunchKernelGGL(dmn::k_preprocess, dim3(grid_for(tot)), dim3(256), 0, n->stream, I, frame,
                     count, x);
  NET_LAUNCHED(n, "k_preprocess");
  return DM_OK;
}

dm_status dmnet_patches(dmnet* n, const float* y, int32_t count, void* patches) {
  if (!n || !y || !patches || count < 1) return DM_E_ARG;
  if (n->failed) return DM_E_STATE;
  const long tot = (long)count * 4 * n->d.size * n->d.size;
  hipLaunchKernelGGL(dmn::k_patches, dim3(grid_for(tot)), dim3(256), 0, n->stream, y, n->d.size,
                     count, reinterpret_cast<float2*>(patches));
  NET_LAUNCHED(n, "k_patches");
  return DM_OK;
}

void dmnet_free(dmnet* n) { delete n; }

const char* dmnet_last_error(const dmnet* n) { return n ? n->err.c_str() : ""; }

}  // extern "C"
