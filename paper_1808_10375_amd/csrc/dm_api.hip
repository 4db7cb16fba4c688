// dm_api.hip -- host side of libdm: the C-ABI declared in include/dm.h.
// Validation, workspace carving, the object-tile -> view lists, and the
// launch sequence of one difference-map iteration (Section II, Eqs. 2-6 of
// arXiv:1808.10375).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dm.h"
#include "dm_kernels.hpp"

using dmk::DevErrors;
static_assert(sizeof(DevErrors) == sizeof(dm_errors), "error record layout");

namespace {

thread_local std::string g_init_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Which transform path a descriptor uses.
bool use_fused(const dm_desc& d) {
  return d.frame <= 128 && !(d.flags & DM_FLAG_MULTIPASS);
}

struct Layout {
  size_t psi, opart, tspec, gscr, P, O, D, num_part, den_part, err_psi, err_obj, err_probe,
      ring, counter, pos, order, tile_ptr, tile_views, tw, total;
  int tile, tiles_x, tiles_y, ntiles, nnz_max, C, chunk, n_psi_parts, n_pblk, cb;
};

// Object tile edge of the gather kernel.
constexpr int kObjTile = 16;

int probe_chunks(const dm_desc& d) {
  const int FF = d.frame * d.frame;
  const int pix_blocks = (FF + 255) / 256;
  int C = (2048 + pix_blocks - 1) / pix_blocks;
  C = std::max(1, std::min(C, d.n_frames));
  return C;
}

int cols_per_block(const dm_desc& d) {
  const int B = d.frame / 16;
  int cb = 1024 / (B * d.n_modes);
  int p = 1;
  while (p * 2 <= cb && p * 2 <= 16) p *= 2;
  return p;
}

Layout make_layout(const dm_desc& d) {
  Layout L{};
  const size_t N = d.n_frames, M = d.n_modes, F = d.frame, FF = F * F;
  const size_t c8 = 8;  // complex64 bytes
  L.tile = kObjTile;
  L.tiles_x = (d.obj_w + L.tile - 1) / L.tile;
  L.tiles_y = (d.obj_h + L.tile - 1) / L.tile;
  L.ntiles = L.tiles_x * L.tiles_y;
  const int span = (int)(F / L.tile) + 1 + (F % L.tile ? 1 : 0);
  L.nnz_max = (int)N * span * span;
  L.C = probe_chunks(d);
  L.chunk = (int)((N + L.C - 1) / L.C);
  L.n_pblk = (int)((FF + 255) / 256);
  const bool fused = use_fused(d);
  const int B = (int)F / 16;
  const int rb = std::min(256 / B, (int)F);
  L.n_psi_parts = fused ? (int)N : (int)N * ((int)F / rb);
  L.cb = fused ? 0 : cols_per_block(d);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.psi = take(N * M * FF * c8);
  L.opart = take(N * FF * c8);
  L.tspec = fused ? 0 : take(N * M * FF * c8);
  L.gscr = fused ? take(N * FF * 4) : 0;
  L.P = take(M * FF * c8);
  L.O = take((size_t)d.obj_h * d.obj_w * c8);
  L.D = take(FF * 4);
  L.num_part = take((size_t)L.C * M * FF * c8);
  L.den_part = take((size_t)L.C * FF * 4);
  L.err_psi = take((size_t)L.n_psi_parts * 2 * 4);
  L.err_obj = take((size_t)L.ntiles * 2 * 4);
  L.err_probe = take((size_t)L.n_pblk * M * 2 * 4);
  L.ring = take(sizeof(DevErrors) * dmk::kRing);
  L.counter = take(2 * sizeof(int));  // [0] iteration counter, [1] flags
  L.pos = take(N * 2 * 4);
  L.order = take(N * 4);
  L.tile_ptr = take(((size_t)L.ntiles + 1) * 4);
  L.tile_views = take((size_t)L.nnz_max * 4);
  L.tw = take(F * c8);
  L.total = off;
  return L;
}

dm_status validate_desc(const dm_desc* d, std::string& why) {
  if (!d) { why = "desc is NULL"; return DM_E_ARG; }
  if (d->n_frames < 1) { why = "n_frames must be >= 1"; return DM_E_ARG; }
  if (d->n_modes < 1) { why = "n_modes must be >= 1"; return DM_E_ARG; }
  if (d->n_modes > DM_MAX_MODES) { why = "n_modes > 16 not supported"; return DM_E_UNSUPPORTED; }
  if (!is_pow2(d->frame) || d->frame < 16 || d->frame > 256) {
    why = "frame must be a power of two in [16, 256]";
    return DM_E_UNSUPPORTED;
  }
  if (d->obj_h < d->frame || d->obj_w < d->frame) { why = "object smaller than a frame"; return DM_E_ARG; }
  if (!(d->beta >= 0.f && d->beta <= 1.f)) { why = "beta must lie in [0, 1]"; return DM_E_ARG; }
  if (d->precision != DM_FP32_FFT && d->precision != DM_BF16X3_DFT) {
    why = "unknown precision";
    return DM_E_UNSUPPORTED;
  }
  if (d->precision == DM_BF16X3_DFT) {
    why = "the BF16x3 DFT form is not built into this library";
    return DM_E_UNSUPPORTED;
  }
  if (d->flags & ~(DM_FLAG_MULTIPASS | DM_FLAG_PHASE_TIMING)) {
    why = "unknown flag bits";
    return DM_E_ARG;
  }
  if ((double)d->obj_h * d->obj_w * 8.0 >= 2147483648.0) {
    why = "object larger than 2^28 pixels";
    return DM_E_UNSUPPORTED;
  }
  if ((double)d->n_frames * d->frame * d->frame >= 2147483648.0) {
    why = "more than 2^31 detector pixels in total";
    return DM_E_UNSUPPORTED;
  }
  return DM_OK;
}

}  // namespace

struct dm_ctx {
  dm_desc d;
  Layout L;
  hipStream_t stream;
  char* ws;
  const float* I;
  bool failed = false;
  std::string err;
  int iters = 0;
  std::vector<int> pos_host;
  // phase timing: event pairs recorded since the last dm_phase_times
  struct Mark { int phase; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  int timed_iters = 0;
  ~dm_ctx() {
    for (auto& m : marks) { event_pool.push_back(m.a); event_pool.push_back(m.b); }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  }
  bool timing() const { return (d.flags & DM_FLAG_PHASE_TIMING) != 0; }

  float2* psi() { return reinterpret_cast<float2*>(ws + L.psi); }
  float2* opart() { return reinterpret_cast<float2*>(ws + L.opart); }
  float2* tspec() { return reinterpret_cast<float2*>(ws + L.tspec); }
  float* gscr() { return reinterpret_cast<float*>(ws + L.gscr); }
  int* order() { return reinterpret_cast<int*>(ws + L.order); }
  float2* P() { return reinterpret_cast<float2*>(ws + L.P); }
  float2* O() { return reinterpret_cast<float2*>(ws + L.O); }
  float* D() { return reinterpret_cast<float*>(ws + L.D); }
  float2* num_part() { return reinterpret_cast<float2*>(ws + L.num_part); }
  float* den_part() { return reinterpret_cast<float*>(ws + L.den_part); }
  float* err_psi() { return reinterpret_cast<float*>(ws + L.err_psi); }
  float* err_obj() { return reinterpret_cast<float*>(ws + L.err_obj); }
  float* err_probe() { return reinterpret_cast<float*>(ws + L.err_probe); }
  DevErrors* ring() { return reinterpret_cast<DevErrors*>(ws + L.ring); }
  int* counter() { return reinterpret_cast<int*>(ws + L.counter); }
  int* flags() { return reinterpret_cast<int*>(ws + L.counter) + 1; }
  int* pos() { return reinterpret_cast<int*>(ws + L.pos); }
  int* tile_ptr() { return reinterpret_cast<int*>(ws + L.tile_ptr); }
  int* tile_views() { return reinterpret_cast<int*>(ws + L.tile_views); }
  float2* tw() { return reinterpret_cast<float2*>(ws + L.tw); }
};

namespace {

dm_status fail_hip(dm_ctx* c, hipError_t e, const char* where) {
  c->failed = true;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return DM_E_HIP;
}

#define DM_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, #call); \
  } while (0)

#define DM_LAUNCHED(ctx, name)                                  \
  do {                                                          \
    hipError_t e_ = hipGetLastError();                          \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, name);     \
  } while (0)

dm_status check_ctx(dm_ctx* c) {
  if (!c) return DM_E_ARG;
  if (c->failed) return DM_E_STATE;
  return DM_OK;
}

// Forward twiddles exp(-2 pi i m / F), computed in double, rounded to float.
std::vector<float2> twiddles(int F) {
  std::vector<float2> t(F);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < F; ++m) {
    const double a = -2.0 * pi * (double)m / (double)F;
    t[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return t;
}

// Lists of views whose window meets each object tile, ascending view order.
void build_tile_lists(const dm_desc& d, const Layout& L, const int* pos, std::vector<int>& ptr,
                      std::vector<int>& views) {
  const int T = L.tile, F = d.frame;
  std::vector<int> count(L.ntiles, 0);
  for (int j = 0; j < d.n_frames; ++j) {
    const int y = pos[2 * j], x = pos[2 * j + 1];
    for (int ty = y / T; ty <= (y + F - 1) / T; ++ty)
      for (int tx = x / T; tx <= (x + F - 1) / T; ++tx) count[ty * L.tiles_x + tx]++;
  }
  ptr.assign(L.ntiles + 1, 0);
  for (int i = 0; i < L.ntiles; ++i) ptr[i + 1] = ptr[i] + count[i];
  views.assign(std::max(ptr[L.ntiles], 1), 0);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int j = 0; j < d.n_frames; ++j) {
    const int y = pos[2 * j], x = pos[2 * j + 1];
    for (int ty = y / T; ty <= (y + F - 1) / T; ++ty)
      for (int tx = x / T; tx <= (x + F - 1) / T; ++tx) views[fill[ty * L.tiles_x + tx]++] = j;
  }
}

hipError_t take_event(dm_ctx* c, hipEvent_t* e) {
  if (!c->event_pool.empty()) {
    *e = c->event_pool.back();
    c->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Record the start of a timed phase; returns the index of its mark or -1.
dm_status phase_begin(dm_ctx* c, int phase, int* idx) {
  *idx = -1;
  if (!c->timing()) return DM_OK;
  dm_ctx::Mark m{phase, nullptr, nullptr};
  DM_HIP(c, take_event(c, &m.a));
  DM_HIP(c, take_event(c, &m.b));
  DM_HIP(c, hipEventRecord(m.a, c->stream));
  c->marks.push_back(m);
  *idx = (int)c->marks.size() - 1;
  return DM_OK;
}

dm_status phase_end(dm_ctx* c, int idx) {
  if (idx < 0) return DM_OK;
  DM_HIP(c, hipEventRecord(c->marks[idx].b, c->stream));
  return DM_OK;
}

// Views sorted along a Z-order curve of their window corners: runs of
// consecutive entries cover compact patches of the object.
std::vector<int> spatial_order(const dm_desc& d, const int* pos) {
  auto spread = [](uint32_t v) {
    uint64_t x = v & 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
  };
  std::vector<std::pair<uint64_t, int>> key(d.n_frames);
  for (int j = 0; j < d.n_frames; ++j) {
    const uint32_t y = (uint32_t)pos[2 * j] / 8u, x = (uint32_t)pos[2 * j + 1] / 8u;
    key[j] = {(spread(y) << 1) | spread(x), j};
  }
  std::stable_sort(key.begin(), key.end());
  std::vector<int> order(d.n_frames);
  for (int j = 0; j < d.n_frames; ++j) order[j] = key[j].second;
  return order;
}

template <int F>
dm_status launch_fourier_fused(dm_ctx* c) {
  const dm_desc& d = c->d;
  hipLaunchKernelGGL(dmk::k_fourier_fused<F>, dim3(d.n_frames), dim3(F * F / 16), 0, c->stream,
                     c->psi(), c->I, c->P(), c->O(), c->pos(), c->order(), c->tw(), c->opart(),
                     c->gscr(), c->err_psi(), d.n_frames, d.n_modes, d.obj_h, d.obj_w, d.beta);
  DM_LAUNCHED(c, "k_fourier_fused");
  return DM_OK;
}

template <int F>
dm_status launch_fourier_multipass(dm_ctx* c) {
  const dm_desc& d = c->d;
  constexpr int B = F / 16, RB = dmk::RowCfg<F>::RB, NT = dmk::RowCfg<F>::NT;
  hipLaunchKernelGGL(dmk::k_rows_fwd<F>, dim3(d.n_frames * d.n_modes, F / RB), dim3(NT), 0,
                     c->stream, c->psi(), c->P(), c->O(), c->pos(), c->tw(), c->tspec(),
                     d.n_modes, d.obj_w);
  DM_LAUNCHED(c, "k_rows_fwd");
  const int cb = c->L.cb;
  const size_t lds = (size_t)cb * d.n_modes * (F + 1) * sizeof(float2);
  hipLaunchKernelGGL(dmk::k_cols<F>, dim3(d.n_frames, F / cb), dim3(cb * B * d.n_modes), lds,
                     c->stream, c->tspec(), c->I, c->tw(), d.n_modes, cb);
  DM_LAUNCHED(c, "k_cols");
  hipLaunchKernelGGL(dmk::k_rows_inv<F>, dim3(d.n_frames, F / RB), dim3(NT), 0, c->stream,
                     c->psi(), c->P(), c->O(), c->pos(), c->tw(), c->tspec(), c->opart(),
                     c->err_psi(), d.n_modes, d.obj_w, d.beta);
  DM_LAUNCHED(c, "k_rows_inv");
  return DM_OK;
}

dm_status launch_views(dm_ctx* c) {
  const int F = c->d.frame;
  if (use_fused(c->d)) {
    switch (F) {
      case 16: return launch_fourier_fused<16>(c);
      case 32: return launch_fourier_fused<32>(c);
      case 64: return launch_fourier_fused<64>(c);
      case 128: return launch_fourier_fused<128>(c);
    }
  } else {
    switch (F) {
      case 16: return launch_fourier_multipass<16>(c);
      case 32: return launch_fourier_multipass<32>(c);
      case 64: return launch_fourier_multipass<64>(c);
      case 128: return launch_fourier_multipass<128>(c);
      case 256: return launch_fourier_multipass<256>(c);
    }
  }
  c->err = "unsupported frame size";
  return DM_E_UNSUPPORTED;
}

#define DM_TRY(expr)              \
  do {                            \
    dm_status s_ = (expr);        \
    if (s_ != DM_OK) return s_;   \
  } while (0)

dm_status launch_iteration(dm_ctx* c) {
  const dm_desc& d = c->d;
  const Layout& L = c->L;
  const int FF = d.frame * d.frame;
  int mk;
  DM_TRY(phase_begin(c, DM_PHASE_VIEWS, &mk));
  DM_TRY(launch_views(c));
  DM_TRY(phase_end(c, mk));
  DM_TRY(phase_begin(c, DM_PHASE_OBJECT, &mk));
  if (L.tile == 16)
    hipLaunchKernelGGL(dmk::k_object<16>, dim3(L.ntiles), dim3(256), 0, c->stream, c->opart(),
                       c->D(), c->O(), c->pos(), c->tile_ptr(), c->tile_views(), d.frame,
                       d.obj_h, d.obj_w, L.tiles_x, c->err_obj());
  else
    hipLaunchKernelGGL(dmk::k_object<32>, dim3(L.ntiles), dim3(256), 0, c->stream, c->opart(),
                       c->D(), c->O(), c->pos(), c->tile_ptr(), c->tile_views(), d.frame,
                       d.obj_h, d.obj_w, L.tiles_x, c->err_obj());
  DM_LAUNCHED(c, "k_object");
  DM_TRY(phase_end(c, mk));
  DM_TRY(phase_begin(c, DM_PHASE_PROBE_PARTIAL, &mk));
  hipLaunchKernelGGL(dmk::k_probe_partial, dim3(L.n_pblk, L.C), dim3(256), 0, c->stream,
                     c->psi(), c->O(), c->pos(), c->order(), d.n_frames, d.n_modes, d.frame,
                     d.obj_w, L.chunk, c->num_part(), c->den_part());
  DM_LAUNCHED(c, "k_probe_partial");
  DM_TRY(phase_end(c, mk));
  DM_TRY(phase_begin(c, DM_PHASE_PROBE_FINAL, &mk));
  hipLaunchKernelGGL(dmk::k_probe_final, dim3(L.n_pblk), dim3(256), 0, c->stream, c->num_part(),
                     c->den_part(), c->P(), c->D(), L.C, d.n_modes, FF, c->err_probe());
  DM_LAUNCHED(c, "k_probe_final");
  DM_TRY(phase_end(c, mk));
  DM_TRY(phase_begin(c, DM_PHASE_ERRORS, &mk));
  hipLaunchKernelGGL(dmk::k_errors, dim3(1), dim3(256), 0, c->stream, c->err_psi(),
                     L.n_psi_parts, c->err_obj(), L.ntiles, c->err_probe(), L.n_pblk, d.n_modes,
                     c->counter(), c->ring(), c->flags());
  DM_LAUNCHED(c, "k_errors");
  DM_TRY(phase_end(c, mk));
  if (c->timing()) c->timed_iters++;
  return DM_OK;
}

dm_status refresh_mode_power(dm_ctx* c) {
  const int FF = c->d.frame * c->d.frame;
  hipLaunchKernelGGL(dmk::k_mode_power, dim3((FF + 255) / 256), dim3(256), 0, c->stream, c->P(),
                     c->D(), c->d.n_modes, FF);
  DM_LAUNCHED(c, "k_mode_power");
  return DM_OK;
}

hipError_t set_cols_lds(int F, int bytes) {
  const void* k = nullptr;
  switch (F) {
    case 16: k = reinterpret_cast<const void*>(dmk::k_cols<16>); break;
    case 32: k = reinterpret_cast<const void*>(dmk::k_cols<32>); break;
    case 64: k = reinterpret_cast<const void*>(dmk::k_cols<64>); break;
    case 128: k = reinterpret_cast<const void*>(dmk::k_cols<128>); break;
    case 256: k = reinterpret_cast<const void*>(dmk::k_cols<256>); break;
  }
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace

extern "C" {

size_t dm_workspace_bytes(const dm_desc* desc) {
  std::string why;
  if (validate_desc(desc, why) != DM_OK) return 0;
  return make_layout(*desc).total;
}

dm_status dm_init(dm_ctx** out, const dm_desc* desc, const float* I_dev, const int32_t* pos_host,
                  const void* probe0_dev, const void* object0_dev, void* workspace_dev,
                  size_t workspace_bytes, void* hip_stream) {
  g_init_error.clear();
  if (!out) { g_init_error = "out is NULL"; return DM_E_ARG; }
  *out = nullptr;
  std::string why;
  dm_status s = validate_desc(desc, why);
  if (s != DM_OK) { g_init_error = why; return s; }
  const dm_desc& d = *desc;
  if (!I_dev || !pos_host || !probe0_dev || !object0_dev || !workspace_dev) {
    g_init_error = "a required pointer is NULL";
    return DM_E_ARG;
  }
  if (!aligned8(I_dev) || !aligned8(probe0_dev) || !aligned8(object0_dev)) {
    g_init_error = "device buffers must be 8-byte aligned";
    return DM_E_ARG;
  }
  if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) {
    g_init_error = "workspace must be 256-byte aligned";
    return DM_E_ARG;
  }
  for (int j = 0; j < d.n_frames; ++j) {
    const int y = pos_host[2 * j], x = pos_host[2 * j + 1];
    if (y < 0 || x < 0 || y > d.obj_h - d.frame || x > d.obj_w - d.frame) {
      char msg[160];
      snprintf(msg, sizeof msg, "view %d at (y=%d, x=%d) leaves the %dx%d object", j, y, x,
               d.obj_h, d.obj_w);
      g_init_error = msg;
      return DM_E_BOUNDS;
    }
  }
  Layout L = make_layout(d);
  if (workspace_bytes < L.total) {
    char msg[160];
    snprintf(msg, sizeof msg, "workspace of %zu bytes, %zu needed", workspace_bytes, L.total);
    g_init_error = msg;
    return DM_E_WORKSPACE;
  }

  dm_ctx* c = new (std::nothrow) dm_ctx();
  if (!c) { g_init_error = "out of host memory"; return DM_E_ARG; }
  c->d = d;
  c->L = L;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char*>(workspace_dev);
  c->I = I_dev;
  c->pos_host.assign(pos_host, pos_host + 2 * (size_t)d.n_frames);

  std::vector<int> ptr, views;
  build_tile_lists(d, L, pos_host, ptr, views);
  if ((int)views.size() > L.nnz_max) {
    g_init_error = "internal: tile list larger than its bound";
    delete c;
    return DM_E_ARG;
  }
  std::vector<float2> tw = twiddles(d.frame);
  std::vector<int> order = spatial_order(d, pos_host);
  const size_t M = d.n_modes, FF = (size_t)d.frame * d.frame;

  auto bail = [&](dm_status st) {
    g_init_error = c->err;
    delete c;
    return st;
  };
  dm_status st;
#define INIT_HIP(call)                                          \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return bail(fail_hip(c, e_, #call));  \
  } while (0)

  INIT_HIP(hipMemcpyAsync(c->pos(), pos_host, 2 * sizeof(int) * d.n_frames,
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->tile_ptr(), ptr.data(), ptr.size() * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->tile_views(), views.data(), views.size() * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->tw(), tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice,
                          c->stream));
  INIT_HIP(hipMemcpyAsync(c->order(), order.data(), order.size() * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->P(), probe0_dev, M * FF * 8, hipMemcpyDeviceToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->O(), object0_dev, (size_t)d.obj_h * d.obj_w * 8,
                          hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->counter(), 2, 0);
  INIT_HIP(hipGetLastError());
  if (!use_fused(d)) {
    const int lds = (int)((size_t)L.cb * d.n_modes * (d.frame + 1) * sizeof(float2));
    INIT_HIP(set_cols_lds(d.frame, lds));
  }
  const size_t nI = (size_t)d.n_frames * FF;
  hipLaunchKernelGGL(dmk::k_check_finite, dim3(1024), dim3(256), 0, c->stream, I_dev, nI,
                     c->flags());
  INIT_HIP(hipGetLastError());
  hipLaunchKernelGGL(dmk::k_init_psi, dim3(d.n_frames * d.n_modes), dim3(256), 0, c->stream,
                     c->psi(), c->P(), c->O(), c->pos(), d.n_modes, d.frame, d.obj_w);
  INIT_HIP(hipGetLastError());
  st = refresh_mode_power(c);
  if (st != DM_OK) return bail(st);
  int flags_host[2] = {0, 0};
  INIT_HIP(hipMemcpyAsync(flags_host, c->counter(), sizeof flags_host, hipMemcpyDeviceToHost,
                          c->stream));
  INIT_HIP(hipStreamSynchronize(c->stream));
  if (flags_host[1] & 2) {
    c->err = "intensities contain NaN or Inf";
    return bail(DM_E_ARG);
  }
#undef INIT_HIP
  *out = c;
  return DM_OK;
}

dm_status dm_iterate(dm_ctx* c, int32_t n_iter) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (n_iter < 0) { c->err = "n_iter < 0"; return DM_E_ARG; }
  for (int i = 0; i < n_iter; ++i) {
    s = launch_iteration(c);
    if (s != DM_OK) return s;
    c->iters++;
  }
  return DM_OK;
}

dm_status dm_get_object(dm_ctx* c, void* dst) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!dst) { c->err = "dst is NULL"; return DM_E_ARG; }
  DM_HIP(c, hipMemcpyAsync(dst, c->O(), (size_t)c->d.obj_h * c->d.obj_w * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  return DM_OK;
}

dm_status dm_get_probe(dm_ctx* c, void* dst) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!dst) { c->err = "dst is NULL"; return DM_E_ARG; }
  DM_HIP(c, hipMemcpyAsync(dst, c->P(), (size_t)c->d.n_modes * c->d.frame * c->d.frame * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  return DM_OK;
}

static dm_status read_errors(dm_ctx* c, int first, int count, dm_errors* out) {
  std::vector<DevErrors> tmp(count);
  int flags_host[2];
  for (int i = 0; i < count; ++i) {
    const int slot = (first - 1 + i) % dmk::kRing;
    DM_HIP(c, hipMemcpyAsync(&tmp[i], c->ring() + slot, sizeof(DevErrors),
                             hipMemcpyDeviceToHost, c->stream));
  }
  DM_HIP(c, hipMemcpyAsync(flags_host, c->counter(), sizeof flags_host, hipMemcpyDeviceToHost,
                           c->stream));
  DM_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, tmp.data(), sizeof(dm_errors) * count);
  if (flags_host[1] & 1) {
    c->err = "a non-finite error norm was produced (the iteration diverged)";
    return DM_E_NUMERIC;
  }
  return DM_OK;
}

dm_status dm_error(dm_ctx* c, dm_errors* out) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!out) { c->err = "out is NULL"; return DM_E_ARG; }
  if (c->iters == 0) {
    std::memset(out, 0, sizeof *out);
    return DM_OK;
  }
  return read_errors(c, c->iters, 1, out);
}

dm_status dm_error_history(dm_ctx* c, int32_t first, int32_t count, dm_errors* out) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!out || count < 0) { c->err = "bad arguments"; return DM_E_ARG; }
  if (count == 0) return DM_OK;
  if (first < 1 || first + count - 1 > c->iters || c->iters - first + 1 > dmk::kRing) {
    c->err = "requested iterations are not in the error ring";
    return DM_E_ARG;
  }
  return read_errors(c, first, count, out);
}

int32_t dm_iterations(const dm_ctx* c) { return c ? c->iters : -1; }

dm_status dm_get_state(dm_ctx* c, void* psi_dst, void* probe_dst, void* object_dst,
                       int32_t* iter_host) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  const dm_desc& d = c->d;
  const size_t FF = (size_t)d.frame * d.frame;
  if (psi_dst)
    DM_HIP(c, hipMemcpyAsync(psi_dst, c->psi(), (size_t)d.n_frames * d.n_modes * FF * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  if (probe_dst)
    DM_HIP(c, hipMemcpyAsync(probe_dst, c->P(), (size_t)d.n_modes * FF * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  if (object_dst)
    DM_HIP(c, hipMemcpyAsync(object_dst, c->O(), (size_t)d.obj_h * d.obj_w * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  DM_HIP(c, hipStreamSynchronize(c->stream));
  if (iter_host) *iter_host = c->iters;
  return DM_OK;
}

dm_status dm_set_state(dm_ctx* c, const void* psi_src, const void* probe_src,
                       const void* object_src, int32_t iter) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!psi_src || !probe_src || !object_src || iter < 0) {
    c->err = "dm_set_state needs psi, probe, object and iter >= 0";
    return DM_E_ARG;
  }
  const dm_desc& d = c->d;
  const size_t FF = (size_t)d.frame * d.frame;
  DM_HIP(c, hipMemcpyAsync(c->psi(), psi_src, (size_t)d.n_frames * d.n_modes * FF * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->P(), probe_src, (size_t)d.n_modes * FF * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->O(), object_src, (size_t)d.obj_h * d.obj_w * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  s = refresh_mode_power(c);
  if (s != DM_OK) return s;
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->counter(), 1, iter);
  DM_LAUNCHED(c, "k_fill_int");
  c->iters = iter;
  return DM_OK;
}

dm_status dm_phase_times(dm_ctx* c, double* ms_host, int32_t* n_iter_host) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!c->timing()) {
    c->err = "phase timing was not enabled (DM_FLAG_PHASE_TIMING)";
    return DM_E_STATE;
  }
  if (!ms_host) { c->err = "ms_host is NULL"; return DM_E_ARG; }
  DM_HIP(c, hipStreamSynchronize(c->stream));
  double acc[DM_N_PHASES] = {0, 0, 0, 0, 0};
  for (auto& m : c->marks) {
    float ms = 0.f;
    DM_HIP(c, hipEventElapsedTime(&ms, m.a, m.b));
    acc[m.phase] += ms;
    c->event_pool.push_back(m.a);
    c->event_pool.push_back(m.b);
  }
  c->marks.clear();
  for (int i = 0; i < DM_N_PHASES; ++i) ms_host[i] = acc[i];
  if (n_iter_host) *n_iter_host = c->timed_iters;
  c->timed_iters = 0;
  return DM_OK;
}

void dm_free(dm_ctx* c) { delete c; }

const char* dm_status_str(dm_status s) {
  switch (s) {
    case DM_OK: return "DM_OK";
    case DM_E_ARG: return "DM_E_ARG: invalid argument";
    case DM_E_UNSUPPORTED: return "DM_E_UNSUPPORTED: configuration not supported";
    case DM_E_BOUNDS: return "DM_E_BOUNDS: a view window leaves the object";
    case DM_E_WORKSPACE: return "DM_E_WORKSPACE: workspace too small";
    case DM_E_HIP: return "DM_E_HIP: HIP runtime error";
    case DM_E_STATE: return "DM_E_STATE: context failed or call out of order";
    case DM_E_NUMERIC: return "DM_E_NUMERIC: non-finite error norm";
  }
  return "unknown dm_status";
}

const char* dm_last_error(const dm_ctx* c) {
  if (!c) return g_init_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
