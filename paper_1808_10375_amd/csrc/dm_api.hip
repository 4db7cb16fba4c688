// dm_api.hip -- host side of libdm: the C-ABI declared in include/dm.h.
// Validation, workspace carving, object-tile -> view lists, spatial view
// order, the launch chain of one difference-map iteration (Section II,
// Eqs. 2-6 of arXiv:1808.10375) for a batch of scans, its hipGraph capture,
// and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dm.h"
#include "dm_kernels.hpp"
#include "dm_mfma.hpp"
#include "dm_mixed.hpp"
#include "dm_order.hpp"
#include "dm_modes.hpp"
#include "dm_ortho.hpp"

using dmk::DevErrors;
using dmk::ScanDev;
static_assert(sizeof(DevErrors) == sizeof(dm_errors), "error record layout");

namespace {

thread_local std::string g_init_error;

constexpr size_t kAlign = 256;
// thread groups per object tile in the Eq. 5 gather (views in flight)
constexpr int kObjGroups = 4;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
// frame edges that are not powers of two: F = R * Q (dm_mixed.hpp)
bool is_mixed(int F) { return F == 188 || F == 200; }

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
int n_pblk(int F) { return (F * F + 255) / 256; }

// view chunks of the probe partial sums: about 1024 blocks of 256 pixels,
// four per compute unit (dm_autotune chose half the earlier 2048 at 2500 x
// 5 x 128^2, 10000 x 8 x 256^2 and 10000 x 4 x 188^2: 0.27 against 0.29 ms
// for the sums and the final division at 128^2, equal at the other two)
int default_chunks(int F) {
  int C = (1024 + n_pblk(F) - 1) / n_pblk(F);
  return std::max(1, std::min(C, DM_MAX_PROBE_CHUNKS));
}

bool is_bf16x3(const dm_desc& d) { return d.precision == DM_BF16X3_DFT; }

// object modes L (n_obj_modes 0 means 1)
int obj_modes(const dm_desc& d) { return d.n_obj_modes > 1 ? d.n_obj_modes : 1; }

// frames per view: the L M pairs (probe mode k, object mode l) of Eqs. 1-5
int frames_per_view(const dm_desc& d) { return d.n_modes * obj_modes(d); }

// Object modes run on the three-kernel path only (its kernels index the
// (k, l) pairs); so do F = 256 and the mixed-radix sizes.
bool has_spectrum_buffer(const dm_desc& d) {
  return d.frame == 256 || is_mixed(d.frame) || (d.flags & DM_FLAG_MULTIPASS) || is_bf16x3(d) ||
         obj_modes(d) > 1;
}

dm_tuning default_tuning(const dm_desc& d) {
  dm_tuning t{};
  t.obj_tile = 16;
  t.probe_chunks = default_chunks(d.frame);
  // F = 128: the streamed kernel with the merged update (the fused one
  // cannot hold a view in registers there); smaller frames: the fused kernel
  t.view_path = (has_spectrum_buffer(d) && !is_bf16x3(d)) ? DM_VIEWS_THREE_KERNEL
                : (d.frame == 128 && !is_bf16x3(d))      ? DM_VIEWS_STREAMED_MERGED
                                                          : DM_VIEWS_FUSED;
  return t;
}

// dynamic LDS of k_cols: the exchange buffer (cb * M lines of
// 16 (F / 16 + 1) + 2 complex) or, aliasing it, the mode-sum and scale rows
// ((M + 1) * cb rows of F + 4 floats), whichever is larger
size_t cols_lds_bytes(int F, int M, int cb) {
  const size_t line = 16 * (F / 16 + 1) + 2;
  return std::max((size_t)cb * M * line * sizeof(float2),
                  (size_t)(M + 1) * cb * (F + 4) * sizeof(float));
}

// columns per block of the power-of-two column kernel: a power of two up to
// 16 with CB * B * M threads at most 256 (at least one column).  With the
// k-major spectrum buffer, smaller blocks let one block's barriers overlap
// another's memory traffic: at 10000 x 8 x 256^2 the view update takes
// 68.5 ms with 256-thread blocks, 69.0 ms with 512 and 69.8 ms with 1024.
int cols_per_block(int F, int M) {
  const int B = F / 16;
  int cb = 256 / (B * M);
  int p = 1;
  while (p * 2 <= cb && p * 2 <= 16 && cols_lds_bytes(F, M, p * 2) <= 160 * 1024) p *= 2;
  return p;
}

// rows per block of the power-of-two row kernels, taken from their own
// RowCfg so that the eps_psi partials they write always fit the buffer sized
// from it
int row_block(int F) {
  switch (F) {
    case 16: return dmk::RowCfg<16>::RB;
    case 32: return dmk::RowCfg<32>::RB;
    case 64: return dmk::RowCfg<64>::RB;
    case 128: return dmk::RowCfg<128>::RB;
    case 256: return dmk::RowCfg<256>::RB;
  }
  return F;
}

// row blocks per frame of the three-kernel path (one eps_psi partial each)
int row_parts(int F) {
  switch (F) {
    case 188: return dmk::Mix<188>::NBLK;
    case 200: return dmk::Mix<200>::NBLK;
  }
  return F / row_block(F);
}

// threads per line of the mixed-radix transforms (Q + 1)
int mix_qt(int F) { return F == 188 ? dmk::Mix<188>::QT : dmk::Mix<200>::QT; }

// columns per block of the mixed-radix column kernel: a power of two up to
// 16 with CB * M * (Q + 1) threads (rounded to whole waves) at most 512.
// The kernel is bound by its arithmetic and barriers, and smaller blocks
// overlap one block's barriers with another's work: at 10000 x 4 x 188^2
// blocks of 384 threads (CB = 2) take 12.6 ms against 15.0 ms with 768
// (CB = 4); with 192 (CB = 1) the view update is 1.3 ms slower again.
int mix_cols_per_block(int F, int M) {
  const int QT = mix_qt(F);
  int p = 1;
  while (p * 2 <= 16 && ((p * 2 * M * QT + 63) / 64) * 64 <= 512) p *= 2;
  return p;
}

int mix_cols_threads(int F, int M, int cb) { return ((cb * M * mix_qt(F) + 63) / 64) * 64; }

// dynamic LDS of the mixed-radix column kernel: cb * M exchange lines of
// Q * R + 2 complex values, the mode powers [M][cb][F], the scale [cb][F]
// and the twiddle tables (F + Q complex)
size_t mix_cols_lds_bytes(int F, int M, int cb) {
  const int Q = mix_qt(F) - 1;
  return (size_t)cb * M * (F + 2) * sizeof(float2) + (size_t)(M + 1) * cb * F * sizeof(float) +
         (size_t)(F + Q) * sizeof(float2);
}

// ---------------------------------------------------------------------------
// workspace carving: a context header, then one region per scan
// ---------------------------------------------------------------------------
struct ScanLayout {
  size_t psi, opart, gscr, tspec, P, O, D, num_part, den_part, err_psi, err_obj, err_probe,
      ring, counter, mode_pow, ortho, pos, order, tile_ptr, tile_views, bytes;
  int ntiles16, nnz16, n_psi_parts_fused, n_psi_parts_multi;
};

int tiles_for(int H, int W, int T) { return ((H + T - 1) / T) * ((W + T - 1) / T); }

int nnz_bound(const dm_desc& d, int T) {
  const int span = d.frame / T + 1 + (d.frame % T ? 1 : 0);
  return d.n_frames * span * span;
}

ScanLayout scan_layout(const dm_desc& d) {
  ScanLayout L{};
  const size_t N = d.n_frames, M = frames_per_view(d), F = d.frame, FF = F * F;
  const size_t NL = obj_modes(d);
  const size_t c8 = 8;
  // eps_psi partial sums per view: 1 (fused), F / row block (three-kernel
  // FFT path), 2 (BF16x3 path, two row halves)
  L.ntiles16 = tiles_for(d.obj_h, d.obj_w, 16);  // the larger of the two tile counts
  L.nnz16 = std::max(nnz_bound(d, 16), nnz_bound(d, 32));
  L.n_psi_parts_fused = (int)N;
  L.n_psi_parts_multi = (int)N * row_parts((int)F);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.psi = take(N * M * FF * c8);
  L.opart = take(N * NL * FF * c8);
  L.gscr = d.frame <= 128 ? take(N * FF * 4) : 0;
  L.tspec = has_spectrum_buffer(d) ? take(N * M * FF * c8) : 0;
  L.P = take(M * FF * c8);
  L.O = take(NL * d.obj_h * d.obj_w * c8);
  L.D = take(FF * 4);
  L.num_part = take((size_t)DM_MAX_PROBE_CHUNKS * d.n_modes * FF * c8);
  L.den_part = take((size_t)DM_MAX_PROBE_CHUNKS * FF * 4);
  L.err_psi = take((size_t)std::max({L.n_psi_parts_fused, L.n_psi_parts_multi, 2 * (int)N}) *
                   2 * 4);
  L.err_obj = take((size_t)L.ntiles16 * NL * 2 * 4);
  L.err_probe = take((size_t)n_pblk((int)F) * d.n_modes * 2 * 4);
  L.ring = take(sizeof(DevErrors) * dmk::kRing);
  L.counter = take(sizeof(int));
  L.mode_pow = take(DM_MAX_MODES * sizeof(double));
  L.ortho = take(dmk::kOrthoScratchBytes);
  L.pos = take(N * 2 * 4);
  L.order = take(N * 4);
  L.tile_ptr = take(((size_t)L.ntiles16 + 1) * 4);
  L.tile_views = take((size_t)L.nnz16 * 4);
  L.bytes = off;
  return L;
}

// persistent workgroups of the streamed view path: one per compute unit of
// an MI355X, fewer when the batch has fewer views
constexpr int kStreamSlots = 256;

int stream_slots(int n_scans, const dm_desc* d) {
  size_t views = 0;
  for (int s = 0; s < n_scans; ++s) views += d[s].n_frames;
  return (int)std::min<size_t>(views, kStreamSlots);
}

struct CtxLayout {
  size_t scans, vmap, tmap, cmap, tw, wf, vscr, flags, header;
  std::vector<size_t> scan_base;
  std::vector<ScanLayout> sl;
  size_t total;
};

CtxLayout ctx_layout(int n_scans, const dm_desc* d) {
  CtxLayout C{};
  size_t views = 0, tiles = 0;
  for (int s = 0; s < n_scans; ++s) {
    views += d[s].n_frames;
    tiles += tiles_for(d[s].obj_h, d[s].obj_w, 16);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  C.scans = take(sizeof(ScanDev) * n_scans);
  C.vmap = take(sizeof(int2) * views);
  C.tmap = take(sizeof(int2) * tiles);
  C.cmap = take(sizeof(int2) * (size_t)DM_MAX_PROBE_CHUNKS * n_scans);
  C.tw = take(sizeof(float2) * d[0].frame);
  C.wf = is_bf16x3(d[0]) ? take(sizeof(uint4) * dmk::kMfWords) : 0;
  // spectra of the view in hand and its modulus scale, per persistent
  // workgroup of the streamed path: [slot]([M][F][F] complex64, [F][F] float)
  C.vscr = (!is_bf16x3(d[0]) && d[0].frame <= 128)
               ? take((size_t)stream_slots(n_scans, d) * d[0].frame * d[0].frame *
                      (8 * (size_t)d[0].n_modes + 4))
               : 0;
  // [0]: bit 2 = non-finite intensities at init; [1 + s]: bit 1 = a
  // non-finite error norm in scan s since its state was last set
  C.flags = take(sizeof(int) * (1 + (size_t)n_scans));
  C.header = off;
  for (int s = 0; s < n_scans; ++s) {
    C.sl.push_back(scan_layout(d[s]));
    C.scan_base.push_back(off);
    off = align_up(off + C.sl.back().bytes);
  }
  C.total = off;
  return C;
}

dm_status validate_desc(const dm_desc* d, std::string& why) {
  if (!d) { why = "desc is NULL"; return DM_E_ARG; }
  if (d->n_frames < 1) { why = "n_frames must be >= 1"; return DM_E_ARG; }
  if (d->n_modes < 1) { why = "n_modes must be >= 1"; return DM_E_ARG; }
  if (d->n_modes > DM_MAX_MODES) { why = "n_modes > 16 not supported"; return DM_E_UNSUPPORTED; }
  if (!(is_pow2(d->frame) && d->frame >= 16 && d->frame <= 256) && !is_mixed(d->frame)) {
    why = "frame must be a power of two in [16, 256], 188 or 200";
    return DM_E_UNSUPPORTED;
  }
  if (d->obj_h < d->frame || d->obj_w < d->frame) { why = "object smaller than a frame"; return DM_E_ARG; }
  if (!(d->beta >= 0.f && d->beta <= 1.f)) { why = "beta must lie in [0, 1]"; return DM_E_ARG; }
  if (d->precision != DM_FP32_FFT && d->precision != DM_BF16X3_DFT) {
    why = "unknown precision";
    return DM_E_UNSUPPORTED;
  }
  if (d->precision == DM_BF16X3_DFT && d->frame != dmk::kMfF) {
    why = "the BF16x3 DFT form is built for 128 x 128 frames";
    return DM_E_UNSUPPORTED;
  }
  if (d->precision == DM_BF16X3_DFT && d->n_modes > dmk::kMfMaxModes) {
    why = "the BF16x3 DFT form takes at most 8 modes";
    return DM_E_UNSUPPORTED;
  }
  if (d->flags &
      ~(DM_FLAG_MULTIPASS | DM_FLAG_PHASE_TIMING | DM_FLAG_GRAPH | DM_FLAG_PSI_ERROR_LAST |
        DM_FLAG_PROBE_FIRST)) {
    why = "unknown flag bits";
    return DM_E_ARG;
  }
  if ((d->flags & DM_FLAG_GRAPH) && (d->flags & DM_FLAG_PHASE_TIMING)) {
    why = "DM_FLAG_GRAPH and DM_FLAG_PHASE_TIMING exclude each other";
    return DM_E_ARG;
  }
  if ((double)d->obj_h * d->obj_w * 8.0 >= 2147483648.0) {
    why = "object larger than 2^28 pixels";
    return DM_E_UNSUPPORTED;
  }
  if (d->n_obj_modes < 0) { why = "n_obj_modes must be >= 0"; return DM_E_ARG; }
  if (obj_modes(*d) > 1) {
    const int L = obj_modes(*d);
    if (L > DM_MAX_OBJ_MODES || L * d->n_modes > DM_MAX_PAIRS) {
      why = "object modes: at most 4, and at most 32 (probe mode, object mode) pairs";
      return DM_E_UNSUPPORTED;
    }
    if (d->precision != DM_FP32_FFT || is_mixed(d->frame)) {
      why = "object modes run on the FP32 three-kernel path with power-of-two frames";
      return DM_E_UNSUPPORTED;
    }
    if ((double)L * d->obj_h * d->obj_w * 8.0 >= 2147483648.0) {
      why = "object modes larger than 2^28 pixels together";
      return DM_E_UNSUPPORTED;
    }
  }
  if ((double)d->n_frames * d->frame * d->frame >= 2147483648.0) {
    why = "more than 2^31 detector pixels in one scan";
    return DM_E_UNSUPPORTED;
  }
  return DM_OK;
}

dm_status validate_batch(int n_scans, const dm_desc* d, std::string& why) {
  if (n_scans < 1 || !d) { why = "need at least one scan"; return DM_E_ARG; }
  for (int s = 0; s < n_scans; ++s) {
    dm_status st = validate_desc(&d[s], why);
    if (st != DM_OK) {
      if (n_scans > 1) why = "scan " + std::to_string(s) + ": " + why;
      return st;
    }
    if (d[s].frame != d[0].frame || d[s].n_modes != d[0].n_modes ||
        d[s].precision != d[0].precision || d[s].flags != d[0].flags ||
        obj_modes(d[s]) != obj_modes(d[0])) {
      why = "all scans of a batch need the same frame, n_modes, n_obj_modes, precision and "
            "flags";
      return DM_E_ARG;
    }
  }
  return DM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct dm_ctx {
  struct Scan {
    dm_desc d;
    ScanLayout L;
    size_t base;
    const float* I;
    const void* P0;  // caller's initial guesses (used again only by dm_autotune)
    const void* O0;
    std::vector<int> pos, order;
    int C = 1, chunk = 1, ntiles = 0, tiles_x = 0;
  };
  std::vector<Scan> scans;
  CtxLayout CL;
  int F = 0, M = 0;
  int L = 1;  // object modes (the views hold L M frames)
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  bool failed = false;
  std::string err;
  int iters = 0;
  // iterations up to this one were not run by this context since its state
  // was last set (dm_set_state): their error records are not valid
  int first_iter = 0;
  int total_views = 0, total_tiles = 0, total_chunks = 0;
  int stream_slots = 0;
  dm_tuning tune{};
  // graph of one iteration
  // graphs of one iteration: [0] without, [1] with the eps_psi partials
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  // phase timing
  struct Mark { int phase; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  int timed_iters = 0;

  ~dm_ctx() {
    for (auto& m : marks) { event_pool.push_back(m.a); event_pool.push_back(m.b); }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k) {
      if (graph_exec[k]) (void)hipGraphExecDestroy(graph_exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
    }
  }
  bool timing() const { return (flags & DM_FLAG_PHASE_TIMING) != 0; }
  template <class T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  template <class T>
  T* sat(int s, size_t off) { return reinterpret_cast<T*>(ws + scans[s].base + off); }
  ScanDev* scan_dev() { return at<ScanDev>(CL.scans); }
  int2* vmap() { return at<int2>(CL.vmap); }
  int2* tmap() { return at<int2>(CL.tmap); }
  int2* cmap() { return at<int2>(CL.cmap); }
  float2* tw() { return at<float2>(CL.tw); }
  float2* vscr() { return at<float2>(CL.vscr); }
  const uint4* wf() { return at<uint4>(CL.wf); }
  bool bf16x3() const { return is_bf16x3(scans[0].d); }
  int* flags_dev() { return at<int>(CL.flags); }
  int n_flags() const { return 1 + (int)scans.size(); }
};

namespace {

dm_status fail_hip(dm_ctx* c, hipError_t e, const char* where) {
  c->failed = true;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return DM_E_HIP;
}

#define DM_HIP(ctx, call)                                    \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, #call); \
  } while (0)

#define DM_LAUNCHED(ctx, name)                              \
  do {                                                      \
    hipError_t e_ = hipGetLastError();                      \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, name); \
  } while (0)

#define DM_TRY(expr)            \
  do {                          \
    dm_status s_ = (expr);      \
    if (s_ != DM_OK) return s_; \
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

// Lists of views whose window meets each T x T object tile, ascending view
// order.
void build_tile_lists(const dm_desc& d, int T, const std::vector<int>& pos,
                      std::vector<int>& ptr, std::vector<int>& views) {
  const int F = d.frame;
  const int tx_n = (d.obj_w + T - 1) / T, ty_n = (d.obj_h + T - 1) / T;
  const int ntiles = tx_n * ty_n;
  std::vector<int> count(ntiles, 0);
  for (int j = 0; j < d.n_frames; ++j) {
    const int y = pos[2 * j], x = pos[2 * j + 1];
    for (int ty = y / T; ty <= (y + F - 1) / T; ++ty)
      for (int tx = x / T; tx <= (x + F - 1) / T; ++tx) count[ty * tx_n + tx]++;
  }
  ptr.assign(ntiles + 1, 0);
  for (int i = 0; i < ntiles; ++i) ptr[i + 1] = ptr[i] + count[i];
  views.assign(std::max(ptr[ntiles], 1), 0);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int j = 0; j < d.n_frames; ++j) {
    const int y = pos[2 * j], x = pos[2 * j + 1];
    for (int ty = y / T; ty <= (y + F - 1) / T; ++ty)
      for (int tx = x / T; tx <= (x + F - 1) / T; ++tx) views[fill[ty * tx_n + tx]++] = j;
  }
}

// Views sorted along a Z-order curve of their window corners: runs of
// consecutive entries cover compact patches of the object.
std::vector<int> spatial_order(const dm_desc& d, const std::vector<int>& pos) {
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

// (Re)build everything that depends on the tuning: tile lists, chunking, the
// scan descriptor table and the block maps; upload them.  Synchronises.
dm_status apply_tuning(dm_ctx* c, const dm_tuning& t) {
  c->tune = t;
  for (int k = 0; k < 2; ++k) {
    if (c->graph_exec[k]) { (void)hipGraphExecDestroy(c->graph_exec[k]); c->graph_exec[k] = nullptr; }
    if (c->graph[k]) { (void)hipGraphDestroy(c->graph[k]); c->graph[k] = nullptr; }
  }
  const int n = (int)c->scans.size();
  std::vector<ScanDev> sd(n);
  std::vector<int2> tmap, cmap;
  // host staging that must outlive the asynchronous copies below
  std::vector<std::vector<int>> ptrs(n), lists(n);
  for (int s = 0; s < n; ++s) {
    auto& S = c->scans[s];
    const ScanLayout& L = S.L;
    build_tile_lists(S.d, t.obj_tile, S.pos, ptrs[s], lists[s]);
    if ((int)lists[s].size() > L.nnz16) {
      c->err = "internal: tile list larger than its bound";
      return DM_E_STATE;
    }
    S.tiles_x = (S.d.obj_w + t.obj_tile - 1) / t.obj_tile;
    S.ntiles = (int)ptrs[s].size() - 1;
    S.C = std::max(1, std::min(t.probe_chunks, S.d.n_frames));
    S.chunk = (S.d.n_frames + S.C - 1) / S.C;
    S.C = (S.d.n_frames + S.chunk - 1) / S.chunk;  // no empty chunks
    DM_HIP(c, hipMemcpyAsync(c->sat<int>(s, L.tile_ptr), ptrs[s].data(),
                             ptrs[s].size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    DM_HIP(c, hipMemcpyAsync(c->sat<int>(s, L.tile_views), lists[s].data(),
                             lists[s].size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    ScanDev& v = sd[s];
    v.psi = c->sat<float2>(s, L.psi);
    v.I = S.I;
    v.P = c->sat<float2>(s, L.P);
    v.O = c->sat<float2>(s, L.O);
    v.pos = c->sat<int>(s, L.pos);
    v.order = c->sat<int>(s, L.order);
    v.opart = c->sat<float2>(s, L.opart);
    v.gscr = S.d.frame <= 128 ? c->sat<float>(s, L.gscr) : nullptr;
    v.tspec = L.tspec ? c->sat<float2>(s, L.tspec) : nullptr;
    v.D = c->sat<float>(s, L.D);
    v.num_part = c->sat<float2>(s, L.num_part);
    v.den_part = c->sat<float>(s, L.den_part);
    v.err_psi = c->sat<float>(s, L.err_psi);
    v.err_obj = c->sat<float>(s, L.err_obj);
    v.err_probe = c->sat<float>(s, L.err_probe);
    v.tile_ptr = c->sat<int>(s, L.tile_ptr);
    v.tile_views = c->sat<int>(s, L.tile_views);
    v.counter = c->sat<int>(s, L.counter);
    v.ring = c->sat<DevErrors>(s, L.ring);
    v.N = S.d.n_frames;
    v.H = S.d.obj_h;
    v.W = S.d.obj_w;
    v.tiles_x = S.tiles_x;
    v.ntiles = S.ntiles;
    v.C = S.C;
    v.chunk = S.chunk;
    v.n_psi_parts = is_bf16x3(S.d)  ? 2 * S.d.n_frames
                    : t.view_path == DM_VIEWS_THREE_KERNEL ? L.n_psi_parts_multi
                                    : L.n_psi_parts_fused;
    v.beta = S.d.beta;
    v.L = obj_modes(S.d);
    for (int i = 0; i < S.ntiles; ++i) tmap.push_back(make_int2(s, i));
    for (int i = 0; i < S.C; ++i) cmap.push_back(make_int2(s, i));
  }
  c->total_tiles = (int)tmap.size();
  c->total_chunks = (int)cmap.size();
  DM_HIP(c, hipMemcpyAsync(c->scan_dev(), sd.data(), sd.size() * sizeof(ScanDev),
                           hipMemcpyHostToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->tmap(), tmap.data(), tmap.size() * sizeof(int2),
                           hipMemcpyHostToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->cmap(), cmap.data(), cmap.size() * sizeof(int2),
                           hipMemcpyHostToDevice, c->stream));
  if (t.view_path == DM_VIEWS_THREE_KERNEL && is_mixed(c->F)) {
    const int lds = (int)mix_cols_lds_bytes(c->F, c->M, mix_cols_per_block(c->F, c->M));
    const void* k = c->F == 188 ? reinterpret_cast<const void*>(dmk::k_mix_cols<188>)
                                : reinterpret_cast<const void*>(dmk::k_mix_cols<200>);
    DM_HIP(c, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  } else if (t.view_path == DM_VIEWS_THREE_KERNEL) {
    const int MT = c->M * c->L;
    const int lds = (int)cols_lds_bytes(c->F, MT, cols_per_block(c->F, MT));
    DM_HIP(c, set_cols_lds(c->F, lds));
  }
  DM_HIP(c, hipStreamSynchronize(c->stream));
  return DM_OK;
}

// ---------------------------------------------------------------------------
// the iteration chain
// ---------------------------------------------------------------------------
hipError_t take_event(dm_ctx* c, hipEvent_t* e) {
  if (!c->event_pool.empty()) {
    *e = c->event_pool.back();
    c->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

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

// Virtual threads per thread of the fused view kernel.  Two at F = 128 (512
// threads, 256 VGPRs each) pass parity but run 1.4x slower than one (1024
// threads, 128 VGPRs), so every frame size uses one.
template <int F>
constexpr int fused_v() { return 1; }

template <int F>
dm_status launch_views_fused(dm_ctx* c) {
  constexpr int V = fused_v<F>();
  hipLaunchKernelGGL((dmk::k_fourier_fused<F, V>), dim3(c->total_views), dim3(F * F / (16 * V)),
                     0, c->stream, c->scan_dev(), c->vmap(), c->total_views, c->tw(), c->M);
  DM_LAUNCHED(c, "k_fourier_fused");
  return DM_OK;
}

// direct: psi' without a second read of psi (the eps_psi partials are not
// formed), as in the merged streamed kernels
template <int F>
dm_status launch_views_multipass(dm_ctx* c, bool direct) {
  constexpr int B = F / 16, RB = dmk::RowCfg<F>::RB, NT = dmk::RowCfg<F>::NT;
  const int M = c->M, MT = c->M * c->L;  // probe modes, frames per view
  hipLaunchKernelGGL(dmk::k_rows_fwd<F>, dim3(c->total_views, F / RB), dim3(NT), 0,
                     c->stream, c->scan_dev(), c->vmap(), c->tw(), M);
  DM_LAUNCHED(c, "k_rows_fwd");
  // the column kernel sums the modulus over all MT frames of a view
  const int cb = cols_per_block(F, MT);
  const size_t lds = cols_lds_bytes(F, MT, cb);
  hipLaunchKernelGGL(dmk::k_cols<F>, dim3(c->total_views * (F / cb)), dim3(cb * B * MT), lds,
                     c->stream, c->scan_dev(), c->vmap(), c->tw(), MT, cb, direct ? 1 : 0);
  DM_LAUNCHED(c, "k_cols");
  if (direct)
    hipLaunchKernelGGL(dmk::k_rows_inv_direct<F>, dim3(c->total_views, F / RB), dim3(NT), 0,
                       c->stream, c->scan_dev(), c->vmap(), c->tw(), M);
  else
    hipLaunchKernelGGL(dmk::k_rows_inv<F>, dim3(c->total_views, F / RB), dim3(NT), 0, c->stream,
                       c->scan_dev(), c->vmap(), c->tw(), M);
  DM_LAUNCHED(c, "k_rows_inv");
  return DM_OK;
}

// Frames of edge F = R * Q (188, 200): the same three passes with the
// mixed-radix line transforms.
template <int F>
dm_status launch_views_mixed(dm_ctx* c, bool direct) {
  using C = dmk::Mix<F>;
  const int M = c->M;
  hipLaunchKernelGGL(dmk::k_mix_rows_fwd<F>, dim3(c->total_views, C::NBLK), dim3(C::NT), 0,
                     c->stream, c->scan_dev(), c->vmap(), c->tw(), M);
  DM_LAUNCHED(c, "k_mix_rows_fwd");
  const int cb = mix_cols_per_block(F, M);
  hipLaunchKernelGGL(dmk::k_mix_cols<F>, dim3(c->total_views * ((F + cb - 1) / cb)),
                     dim3(mix_cols_threads(F, M, cb)), mix_cols_lds_bytes(F, M, cb), c->stream,
                     c->scan_dev(), c->vmap(), c->tw(), M, cb, direct ? 1 : 0);
  DM_LAUNCHED(c, "k_mix_cols");
  if (direct)
    hipLaunchKernelGGL(dmk::k_mix_rows_inv_direct<F>, dim3(c->total_views, C::NBLK),
                       dim3(C::NT), 0, c->stream, c->scan_dev(), c->vmap(), c->tw(), M);
  else
    hipLaunchKernelGGL(dmk::k_mix_rows_inv<F>, dim3(c->total_views, C::NBLK), dim3(C::NT), 0,
                       c->stream, c->scan_dev(), c->vmap(), c->tw(), M);
  DM_LAUNCHED(c, "k_mix_rows_inv");
  return DM_OK;
}

// BF16x3 form: three persistent kernels, one block per CU, each holding the
// split DFT matrix in LDS
constexpr size_t kMfLdsW = sizeof(uint4) * dmk::kMfWords;
constexpr size_t kMfLdsCols = kMfLdsW + 2 * 4 * dmk::kMfKs * 64 * 16;  // 160 KB

hipError_t set_mfma_lds() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(dmk::k_mf_rows_fwd),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMfLdsW);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(dmk::k_mf_cols),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMfLdsCols);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(dmk::k_mf_rows_inv),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMfLdsW);
  return e;
}

// The split DFT matrix in B-fragment order (see dm_mfma.hpp): W[a][b] =
// exp(-2 pi i ab / F) in double, rounded to float, split into bfloat16 hi
// and lo = bf16(x - hi), both rounded to nearest even.
std::vector<uint4> mfma_dft_table() {
  constexpr int F = dmk::kMfF;
  auto rne = [](float f) -> uint32_t {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  };
  auto bf = [](uint32_t h) -> float {
    const uint32_t u = h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
  };
  std::vector<uint16_t> half(4 * (size_t)dmk::kMfFrag * 8);
  const double pi = 3.14159265358979323846;
  for (int ks = 0; ks < dmk::kMfKs; ++ks)
    for (int nt = 0; nt < dmk::kMfNt; ++nt)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int k = 32 * ks + 8 * (lane / 16) + e, n = 16 * nt + lane % 16;
          const double ang = -2.0 * pi * (double)((k * n) % F) / (double)F;
          const float v[2] = {(float)std::cos(ang), (float)std::sin(ang)};
          for (int part = 0; part < 2; ++part) {
            const uint32_t hi = rne(v[part]);
            const uint32_t lo = rne(v[part] - bf(hi));
            const size_t slot = (((size_t)ks * dmk::kMfNt + nt) * 64 + lane) * 8 + e;
            half[(size_t)(2 * part) * dmk::kMfFrag * 8 + slot] = (uint16_t)hi;
            half[(size_t)(2 * part + 1) * dmk::kMfFrag * 8 + slot] = (uint16_t)lo;
          }
        }
  std::vector<uint4> out(dmk::kMfWords);
  std::memcpy(out.data(), half.data(), out.size() * sizeof(uint4));
  return out;
}

int mfma_grid(dm_ctx* c, int items) {
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        v > 0)
      cus = v;
  }
  (void)c;
  return std::max(1, std::min(items, cus));
}

dm_status launch_views_mfma(dm_ctx* c) {
  const int M = c->M, nv = c->total_views;
  hipLaunchKernelGGL(dmk::k_mf_rows_fwd, dim3(mfma_grid(c, nv * M)),
                     dim3(dmk::kMfRowsThreads), kMfLdsW,
                     c->stream, c->scan_dev(), c->vmap(), nv, M, c->wf());
  DM_LAUNCHED(c, "k_mf_rows_fwd");
  hipLaunchKernelGGL(dmk::k_mf_cols, dim3(mfma_grid(c, nv * dmk::kMfNt)),
                     dim3(dmk::kMfColsThreads), kMfLdsCols,
                     c->stream, c->scan_dev(), c->vmap(), nv, M, c->wf());
  DM_LAUNCHED(c, "k_mf_cols");
  hipLaunchKernelGGL(dmk::k_mf_rows_inv, dim3(mfma_grid(c, nv)), dim3(dmk::kMfRowsThreads),
                     kMfLdsW,
                     c->stream, c->scan_dev(), c->vmap(), nv, M, c->wf());
  DM_LAUNCHED(c, "k_mf_rows_inv");
  return DM_OK;
}

template <int F, bool PE>
void launch_merged(dm_ctx* c, int grid, int v) {
  if (v == 2)
    hipLaunchKernelGGL((dmk::k_fourier_stream<F, (F >= 32 ? 2 : 1), true, true, PE>), dim3(grid),
                       dim3(F * F / (16 * (F >= 32 ? 2 : 1))), 0, c->stream, c->scan_dev(),
                       c->vmap(), c->total_views, c->tw(), c->M, c->vscr());
  else
    hipLaunchKernelGGL((dmk::k_fourier_stream<F, 1, true, true, PE>), dim3(grid), dim3(F * F / 16),
                       0, c->stream, c->scan_dev(), c->vmap(), c->total_views, c->tw(), c->M,
                       c->vscr());
}

template <int F>
dm_status launch_views_streamed(dm_ctx* c, int vp, bool psi_err) {
  const int grid = std::min(c->total_views, c->stream_slots);
  if (vp == DM_VIEWS_STREAMED)
    hipLaunchKernelGGL((dmk::k_fourier_stream<F, 1, true, false>), dim3(grid), dim3(F * F / 16),
                       0, c->stream, c->scan_dev(), c->vmap(), c->total_views, c->tw(), c->M,
                       c->vscr());
  else if (vp == DM_VIEWS_STREAMED_CACHED)
    hipLaunchKernelGGL((dmk::k_fourier_stream<F, 1, false, false>), dim3(grid), dim3(F * F / 16),
                       0, c->stream, c->scan_dev(), c->vmap(), c->total_views, c->tw(), c->M,
                       c->vscr());
  else {
    const int v = (vp == DM_VIEWS_STREAMED_WIDE) ? 2 : 1;
    if (psi_err) launch_merged<F, true>(c, grid, v);
    else launch_merged<F, false>(c, grid, v);
  }
  DM_LAUNCHED(c, "k_fourier_stream");
  return DM_OK;
}

// *psi_valid: whether the launched kernels formed the eps_psi partials
dm_status launch_views(dm_ctx* c, bool psi_err, bool* psi_valid) {
  *psi_valid = true;
  if (c->bf16x3()) return launch_views_mfma(c);
  const int vp = c->tune.view_path;
  if (vp >= DM_VIEWS_STREAMED) {
    if (vp >= DM_VIEWS_STREAMED_MERGED) *psi_valid = psi_err;
    switch (c->F) {
      case 16: return launch_views_streamed<16>(c, vp, psi_err);
      case 32: return launch_views_streamed<32>(c, vp, psi_err);
      case 64: return launch_views_streamed<64>(c, vp, psi_err);
      case 128: return launch_views_streamed<128>(c, vp, psi_err);
    }
  }
  if (vp == DM_VIEWS_FUSED) {
    switch (c->F) {
      case 16: return launch_views_fused<16>(c);
      case 32: return launch_views_fused<32>(c);
      case 64: return launch_views_fused<64>(c);
      case 128: return launch_views_fused<128>(c);
    }
  } else {
    *psi_valid = psi_err;
    const bool direct = !psi_err;
    switch (c->F) {
      case 16: return launch_views_multipass<16>(c, direct);
      case 32: return launch_views_multipass<32>(c, direct);
      case 64: return launch_views_multipass<64>(c, direct);
      case 128: return launch_views_multipass<128>(c, direct);
      case 256: return launch_views_multipass<256>(c, direct);
      case 188: return launch_views_mixed<188>(c, direct);
      case 200: return launch_views_mixed<200>(c, direct);
    }
  }
  c->err = "unsupported frame size for this transform path";
  return DM_E_UNSUPPORTED;
}

// psi_err: form the eps_psi partial sums in this iteration (without them the
// merged streamed kernels and the three-kernel paths skip the second read of
// psi)
dm_status launch_iteration(dm_ctx* c, bool psi_err) {
  const int F = c->F, M = c->M, FF = F * F, nb = n_pblk(F);
  const int n = (int)c->scans.size();
  int mk;
  DM_TRY(phase_begin(c, DM_PHASE_VIEWS, &mk));
  bool psi_valid = true;
  DM_TRY(launch_views(c, psi_err, &psi_valid));
  DM_TRY(phase_end(c, mk));
  // Eq. 5 gather of the per-view numerators (with DM_FLAG_PROBE_FIRST the
  // numerators are formed again with the new probe first)
  auto object = [&]() -> dm_status {
    DM_TRY(phase_begin(c, DM_PHASE_OBJECT, &mk));
    if (c->flags & DM_FLAG_PROBE_FIRST) {
      hipLaunchKernelGGL(dmk::k_view_numerators, dim3(c->total_views, nb, c->L), dim3(256), 0,
                         c->stream, c->scan_dev(), c->vmap(), M, FF);
      DM_LAUNCHED(c, "k_view_numerators");
    }
    if (c->tune.obj_tile == 16)
      hipLaunchKernelGGL((dmk::k_object<16, kObjGroups>), dim3(c->total_tiles, c->L),
                         dim3(256 * kObjGroups), 0, c->stream, c->scan_dev(), c->tmap(), F);
    else
      hipLaunchKernelGGL((dmk::k_object<32, kObjGroups>), dim3(c->total_tiles, c->L),
                         dim3(256 * kObjGroups), 0, c->stream, c->scan_dev(), c->tmap(), F);
    DM_LAUNCHED(c, "k_object");
    return phase_end(c, mk);
  };
  // Eq. 4 from the new views and the object as it stands
  auto probe = [&]() -> dm_status {
    DM_TRY(phase_begin(c, DM_PHASE_PROBE_PARTIAL, &mk));
    hipLaunchKernelGGL(dmk::k_probe_partial, dim3(nb, c->total_chunks), dim3(256), 0, c->stream,
                       c->scan_dev(), c->cmap(), M, F);
    DM_LAUNCHED(c, "k_probe_partial");
    DM_TRY(phase_end(c, mk));
    DM_TRY(phase_begin(c, DM_PHASE_PROBE_FINAL, &mk));
    hipLaunchKernelGGL(dmk::k_probe_final, dim3(nb, n), dim3(256), 0, c->stream, c->scan_dev(),
                       M, FF);
    DM_LAUNCHED(c, "k_probe_final");
    return phase_end(c, mk);
  };
  if (c->flags & DM_FLAG_PROBE_FIRST) {
    DM_TRY(probe());
    DM_TRY(object());
  } else {
    DM_TRY(object());
    DM_TRY(probe());
  }
  DM_TRY(phase_begin(c, DM_PHASE_ERRORS, &mk));
  hipLaunchKernelGGL(dmk::k_errors, dim3(n), dim3(256), 0, c->stream, c->scan_dev(), nb, M,
                     c->flags_dev(), psi_valid ? 1 : 0);
  DM_LAUNCHED(c, "k_errors");
  DM_TRY(phase_end(c, mk));
  if (c->timing()) c->timed_iters++;
  return DM_OK;
}

// One iteration as a replayed graph (captured on first use; one graph with
// and one without the eps_psi partials).
dm_status graph_iteration(dm_ctx* c, bool psi_err) {
  const int k = psi_err ? 1 : 0;
  if (!c->graph_exec[k]) {
    DM_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    dm_status s = launch_iteration(c, psi_err);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (s != DM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail_hip(c, e, "hipStreamEndCapture");
    c->graph[k] = g;
    DM_HIP(c, hipGraphInstantiate(&c->graph_exec[k], c->graph[k], nullptr, nullptr, 0));
  }
  DM_HIP(c, hipGraphLaunch(c->graph_exec[k], c->stream));
  return DM_OK;
}

// Set-up kernels of one scan: views psi = P0 * O0, mode power, counter.
dm_status init_scan_state(dm_ctx* c, int s) {
  auto& S = c->scans[s];
  const ScanLayout& L = S.L;
  const size_t M = S.d.n_modes, FF = (size_t)S.d.frame * S.d.frame;
  const int NL = obj_modes(S.d);
  DM_HIP(c, hipMemcpyAsync(c->sat<float2>(s, L.P), S.P0, M * FF * 8, hipMemcpyDeviceToDevice,
                           c->stream));
  DM_HIP(c, hipMemcpyAsync(c->sat<float2>(s, L.O), S.O0,
                           (size_t)NL * S.d.obj_h * S.d.obj_w * 8, hipMemcpyDeviceToDevice,
                           c->stream));
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->sat<int>(s, L.counter),
                     1, 0);
  DM_LAUNCHED(c, "k_fill_int");
  hipLaunchKernelGGL(dmk::k_init_psi, dim3(S.d.n_frames * S.d.n_modes * NL), dim3(256), 0,
                     c->stream, c->sat<float2>(s, L.psi), c->sat<float2>(s, L.P),
                     c->sat<float2>(s, L.O), c->sat<int>(s, L.pos), S.d.n_modes, S.d.frame,
                     S.d.obj_w, NL, S.d.obj_h);
  DM_LAUNCHED(c, "k_init_psi");
  hipLaunchKernelGGL(dmk::k_mode_power, dim3((FF + 255) / 256), dim3(256), 0, c->stream,
                     c->sat<float2>(s, L.P), c->sat<float>(s, L.D), S.d.n_modes, (int)FF);
  DM_LAUNCHED(c, "k_mode_power");
  return DM_OK;
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Orthogonal probe modes (dm_ortho.hpp): the modes' Gram matrix, its
// eigen-decomposition and the mix of the probe and of every view, enqueued
// on `st`; `scr` holds dmk::kOrthoScratchBytes; the eigenvalues (the new
// modes' powers, descending) go to lam_dev if it is not NULL.
hipError_t launch_ortho(float2* P, float2* psi, int n_views, int M, int F, void* scr,
                        double* lam_dev, hipStream_t st) {
  const int FF = F * F, npairs = M * (M + 1) / 2;
  double2* w = reinterpret_cast<double2*>(scr);
  hipLaunchKernelGGL(dmk::k_gram_partial, dim3(npairs, dmk::kOrthoChunks), dim3(256), 0, st, P,
                     M, FF, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dmk::k_ortho_eig, dim3(1), dim3(64), 0, st, M, w, lam_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int sets = n_views + 1;
  hipLaunchKernelGGL(dmk::k_mix_modes, dim3((FF + 255) / 256, std::min(sets, 65535)), dim3(256), 0,
                     st, psi, P, n_views, M, FF, w);
  return hipGetLastError();
}

dm_status batch_init(dm_ctx** out, int n_scans, const dm_desc* descs, const float* const* Is,
                     const int32_t* const* poss, const void* const* P0s, const void* const* O0s,
                     void* ws, size_t ws_bytes, void* stream) {
  g_init_error.clear();
  if (!out) { g_init_error = "out is NULL"; return DM_E_ARG; }
  *out = nullptr;
  std::string why;
  dm_status st = validate_batch(n_scans, descs, why);
  if (st != DM_OK) { g_init_error = why; return st; }
  if (!Is || !poss || !P0s || !O0s || !ws) {
    g_init_error = "a required pointer is NULL";
    return DM_E_ARG;
  }
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) {
    g_init_error = "workspace must be 256-byte aligned";
    return DM_E_ARG;
  }
  if ((descs[0].flags & DM_FLAG_GRAPH) && !stream) {
    g_init_error = "DM_FLAG_GRAPH needs a non-NULL stream";
    return DM_E_ARG;
  }
  for (int s = 0; s < n_scans; ++s) {
    const dm_desc& d = descs[s];
    if (!Is[s] || !poss[s] || !P0s[s] || !O0s[s]) {
      g_init_error = "scan " + std::to_string(s) + ": a required pointer is NULL";
      return DM_E_ARG;
    }
    if (!aligned8(Is[s]) || !aligned8(P0s[s]) || !aligned8(O0s[s])) {
      g_init_error = "device buffers must be 8-byte aligned";
      return DM_E_ARG;
    }
    for (int j = 0; j < d.n_frames; ++j) {
      const int y = poss[s][2 * j], x = poss[s][2 * j + 1];
      if (y < 0 || x < 0 || y > d.obj_h - d.frame || x > d.obj_w - d.frame) {
        char msg[200];
        snprintf(msg, sizeof msg, "scan %d: view %d at (y=%d, x=%d) leaves the %dx%d object", s,
                 j, y, x, d.obj_h, d.obj_w);
        g_init_error = msg;
        return DM_E_BOUNDS;
      }
    }
  }
  CtxLayout CL = ctx_layout(n_scans, descs);
  if (ws_bytes < CL.total) {
    char msg[160];
    snprintf(msg, sizeof msg, "workspace of %zu bytes, %zu needed", ws_bytes, CL.total);
    g_init_error = msg;
    return DM_E_WORKSPACE;
  }
  dm_ctx* c = new (std::nothrow) dm_ctx();
  if (!c) { g_init_error = "out of host memory"; return DM_E_ARG; }
  c->CL = CL;
  c->F = descs[0].frame;
  c->M = descs[0].n_modes;
  c->L = obj_modes(descs[0]);
  c->flags = descs[0].flags;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(ws);
  std::vector<int2> vmap;
  for (int s = 0; s < n_scans; ++s) {
    dm_ctx::Scan S;
    S.d = descs[s];
    S.L = CL.sl[s];
    S.base = CL.scan_base[s];
    S.I = Is[s];
    S.P0 = P0s[s];
    S.O0 = O0s[s];
    S.pos.assign(poss[s], poss[s] + 2 * (size_t)S.d.n_frames);
    S.order = spatial_order(S.d, S.pos);
    for (int j : S.order) vmap.push_back(make_int2(s, j));
    c->scans.push_back(std::move(S));
  }
  c->total_views = (int)vmap.size();
  c->stream_slots = stream_slots(n_scans, descs);
  auto bail = [&](dm_status e) {
    g_init_error = c->err;
    delete c;
    return e;
  };
#define INIT_HIP(call)                                         \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return bail(fail_hip(c, e_, #call)); \
  } while (0)
  std::vector<float2> tw = twiddles(c->F);
  INIT_HIP(hipMemcpyAsync(c->tw(), tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice,
                          c->stream));
  std::vector<uint4> wtab;
  if (c->bf16x3()) {
    wtab = mfma_dft_table();
    INIT_HIP(hipMemcpyAsync(const_cast<uint4*>(c->wf()), wtab.data(), wtab.size() * sizeof(uint4),
                            hipMemcpyHostToDevice, c->stream));
    INIT_HIP(set_mfma_lds());
  }
  INIT_HIP(hipMemcpyAsync(c->vmap(), vmap.data(), vmap.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flags_dev(),
                     c->n_flags(), 0);
  INIT_HIP(hipGetLastError());
  for (int s = 0; s < n_scans; ++s) {
    auto& S = c->scans[s];
    INIT_HIP(hipMemcpyAsync(c->sat<int>(s, S.L.pos), S.pos.data(), S.pos.size() * sizeof(int),
                            hipMemcpyHostToDevice, c->stream));
    INIT_HIP(hipMemcpyAsync(c->sat<int>(s, S.L.order), S.order.data(),
                            S.order.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    const size_t nI = (size_t)S.d.n_frames * S.d.frame * S.d.frame;
    hipLaunchKernelGGL(dmk::k_check_finite, dim3(1024), dim3(256), 0, c->stream, S.I, nI,
                       c->flags_dev());
    INIT_HIP(hipGetLastError());
    st = init_scan_state(c, s);
    if (st != DM_OK) return bail(st);
  }
  st = apply_tuning(c, default_tuning(descs[0]));  // synchronises
  if (st != DM_OK) return bail(st);
  int flags_host = 0;
  INIT_HIP(hipMemcpy(&flags_host, c->flags_dev(), sizeof(int), hipMemcpyDeviceToHost));
  if (flags_host & 2) {
    c->err = "intensities contain NaN or Inf";
    return bail(DM_E_ARG);
  }
#undef INIT_HIP
  *out = c;
  return DM_OK;
}

dm_status read_errors(dm_ctx* c, int s, int first, int count, dm_errors* out) {
  std::vector<DevErrors> tmp(count);
  DevErrors* ring = c->sat<DevErrors>(s, c->scans[s].L.ring);
  for (int i = 0; i < count; ++i) {
    const int slot = (first - 1 + i) % dmk::kRing;
    DM_HIP(c, hipMemcpyAsync(&tmp[i], ring + slot, sizeof(DevErrors), hipMemcpyDeviceToHost,
                             c->stream));
  }
  int flags_host = 0;
  DM_HIP(c, hipMemcpyAsync(&flags_host, c->flags_dev() + 1 + s, sizeof(int),
                           hipMemcpyDeviceToHost, c->stream));
  DM_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, tmp.data(), sizeof(dm_errors) * count);
  if (flags_host & 1) {
    c->err = "a non-finite error norm was produced (the iteration diverged)";
    return DM_E_NUMERIC;
  }
  return DM_OK;
}

dm_status check_scan(dm_ctx* c, int scan) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (scan < 0 || scan >= (int)c->scans.size()) {
    c->err = "scan index out of range";
    return DM_E_ARG;
  }
  return DM_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
std::string tune_key(dm_ctx* c) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "gfx";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  int nb = 0;
  while ((1 << (nb + 1)) <= c->total_views) ++nb;
  char k[200];
  snprintf(k, sizeof k, "%s:F%d:M%d:N2^%d:S%zu:flags%u:prec%d", arch.c_str(), c->F, c->M, nb,
           c->scans.size(), c->flags & DM_FLAG_MULTIPASS, (int)c->scans[0].d.precision);
  return k;
}

bool cache_lookup(const char* path, const std::string& key, dm_tuning* t) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[256];
    int tile, chunks, multi;
    if (sscanf(line,
               "{\"key\": \"%255[^\"]\", \"obj_tile\": %d, \"probe_chunks\": %d, "
               "\"view_path\": %d",
               k, &tile, &chunks, &multi) == 4 &&
        key == k) {
      t->obj_tile = tile;
      t->probe_chunks = chunks;
      t->view_path = multi;
      t->reserved = 0;
      found = true;  // the last entry for a key wins
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const dm_tuning& t, double ms) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"key\": \"%s\", \"obj_tile\": %d, \"probe_chunks\": %d, \"view_path\": %d, "
          "\"ms_per_iter\": %.6f}\n",
          key.c_str(), t.obj_tile, t.probe_chunks, t.view_path, ms);
  fclose(f);
}

dm_status valid_tuning(dm_ctx* c, const dm_tuning& t) {
  if (t.obj_tile != 16 && t.obj_tile != 32) {
    c->err = "obj_tile must be 16 or 32";
    return DM_E_ARG;
  }
  if (t.probe_chunks < 1 || t.probe_chunks > DM_MAX_PROBE_CHUNKS) {
    c->err = "probe_chunks out of range";
    return DM_E_ARG;
  }
  if (t.reserved != 0 || t.view_path < DM_VIEWS_FUSED || t.view_path > DM_VIEWS_STREAMED_WIDE) {
    c->err = "bad tuning fields";
    return DM_E_ARG;
  }
  const bool have_spec = c->scans[0].L.tspec != 0;
  if (t.view_path != DM_VIEWS_FUSED && c->bf16x3()) {
    c->err = "the BF16x3 form has its own transform path (view_path must be 0)";
    return DM_E_ARG;
  }
  if (t.view_path == DM_VIEWS_THREE_KERNEL && !have_spec) {
    c->err = "the three-kernel path needs DM_FLAG_MULTIPASS at init";
    return DM_E_ARG;
  }
  if (t.view_path != DM_VIEWS_THREE_KERNEL && c->F > 128) {
    c->err = "frames above 128 only have the three-kernel path";
    return DM_E_ARG;
  }
  if (t.view_path != DM_VIEWS_THREE_KERNEL && c->L > 1) {
    c->err = "object modes only have the three-kernel path";
    return DM_E_ARG;
  }
  return DM_OK;
}

// Median per-iteration time (ms) of `reps` iterations with tuning t.
dm_status time_tuning(dm_ctx* c, const dm_tuning& t, int reps, double* ms) {
  DM_TRY(apply_tuning(c, t));
  const uint32_t saved_flags = c->flags;
  c->flags &= ~DM_FLAG_PHASE_TIMING;
  // time the form the context's iterations run (with the eps_psi partials
  // unless DM_FLAG_PSI_ERROR_LAST)
  const bool psi_err = !(c->flags & DM_FLAG_PSI_ERROR_LAST);
  dm_status s = launch_iteration(c, psi_err);  // warm-up
  std::vector<double> v;
  for (int r = 0; r < reps && s == DM_OK; ++r) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = take_event(c, &a);
    if (e == hipSuccess) e = take_event(c, &b);
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    if (e != hipSuccess) { s = fail_hip(c, e, "autotune events"); break; }
    s = launch_iteration(c, psi_err);
    if (s != DM_OK) break;
    e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float x = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, a, b);
    if (e != hipSuccess) { s = fail_hip(c, e, "autotune timing"); break; }
    v.push_back(x);
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
  }
  c->flags = saved_flags;
  if (s != DM_OK) return s;
  std::sort(v.begin(), v.end());
  *ms = v[v.size() / 2];
  return DM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing
// (dm_orthogonalize_modes_noalloc): a static device array, one copy per GPU
// for the life of the process.  Its name is a host-side stand-in; the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[dmk::kOrthoScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices] = {};

hipError_t scratch_address(void** out, std::string& why) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    why = "hipGetDevice";
    return e;
  }
  if (dev < 0 || dev >= kScratchDevices) {
    why = "device index beyond the scratch table";
    return hipErrorInvalidDevice;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      why = "hipGetSymbolAddress(scratch)";
      return e;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t dm_workspace_bytes(const dm_desc* desc) { return dm_batch_workspace_bytes(1, desc); }

size_t dm_batch_workspace_bytes(int32_t n_scans, const dm_desc* descs) {
  std::string why;
  if (validate_batch(n_scans, descs, why) != DM_OK) return 0;
  return ctx_layout(n_scans, descs).total;
}

dm_status dm_init(dm_ctx** out, const dm_desc* desc, const float* I_dev, const int32_t* pos_host,
                  const void* probe0_dev, const void* object0_dev, void* workspace_dev,
                  size_t workspace_bytes, void* hip_stream) {
  const float* Is[1] = {I_dev};
  const int32_t* ps[1] = {pos_host};
  const void* P0s[1] = {probe0_dev};
  const void* O0s[1] = {object0_dev};
  return batch_init(out, 1, desc, Is, ps, P0s, O0s, workspace_dev, workspace_bytes, hip_stream);
}

dm_status dm_batch_init(dm_ctx** out, int32_t n_scans, const dm_desc* descs,
                        const float* const* I_devs, const int32_t* const* pos_hosts,
                        const void* const* probe0_devs, const void* const* object0_devs,
                        void* workspace_dev, size_t workspace_bytes, void* hip_stream) {
  return batch_init(out, n_scans, descs, I_devs, pos_hosts, probe0_devs, object0_devs,
                    workspace_dev, workspace_bytes, hip_stream);
}

dm_status dm_iterate(dm_ctx* c, int32_t n_iter) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (n_iter < 0) { c->err = "n_iter < 0"; return DM_E_ARG; }
  for (int i = 0; i < n_iter; ++i) {
    const bool psi_err = (i == n_iter - 1) || !(c->flags & DM_FLAG_PSI_ERROR_LAST);
    s = (c->flags & DM_FLAG_GRAPH) ? graph_iteration(c, psi_err) : launch_iteration(c, psi_err);
    if (s != DM_OK) return s;
    c->iters++;
  }
  return DM_OK;
}

dm_status dm_scan_get_object(dm_ctx* c, int32_t scan, void* dst) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  if (!dst) { c->err = "dst is NULL"; return DM_E_ARG; }
  const auto& S = c->scans[scan];
  DM_HIP(c, hipMemcpyAsync(dst, c->sat<float2>(scan, S.L.O),
                           (size_t)obj_modes(S.d) * S.d.obj_h * S.d.obj_w * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  return DM_OK;
}

dm_status dm_scan_get_probe(dm_ctx* c, int32_t scan, void* dst) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  if (!dst) { c->err = "dst is NULL"; return DM_E_ARG; }
  const auto& S = c->scans[scan];
  DM_HIP(c, hipMemcpyAsync(dst, c->sat<float2>(scan, S.L.P),
                           (size_t)S.d.n_modes * S.d.frame * S.d.frame * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  return DM_OK;
}

dm_status dm_scan_mode_power(dm_ctx* c, int32_t scan, double* power_host) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  if (!power_host) { c->err = "power_host is NULL"; return DM_E_ARG; }
  const auto& S = c->scans[scan];
  double* dev = c->sat<double>(scan, S.L.mode_pow);
  hipLaunchKernelGGL(dmk::k_mode_sums, dim3(S.d.n_modes), dim3(256), 0, c->stream,
                     c->sat<float2>(scan, S.L.P), S.d.frame * S.d.frame, dev);
  DM_LAUNCHED(c, "k_mode_sums");
  DM_HIP(c, hipMemcpyAsync(power_host, dev, (size_t)S.d.n_modes * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  DM_HIP(c, hipStreamSynchronize(c->stream));
  return DM_OK;
}

dm_status dm_mode_power(dm_ctx* c, double* power_host) {
  return dm_scan_mode_power(c, 0, power_host);
}

dm_status dm_scan_orthogonalize_modes(dm_ctx* c, int32_t scan, double* power_host) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  const auto& S = c->scans[scan];
  const ScanLayout& L = S.L;
  const int M = S.d.n_modes, F = S.d.frame;
  double* lam = c->sat<double>(scan, L.mode_pow);
  // the views' frames come in runs of M probe modes, one run per object mode
  DM_HIP(c, launch_ortho(c->sat<float2>(scan, L.P), c->sat<float2>(scan, L.psi),
                         S.d.n_frames * obj_modes(S.d), M, F, c->sat<void>(scan, L.ortho), lam,
                         c->stream));
  // the mode power D = sum_k |P_k|^2 of the Eq. 5 normaliser, formed again
  // from the mixed modes
  hipLaunchKernelGGL(dmk::k_mode_power, dim3((F * F + 255) / 256), dim3(256), 0, c->stream,
                     c->sat<float2>(scan, L.P), c->sat<float>(scan, L.D), M, F * F);
  DM_LAUNCHED(c, "k_mode_power");
  if (power_host) {
    DM_HIP(c, hipMemcpyAsync(power_host, lam, (size_t)M * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    DM_HIP(c, hipStreamSynchronize(c->stream));
  }
  return DM_OK;
}

dm_status dm_orthogonalize_modes(dm_ctx* c, double* power_host) {
  return dm_scan_orthogonalize_modes(c, 0, power_host);
}

dm_status dm_orthogonalize_modes_noalloc(void* probe_dev, void* psi_dev, int32_t n_views,
                                         int32_t n_modes, int32_t frame, double* power_dev,
                                         void* hip_stream) {
  g_init_error.clear();
  if (n_modes > dmk::kOrthoMaxModes) {
    g_init_error = "n_modes = " + std::to_string(n_modes) +
                   " exceeds the 16 modes the static scratch holds";
    return DM_E_UNSUPPORTED;
  }
  if (n_modes < 1 || frame < 1 || n_views < 0) {
    g_init_error = "need n_modes >= 1, frame >= 1 and n_views >= 0";
    return DM_E_ARG;
  }
  if ((double)frame * frame >= 2147483648.0 ||
      (double)n_views * n_modes * frame * frame >= 9.2e18 / 8) {
    g_init_error = "frame or view count too large";
    return DM_E_UNSUPPORTED;
  }
  if (!probe_dev || !aligned8(probe_dev) || (n_views > 0 && (!psi_dev || !aligned8(psi_dev))) ||
      (power_dev && !aligned8(power_dev))) {
    g_init_error = "probe (and psi when n_views > 0) must be non-NULL 8-byte aligned device "
                   "pointers, power_dev NULL or 8-byte aligned";
    return DM_E_ARG;
  }
  void* scr = nullptr;
  std::string why;
  hipError_t e = scratch_address(&scr, why);
  if (e == hipSuccess)
    e = launch_ortho(reinterpret_cast<float2*>(probe_dev), reinterpret_cast<float2*>(psi_dev),
                     n_views, n_modes, frame, scr, power_dev,
                     reinterpret_cast<hipStream_t>(hip_stream));
  else
    why += ": ";
  if (e != hipSuccess) {
    g_init_error = why + hipGetErrorString(e);
    return DM_E_HIP;
  }
  return DM_OK;
}

dm_status dm_scan_warm_start(dm_ctx* c, int32_t scan, const void* patches_dev) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  if (!patches_dev || !aligned8(patches_dev)) {
    c->err = "warm start needs an 8-byte aligned device array of patches";
    return DM_E_ARG;
  }
  auto& S = c->scans[scan];
  if (obj_modes(S.d) > 1) {
    c->err = "the warm start replaces a single object mode";
    return DM_E_UNSUPPORTED;
  }
  const ScanLayout& L = S.L;
  const int FF = S.d.frame * S.d.frame;
  const size_t total = (size_t)S.d.n_frames * FF;
  hipLaunchKernelGGL(dmk::k_warm_opart, dim3((unsigned)std::min<size_t>((total + 255) / 256, 8192)),
                     dim3(256), 0, c->stream, c->sat<float2>(scan, L.opart),
                     c->sat<float>(scan, L.D), reinterpret_cast<const float2*>(patches_dev),
                     S.d.n_frames, FF);
  DM_LAUNCHED(c, "k_warm_opart");
  // the object gather over this scan's tiles only: they are a contiguous
  // range of the tile map
  int first = 0;
  for (int t = 0; t < scan; ++t) first += c->scans[t].ntiles;
  if (c->tune.obj_tile == 16)
    hipLaunchKernelGGL((dmk::k_object<16, kObjGroups>), dim3(S.ntiles), dim3(256 * kObjGroups), 0, c->stream, c->scan_dev(),
                       c->tmap() + first, S.d.frame);
  else
    hipLaunchKernelGGL((dmk::k_object<32, kObjGroups>), dim3(S.ntiles), dim3(256 * kObjGroups), 0, c->stream, c->scan_dev(),
                       c->tmap() + first, S.d.frame);
  DM_LAUNCHED(c, "k_object (warm start)");
  hipLaunchKernelGGL(dmk::k_init_psi, dim3(S.d.n_frames * S.d.n_modes), dim3(256), 0, c->stream,
                     c->sat<float2>(scan, L.psi), c->sat<float2>(scan, L.P),
                     c->sat<float2>(scan, L.O), c->sat<int>(scan, L.pos), S.d.n_modes,
                     S.d.frame, S.d.obj_w, 1, S.d.obj_h);
  DM_LAUNCHED(c, "k_init_psi");
  return DM_OK;
}

dm_status dm_warm_start(dm_ctx* c, const void* patches_dev) {
  return dm_scan_warm_start(c, 0, patches_dev);
}

dm_status dm_get_object(dm_ctx* c, void* dst) { return dm_scan_get_object(c, 0, dst); }
dm_status dm_get_probe(dm_ctx* c, void* dst) { return dm_scan_get_probe(c, 0, dst); }

dm_status dm_scan_error_history(dm_ctx* c, int32_t scan, int32_t first, int32_t count,
                                dm_errors* out) {
  dm_status s = check_scan(c, scan);
  if (s != DM_OK) return s;
  if (!out || count < 0) { c->err = "bad arguments"; return DM_E_ARG; }
  if (count == 0) return DM_OK;
  if (first <= c->first_iter || first + count - 1 > c->iters ||
      c->iters - first + 1 > dmk::kRing) {
    c->err = "requested iterations are not in the error ring (or precede the last dm_set_state)";
    return DM_E_ARG;
  }
  return read_errors(c, scan, first, count, out);
}

dm_status dm_error(dm_ctx* c, dm_errors* out) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!out) { c->err = "out is NULL"; return DM_E_ARG; }
  if (c->iters == c->first_iter) {
    // no iteration since the start or the last dm_set_state
    std::memset(out, 0, sizeof *out);
    out->iter = c->iters;
    return DM_OK;
  }
  return read_errors(c, 0, c->iters, 1, out);
}

dm_status dm_error_history(dm_ctx* c, int32_t first, int32_t count, dm_errors* out) {
  return dm_scan_error_history(c, 0, first, count, out);
}

int32_t dm_iterations(const dm_ctx* c) { return c ? c->iters : -1; }
int32_t dm_n_scans(const dm_ctx* c) { return c ? (int32_t)c->scans.size() : -1; }

dm_status dm_get_state(dm_ctx* c, void* psi_dst, void* probe_dst, void* object_dst,
                       int32_t* iter_host) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (c->scans.size() != 1) {
    c->err = "dm_get_state needs a batch of one";
    return DM_E_STATE;
  }
  const auto& S = c->scans[0];
  const size_t FF = (size_t)S.d.frame * S.d.frame;
  const size_t NL = obj_modes(S.d);
  if (psi_dst)
    DM_HIP(c, hipMemcpyAsync(psi_dst, c->sat<float2>(0, S.L.psi),
                             (size_t)S.d.n_frames * S.d.n_modes * NL * FF * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  if (probe_dst)
    DM_HIP(c, hipMemcpyAsync(probe_dst, c->sat<float2>(0, S.L.P), (size_t)S.d.n_modes * FF * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  if (object_dst)
    DM_HIP(c, hipMemcpyAsync(object_dst, c->sat<float2>(0, S.L.O),
                             NL * S.d.obj_h * S.d.obj_w * 8, hipMemcpyDeviceToDevice,
                             c->stream));
  DM_HIP(c, hipStreamSynchronize(c->stream));
  if (iter_host) *iter_host = c->iters;
  return DM_OK;
}

dm_status dm_set_state(dm_ctx* c, const void* psi_src, const void* probe_src,
                       const void* object_src, int32_t iter) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (c->scans.size() != 1) {
    c->err = "dm_set_state needs a batch of one";
    return DM_E_STATE;
  }
  if (!psi_src || !probe_src || !object_src || iter < 0) {
    c->err = "dm_set_state needs psi, probe, object and iter >= 0";
    return DM_E_ARG;
  }
  const auto& S = c->scans[0];
  const size_t FF = (size_t)S.d.frame * S.d.frame;
  const size_t NL = obj_modes(S.d);
  DM_HIP(c, hipMemcpyAsync(c->sat<float2>(0, S.L.psi), psi_src,
                           (size_t)S.d.n_frames * S.d.n_modes * NL * FF * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->sat<float2>(0, S.L.P), probe_src, (size_t)S.d.n_modes * FF * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  DM_HIP(c, hipMemcpyAsync(c->sat<float2>(0, S.L.O), object_src,
                           NL * S.d.obj_h * S.d.obj_w * 8, hipMemcpyDeviceToDevice,
                           c->stream));
  hipLaunchKernelGGL(dmk::k_mode_power, dim3((FF + 255) / 256), dim3(256), 0, c->stream,
                     c->sat<float2>(0, S.L.P), c->sat<float>(0, S.L.D), S.d.n_modes, (int)FF);
  DM_LAUNCHED(c, "k_mode_power");
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream,
                     c->sat<int>(0, S.L.counter), 1, iter);
  DM_LAUNCHED(c, "k_fill_int");
  // a restored state starts a new run: its numeric flag is clear and the
  // error records of earlier iterations are no longer this run's
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flags_dev() + 1, 1, 0);
  DM_LAUNCHED(c, "k_fill_int");
  c->iters = iter;
  c->first_iter = iter;
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

dm_status dm_get_tuning(const dm_ctx* c, dm_tuning* out) {
  if (!c || !out) return DM_E_ARG;
  *out = c->tune;
  return DM_OK;
}

dm_status dm_set_tuning(dm_ctx* c, const dm_tuning* t) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (!t) { c->err = "tuning is NULL"; return DM_E_ARG; }
  DM_TRY(valid_tuning(c, *t));
  return apply_tuning(c, *t);
}

dm_status dm_autotune(dm_ctx* c, int32_t reps, const char* cache_path, dm_tuning* out) {
  dm_status s = check_ctx(c);
  if (s != DM_OK) return s;
  if (reps < 1) { c->err = "reps must be >= 1"; return DM_E_ARG; }
  const std::string key = tune_key(c);
  dm_tuning best = c->tune;
  if (cache_path && cache_lookup(cache_path, key, &best) && valid_tuning(c, best) == DM_OK) {
    DM_TRY(apply_tuning(c, best));
    if (out) *out = best;
    return DM_OK;
  }
  const dm_tuning base = default_tuning(c->scans[0].d);
  std::vector<dm_tuning> cand;
  const int chunk_opts[3] = {std::max(1, base.probe_chunks / 2), base.probe_chunks,
                             std::min(DM_MAX_PROBE_CHUNKS, base.probe_chunks * 2)};
  const bool have_spec = c->scans[0].L.tspec != 0 && !c->bf16x3();
  for (int mp = DM_VIEWS_FUSED; mp <= DM_VIEWS_STREAMED_WIDE; ++mp) {
    if (c->bf16x3() && mp != DM_VIEWS_FUSED) continue;
    if (mp == DM_VIEWS_THREE_KERNEL && !have_spec) continue;
    if (mp != DM_VIEWS_THREE_KERNEL && (c->F > 128 || c->L > 1)) continue;
    for (int tile : {16, 32})
      for (int ch : chunk_opts) {
        dm_tuning t{tile, ch, mp, 0};
        bool dup = false;
        for (auto& u : cand)
          if (u.obj_tile == t.obj_tile && u.probe_chunks == t.probe_chunks &&
              u.view_path == t.view_path)
            dup = true;
        if (!dup) cand.push_back(t);
      }
  }
  double best_ms = 1e30;
  for (const auto& t : cand) {
    double ms = 0;
    DM_TRY(time_tuning(c, t, reps, &ms));
    // strictly faster wins; within 0.1% the smaller tile wins
    if (ms < best_ms * 0.999 || (ms <= best_ms * 1.001 && t.obj_tile < best.obj_tile)) {
      best_ms = std::min(ms, best_ms);
      best = t;
    }
  }
  DM_TRY(apply_tuning(c, best));
  // rebuild the initial state and forget the timed iterations
  for (int sidx = 0; sidx < (int)c->scans.size(); ++sidx) DM_TRY(init_scan_state(c, sidx));
  hipLaunchKernelGGL(dmk::k_fill_int, dim3(1), dim3(64), 0, c->stream, c->flags_dev(),
                     c->n_flags(), 0);
  DM_LAUNCHED(c, "k_fill_int");
  DM_HIP(c, hipStreamSynchronize(c->stream));
  c->iters = 0;
  c->first_iter = 0;
  for (auto& m : c->marks) { c->event_pool.push_back(m.a); c->event_pool.push_back(m.b); }
  c->marks.clear();
  c->timed_iters = 0;
  if (cache_path) cache_store(cache_path, key, best, best_ms);
  if (out) *out = best;
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
  if (!c) return g_init_error.c_str();  // dm_init and the context-free calls
  return c->err.c_str();
}

}  // extern "C"
