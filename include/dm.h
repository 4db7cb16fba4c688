/*
 * dm.h -- C-ABI of libdm: one multi-mode difference-map (DM) ptychography
 * iteration on an MI355X (gfx950), after Section II of Dong, Fang et al.,
 * "High-Performance Multi-Mode Ptychography Reconstruction on Distributed
 * GPUs" (arXiv:1808.10375).
 *
 * Problem (Section II, Eqs. 1-2): N views j with integer top-left corners
 * (y_j, x_j), measured intensities I_j, probe modes P_k (k < M) and one object
 * O (by default a single object mode).  The exit wave of view j, mode k is
 * psi_{j,k} = P_k * O[window_j].  With L object modes O_l (dm_desc.n_obj_modes)
 * the views hold the pairs psi_{j,(k,l)} = P_k * O_l[window_j] at mode index
 * l M + k, F_c sums over all pairs, Eq. 5 updates each O_l from its pairs and
 * Eq. 4 sums over l as well.  One iteration (dm_iterate) computes:
 *   1. views   psi <- psi + beta (F^-1 F_c[2 P O - psi] - P O)       (Eq. 3)
 *              F_c rescales every mode of a view by
 *              sqrt(I_j / sum_k |F[.]_k|^2) and keeps the phase  (F_c, Eq. 3)
 *   2. object  O <- sum_j sum_k conj(P_k) psi / sum_j sum_k |P_k|^2  (Eq. 5)
 *   3. probe   P_k <- sum_j conj(O[win_j]) psi_{j,k}
 *                     / sum_j |O[win_j]|^2, with the new O            (Eq. 4)
 *   4. errors  relative L2 change between iterations                  (Eq. 6)
 * Transform convention: unnormalised forward DFT exp(-2 pi i (ku+lv)/F),
 * inverse with 1/F^2, detector DC at [0,0] (no fftshift).  Zero mode sums in
 * F_c give 0; zero denominators in Eqs. 4-5 keep the previous value.
 *
 * Layouts (all row-major, complex64 = interleaved {float re, float im}):
 *   I      float32   [N][F][F]
 *   pos    int32     [N][2]      (y, x) top-left of each F x F window
 *   probe  complex64 [M][F][F]
 *   object complex64 [H][W], or [L][H][W] with L object modes
 *   psi    complex64 [N][M][F][F], or [N][L M][F][F] with L object modes
 *
 * Memory ownership: every device buffer is the caller's.  I is read in place
 * and must stay alive and unchanged until dm_free.  probe0/object0 are
 * copied at dm_init.  All iteration state (psi, P, O, partial sums, error
 * ring) lives in the caller's workspace of at least dm_workspace_bytes().
 * The library allocates no device memory; its host-side context is freed by
 * dm_free.
 *
 * Streams: every call enqueues its work on the stream given to dm_init
 * (a hipStream_t passed as void*; NULL = the default stream).  Only dm_init,
 * dm_error, dm_error_history and dm_get_state synchronise with that stream.
 *
 * Errors: calls return a dm_status and never abort.  After a HIP runtime
 * error the context is failed for good: every later call returns DM_E_STATE
 * and dm_last_error() holds the message.  A non-finite error norm (the
 * iteration diverged) is reported as DM_E_NUMERIC by dm_error.
 *
 * Threading: one host thread at a time per context; several contexts may
 * share a GPU and a stream.
 */
#ifndef DM_H_
#define DM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dm_ctx dm_ctx; /* opaque */

typedef enum {
  DM_OK = 0,
  DM_E_ARG = -1,          /* bad descriptor value, null/misaligned pointer,
                             non-finite intensity                          */
  DM_E_UNSUPPORTED = -2,  /* valid in the paper but not built: F neither a
                             power of two in [16, 256] nor 188 or 200,
                             M > 16, unknown precision                     */
  DM_E_BOUNDS = -3,       /* a window leaves the object                     */
  DM_E_WORKSPACE = -4,    /* workspace smaller than dm_workspace_bytes()    */
  DM_E_HIP = -5,          /* HIP runtime error (context becomes failed)     */
  DM_E_STATE = -6,        /* call on a failed or freed context, or out of
                             order                                          */
  DM_E_NUMERIC = -7       /* non-finite error norm: the iteration diverged  */
} dm_status;

typedef enum {
  DM_FP32_FFT = 0,        /* FP32 radix FFTs on the vector ALUs             */
  DM_BF16X3_DFT = 1       /* F = 128 and M <= 8 only (else
                             DM_E_UNSUPPORTED): each 2-D DFT as dense
                             complex matrix products with the DFT matrix on
                             MFMA, every real product split into
                             hi*hi + hi*lo + lo*hi of BF16 pieces, FP32
                             accumulation; the modulus scale, error norms
                             and updates stay FP32 and the object
                             normaliser sum_j sum_k |P_k|^2 accumulates in
                             FP64 (as on every path).  Uses a spectrum
                             buffer; DM_FLAG_MULTIPASS has no effect.     */
} dm_precision;

/* dm_desc.flags bits */
#define DM_FLAG_MULTIPASS 1u     /* use the three-kernel transform path for any
                                    F (it is always used for F = 256, 188
                                    and 200)                                */
#define DM_FLAG_PHASE_TIMING 2u  /* bracket every phase launch of
                                    dm_iterate with HIP events on the
                                    context's stream (read by
                                    dm_phase_times)                          */

#define DM_FLAG_GRAPH 4u         /* capture one iteration's launches (all
                                    scans) into a hipGraph at the first
                                    dm_iterate and replay it once per
                                    iteration; needs a non-NULL stream and
                                    excludes DM_FLAG_PHASE_TIMING           */

#define DM_FLAG_PSI_ERROR_LAST 8u /* form eps_psi only in the last iteration
                                    of each dm_iterate call (by default:
                                    every iteration).  The other iterations
                                    then run the merged streamed view kernels
                                    (F <= 128) and the three-kernel paths
                                    (rows / columns / rows, all F) without a
                                    second read of psi (the fused view kernel
                                    and the BF16x3 form still read it):
                                    psi' = (2 - beta) P O + F^-1[(beta g -
                                    1/F^2) F(2 P O - psi)], g the F_c scale,
                                    which is Eq. 3 rewritten; psi' - psi is
                                    not formed there and eps_psi is reported
                                    as NaN.                                 */

#define DM_FLAG_PROBE_FIRST 16u  /* overlap projection probe first: the
                                    probe (Eq. 4) from the new views and the
                                    current object, then the object (Eq. 5)
                                    from the new views and the new probe,
                                    the order Eqs. 4-5 are written in, i.e.
                                    the order before the swap Section III
                                    describes.  The default, object first
                                    and then the probe from the new object,
                                    is the swapped order: the object update
                                    of a view then needs only that view's
                                    new exit waves and the current probe, so
                                    every view's contribution is formed in
                                    the view kernel right after its update
                                    (the paper's overlap of one batch's
                                    object embedding with the next batch's
                                    view update, at the grain of single
                                    views) and only the gather over views is
                                    left.  Probe first costs one more read
                                    of psi' (the object numerators are
                                    formed again with the new probe).       */

/* Phases of one iteration, in launch order (indices of dm_phase_times;
 * with DM_FLAG_PROBE_FIRST the two probe phases run before the object
 * phase). */
#define DM_PHASE_VIEWS 0         /* Eq. 3 with F_c: exit waves, transforms,
                                    modulus projection, view update         */
#define DM_PHASE_OBJECT 1        /* Eq. 5: object gather (probe first: with
                                    the numerators formed again before it)  */
#define DM_PHASE_PROBE_PARTIAL 2 /* Eq. 4: per-chunk probe sums              */
#define DM_PHASE_PROBE_FINAL 3   /* Eq. 4: division, next mode power        */
#define DM_PHASE_ERRORS 4        /* Eq. 6: error norms into the ring        */
#define DM_N_PHASES 5

typedef struct {
  int32_t n_frames;   /* N >= 1                                          */
  int32_t frame;      /* F: power of two, 16 <= F <= 256, or 188 or 200
                         (the paper's frame sizes: 4 x 47, 8 x 25; these
                         run the three-kernel path with mixed-radix line
                         transforms and take extra workspace for the
                         spectrum buffer, N M F^2 complex values)        */
  int32_t n_modes;    /* M: 1 <= M <= 16 probe modes                     */
  int32_t obj_h;      /* H >= F                                          */
  int32_t obj_w;      /* W >= F                                          */
  float beta;         /* relaxation, 0 <= beta <= 1 (Eq. 3; usually 0.8) */
  int32_t precision;  /* dm_precision                                    */
  uint32_t flags;     /* DM_FLAG_* bits, others must be 0                */
  int32_t n_obj_modes; /* L: object modes of Eqs. 1-5; 0 or 1 = one.  L > 1
                         (at most DM_MAX_OBJ_MODES, and L M at most
                         DM_MAX_PAIRS) runs the FP32 three-kernel path
                         with power-of-two F (the spectrum buffer then
                         holds N L M F^2 complex values); other precisions
                         and frame sizes give DM_E_UNSUPPORTED, and so
                         does the warm start                             */
} dm_desc;

#define DM_MAX_MODES 16
#define DM_MAX_OBJ_MODES 4
#define DM_MAX_PAIRS 32
#define DM_MAX_PROBE_CHUNKS 64

/* dm_tuning.view_path values */
#define DM_VIEWS_FUSED 0           /* one workgroup per view, transforms
                                      recomputed instead of stored (F <= 128) */
#define DM_VIEWS_THREE_KERNEL 1    /* rows / columns / rows through the
                                      spectrum buffer                        */
#define DM_VIEWS_STREAMED 2        /* persistent workgroups, spectra in a
                                      per-workgroup scratch slot, psi loaded
                                      and stored with the non-temporal hint
                                      (F <= 128)                             */
#define DM_VIEWS_STREAMED_CACHED 3 /* the same with ordinary psi accesses    */
#define DM_VIEWS_STREAMED_MERGED 4 /* DM_VIEWS_STREAMED with the view update
                                      right after each inverse transform (the
                                      updated spectra make one trip through
                                      the slot instead of two)               */
#define DM_VIEWS_STREAMED_WIDE 5   /* DM_VIEWS_STREAMED_MERGED with half the
                                      threads, each running two columns of
                                      the transform (F >= 32; one at F = 16):
                                      twice the registers per thread keep the
                                      modulus scale out of the slot          */

/* Launch shapes chosen per context (dm_set_tuning / dm_autotune).  They
 * change the speed of an iteration and the summation order of the probe
 * sums (results agree to rounding), nothing else. */
typedef struct {
  int32_t obj_tile;      /* edge of the object tiles of the Eq. 5 gather:
                            16 or 32                                      */
  int32_t probe_chunks;  /* runs of views summed separately in the Eq. 4
                            partial sums, 1..DM_MAX_PROBE_CHUNKS (capped at
                            each scan's view count)                       */
  int32_t view_path;     /* transform path of the view update (Eq. 3):
                            DM_VIEWS_FUSED, DM_VIEWS_THREE_KERNEL (only
                            where the workspace holds its spectrum buffer:
                            F = 256, 188, 200 or DM_FLAG_MULTIPASS at init;
                            forced for F = 256, 188 and 200), or one of the DM_VIEWS_STREAMED*
                            paths (F <= 128); ignored by
                            the BF16x3 form, which must be given 0        */
  int32_t reserved;      /* must be 0                                     */
} dm_tuning;

typedef struct {
  int32_t iter;        /* 1-based index of the iteration these belong to  */
  float eps_psi;       /* ||psi' - psi|| / ||psi'||; NaN where not formed
                          (see DM_FLAG_PSI_ERROR_LAST)                    */
  float eps_obj;       /* ||O' - O|| / ||O'|| over covered object pixels  */
  float eps_probe;     /* Eq. 6 with the mode sum inside both norms; the
                          convergence error "err"                        */
  float eps_probe_mode[DM_MAX_MODES]; /* Eq. 6 per probe mode          */
} dm_errors;

/* Bytes of device workspace dm_init needs for this problem; 0 if the
 * descriptor is invalid.  Pure host computation. */
size_t dm_workspace_bytes(const dm_desc* desc);

/* Validate, build the object-tile -> view lists, copy probe0/object0 into
 * the workspace and set the initial views psi_j = P0 * O0[window_j]
 * (Section II: the initial fields are built from the initial guesses).
 *   out       receives the new context (set to NULL on failure)
 *   I_dev     device, float32 [N][F][F]; negative values act as 0; any NaN
 *             or Inf -> DM_E_ARG
 *   pos_host  host, int32 [N][2] (y, x); 0 <= y <= H-F and 0 <= x <= W-F,
 *             otherwise DM_E_BOUNDS; copied
 *   probe0_dev, object0_dev  device complex64, copied
 *   workspace_dev  device, >= dm_workspace_bytes(desc) bytes, 256-byte
 *             aligned; owned by the caller, used until dm_free
 *   hip_stream     hipStream_t or NULL
 * Synchronises the stream once (to read the intensity check). */
dm_status dm_init(dm_ctx** out, const dm_desc* desc, const float* I_dev,
                  const int32_t* pos_host, const void* probe0_dev,
                  const void* object0_dev, void* workspace_dev,
                  size_t workspace_bytes, void* hip_stream);

/* Enqueue n_iter >= 0 DM iterations (steps 1-4 above) on the context's
 * stream.  Asynchronous; the error norms of every iteration go to a device
 * ring of the last 4096 iterations. */
dm_status dm_iterate(dm_ctx* ctx, int32_t n_iter);

/* Enqueue a device-to-device copy of the current object, complex64 [H][W]
 * ([L][H][W] with L object modes). */
dm_status dm_get_object(dm_ctx* ctx, void* dst_dev);

/* Enqueue a device-to-device copy of the current probe, complex64 [M][F][F]. */
dm_status dm_get_probe(dm_ctx* ctx, void* dst_dev);

/* Synchronise and return the power of each probe mode, sum over pixels of
 * |P_k|^2 (FP64 sums on the device), k < M, in power_host[M].  The paper
 * (Section II, after Eq. 6) picks the number of probe modes by adding
 * modes in trial runs while each one carries at least 1% of the total
 * intensity; its share is power[k] / sum(power). */
dm_status dm_mode_power(dm_ctx* ctx, double* power_host);

/* Synchronise and return the error norms of the latest iteration
 * (iter = 0 and zeros before the first).  DM_E_NUMERIC if any is not
 * finite. */
dm_status dm_error(dm_ctx* ctx, dm_errors* out_host);

/* Synchronise and copy the error norms of iterations first..first+count-1
 * (1-based; each must be among the last 4096 run) to out_host[count]. */
dm_status dm_error_history(dm_ctx* ctx, int32_t first, int32_t count,
                           dm_errors* out_host);

/* Number of iterations run so far (host-side count of enqueued ones). */
int32_t dm_iterations(const dm_ctx* ctx);

/* Copy the full state out (device destinations; any may be NULL to skip):
 * psi [N][M][F][F], probe [M][F][F], object [H][W] (with L object modes psi
 * [N][L M][F][F] and object [L][H][W]); *iter_host gets the iteration count.
 * Synchronises. */
dm_status dm_get_state(dm_ctx* ctx, void* psi_dst_dev, void* probe_dst_dev,
                       void* object_dst_dev, int32_t* iter_host);

/* Replace the state (device sources in the layouts of dm_get_state; all
 * three required) and set the iteration count: exact resume, or a one-step
 * comparison from a given state.  Asynchronous. */
dm_status dm_set_state(dm_ctx* ctx, const void* psi_dev, const void* probe_dev,
                       const void* object_dev, int32_t iter);

/* With DM_FLAG_PHASE_TIMING: synchronise, then write to ms_host[DM_N_PHASES]
 * the GPU time (milliseconds, from HIP events) spent in each phase by all
 * iterations enqueued since the previous call, and to *n_iter_host their
 * number; the accumulators restart.  Without the flag: DM_E_STATE. */
dm_status dm_phase_times(dm_ctx* ctx, double* ms_host, int32_t* n_iter_host);

/* ---- batches: many scans, one launch chain per iteration ------------------
 * All scans of a batch share F, M, L, precision and flags; each has its own
 * views, positions, intensities, probe, object, beta and error ring.  One
 * dm_iterate advances every scan by one DM iteration with one launch per
 * phase for the whole batch (one graph launch with DM_FLAG_GRAPH).  The
 * single-scan calls above act on scan 0; dm_get_state/dm_set_state need a
 * batch of one. */
size_t dm_batch_workspace_bytes(int32_t n_scans, const dm_desc* descs);

/* Like dm_init for n_scans scans; arrays of n_scans pointers (I, positions,
 * probe0, object0 per scan); one workspace for the batch. */
dm_status dm_batch_init(dm_ctx** out, int32_t n_scans, const dm_desc* descs,
                        const float* const* I_devs, const int32_t* const* pos_hosts,
                        const void* const* probe0_devs,
                        const void* const* object0_devs, void* workspace_dev,
                        size_t workspace_bytes, void* hip_stream);

int32_t dm_n_scans(const dm_ctx* ctx);
dm_status dm_scan_get_object(dm_ctx* ctx, int32_t scan, void* dst_dev);
dm_status dm_scan_get_probe(dm_ctx* ctx, int32_t scan, void* dst_dev);
dm_status dm_scan_error_history(dm_ctx* ctx, int32_t scan, int32_t first,
                                int32_t count, dm_errors* out_host);
dm_status dm_scan_mode_power(dm_ctx* ctx, int32_t scan, double* power_host);

/* ---- orthogonal probe modes ----------------------------------------------- */
/* Replace the probe modes by the eigenmodes of their overlap matrix
 * G[k][l] = sum_r conj(P_k(r)) P_l(r).  With G = V diag(lam) V^H, lam
 * descending, mode a becomes sum_k V[k][a] P_k and every view is mixed the
 * same way, psi_{j,a} <- sum_k V[k][a] psi_{j,k}.  The intensity model of
 * Eq. 1 is a sum over modes, so the modulus projection F_c and the updates
 * of Eqs. 4-5 do not change under such a unitary mix: the iteration goes on
 * from an equivalent state whose modes are orthogonal and ordered by power
 * (Section II treats the modes as mutually incoherent and cites the
 * mixed-state method, which works with these eigenmodes).  Each column of V
 * gets a fixed phase: its entry of largest modulus (the first such) is made
 * real and positive.  Overlaps, eigen-decomposition (cyclic Jacobi) and mix
 * run in FP64 on the device; the results are rounded to FP32 once.
 *   power_host  NULL, or host array of M doubles: the eigenvalues, i.e. the
 *               new modes' powers sum_r |P_a(r)|^2, descending (the call then
 *               synchronises with the context's stream).
 * Enqueued on the context's stream.  The iteration counter and the error
 * ring are kept.  DM_E_ARG: scan index out of range. */
dm_status dm_orthogonalize_modes(dm_ctx* ctx, double* power_host);
dm_status dm_scan_orthogonalize_modes(dm_ctx* ctx, int32_t scan, double* power_host);

/* The same orthogonalisation without a context, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): it calls no allocator.  Its scratch (the
 * overlap partial sums, V and the eigenvalues: 39,168 bytes) is a static
 * device array that each GPU the library runs on holds until the process
 * ends; the device address is looked up once per device.  Every call on a
 * GPU shares that array, so calls that overlap in time on one GPU (other
 * streams, other host threads) race; calls on one stream are ordered.  The
 * kernels overwrite all the scratch they read, so nothing carries over from
 * an earlier call.  Same kernels, launch shapes and results as
 * dm_orthogonalize_modes; it does not form the Eq. 5 mode power (no context).
 *   probe_dev  complex64 [n_modes][frame][frame], device, mixed in place
 *   psi_dev    complex64 [n_views][n_modes][frame][frame], device, mixed in
 *              place; may be NULL when n_views = 0 (probe only)
 *   power_dev  NULL, or device array of n_modes doubles: the eigenvalues
 *              (the new modes' powers), descending
 *   hip_stream hipStream_t of the current device (NULL: default stream)
 * Enqueued on hip_stream; never synchronises.  The stream must belong to the
 * current device.  DM_E_UNSUPPORTED: n_modes above 16 (the limit of the
 * static scratch) or more than 2^31 pixels per frame; DM_E_ARG: other bad
 * sizes or NULL/misaligned pointers; DM_E_HIP: a launch failed.  Messages
 * through dm_last_error(NULL). */
dm_status dm_orthogonalize_modes_noalloc(void* probe_dev, void* psi_dev, int32_t n_views,
                                         int32_t n_modes, int32_t frame, double* power_dev,
                                         void* hip_stream);

/* ---- warm start ------------------------------------------------------------ */
/* Replace the object with patches stitched by the object update (Section II,
 * Eq. 5) applied to the exit waves psi_{j,k} = P_k * patch_j with the current
 * probe; the paper allows initial guesses taken from pre-existing results
 * (Section III).  Pixels under no window keep their value.  Then reset every
 * view to psi = P * O[window] (the initial state of Section II).
 *   patches_dev  complex64 [N][F][F], device, caller-owned; patch j is the
 *                object guess under view j's window, indexed like the frame.
 * Enqueued on the context's stream; the iteration counter is kept.
 * DM_E_ARG: NULL or misaligned patches, or a scan index out of range;
 * DM_E_UNSUPPORTED: more than one object mode. */
dm_status dm_warm_start(dm_ctx* ctx, const void* patches_dev);
dm_status dm_scan_warm_start(dm_ctx* ctx, int32_t scan, const void* patches_dev);

/* ---- launch tuning -------------------------------------------------------- */
dm_status dm_get_tuning(const dm_ctx* ctx, dm_tuning* out);

/* Apply a tuning (re-uploads the object tile lists; synchronises). */
dm_status dm_set_tuning(dm_ctx* ctx, const dm_tuning* tuning);

/* Time every candidate tuning (object tile 16/32, probe chunks
 * {1/2, 1, 2} x default, transform path where available) over `reps`
 * iterations each (median of per-iteration HIP-event times, ties to the
 * smaller tile), apply the fastest and write it to *out.  With cache_path,
 * a previous result for the same (GPU architecture, F, M, view-count bucket,
 * scan count) is read from that JSON-lines file instead, and a new result is
 * appended to it.  The timed iterations advance the state; afterwards the
 * state is rebuilt from probe0/object0 as at init, so call it right after
 * init, while those buffers are still alive and unchanged.  Synchronises. */
dm_status dm_autotune(dm_ctx* ctx, int32_t reps, const char* cache_path, dm_tuning* out);

/* Release the host-side context.  Does not touch the caller's buffers.
 * NULL is a no-op. */
void dm_free(dm_ctx* ctx);

/* Static text for a status code. */
const char* dm_status_str(dm_status s);

/* Last error message of a context ("" if none); valid until the next call
 * on it.  With NULL: the last message of a failed dm_init or context-free
 * call (dm_orthogonalize_modes_noalloc) on this thread. */
const char* dm_last_error(const dm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DM_H_ */
