/*
 * mvd.h — C ABI of the plane-wise multi-view Richardson-Lucy deconvolution
 * library for AMD Instinct MI355X (gfx950).
 *
 * Method (Schmid & Huisken, "Real-time multi-view deconvolution"):
 *   ψ^{t+1} = ψ^t · Π_v [ (φ_v / (ψ^t ∗ P_v)) ∗ X_v ]
 * (Supplementary Note 1, update equation; Supplementary Note 2 §1 for the
 * back-projector X_v), applied independently to every plane orthogonal to the
 * rotation axis with a 2D PSF per view (Results, second paragraph; Fig. 1a).
 *
 * Conventions shared by every entry point
 *   - A volume is Y planes of Z rows × X columns.  The rotation axis is Y, the
 *     camera row axis: plane y is the Z×X image made of camera row y of every
 *     slice z.  Plane data is row-major "[Y][Z][X]" (X fastest).  Camera-ordered
 *     stacks are "[Z][Y][X]".
 *   - PSF taps are host float32 "[kz][kx]" (rows = Z offsets, columns = X
 *     offsets), odd sides in [1, MVD_MAX_K], finite, non-negative, not all 0.
 *     The centre tap is (kz-1)/2, (kx-1)/2.  Taps are used as given (no
 *     renormalisation).
 *   - Convolution (a ∗ k)[z][x] = Σ_j Σ_i k[j][i] · ã[z+Rz−j][x+Rx−i] with ã
 *     zero outside the plane (MVD_BOUNDARY_ZERO: the linear convolution that a
 *     Fourier convolution padded to data + PSF size computes, Supplementary
 *     Table 1 caption) or wrapped (MVD_BOUNDARY_PERIODIC).
 *   - Ratio guard: φ/b where b > 1e-6, else 1.
 *   - Every call that takes a stream only enqueues work on it (the library's
 *     calls are asynchronous, Supplementary Note 2 §3); the caller keeps the
 *     buffers alive until the stream has completed.  stream may be NULL (the
 *     device's null stream).
 *   - Device buffers (observations, estimate, checkpoints, workspace,
 *     gradients) belong to the caller.  A context owns only host copies of the
 *     taps, their derived 1D factors and a few KB of device memory for taps.
 *   - Errors: every call returns an mvd_status.  On MVD_ERR_ARG, MVD_ERR_STATE
 *     or MVD_ERR_WORKSPACE nothing has been enqueued.  mvd_last_error() gives a
 *     message.  A context is not thread-safe; separate contexts may be used
 *     from separate threads and streams.
 */
#ifndef MVD_H
#define MVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MVD_ABI_VERSION 3
#define MVD_MAX_VIEWS 8
#define MVD_MAX_K 63
#define MVD_DEVICE_NONE (-1) /* host-only context: PSF setup and validation only */
#define MVD_MAX_PLANE_X 65536 /* widest plane row (X) a context accepts */

typedef struct mvd_ctx mvd_ctx;

typedef enum {
  MVD_OK = 0,
  MVD_ERR_ARG = -1,         /* invalid argument; nothing enqueued */
  MVD_ERR_STATE = -2,       /* call out of order (e.g. a PSF not set) */
  MVD_ERR_WORKSPACE = -3,   /* workspace missing or too small */
  MVD_ERR_DEVICE = -4,      /* no usable GPU / host-only context */
  MVD_ERR_LAUNCH = -5,      /* HIP launch or runtime failure */
  MVD_ERR_UNSUPPORTED = -6, /* valid but not supported combination */
  MVD_ERR_ALLOC = -7,       /* small internal allocation failed */
  MVD_ERR_IO = -8           /* a file read or write failed (disk-to-disk form) */
} mvd_status;

typedef enum { MVD_U16 = 1, MVD_F32 = 2 } mvd_dtype;

typedef enum {
  MVD_STACK_ZYX = 1,  /* camera-ordered stack [Z][Y][X]; resliced on the device */
  MVD_PLANES_YZX = 2  /* already planes [Y][Z][X] */
} mvd_layout;

/* Back-projector X_v (Supplementary Note 2 §1).  Compound kernels are built
 * on the host in float64 from all views' PSFs, cropped to the view's PSF size
 * and normalised to unit sum:
 *   FLIPPED          X_v = P_v^*  ("Independent")
 *   EFFICIENT_BAYES  X_v = N( P_v^* ⊙ Π_{w≠v} C(P_v^* ⊛ P_w ⊛ P_w^*) )
 *   OPT1             X_v = N( P_v^* ⊙ Π_{w≠v} C(P_v^* ⊛ P_w) )
 *   OPT2             X_v = N( (P_v^*)^{⊙V} )
 *   EXPLICIT         X_v given by the caller, used as is.                    */
typedef enum {
  MVD_BACK_FLIPPED = 0,
  MVD_BACK_EFFICIENT_BAYES = 1,
  MVD_BACK_OPT1 = 2,
  MVD_BACK_OPT2 = 3,
  MVD_BACK_EXPLICIT = 4
} mvd_back;

/* SIMULTANEOUS: all views' corrections from the same ψ^t, multiplied together
 * (the printed update).  SEQUENTIAL: each view's correction is multiplied
 * into ψ before the next view is blurred (stable for V ≥ 3). */
typedef enum { MVD_UPDATE_SIMULTANEOUS = 0, MVD_UPDATE_SEQUENTIAL = 1 } mvd_update;
typedef enum { MVD_BOUNDARY_ZERO = 0, MVD_BOUNDARY_PERIODIC = 1 } mvd_boundary;

/* ψ^0: mean of the views' observations (averaging fusion), the estimate
 * passed in `est`, or a constant. */
typedef enum { MVD_INIT_MEAN = 0, MVD_INIT_GIVEN = 1, MVD_INIT_CONST = 2 } mvd_init;

/* mvd_run.flags */
#define MVD_FLAG_FORCE_2D 0x1u /* use the general K×K kernels even for rank-1 PSFs */
#define MVD_FLAG_TIMING 0x2u   /* record HIP events around every launch (see mvd_get_timing) */
#define MVD_FLAG_GRAPH 0x4u    /* capture the whole run into a HIP graph on first use and replay it
                                  (per context, keyed by every pointer and parameter of the run;
                                  not with MVD_FLAG_TIMING) */
#define MVD_FLAG_NORMALIZE 0x10u /* divide each view's back-projection by X_v ⊛ 1 (the
                                    sensitivity Aᵀ1; below the tap sum within R of the edges
                                    under the zero boundary): the EM form of the update for a
                                    zero-extended convolution.  Rank-one back-projectors take
                                    it in the backward pass's epilogue (separable sensitivity);
                                    others, and MVD_FLAG_FORCE_2D runs, store each view's
                                    back-projection and divide by a sensitivity plane computed
                                    by the same pass (more workspace: mvd_workspace_bytes).
                                    Supplementary Note 1 (the update assumes unit column
                                    sums) */
#define MVD_FLAG_TUNE 0x8u     /* choose launch shapes (row-segment length, views per launch,
                                  columns per thread, occupancy; for simultaneous two-view runs
                                  with rank-one PSFs of at most 31 taps also whether each
                                  iteration runs as one fused launch) by timing candidates on one
                                  iteration of this run's own data at the first run of a workload
                                  shape; the choice is cached for the process.  That first call
                                  synchronises its stream and overwrites est while it times (so
                                  runs with MVD_INIT_GIVEN are not tuned).  Results can differ from
                                  untuned runs by float32 rounding only. */

/* Parameters of one deconvolution run.  struct_size must be sizeof(mvd_run). */
typedef struct {
  uint32_t struct_size;
  uint32_t flags;             /* MVD_FLAG_* */
  int32_t n_planes;           /* Y ≥ 1 */
  int32_t n_iters;            /* T ≥ 0 (chosen by the user; no convergence test) */
  int32_t update;             /* mvd_update */
  int32_t boundary;           /* mvd_boundary */
  int32_t init;               /* mvd_init */
  float init_const;           /* ψ^0 for MVD_INIT_CONST, must be > 0 */
  int32_t obs_dtype;          /* mvd_dtype of the observations */
  int32_t obs_layout;         /* mvd_layout of the observations */
  const float *view_weights;  /* host [V] in [0,1], or NULL = all 1.  Each view's
                                 correction c is tempered as w·c + (1 − w). */
  float *checkpoints;         /* device [T][Y][Z][X] float32 receiving ψ^0..ψ^{T−1},
                                 or NULL.  Needed later by mvd_backward. */
  void *workspace;            /* device scratch of mvd_workspace_bytes() bytes */
  size_t workspace_bytes;
  const float *const *weight_planes; /* host array of V device pointers to float32
                                 [Y][Z][X] per-pixel weights ω_v in [0,1], or NULL.  Each
                                 pixel's correction is tempered as ω·c + (1 − ω) with
                                 ω = view_weights[v] · ω_v(pixel) (the memory table's
                                 per-pixel, per-view weights, Supplementary Note 2; their
                                 formula is not given).  Back-projectors that are not rank
                                 one, and MVD_FLAG_FORCE_2D runs, apply them in a pointwise
                                 update after storing each view's back-projection.  Streamed and
                                 disk-to-disk runs read them in place, each plane batch
                                 its own planes: there they must be device memory
                                 (MVD_ERR_ARG otherwise).  Read only, kept alive until
                                 the stream is done. */
} mvd_run;

/* Library version (MVD_ABI_VERSION). */
int mvd_version(void);

/* Human-readable name of a status code (static string). */
const char *mvd_status_string(mvd_status s);

/* Create a context for V views of Z×X planes on HIP device `device`
 * (or MVD_DEVICE_NONE for a host-only context).  *out receives the context,
 * owned by the caller and released with mvd_destroy().
 * Errors: MVD_ERR_ARG (null out, V outside [1, MVD_MAX_VIEWS], Z or X < 1,
 * X > MVD_MAX_PLANE_X, Z·X > 2^31), MVD_ERR_DEVICE (device does not exist). */
mvd_status mvd_create(mvd_ctx **out, int n_views, int n_z, int n_x, int device);

/* Release a context (NULL is ignored).  Waits for nothing: the caller must
 * have synchronised the streams it used with this context. */
void mvd_destroy(mvd_ctx *ctx);

/* Set view `view`'s PSF P_v (host float32 [kz][kx], copied) and its
 * back-projector mode (mvd_back).  back_taps: host float32 [kz][kx] for
 * MVD_BACK_EXPLICIT, else ignored (may be NULL).  Back-projectors, compound
 * ones included, are (re)built by the call that completes the set of PSFs and
 * by every later call.  Rank-one taps (to 1e-6 relative) are run as two 1D
 * passes; taps whose SVD gives at most 6 rank-one terms reproducing them to
 * 1e-6 of the largest as that many pairs of 1D passes; others
 * as K×K passes (mvd_psf_info).
 * Errors: MVD_ERR_ARG (bad view, sides even or outside [1, MVD_MAX_K], taps
 * negative/non-finite/all zero, missing explicit taps), MVD_ERR_ALLOC. */
mvd_status mvd_set_psf(mvd_ctx *ctx, int view, const float *taps, int kz, int kx,
                       int back_mode, const float *back_taps);

/* Host copy of the effective back-projector X_v (float32 [kz][kx] of view v's
 * PSF size) after compound kernels are built.  `out` holds kz·kx floats.
 * Errors: MVD_ERR_ARG, MVD_ERR_STATE (some view has no PSF). */
mvd_status mvd_get_back_taps(mvd_ctx *ctx, int view, float *out);

/* How view v's forward PSF and back-projector run: 1 = rank one (two 1D
 * passes); r ≥ 2 = a sum of r rank-one terms from the kernel's SVD (at most
 * 6 terms, every tap reproduced to 1e-6 of the largest; r pairs of 1D passes
 * accumulated before the ratio or the update, Supplementary Note 2 §4 convolves
 * with measured PSFs); 0 = K×K passes.  Either pointer may be NULL. */
mvd_status mvd_psf_info(mvd_ctx *ctx, int view, int *separable_psf, int *separable_back);

/* Device workspace needed by mvd_deconvolve_planes() for `run`, in bytes:
 * V float32 plane sets for the observations, resliced/converted and clamped
 * at 0 (filled only when some view's PSF is not rank one; the rank-one
 * passes read the observations as given, through their layout's strides),
 * plus the ratio planes (V sets for MVD_UPDATE_SIMULTANEOUS, one for
 * sequential; none when n_iters = 0), plus one set for partial sums where a
 * kernel runs as a sum of rank-one terms.  Errors: MVD_ERR_ARG. */
mvd_status mvd_workspace_bytes(const mvd_ctx *ctx, const mvd_run *run, size_t *bytes);

/* Reslice one camera-ordered stack (device [Z][Y][X], u16 or f32) into device
 * float32 planes [Y][Z][X] (Fig. 1a: one plane per camera line).  uint16
 * converts exactly; float values are clamped below at 0 (NaN → 0).
 * Errors: MVD_ERR_ARG, MVD_ERR_DEVICE, MVD_ERR_LAUNCH. */
mvd_status mvd_reslice(mvd_ctx *ctx, const void *stack, int dtype, int n_planes,
                       float *planes, void *stream);

/* Plane-wise MV-RL on all planes.
 *   obs: host array of V device pointers, one per view, in run->obs_layout
 *        and run->obs_dtype (Y = run->n_planes).  Read only.
 *   est: device float32 [Y][Z][X]; ψ^0 on entry for MVD_INIT_GIVEN, ψ^T on exit.
 * Steps: ψ^0 (and, for K×K forward passes, the observations resliced and
 * converted into the workspace), then T iterations (2 passes per iteration
 * for SIMULTANEOUS, 2V for SEQUENTIAL) that read the observations in place:
 * they must stay unchanged until the stream has finished the run.  uint16
 * values convert exactly, float values are clamped below at 0 (NaN → 0).
 * ψ stays ≥ 0 for non-negative data.
 * Errors: MVD_ERR_ARG, MVD_ERR_STATE (PSF missing), MVD_ERR_WORKSPACE,
 * MVD_ERR_DEVICE, MVD_ERR_LAUNCH. */
mvd_status mvd_deconvolve_planes(mvd_ctx *ctx, const void *const *obs, float *est,
                                 const mvd_run *run, void *stream);

/* Allocation-free form of mvd_deconvolve_planes, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results (bitwise)
 * except that run->workspace must be NULL and run->workspace_bytes 0: the
 * workspace is a static device array of MVD_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends.  Planes are
 * independent, so the volume goes through all T iterations in batches of as
 * many planes as fit the scratch (mvd_workspace_bytes of a batch ≤
 * MVD_SCRATCH_BYTES).  The call makes no device allocation: no hipMalloc,
 * events or graphs (MVD_FLAG_TIMING, MVD_FLAG_GRAPH and MVD_FLAG_TUNE are
 * rejected).  Every call on a GPU shares that GPU's scratch, which keeps the
 * last call's contents (every value a run reads from it, it has written
 * first): calls that overlap on one GPU (several streams or threads) race.
 * Errors: as mvd_deconvolve_planes; MVD_ERR_WORKSPACE when one plane's
 * workspace exceeds MVD_SCRATCH_BYTES, MVD_ERR_ARG with a workspace or one of
 * those flags. */
#define MVD_SCRATCH_BYTES (64u << 20)
mvd_status mvd_deconvolve_planes_static(mvd_ctx *ctx, const void *const *obs, float *est,
                                        const mvd_run *run, void *stream);

/* ---- streamed form ---------------------------------------------------------
 * The whole run of mvd_deconvolve_planes on camera-ordered stacks that stay in
 * host memory: planes are independent, so the volume is processed in batches
 * of `batch_planes` consecutive planes, each copied to the device, resliced,
 * deconvolved for all T iterations and (for a host estimate) copied back,
 * with the copies of one batch overlapping the iterations of another
 * (Supplementary Note 2 §3, which interleaves per-plane transfers and RL steps
 * on several streams; here copies in, compute and copies out run on three
 * streams, two batches in flight).  Results equal those of
 * mvd_deconvolve_planes on the whole volume bitwise.
 *
 * mvd_stream_workspace_bytes: device workspace for mvd_deconvolve_stream
 * with this run, batch size and estimate placement (est_on_host ≠ 0 when est
 * will be host memory): two staging slots of V observation batches (+ one
 * estimate batch for a host estimate) and one batch run's workspace.
 * Errors: MVD_ERR_ARG. */
mvd_status mvd_stream_workspace_bytes(const mvd_ctx *ctx, const mvd_run *run, int batch_planes,
                                      int est_on_host, size_t *bytes);

/* Streamed run.
 *   obs: host array of V pointers to camera-ordered stacks [Z][Y][X] of
 *        run->obs_dtype (Y = run->n_planes), in page-locked host memory
 *        (hipHostMalloc) or device memory.  Read only.  run->obs_layout must
 *        be MVD_STACK_ZYX.
 *   est: float32 [Y][Z][X], device or page-locked host memory; ψ^0 on entry
 *        for MVD_INIT_GIVEN, ψ^T on exit.
 *   run: as for mvd_deconvolve_planes except checkpoints (must be NULL) and
 *        MVD_FLAG_GRAPH (not allowed); run->workspace of
 *        mvd_stream_workspace_bytes() bytes.
 *   batch_planes: planes per batch, ≥ 1 (the last batch may be shorter).
 * Compute runs on `stream`; the copies run on two streams the context owns,
 * ordered after the work already on `stream`, and `stream` waits for them
 * before it completes, so synchronising `stream` covers the whole call.
 * Pageable host memory is rejected (MVD_ERR_ARG).
 * Errors: MVD_ERR_ARG, MVD_ERR_STATE, MVD_ERR_WORKSPACE, MVD_ERR_DEVICE,
 * MVD_ERR_LAUNCH, MVD_ERR_ALLOC (streams or events). */
mvd_status mvd_deconvolve_stream(mvd_ctx *ctx, const void *const *obs, float *est,
                                 const mvd_run *run, int batch_planes, void *stream);

/* ---- disk-to-disk form ------------------------------------------------------
 * The streamed run with the stacks read from files and the estimate written to
 * a file (Supplementary Note 2 §3, Algorithm 1: planes are loaded from disk into
 * main memory, copied to the GPU, deconvolved and saved back, with the disk
 * traffic of some planes hidden behind the iterations of others).  Here a
 * reader thread fills `host_slots` page-locked input batches, the caller's
 * thread enqueues copies and iterations exactly as mvd_deconvolve_stream does,
 * and a writer thread drains `host_slots` page-locked output batches to the
 * estimate file; each read or write is split over `io_threads` threads.
 * Results equal those of mvd_deconvolve_stream (and of mvd_deconvolve_planes)
 * bitwise. */
#define MVD_FILES_SYNC 0x1        /* fdatasync the estimate file before returning */
#define MVD_FILES_DROP_CACHE 0x2  /* after each read and each (flushed) write, drop the
                                     file range from the page cache (posix_fadvise), so
                                     the run is timed against the disk, not the cache */
typedef struct {
  uint32_t struct_size;           /* sizeof(mvd_files) */
  uint32_t flags;                 /* MVD_FILES_* */
  int32_t obs_fd[MVD_MAX_VIEWS];  /* per view: descriptor of a regular file open for reading */
  int64_t obs_offset[MVD_MAX_VIEWS]; /* byte offset of view v's stack [Z][Y][X] of run->obs_dtype
                                        (native byte order, no padding) in its file */
  int32_t est_fd;                 /* regular file open for writing */
  int64_t est_offset;             /* byte offset of ψ^T, float32 planes [Y][Z][X] (the file
                                     grows as needed; other bytes are left alone) */
  int32_t host_slots;             /* page-locked batches on each side: 0 → 3 (the paper's
                                     stream count), else 2..8 */
  int32_t io_threads;             /* threads per batch read or write: 0 → 4, else 1..64 */
  /* out, filled on MVD_OK: */
  double seconds[4];              /* reader busy, writer busy (with SYNC: incl. fdatasync),
                                     caller's thread waiting for reads, wall time of the call */
  int64_t bytes[2];               /* bytes read, bytes written */
} mvd_files;

/* Disk-to-disk run.
 *   io: the files (see mvd_files); the library reads obs with pread and writes
 *       the estimate with pwrite, and never closes the descriptors.
 *   run: as for mvd_deconvolve_stream, except run->init: MVD_INIT_MEAN or
 *        MVD_INIT_CONST (MVD_INIT_GIVEN has no source here: MVD_ERR_ARG);
 *        run->workspace: device memory of mvd_stream_workspace_bytes(ctx, run,
 *        batch_planes, 1) bytes.
 *   batch_planes: planes per batch, ≥ 1.
 * Synchronous: returns when every plane has been written (and `stream`, on
 * which the iterations run, has completed).  Page-locked host batches
 * (host_slots × (V input + 1 output) batches) are allocated on first use and
 * kept by the context, which frees them in mvd_destroy.
 * Errors: MVD_ERR_ARG (bad descriptor, not a regular file, a file shorter than
 * its stack, bad offsets or counts; checked before any device work),
 * MVD_ERR_STATE, MVD_ERR_DEVICE, MVD_ERR_WORKSPACE, MVD_ERR_ALLOC (host
 * batches, threads, streams or events), MVD_ERR_IO (a read or write failed or
 * came up short: the estimate file is then incomplete), MVD_ERR_LAUNCH. */
mvd_status mvd_deconvolve_files(mvd_ctx *ctx, mvd_files *io, const mvd_run *run, int batch_planes,
                                void *stream);

/* Launch timings of runs made with MVD_FLAG_TIMING since the last reset:
 * summed HIP-event durations (ms) and launch counts per kind.  Kinds: 0 forward
 * pass (blur + ratio), 1 backward pass (back-projection + update), 2 the rest
 * (reslice/convert, ψ^0), 3 reverse-sweep passes (mvd_backward), 4 tap-gradient
 * correlations, 5 fused iterations (forward and backward passes of both views
 * in one launch: simultaneous two-view runs with rank-one PSFs of at most 31
 * taps under the zero boundary, without normalisation or weight planes).
 * Events are recorded on the run's stream around each launch; this call waits
 * for the last of them.  reset ≠ 0 clears the record.
 * Errors: MVD_ERR_ARG, MVD_ERR_LAUNCH. */
#define MVD_TIMING_KINDS 6
typedef struct {
  uint32_t struct_size;
  int32_t count[MVD_TIMING_KINDS];
  double ms[MVD_TIMING_KINDS];
} mvd_timing;
mvd_status mvd_get_timing(mvd_ctx *ctx, mvd_timing *out, int reset);

/* Device workspace needed by mvd_backward() for `run`, in bytes.
 * Errors: MVD_ERR_ARG, MVD_ERR_STATE. */
mvd_status mvd_backward_workspace_bytes(const mvd_ctx *ctx, const mvd_run *run, size_t *bytes);

/* Reverse sweep (adjoint) of mvd_deconvolve_planes: gradients of a loss L
 * with respect to the taps of every view's PSF P_v and back-projector X_v,
 * the view weights and ψ^0, given ∂L/∂ψ^T.  The chain rule of the update
 * (Supplementary Note 1 / Note 2 §1) is applied backwards through every
 * iteration, recomputing each iteration's intermediates from its checkpoint.
 *   obs, run: exactly as in the forward call (same n_iters, update, boundary,
 *        weights, observations); run->checkpoints must hold ψ^0 … ψ^{T−1} as
 *        written by that call; run->workspace of mvd_backward_workspace_bytes().
 *   grad_est: device [Y][Z][X], ∂L/∂ψ^T (read only).
 *   grad_psf, grad_back: host arrays of V device pointers to float32 [kz][kx]
 *        of each view's PSF size, receiving ∂L/∂P_v and ∂L/∂X_v (X_v taken as
 *        an independent kernel; for X_v = P_v^* add the flipped grad_back to
 *        grad_psf).  Either array may be NULL (not computed).
 *   grad_weights: device [V] or NULL.  grad_init: device [Y][Z][X], ∂L/∂ψ^0,
 *        or NULL.  Outputs are overwritten, in float32 from float64 sums in a
 *        fixed order (bitwise reproducible).
 * PSFs and back-projectors of every form are differentiated: rank one,
 * sums of a few rank-one terms (summed term by term) and general K×K kernels
 * (the K×K passes); the tap gradients always cover the whole K×K kernel, and
 * the reverse sweep may use other pass forms than the forward call
 * (MVD_FLAG_FORCE_2D), which changes float32 rounding only.  With
 * MVD_FLAG_NORMALIZE the chain rule also runs through the sensitivity
 * 1 ⊛ X_v, which depends on the back-projector's taps.  Per-pixel
 * weight planes (run->weight_planes) are taken as in the forward call: each
 * pixel's correction tempered by o = w_v · ω_v(pixel); grad_weights is then
 * ∂L/∂w_v with the planes held fixed (mvd_backward_grads also returns ∂L/∂ω_v).
 * Where a run of the same workload was tuned (MVD_FLAG_TUNE) in this process,
 * the passes take its launch shapes.
 * Errors: MVD_ERR_ARG, MVD_ERR_STATE, MVD_ERR_WORKSPACE, MVD_ERR_UNSUPPORTED,
 * MVD_ERR_DEVICE, MVD_ERR_LAUNCH. */
mvd_status mvd_backward(mvd_ctx *ctx, const void *const *obs, const float *grad_est,
                        const mvd_run *run, float *const *grad_psf, float *const *grad_back,
                        float *grad_weights, float *grad_init, void *stream);

/* The outputs of a reverse sweep (every field NULL: not computed). */
typedef struct {
  uint32_t struct_size;              /* sizeof(mvd_grads) */
  float *const *grad_psf;            /* host array of V device pointers, float32 [kz][kx] */
  float *const *grad_back;           /* host array of V device pointers, float32 [kz][kx] */
  float *grad_weights;               /* device [V] */
  float *grad_init;                  /* device [Y][Z][X] */
  float *const *grad_weight_planes;  /* host array of V device pointers, float32 [Y][Z][X]:
                                        ∂L/∂ω_v pixel by pixel, summed over the iterations
                                        (float32 sums in iteration order); needs
                                        run->weight_planes, 16-byte aligned for full speed */
} mvd_grads;

/* mvd_backward with its outputs in a struct, and the gradient of the
 * per-pixel weight planes ω_v (the per-pixel, per-view weights of
 * Supplementary Note 2's memory table, with the forward call's tempering
 * o = w_v · ω_v): ∂L/∂ω_v(pixel) = Σ_t c̄_v(pixel) (q_v(pixel) − 1) w_v.
 * Arguments and errors as mvd_backward; MVD_ERR_ARG also for a NULL `out`, a
 * wrong struct_size, grad_weight_planes without run->weight_planes, or a NULL
 * entry in it. */
mvd_status mvd_backward_grads(mvd_ctx *ctx, const void *const *obs, const float *grad_est,
                              const mvd_run *run, const mvd_grads *out, void *stream);

/* ---- batched form --------------------------------------------------------
 * Several deconvolutions (volumes of different plane sizes, view counts and
 * PSF sizes, each with its own context, observations, estimate and run
 * parameters) in one launch.  Planes are independent (Results, second
 * paragraph), so the batch is a queue of work items, one per (volume, phase,
 * plane, tile): ψ^0, then every forward and backward pass of every iteration
 * in the volume's update order, each pass cut into row-segment × column-strip
 * tiles.  One persistent kernel takes items from an atomic queue head; an
 * item waits until every tile of its plane's previous phase is complete
 * (per-plane counters), and the table lists items in that dependency order,
 * so a work-group only waits for items already taken by running ones.  The
 * volumes advance together (their item lists are merged in proportion).
 * Items that the persistent kernel does not take (K×K or > 41-tap passes,
 * normalised or per-pixel-weighted updates, checkpoints, rows that are not
 * whole 16-byte units) make the batch a HIP graph instead: every volume's
 * whole iteration loop as one branch.  Results equal mvd_deconvolve_planes
 * bitwise in both forms.  Items are copied; their device buffers must stay
 * valid and unchanged in address while the batch exists. */
typedef struct {
  mvd_ctx *ctx;
  const void *const *obs;   /* host array of the context's V device pointers */
  float *est;
  const mvd_run *run;       /* flags must not include MVD_FLAG_TIMING or MVD_FLAG_GRAPH */
} mvd_item;

typedef struct mvd_batch mvd_batch;

#define MVD_BATCH_TUNE 0x1u /* graph form: time launch-shape candidates per item before capture
                               (runs one iteration of each item on `stream`, synchronously;
                               items with MVD_INIT_GIVEN keep the default shapes).  The choice is
                               cached per workload shape for the process.  Where the persistent
                               form applies too, both forms are built and timed (three whole
                               launches each on `stream`, overwriting the items' estimates) and
                               the faster is kept; not when an item's ψ^0 is given
                               (MVD_INIT_GIVEN), which keeps the persistent form. */
#define MVD_BATCH_GRAPH 0x2u /* use the graph form even where the persistent form applies */

/* Validate every item, optionally autotune, and capture the batch graph.
 * All items must be on one device.  Errors: MVD_ERR_ARG (item index in
 * mvd_last_error(NULL)), MVD_ERR_WORKSPACE, MVD_ERR_STATE, MVD_ERR_DEVICE,
 * MVD_ERR_LAUNCH, MVD_ERR_ALLOC. */
mvd_status mvd_batch_create(mvd_batch **out, const mvd_item *items, int n_items, uint32_t flags,
                            void *stream);

/* Launch the batch on `stream` (asynchronous; one kernel launch in the
 * persistent form).  Calls that overlap on one batch race (they share its
 * queue).  The batch holds each
 * item's taps as they were at creation: after mvd_set_psf or mvd_destroy on an
 * item's context the batch must be recreated (MVD_ERR_STATE, nothing launched). */
mvd_status mvd_batch_launch(mvd_batch *b, void *stream);

/* Wait for the batch's work on `stream` and report its status: MVD_ERR_LAUNCH
 * when a persistent launch's wait for a dependency gave up (the flag is then
 * cleared) or the stream failed.  Errors: MVD_ERR_ARG, MVD_ERR_LAUNCH. */
mvd_status mvd_batch_wait(mvd_batch *b, void *stream);

/* Form of the batch: out[4] = persistent (1) or graph (0), work items,
 * work-groups of the persistent launch, its LDS bytes per work-group. */
mvd_status mvd_batch_info(const mvd_batch *b, int *out);

/* Launch durations (ms, HIP events, mean of two launches) that a batch made
 * with MVD_BATCH_TUNE measured for its two forms when it chose between them:
 * out[0] persistent, out[1] graph; both 0 where no choice was timed.
 * Errors: MVD_ERR_ARG. */
mvd_status mvd_batch_form_times(const mvd_batch *b, double *out);

/* Launch shapes chosen for item `item`: out[5] = forward occupancy, forward
 * views per launch, backward inputs per launch, segment scale, columns per
 * thread (0 = default in every field). */
mvd_status mvd_batch_tuning(const mvd_batch *b, int item, int *out);

/* Release a batch (the caller has synchronised its launches). */
void mvd_batch_destroy(mvd_batch *b);

/* One-shot: create (no tuning), launch, wait for completion, destroy. */
mvd_status mvd_batch_run(const mvd_item *items, int n_items, void *stream);

/* Per-context message of the last failing call (empty if none); valid until
 * the next call on the context.  ctx NULL gives the last message of a call
 * that had no context (mvd_create). */
const char *mvd_last_error(const mvd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MVD_H */
