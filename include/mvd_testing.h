/*
 * mvd_testing.h — test and tuning hooks of libmvd (not part of the stable
 * ABI in mvd.h).
 *
 * These entry points expose the host planner's launch geometry so that CPU
 * tests can check every index the kernels compute against its buffer, and let
 * one process switch the launch-shape overrides that the MVD_TUNE environment
 * variable otherwise sets once.  They may change with MVD_TESTING_VERSION;
 * callers check mvd_internal_version() first.  Only mvd_internal_batch_raise_giveup
 * and mvd_internal_stream_probe touch a device.
 * Return values are mvd_status codes (0 ok, MVD_ERR_ARG on a bad argument,
 * MVD_ERR_UNSUPPORTED where the asked-for form does not apply).
 */
#ifndef MVD_TESTING_H
#define MVD_TESTING_H

#include <stddef.h>

#include "mvd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MVD_TESTING_VERSION 2

/* MVD_TESTING_VERSION of the library. */
int mvd_internal_version(void);

/* Launch plan of a separable pass over n_planes planes of ctx's size with a
 * k-tap kernel under `boundary` (k < 0: the one-ring form for −k taps, which
 * the forward pass and the one-plane backward use).  out[13]: bucket, columns
 * per thread, threads, occupancy, row-segment length, segments, outputs per
 * strip, strips, halo, z-pass columns, LDS row pitch, 16-byte row-pass access
 * (for 16-byte aligned buffers), LDS bytes per view. */
int mvd_internal_sep_plan(const mvd_ctx *ctx, int n_planes, int k, int boundary, int *out);

/* The split-view two-plane backward's plan (same out[] layout), or
 * MVD_ERR_UNSUPPORTED where the form does not apply. */
int mvd_internal_split_plan(const mvd_ctx *ctx, int n_planes, int k, int *out);

/* The fused iteration (forward and backward passes of both views in one
 * launch) for a context of ctx's plane size and kernel bucket kb.  out[8]:
 * bucket, output columns per strip, strips, halo R, forward output margin,
 * LDS row pitch, LDS bytes, threads per work-group.  MVD_ERR_UNSUPPORTED
 * where the bucket has no fused form. */
int mvd_internal_fused_plan(const mvd_ctx *ctx, int kb, int *out);

/* The matrix-core K×K pass for a kz × kx kernel.  out[3]: column steps, input
 * tile row pitch, LDS bytes. */
int mvd_internal_mfma_plan(int kz, int kx, int *out);

/* The matrix-core tap-gradient correlation for a volume of n_planes × Z × X
 * and a kz × kx kernel.  out[7]: padded lags (z, x), tile width, tiles per
 * z run, work items, work-groups, LDS bytes. */
int mvd_internal_corr_plan(int n_planes, int Z, int X, int kz, int kx, long *out);

/* Replace the process-wide launch-shape overrides (MVD_TUNE syntax,
 * "key=value,..."; NULL re-reads the environment).  Affects every context of
 * the process from the next enqueued run on; not thread-safe against calls
 * running in other threads. */
int mvd_internal_set_tune(const char *spec);

/* The 1D factors view `view`'s PSF (which = 0) or back-projector (1) runs
 * with: R terms, each kz z-taps then kx x-taps (float32), into out[R·(kz+kx)]
 * (at most `cap` terms written).  Returns R: 1 for a rank-one kernel, the
 * number of terms for a sum of rank-one terms, 0 for the K×K passes; or a
 * negative mvd_status. */
int mvd_internal_psf_terms(mvd_ctx *ctx, int view, int which, float *out, int cap);

/* Polls a persistent batch's work-group makes before it gives up waiting for
 * a dependency (0: the default, about 2^24).  Lets a test make the wait give
 * up at once, so the failure report is exercised with every kernel ending
 * normally. */
int mvd_internal_set_pq_spin(unsigned polls);

/* Raise a persistent batch's give-up flag from the host, as a wait that gave
 * up would: the next launch's work-groups skip every item and end, and
 * mvd_batch_wait reports MVD_ERR_LAUNCH.  MVD_ERR_ARG for a graph batch. */
int mvd_internal_batch_raise_giveup(mvd_batch *b);

/* The persistent form's item order for jobs of n_planes[k] planes cut into
 * nseg[k] row segments × nstrip[k] column strips (tile = (plane·nseg + seg)·
 * nstrip + strip), two tiles per item where pair[k] ≠ 0, per_iter[k] phases
 * per iteration over iters[k] iterations (plus the ψ^0 phase), windows of
 * `window` planes (0: whole volumes): up to `cap` items (job, phase, tile,
 * second tile or −1) into out[4·cap].  Returns the number of items (or a
 * negative mvd_status). */
long mvd_internal_pq_order(int n_jobs, const int *n_planes, const int *nseg, const int *nstrip, const int *pair,
                           const int *per_iter, const int *iters, int window, int *out, long cap);

/* Workspace bytes that the launch-shape tuner's probe (one iteration of the
 * run, made for MVD_FLAG_TUNE) would use, or 0 when the run makes no probe
 * (n_iters = 0).  Never more than mvd_workspace_bytes() of the same run. */
int mvd_internal_tune_probe_bytes(const mvd_ctx *ctx, const mvd_run *run, size_t *bytes);

/* Calibration kernels of known traffic, launched on `stream` (a hipStream_t,
 * NULL for the null stream) of the current device: kind 0 copies `bytes` from
 * src to dst, reading and writing every byte once; kind 1 only reads them
 * (dst then receives at most 2048 floats, and only for data holding NaNs).
 * bytes is a multiple of 16, src and dst 16-byte aligned device buffers.
 * They give the bandwidth a plain streaming kernel reaches on the device, the
 * yardstick beside the peak for the passes.  Returns MVD_OK, MVD_ERR_ARG or
 * MVD_ERR_LAUNCH (asynchronous: completion is the stream's). */
int mvd_internal_stream_probe(int kind, const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MVD_TESTING_H */
