// Internal interface between the host runtime (mvd_api.cpp, psf.cpp) and the
// HIP kernel launchers (k_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mvd {

constexpr int kMaxViews = 8;
constexpr int kMaxK = 63;
constexpr int kMaxPlaneX = 65536;   // plane width limit (row of zeros of this size; mvd_create enforces it)
constexpr float kEps = 1e-6f;   // ratio guard: φ/b where b > kEps, else 1

// Quotient n / d by the reciprocal refined with one Newton-Raphson correction
// of the quotient (Markstein's method): within 1 ulp of the IEEE quotient for
// d > ε and finite n, and exactly 1 when n = d (the exact FMA residual then
// carries the whole error of the first quotient).  Every kernel that forms a
// ratio uses this one definition, so their results agree bitwise.
__device__ __forceinline__ float nr_quotient(float n, float d) {
  const float y = __builtin_amdgcn_rcpf(d);
  const float q0 = n * y;
  return fmaf(fmaf(-d, q0, n), y, q0);
}

// Guarded ratio φ / b for b > ε, else 1.
__device__ __forceinline__ float guarded_ratio(float phi, float b) {
  const float q = nr_quotient(phi, b);
  return b > kEps ? q : 1.f;
}

// Views handled by one separable pass launch.
constexpr int kSepFwdViews = 2;
constexpr int kSepBwdViews = 2;
// Views handled by one general (K×K) pass launch.
constexpr int k2dViews = 4;

// Kernel-size buckets of the separable kernels: the 1D factors are
// zero-padded (centred) to the bucket size.  Adding 0·a is exact, so padding
// does not change results.
constexpr int kSepBuckets[] = {3, 7, 11, 15, 21, 31, 41, 63};
constexpr int kNumSepBuckets = sizeof(kSepBuckets) / sizeof(int);

inline int sep_bucket(int k) {
  for (int b : kSepBuckets)
    if (k <= b) return b;
  return -1;
}

// Geometry of one plane set.
struct PlaneGeom {
  int Y, Z, X;
};

// One forward (blur + ratio) or backward (back-projection + update) pass.
//
// Forward:  for each view v of the pass: b = in0 ⊛ P_v; out[v] = guard(φ_v / b).
// Backward: for each view v of the pass: q = in[v] ⊛ X_v; c = w_v·q + (1 − w_v);
//           psi_out = psi_in · Π_v c.
struct SepPassArgs {
  PlaneGeom g;
  int boundary;       // 0 zero, 1 periodic
  int nviews;         // views in this launch
  int zseg;           // output rows per work-group (multiple of the row group)
  int nseg;           // z segments per plane
  int x_out;          // output columns per strip
  int nstrip;         // strips per plane row
  int halo;           // 0: strip is the whole row (pads from the boundary rule); R: halo columns computed
  int ncols;          // z-pass columns per work-group (x_out + 2·halo)
  int ldsw;           // LDS row pitch in floats
  int vec;            // every plane pointer of the pass is 16-byte aligned
  const float *in[kSepFwdViews];      // forward: in[0] = ψ; backward: in[v] = r_v
  const float *phi[kSepFwdViews];     // adjoint recompute: staged observations (float32 planes)
  const void *obs[kSepFwdViews];      // forward: observations as given, float32 or uint16 (obs_u16)
  long obs_sy, obs_sz;                // element (y, z, x) of obs[v] at y·obs_sy + z·obs_sz + x
  int obs_u16;
  float *out[kSepFwdViews];           // forward: ratio planes
  float *out2[kSepFwdViews];          // second output (adjoint recompute: ratio planes)
  const float *aux0[kSepFwdViews];    // epilogue operands (adjoint passes)
  const float *aux1[kSepFwdViews];
  const float *psi_in;                // backward
  float *psi_out;                     // backward
  float w[kSepFwdViews];              // backward: view weights
  const float *nsz[kSepFwdViews];     // backward with normalisation: 1 ⊛ X_v = nsz[z]·nsx[x]
  const float *nsx[kSepFwdViews];     //   (separable; null: no normalisation)
  const float *wpl[kSepFwdViews];     // backward: per-pixel weights (plane sets), or null
  float tz[kSepFwdViews][kMaxK];      // z factor, padded to the bucket
  float tx[kSepFwdViews][kMaxK];      // x factor, padded to the bucket
};

// One fused iteration of the simultaneous two-view update (forward and
// backward passes in one launch; k_fused.hip).  `f` carries the geometry
// (x_out: output columns per strip, nstrip, halo = R, ldsw: LDS row pitch),
// the observations, ψ in (f.psi_in, also f.in[0]) and out (f.psi_out, a
// different plane set unless nstrip = 1), the weights and the PSF factors
// (f.tz, f.tx); the back-projector factors follow.
struct FusedArgs {
  SepPassArgs f;
  float btz[kSepFwdViews][kMaxK];
  float btx[kSepFwdViews][kMaxK];
};
constexpr int kFusedStrip = 256;     // output columns per work-group of the fused iteration
constexpr int kFusedThreads = 960;   // its work-group: three roles of 320 threads
size_t fused_lds_bytes(int kb, int pitch);
hipError_t launch_fused(const FusedArgs &a, int kb, hipStream_t s);

// General K×K pass (same semantics as SepPassArgs).
struct TwoDPassArgs {
  PlaneGeom g;
  int boundary;
  int nviews;
  int kz, kx;                          // common (padded) kernel size of this pass
  const float *in[k2dViews];
  const float *phi[k2dViews];          // forward: φ_v, or null to store the convolution itself
  float *out[k2dViews];
  const float *psi_in;
  float *psi_out;
  float w[k2dViews];
  const float *taps[k2dViews];        // device [kz][kx] per view
  int mfma;                            // 1: matrix-core kernels, 0: vector-ALU kernels
};

// Matrix-core general passes.  Column steps of 4 covering the 16 + kx − 1 input
// columns of a 16-column block, rounded up to the compiled sizes (extra steps
// meet zero taps); -1 beyond them.
__host__ __device__ constexpr int mfma_chunks(int kx) {
  return (15 + kx + 3) / 4 <= 6 ? 6
       : (15 + kx + 3) / 4 <= 8 ? 8
       : (15 + kx + 3) / 4 <= 12 ? 12
       : (15 + kx + 3) / 4 <= 16 ? 16
       : (15 + kx + 3) / 4 <= 20 ? 20 : -1;
}
// Input-tile row pitch: covers columns up to 48 + 4·nck − 1 and is ≡ 2 (mod 32).
__host__ __device__ constexpr int mfma_tile_width(int nck) {
  return 48 + 4 * nck + ((2 - (48 + 4 * nck) % 32) % 32 + 32) % 32;
}
// LDS bytes of one work-group (input tile + one view's tap rows).
size_t mfma_lds_bytes(int kz, int kx);

// Epilogues of the single-input separable pass.
constexpr int kEpRatio = 0;   // out = φ / conv (guarded); φ float32 at obs (clamped at 0 when read)
constexpr int kEpRatioU16 = 5;  // the same with φ uint16 at obs
constexpr int kEpStore = 1;   // out = conv
constexpr int kEpBR = 2;      // out = conv, out2 = φ / conv
constexpr int kEpBbar = 3;    // out = −conv · aux0 / aux1 where aux1 > ε, else 0
constexpr int kEpAccum = 4;   // out = aux0 + conv
// Last term of a kernel that runs as a sum of rank-one terms (aux0: the sum of
// the earlier terms):
constexpr int kEpAccumRatio = 6;   // b = aux0 + conv; out = φ / b (guarded), φ float32 at aux1
constexpr int kEpAccumUpdate = 7;  // q = aux0 + conv; out = ψ · (w q + 1 − w), ψ at aux1 (may be out)
// Two terms of one kernel in one launch (nviews = 2: tz/tx of both terms, one
// input; the outputs, operands and weight of slot 0; aux0 may be null):
constexpr int kEpTermsSum = 8;     // out = [aux0 +] conv_0 + conv_1
constexpr int kEpTermsRatio = 9;   // b = [aux0 +] conv_0 + conv_1; out = φ / b (guarded), φ float32 at aux1
constexpr int kEpTermsUpdate = 10; // q = [aux0 +] conv_0 + conv_1; out = ψ · (w q + 1 − w), ψ at aux1
__host__ __device__ constexpr bool ep_terms(int ep) { return ep >= kEpTermsSum && ep <= kEpTermsUpdate; }

// Launch configuration chosen by the host for a separable pass.
struct SepPlan {
  int bucket;     // KB
  int cols;       // columns per thread (1 or 2)
  int threads;    // work-group size
  int vin;        // backward: inputs per launch (1 or 2)
  int occ;        // register budget: 4 waves/SIMD (128 VGPRs) or 2 (256)
};

// --- launchers (return hipSuccess or the launch error) ---------------------
hipError_t launch_sep_forward(const SepPassArgs &a, const SepPlan &p, hipStream_t s);
hipError_t launch_sep_backward(const SepPassArgs &a, const SepPlan &p, hipStream_t s);
hipError_t launch_2d_forward(const TwoDPassArgs &a, hipStream_t s);
hipError_t launch_2d_backward(const TwoDPassArgs &a, hipStream_t s);

// Reverse sweep: pointwise step of the update (simultaneous: all views;
// sequential: one view, nv = 1).
struct AdjPointArgs {
  size_t n;
  int nv;
  const float *psi;
  const float *gbar_in;
  float *gbar_out;
  float *q[kMaxViews];   // in: q_v, out: q̄_v
  float w[kMaxViews];
  double *wpart;         // [blocks][nv]
  int wp;                // 0 scalar weights, 1 per-pixel weight planes, 2 planes and their gradients
  const float *wpl[kMaxViews];   // ω_v (wp ≥ 1)
  float *gwpl[kMaxViews];        // ∂L/∂ω_v, accumulated (wp = 2)
  // EM-normalised back-projection: q_v holds the raw back-projection, divided
  // here by s_v(z, x) = nsz_v[z] · nsx_v[x] where that exceeds ε; s̄_v is written
  int nrm;
  int Z, X;
  const float *nsz[kMaxViews];
  const float *nsx[kMaxViews];
  const float *nsp[kMaxViews];   // a sensitivity plane [Z][X] instead of the factors (back-projectors not rank one)
  float *sbar[kMaxViews];
};

// Tap-gradient correlation over all planes: part[block][j][i] partial sums of
// Σ gbar[z][x] · s̃rc[z+rz−j][x+rx−i] for lags padded to kzp × kxp.
struct CorrArgs {
  PlaneGeom g;
  int boundary;
  int rz, rx;
  int kzp, kxp;
  int tw, zch;       // matrix-core form: columns x' per tile, tiles per run down z
  const float *gbar;
  const float *src;
  float *part;
};

hipError_t launch_sep_single_dispatch(const SepPassArgs &a, const SepPlan &p, int ep, hipStream_t s);
hipError_t launch_pointwise_sim(const AdjPointArgs &a, int nblocks, hipStream_t s);
hipError_t launch_pointwise_seq(const AdjPointArgs &a, int nblocks, hipStream_t s);
hipError_t launch_sum_partials(const double *part, int nblocks, int nv, double *acc, hipStream_t s);
// Pointwise ends of the reverse sweep's passes for kernels summed term by term:
// r = φ / b (guarded), and b ← −sum · r / b (0 where b ≤ ε).
hipError_t launch_ratio_plane(const float *phi, const float *b, float *r, size_t n, hipStream_t s);
hipError_t launch_bbar_plane(const float *sum, const float *r, float *b, size_t n, hipStream_t s);
// dst += src, element by element.
hipError_t launch_add_plane(float *dst, const float *src, size_t n, hipStream_t s);
hipError_t launch_corr(const CorrArgs &a, int nblocks, hipStream_t s);
// Matrix-core form: padded lags, tile width, z-run length and grid from
// corr_mfma_shape (at most max_blocks work-groups, one resident wave of them).
struct CorrMfmaShape {
  int kzp, kxp, tw, zch;
  long nitems;
  int nblocks;
  size_t lds;
};
hipError_t launch_corr_mfma(const CorrArgs &a, int nblocks, hipStream_t s);
int corr_mfma_pad(int k);
CorrMfmaShape corr_mfma_shape(const PlaneGeom &g, int kz, int kx, int max_blocks);
size_t corr_mfma_lds_bytes(int kzp, int kxp, int tw);
hipError_t launch_corr_finalize(const float *part, int nblocks, int kzp, int kxp, int kz, int kx, double *acc,
                                hipStream_t s);
hipError_t launch_to_f32(const double *src, float *dst, int n, hipStream_t s);
hipError_t launch_zero_f64(double *dst, int n, hipStream_t s);
int corr_pad(int k, int unit);   // smallest unit·2^n ≥ k
size_t corr_lds_bytes(int kzp, int kxp);
int corr_threads(int kzp, int kxp);

// Observations → float32 planes.  layout 1 = stack [Z][Y][X], 2 = planes.
hipError_t launch_stage_obs(const void *src, int dtype, int layout, PlaneGeom g, float *dst,
                            hipStream_t s);
// Every view's observations → float32 planes dst[v] in one pass, and
// ψ^0 = (1/V) Σ_v φ_v into `mean` when it is not null.
// Observations → float32 planes dst[v] (dst null: none written) and their mean (mean null: none).
// A camera stack source may hold more planes than g.Y (ysrc; 0: g.Y), src pointing at plane y0.
hipError_t launch_stage_views(const void *const *src, int nv, int dtype, int layout, PlaneGeom g,
                              float *const *dst, float *mean, hipStream_t s, int ysrc = 0);
// ψ^0 = (1/V) Σ_v φ_v
hipError_t launch_init_mean(const float *const *phis, int nv, size_t n, float *dst,
                            hipStream_t s);
hipError_t launch_fill(float *dst, size_t n, float value, hipStream_t s);
hipError_t launch_copy(const float *src, float *dst, size_t n, hipStream_t s);
// ψ_out = ψ_in · (o q' + 1 − o) over n elements: q' = q / splane[i mod zx] where
// that exceeds ε (splane null: q), o = w · wpl[i] (wpl null: w).
hipError_t launch_update_plane(const float *psi_in, float *psi_out, const float *q, const float *splane, size_t zx,
                               const float *wpl, float w, size_t n, hipStream_t s);
// Calibration kernels: kind 0 copies `bytes` from src to dst, kind 1 reads
// them (dst: kProbeBlocks floats, written only for non-finite sums).  bytes is
// a multiple of 16, both pointers 16-byte aligned.
constexpr int kProbeBlocks = 2048;
hipError_t launch_stream_probe(int kind, const void *src, void *dst, size_t bytes, hipStream_t s);

// Work-group / LDS parameters of the separable kernels (shared by launchers
// and the host planner).
constexpr int kRowGroup = 8;          // output rows produced per ring step
constexpr int kSepMaxThreads = 512;

// ---- persistent batched form (k_pq.hip) ------------------------------------
// One volume of a persistent batch.  Every pass of the volume uses one tiling
// of its planes (row segments × column strips, one column per thread): tile b
// of a pass is (plane, segment, strip) as in SepPassArgs.  Phase 0 is ψ^0; then per iteration `per_iter` phases: for the
// simultaneous update the nf forward passes (views in pairs) and then one
// backward pass per view, for the sequential update F_0, B_0, F_1, B_1, ….
constexpr int kPqThreads = 1024;   // persistent work-groups: one wide tile or two tiles of ≤ 512 threads

struct PqJob {
  PlaneGeom g;
  int kb;                      // kernel-size bucket of every pass
  int pair;                    // 1: tiles of ≤ kPqThreads/2 threads, two per item; 0: one tile per item
  int lds_floats;              // LDS of one tile (floats; the second tile of a pair starts there)
  int nseg, nstrip, zseg, x_out, ntiles;   // tiling (ntiles = nseg · nstrip per plane)
  int sim, nf, per_iter;
  int fkind[kMaxViews];        // forward pass variant: 0/1 float32 obs with 1/2 views, 2/3 uint16
  // ψ^0
  int init;                    // 0 mean of the views, 1 given (nothing to do), 2 constant
  float init_const;
  int nv, obs_u16;
  long obs_sy, obs_sz;
  const void *obs[kMaxViews];
  float *est;
  unsigned *done;              // [Y] tiles completed per plane (zero between launches)
  SepPassArgs f[kMaxViews];    // forward passes of an iteration
  SepPassArgs b[kMaxViews];    // backward passes (one ratio plane each)
};

struct PqQueue {
  const int4 *items;           // (job, phase, tile, second tile or −1) in dependency order; tile = plane·ntiles + t
  int n_items, n_jobs;
  const PqJob *jobs;
  unsigned *head, *exited;     // queue head; work-groups that have left (zero between launches)
  unsigned *giveup;            // raised when a wait exceeds spin_limit polls
  unsigned spin_limit;
};

size_t pq_lds_bytes(const PqJob &j);
hipError_t launch_pq(const PqQueue &q, int nblocks, size_t lds, hipStream_t s);
hipError_t pq_occupancy(size_t lds, int *blocks_per_cu);

}  // namespace mvd
