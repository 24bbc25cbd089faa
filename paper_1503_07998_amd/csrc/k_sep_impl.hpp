// Separable (rank-one PSF) forward and backward passes of plane-wise MV-RL.
//
// One work-group owns a strip of columns of one plane (normally the whole row)
// over a segment of rows, and walks down the segment in groups of G rows:
//
//   z pass  each thread owns one or two columns and keeps a ring of input rows
//           in registers; every group it loads G new rows (issued one group
//           ahead, so the loads overlap the arithmetic of the current group)
//           and computes G outputs of the K-tap column convolution with
//           compile-time ring indices.  Results go to LDS, one row per output.
//   x pass  threads read 8 consecutive row values plus the K−1 halo values with
//           128-bit LDS reads and compute the K-tap row convolution on the
//           matrix cores (two 4-output blocks), then run the fused epilogue.
//
// Forward epilogue:  r_v = φ_v / b_v  (b_v = ψ ⊛ P_v; 1 where b_v ≤ ε).  φ_v are
//                    read where the caller left them (uint16, or float32
//                    clamped at 0), through the layout's strides.
// Backward epilogue: ψ' = ψ · Π_v (w_v · q_v + 1 − w_v)  (q_v = r_v ⊛ X_v).
// (Supplementary Note 1 update; Supplementary Note 2 §1 back-projector.)
//
// The update reads ψ only at the output pixel, so ψ' may overwrite ψ.
// Included by k_sep_<K>.hip with MVD_KB defined: one compilation unit per
// kernel-size bucket.
#pragma once

#include <utility>

#include "mvd_internal.hpp"

// Rows per ring step and the namespace of this instantiation: the split-view
// backward kernels are compiled with 16-row groups in translation units of
// their own.
#ifndef MVD_SEP_G
#define MVD_SEP_G 8
#endif
#ifndef MVD_SEP_NS
#define MVD_SEP_NS sepk
#endif

namespace mvd {
namespace MVD_SEP_NS {

// Kernel arguments are read through the kernarg segment pointer (constant
// address space): per-view fields are indexed with a runtime view number, and
// indexing the by-value parameter that way would make the compiler copy the
// whole argument block to scratch.  Through this pointer the loads are
// uniform scalar loads.
typedef __attribute__((address_space(4))) const SepPassArgs KArg;
typedef __attribute__((address_space(4))) const float KFloat;

__device__ __forceinline__ KArg *kargs() {
  return (KArg *)__builtin_amdgcn_kernarg_segment_ptr();
}

constexpr int G = MVD_SEP_G;   // rows per ring step
constexpr int NX = 8;          // x-pass outputs per work item

template <int KB>
struct Shape {
  static constexpr int R = (KB - 1) / 2;
  // ring slots: the current group's G+K−1 rows plus the next group's G rows
  static constexpr int M = G * ((2 * G + KB - 1 + G - 1) / G);
  static constexpr int U = M / G;                  // ring phases
  static constexpr int NIN4 = (NX + KB - 1 + 3) / 4;
  // column pass on the matrix cores: a block of 4 output rows takes input rows
  // k = 0 … KB + 2 of its window; per view a [4][NK] tap table in LDS
  static constexpr int NK = (KB + 3 + 3) / 4 * 4;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Tap table of the matrix-core column pass: TT[i][k] = tz[i + KB − 1 − k], the
// tap that input row k of a 4-row block contributes to its output row i (zero
// off the kernel).  Filled once per work-group; the caller synchronises.
template <int KB>
__device__ __forceinline__ void fill_tap_table(float *TT, KArg *a, int nviews, int t, int nt) {
  constexpr int NK = Shape<KB>::NK;
  for (int e = t; e < nviews * 8 * NK; e += nt) {
    const int v = e / (8 * NK), x = (e / (4 * NK)) & 1, i = (e / NK) % 4, k = e % NK;
    const int j = i + KB - 1 - k;
    TT[e] = (j >= 0 && j < KB) ? (x ? a->tx[v][j] : a->tz[v][j]) : 0.f;
  }
}

// Tap tables of view v: [4][NK] for the column pass, then [4][NK] for the row pass.
template <int KB>
__device__ __forceinline__ const float *ztab(const float *tt, int v) { return tt + v * 8 * Shape<KB>::NK; }
template <int KB>
__device__ __forceinline__ const float *xtab(const float *tt, int v) {
  return tt + v * 8 * Shape<KB>::NK + 4 * Shape<KB>::NK;
}

// LDS-only barrier: waits for this wave's LDS traffic, not for its global
// loads, so the next group's prefetched rows stay in flight across it.
__device__ __forceinline__ void lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Work-groups are dealt round-robin to the 8 XCDs; remap so that each XCD
// gets a contiguous run of (plane, segment, strip) tiles and neighbouring
// segments share its L2.
__device__ __forceinline__ int logical_block() {
  const int n = gridDim.x, b = blockIdx.x;
  if ((n & 7) == 0) return (b & 7) * (n >> 3) + (b >> 3);
  return b;
}

struct Geo {
  int y, zs, ze, ngroups, xo0, xout;
  size_t plane_off;
};

// Geometry of tile b of a pass: (plane, segment, strip), strip fastest.
__device__ __forceinline__ Geo tile_geo(KArg *a, int b) {
  Geo o;
  const int strip = b % a->nstrip;
  b /= a->nstrip;
  const int seg = b % a->nseg;
  const int y = b / a->nseg;
  o.zs = seg * a->zseg;
  o.ze = min(o.zs + a->zseg, a->g.Z);
  o.ngroups = (o.ze - o.zs + G - 1) / G;
  o.xo0 = strip * a->x_out;
  o.xout = min(a->x_out, a->g.X - o.xo0);
  o.y = y;
  o.plane_off = (size_t)y * a->g.Z * a->g.X;
  return o;
}

// Barriers a tile executes: one after its set-up, one per row group.
__device__ __forceinline__ int tile_barriers(KArg *a, int b) { return 1 + tile_geo(a, b).ngroups; }

// Column bookkeeping of the z pass for one thread.
template <int C, int R>
struct Cols {
  int gx[C];     // source column in the plane
  int lcol[C];   // LDS column
  bool act[C];   // thread owns a z-pass column
  bool ok[C];    // column lies in the plane (else its values are 0)

  __device__ __forceinline__ Cols(KArg *a, const Geo &o, int t, int nt) {
    const bool halo = a->halo != 0;
    const int ncz = halo ? o.xout + 2 * R : o.xout;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int lc = t + c * nt;
      act[c] = lc < ncz;
      int x = halo ? o.xo0 - R + lc : lc;
      if (a->boundary == 0) {
        ok[c] = act[c] && x >= 0 && x < a->g.X;
      } else {
        ok[c] = act[c];
        x = wrapi(x, a->g.X);
      }
      gx[c] = ok[c] ? x : 0;   // always a valid address; the value is dropped when !ok
      lcol[c] = halo ? lc : lc + R;
    }
  }
};

// Zero the LDS pad columns of a whole-row strip: [0, R) and [R+X, ldsw).
template <int R>
__device__ __forceinline__ void zero_pads(float *lds, int nrows, KArg *a, int t,
                                          int nt) {
  const int right = a->ldsw - (R + a->g.X);
  const int per = R + right;
  for (int e = t; e < nrows * per; e += nt) {
    const int row = e / per, p = e - row * per;
    const int col = p < R ? p : R + a->g.X + (p - R);
    lds[row * a->ldsw + col] = 0.f;
  }
}

// A row of zeros standing in for the rows outside the plane under the zero
// boundary (zero-initialised device memory, never written).
__device__ float kZeroRow[kMaxPlaneX];

// Load input row `rr` (plane coordinates, may lie outside) for this thread's
// columns.  The row pointer is chosen per row (uniform): the plane row, its
// wrapped copy, or the zero row.  Every lane loads from a valid address and the
// loaded value is used as is, so the loads stay unconditional and the compiler
// waits for them only where the ring slot is consumed, a group later.  Columns
// outside the plane are zeroed when the column-pass result is stored.
template <int C, int R>
__device__ __forceinline__ void load_row(const float *__restrict__ src, int rr, KArg *a,
                                         const Cols<C, R> &cl, float *dst /* [C] stride M */,
                                         int stride) {
  const int Z = a->g.Z;
  const float *row;
  if (a->boundary == 0) {
    // a plane holds at most 2^31 elements (checked when a context is made),
    // so the row offset fits 32 unsigned bits
    row = (unsigned)rr < (unsigned)Z ? src + (unsigned)rr * (unsigned)a->g.X : kZeroRow;
  } else {
    // a real branch: the modulo of the periodic rule is not evaluated for
    // zero-boundary rows (a select would compute it for every row)
    row = src + (size_t)wrapi(rr, Z) * a->g.X;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) dst[c * stride] = row[cl.gx[c]];
}

// LDS row pitch as an opaque per-use value: keeps the compiler from hoisting
// one precomputed LDS address per row into registers across the whole loop
// (an add per store is far cheaper than the registers).
__device__ __forceinline__ int lds_pitch(KArg *a) {
  int p = a->ldsw;
  asm volatile("" : "+s"(p));
  return p;
}

// Write one z-pass output (row g of the current buffer).  Whole-row strips
// (no x halo) are planned for the zero boundary only, so their pad columns
// stay zero and every active column lies in the plane; strips with a halo
// zero the columns outside the plane (zero boundary) or hold wrapped columns.
template <int C, int R, bool MASK>
__device__ __forceinline__ void store_mid(float *B, int g, KArg *a, const Cols<C, R> &cl,
                                          int c, float v) {
  if (!cl.act[c]) return;
  if (MASK) v = cl.ok[c] ? v : 0.f;   // column outside the plane (zero boundary)
  B[g * lds_pitch(a) + cl.lcol[c]] = v;
}

// K-tap row convolution of 8 consecutive outputs from one LDS row.
// Inputs are streamed 4 at a time (one 128-bit LDS read) and each is used for
// every output it touches before the next read, so only a handful of inputs
// are live: out[n] = Σ_i taps[i] · L[n + K − 1 − i].
template <int KB>
__device__ __forceinline__ void xconv_valu(const float *L, KFloat *taps, float (&out)[NX]) {
  using S = Shape<KB>;
#pragma unroll
  for (int n = 0; n < NX; ++n) out[n] = 0.f;
#pragma unroll
  for (int q = 0; q < S::NIN4; ++q) {
    const float4 f = *reinterpret_cast<const float4 *>(L + 4 * q);
    const float in4[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int p = 4 * q + e;
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const int i = n + KB - 1 - p;
        if (i >= 0 && i < KB) out[n] = fmaf(taps[i], in4[e], out[n]);
      }
    }
  }
}

// The same 8 outputs on the matrix cores, in two blocks of 4 (outputs 4b + i):
// out[4b + i] = Σ_k TX[i][k] · L[4b + k], TX[i][k] = taps[i + K − 1 − k], the
// row-pass form of the column pass's v_mfma_f32_4x4x1f32 scheme (B = this
// lane's own input, A = TX[lane % 4][k]); K + 3 steps per block against 4K
// vector multiply-adds.  Inputs are read 4 at a time; block 0 takes step k of
// chunk k / 4, block 1 the step that input fed block 0 four steps earlier.
// Every lane of the wave must take part (the caller keeps the loop uniform).
template <int KB>
__device__ __forceinline__ void xconv_mfma(const float *L, const float *TX, float (&out)[NX]) {
  using S = Shape<KB>;
  constexpr int NK = S::NK, KS = KB + 3;   // steps per block
  const float *tl = TX + (threadIdx.x & 3) * NK;
  f32x4 d0 = f32x4{0.f, 0.f, 0.f, 0.f}, d1 = f32x4{0.f, 0.f, 0.f, 0.f};
  float tp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < S::NIN4; ++q) {
    const float4 f = *reinterpret_cast<const float4 *>(L + 4 * q);
    const float in4[4] = {f.x, f.y, f.z, f.w};
    float tc[4] = {0.f, 0.f, 0.f, 0.f};
    if (4 * q < KS) {
      const float4 t4 = *reinterpret_cast<const float4 *>(tl + 4 * q);
      tc[0] = t4.x;
      tc[1] = t4.y;
      tc[2] = t4.z;
      tc[3] = t4.w;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (4 * q + e < KS) d0 = __builtin_amdgcn_mfma_f32_4x4x1f32(tc[e], in4[e], d0, 0, 0, 0);
      if (q >= 1 && 4 * (q - 1) + e < KS) d1 = __builtin_amdgcn_mfma_f32_4x4x1f32(tp[e], in4[e], d1, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tp[e] = tc[e];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[i] = d0[i];
    out[4 + i] = d1[i];
  }
}

#ifndef MVD_ROW_MFMA
#define MVD_ROW_MFMA 1
#endif

// Row pass of one item from LDS row L: matrix cores (default) or vector ALUs.
template <int KB>
__device__ __forceinline__ void xconv(const float *L, const float *TX, KFloat *taps, float (&out)[NX]) {
#if MVD_ROW_MFMA
  xconv_mfma<KB>(L, TX, out);
#else
  xconv_valu<KB>(L, taps, out);
#endif
}

// Per-work-group constants of a pass.
struct Loop {
  int t, nt, bufsz, rbase, nxb, nitems;
  bool vec;          // whole 8-wide items, 16-byte aligned rows: 128-bit loads and stores
  const float *tt;   // tap tables of the column pass, [views][4][NK]
};

// Geometry of one row-pass work item (row g of the group, 8 output columns).
struct Item {
  bool valid;
  int g, ox, nvalid;
  int z, x;      // row and first column in the plane (clamped like off)
  size_t off;    // in the plane set
  size_t soff;   // in the forward pass's observations
};

// Items are dealt to lanes in pairs of rows: lane pairs (2p, 2p+1) take the same
// 8 columns of rows 2q and 2q+1.  The LDS row pitch is 4 (mod 8) floats, so of
// the 8 lanes that share an LDS cycle, those on the odd row read 16-byte
// chunks in the bank groups the even-row lanes leave free.
__device__ __forceinline__ Item item_at(int it, const Loop &st, const Geo &o, int i, KArg *a) {
  Item r;
  const int itc = min(it, st.nitems - 1);
  const int pr = itc >> 1;
  const int gp = pr / st.nxb;
  const int xb = pr - gp * st.nxb;
  r.g = 2 * gp + (itc & 1);
  const int z = o.zs + i * G + r.g;
  r.valid = it < st.nitems && z < o.ze;
  r.ox = xb * NX;
  r.nvalid = min(NX, o.xout - r.ox);
  // rows past the segment are clamped to its first row: a valid address whose data is unused
  const int zc = r.valid ? z : o.zs;
  r.z = zc;
  r.x = o.xo0 + r.ox;
  r.off = o.plane_off + (size_t)zc * a->g.X + o.xo0 + r.ox;
  r.soff = (size_t)o.y * a->obs_sy + (size_t)zc * a->obs_sz + o.xo0 + r.ox;
  return r;
}

// Row-pass access mode: VM = 1 two 128-bit accesses per item (every item is
// whole and 16-byte aligned), 0 element-wise within the row, 2 chosen at run
// time from `vec`.  A run-time choice makes both forms join in the same
// registers, and the copies at the join wait for the loads at once; the fixed
// forms let the loads stay in flight until their values are used.
template <int VM>
__device__ __forceinline__ bool vec_mode(bool vec) {
  return VM == 2 ? vec : VM == 1;
}

// 8 values at p (see vec_mode).
template <int VM>
__device__ __forceinline__ void load8(const float *__restrict__ p, int nvalid, bool vec, float (&v)[NX]) {
  if (vec_mode<VM>(vec)) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int n = 0; n < NX; ++n) v[n] = n < nvalid ? p[n] : 0.f;
  }
}

template <int VM>
__device__ __forceinline__ void store8(float *__restrict__ p, int nvalid, bool vec, const float (&v)[NX]) {
  if (vec_mode<VM>(vec)) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4 *>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int n = 0; n < NX; ++n)
      if (n < nvalid) p[n] = v[n];
  }
}

// Column pass of one group for one input ring: G output rows per column, on the
// matrix cores.  v_mfma_f32_4x4x1f32 treats the wave as 16 blocks of 4 lanes:
// lane 4b + i supplies A[i] and lane 4b + j supplies B[j] of block b, and
// register i of lane 4b + j receives D[i][j] += A[i]·B[j].  With B = this
// lane's ring register of input row k (its own column) and A = TT[lane % 4][k],
// register i of every lane accumulates output row g0 + i of its own column:
// Σ_k tz[i + KB − 1 − k] · in[g0 + k].  A 4-row block needs input rows
// k = 0 … KB + 2 only (all in the current group's window), KB + 3 steps against
// 4·KB multiply-adds on the vector ALUs.
template <int KB, int C, int u>
__device__ __forceinline__ void zpass(const float *TT, const float (&ring)[C][Shape<KB>::M], float (&acc)[C][G]) {
  constexpr int M = Shape<KB>::M, NK = Shape<KB>::NK, NB = G / 4;
  const float *tl = TT + (threadIdx.x & 3) * NK;
  f32x4 d[C][NB];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) d[c][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kq = 0; kq < NK / 4; ++kq) {
    const float4 t4 = *reinterpret_cast<const float4 *>(tl + 4 * kq);
    const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * kq + e;
      if (k > KB + 2) continue;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < C; ++c)
          d[c][b] = __builtin_amdgcn_mfma_f32_4x4x1f32(tv[e], ring[c][(u * G + 4 * b + k) % M], d[c][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[c][4 * b + i] = d[c][b][i];
}

template <int KB, int C>
__device__ __forceinline__ void store_group(float *B, KArg *a, const Cols<C, Shape<KB>::R> &cl,
                                            const float (&acc)[C][G]) {
  if (a->halo == 0) {   // uniform: whole rows need no mask
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < C; ++c) store_mid<C, Shape<KB>::R, false>(B, g, a, cl, c, acc[c][g]);
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < C; ++c) store_mid<C, Shape<KB>::R, true>(B, g, a, cl, c, acc[c][g]);
  }
}

// ---------------------------------------------------------------------------
// Single-input passes: one input plane set convolved with NV views' kernels,
// each view's result finished by the epilogue EP:
//   kRatio  out = φ / conv (guarded)                 forward pass of the update
//   kStore  out = conv                               (adjoint: q = r ⊛ X)
//   kBR     out = conv (b), out2 = φ / conv (r)      (adjoint: recompute b and r)
//   kBbar   out = −conv · r / b where b > ε, else 0 (adjoint: b̄ from r̄)
//   kAccum  out = aux0 + conv                        (adjoint: ψ̄ += b̄ ⊛ P^*; the
//                                                    middle terms of a low-rank kernel)
//   kAccumRatio   out = φ / (aux0 + conv), φ at aux1 (last term of a low-rank P_v)
//   kAccumUpdate  out = ψ · (w (aux0 + conv) + 1 − w), ψ at aux1 (last term of a
//                 low-rank X_v; out may be ψ itself: read and written at one pixel)
// ---------------------------------------------------------------------------
template <int EP>
struct Epi {
  static constexpr int nops = (EP == kEpBbar || EP == kEpAccumRatio || EP == kEpAccumUpdate ||
                               EP == kEpTermsRatio || EP == kEpTermsUpdate) ? 2
                              : (EP == kEpStore ? 0 : 1);
  static constexpr int nbuf = nops > 0 ? nops : 1;
};

// Epilogue operands of one item: float32 values, or for uint16 observations
// the raw 16-bit pairs (converted where they are used, so the loads can stay
// in flight through the column pass).
template <int EP, int NV>
struct Ops {
  float f[NV][Epi<EP>::nbuf][NX];
};
template <int NV>
struct Ops<kEpRatioU16, NV> {
  uint32_t u[NV][NX / 2];
};

template <int EP>
__device__ __forceinline__ const float *op_ptr(KArg *a, int v, int k) {
  if (EP == kEpBR) return a->phi[v];
  return k == 0 ? a->aux0[v] : a->aux1[v];
}

// φ of element n of an item for the ratio epilogues.
template <int EP, int NV>
__device__ __forceinline__ float obs_at(const Ops<EP, NV> &ops, int v, int n) {
  if constexpr (EP == kEpRatioU16)
    return (float)((ops.u[v][n >> 1] >> (16 * (n & 1))) & 0xffffu);
  else if constexpr (EP == kEpRatio)
    return fmaxf(ops.f[v][0][n], 0.f);
  else
    return ops.f[v][0][n];
}

// Row pass and epilogue of one item for every view; the row pass runs on every
// lane (invalid items at clamped addresses), only valid items store.
template <int KB, int NV, int EP, int VM>
__device__ __forceinline__ void single_epilogue(KArg *a, const float *buf, const float *tt, const Item &itm,
                                                bool vec, const Ops<EP, NV> &ops) {
  if constexpr (ep_terms(EP)) {
    // the terms of one kernel: their sum (after the partial sum of earlier
    // terms, in term order) finishes one output; operands in slot 0
    float s[NX];
#pragma unroll
    for (int n = 0; n < NX; ++n) s[n] = ops.f[0][0][n];   // zeros without a partial sum
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float b[NX];
      xconv<KB>(buf + (v * G + itm.g) * lds_pitch(a) + itm.ox, xtab<KB>(tt, v), a->tx[v], b);
#pragma unroll
      for (int n = 0; n < NX; ++n) s[n] += b[n];
    }
    if (!itm.valid) return;
    float r[NX];
    if constexpr (EP == kEpTermsSum) {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = s[n];
    } else if constexpr (EP == kEpTermsRatio) {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = guarded_ratio(ops.f[0][1][n], s[n]);
    } else {
      const float w = a->w[0], w1 = 1.f - w;
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = ops.f[0][1][n] * fmaf(w, s[n], w1);
    }
    store8<VM>(a->out[0] + itm.off, itm.nvalid, vec, r);
    return;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float b[NX];
    xconv<KB>(buf + (v * G + itm.g) * lds_pitch(a) + itm.ox, xtab<KB>(tt, v), a->tx[v], b);
    if (!itm.valid) continue;
    float r[NX];
    if constexpr (EP == kEpRatio || EP == kEpRatioU16) {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = guarded_ratio(obs_at(ops, v, n), b[n]);
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, r);
    } else if constexpr (EP == kEpStore) {
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, b);
    } else if constexpr (EP == kEpBR) {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = guarded_ratio(obs_at(ops, v, n), b[n]);
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, b);
      store8<VM>(a->out2[v] + itm.off, itm.nvalid, vec, r);
    } else if constexpr (EP == kEpBbar) {
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const float bb = ops.f[v][1][n];
        const float q = nr_quotient(b[n] * ops.f[v][0][n], bb);
        r[n] = bb > kEps ? -q : 0.f;
      }
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, r);
    } else if constexpr (EP == kEpAccumRatio) {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = guarded_ratio(ops.f[v][1][n], ops.f[v][0][n] + b[n]);
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, r);
    } else if constexpr (EP == kEpAccumUpdate) {
      const float w = a->w[v], w1 = 1.f - w;
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = ops.f[v][1][n] * fmaf(w, ops.f[v][0][n] + b[n], w1);
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, r);
    } else {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = ops.f[v][0][n] + b[n];
      store8<VM>(a->out[v] + itm.off, itm.nvalid, vec, r);
    }
  }
}

template <int NV, int EP, int VM>
__device__ __forceinline__ void load_ops(KArg *a, const Item &itm, bool vec, Ops<EP, NV> &ops) {
  if constexpr (ep_terms(EP)) {
    // one output: the partial sum (aux0, or zeros) and the ratio's φ or the update's ψ (aux1)
    if (a->aux0[0]) {
      load8<VM>(a->aux0[0] + itm.off, itm.nvalid, vec, ops.f[0][0]);
    } else {
#pragma unroll
      for (int n = 0; n < NX; ++n) ops.f[0][0][n] = 0.f;
    }
    if constexpr (Epi<EP>::nops > 1) load8<VM>(a->aux1[0] + itm.off, itm.nvalid, vec, ops.f[0][1]);
    return;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (EP == kEpRatioU16) {
      const uint16_t *p = static_cast<const uint16_t *>(a->obs[v]) + itm.soff;
      if (vec_mode<VM>(vec)) {
        const uint4 w = *reinterpret_cast<const uint4 *>(p);
        ops.u[v][0] = w.x;
        ops.u[v][1] = w.y;
        ops.u[v][2] = w.z;
        ops.u[v][3] = w.w;
      } else {
#pragma unroll
        for (int h = 0; h < NX / 2; ++h) {
          const uint32_t lo = 2 * h < itm.nvalid ? p[2 * h] : 0u;
          const uint32_t hi = 2 * h + 1 < itm.nvalid ? p[2 * h + 1] : 0u;
          ops.u[v][h] = lo | (hi << 16);
        }
      }
    } else if constexpr (EP == kEpRatio) {
      load8<VM>(static_cast<const float *>(a->obs[v]) + itm.soff, itm.nvalid, vec, ops.f[v][0]);
    } else {
#pragma unroll
      for (int k = 0; k < Epi<EP>::nops; ++k)
        load8<VM>(op_ptr<EP>(a, v, k) + itm.off, itm.nvalid, vec, ops.f[v][k]);
    }
  }
}

// One ring phase: group i = i0 + u.  u is a compile-time constant so every
// ring index below is one too and the ring stays in registers.
template <int KB, int C, int NV, int EP, int VM, int u>
__device__ __forceinline__ void fwd_group(KArg *a, const Geo &o, const Cols<C, Shape<KB>::R> &cl,
                                          const float *__restrict__ src, float *lds, const Loop &st,
                                          float (&ring)[C][Shape<KB>::M], int i0) {
  constexpr int M = Shape<KB>::M, R = Shape<KB>::R;
  const int i = i0 + u;
  if (i >= o.ngroups) return;
  // 1. loads issued now and consumed later: this thread's first row-pass
  //    operands, then the next group's rows (past the segment end they are
  //    clamped and unused).  The column pass below covers their latency.
  //    Memory loads retire in issue order, so the operands go first: the row
  //    pass can then wait for them while the rows stay in flight.
  const Item first = item_at(st.t, st, o, i, a);
  Ops<EP, NV> ops;
  load_ops<NV, EP, VM>(a, first, st.vec, ops);
#pragma unroll
  for (int g = 0; g < G; ++g)
    load_row<C, R>(src, st.rbase + (i + 1) * G + KB - 1 + g, a, cl,
                   &ring[0][((u + 1) * G + KB - 1 + g) % M], M);
  // 2. column pass → LDS
  float *buf = lds + (i & 1) * st.bufsz;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float acc[C][G];
    zpass<KB, C, u>(ztab<KB>(st.tt, v), ring, acc);
    store_group<KB, C>(buf + v * G * lds_pitch(a), a, cl, acc);
  }
  lds_sync();
  // 3. row pass + epilogue, in wave-uniform steps over the items
  single_epilogue<KB, NV, EP, VM>(a, buf, st.tt, first, st.vec, ops);
  for (int base = st.nt; base < st.nitems; base += st.nt) {
    const Item itm = item_at(base + st.t, st, o, i, a);
    Ops<EP, NV> q;
    load_ops<NV, EP, VM>(a, itm, st.vec, q);
    single_epilogue<KB, NV, EP, VM>(a, buf, st.tt, itm, st.vec, q);
  }
}

template <int KB, int C, int NV, int EP, int VM, int... us>
__device__ __forceinline__ void fwd_phases(KArg *a, const Geo &o, const Cols<C, Shape<KB>::R> &cl,
                                           const float *__restrict__ src, float *lds, const Loop &st,
                                           float (&ring)[C][Shape<KB>::M], int i0,
                                           std::integer_sequence<int, us...>) {
  (fwd_group<KB, C, NV, EP, VM, us>(a, o, cl, src, lds, st, ring, i0), ...);
}

// One tile of a single-input pass (the forward pass and the adjoint's
// single-view passes) by threads t = 0 … nt−1 (whole waves) with LDS at `lds`.
// Every wave of the work-group must execute the same barriers: 1 + the tile's
// row groups (tile_barriers).
template <int KB, int C, int NV, int EP, int VM>
__device__ __forceinline__ void fwd_tile(KArg *a, int b, int t, int nt, float *lds) {
  using S = Shape<KB>;
  constexpr int R = S::R, M = S::M, U = S::U;
  const Geo o = tile_geo(a, b);
  const Cols<C, R> cl(a, o, t, nt);
  if (a->halo == 0) zero_pads<R>(lds, 2 * NV * G, a, t, nt);
  const int nxb = (o.xout + NX - 1) / NX;
  float *tt = lds + 2 * NV * G * a->ldsw;
  fill_tap_table<KB>(tt, a, NV, t, nt);
  lds_sync();
  const Loop st{t, nt, NV * G * a->ldsw, o.zs - R, nxb, G * nxb, a->vec != 0, tt};
  const float *__restrict__ src = a->in[0] + o.plane_off;
  float ring[C][M];
#pragma unroll
  for (int m = 0; m < G + KB - 1; ++m) load_row<C, R>(src, st.rbase + m, a, cl, &ring[0][m], M);
  for (int i0 = 0; i0 < o.ngroups; i0 += U)
    fwd_phases<KB, C, NV, EP, VM>(a, o, cl, src, lds, st, ring, i0, std::make_integer_sequence<int, U>{});
}

// OCC: minimum waves per SIMD the register budget must allow (second
// launch-bounds argument): 4 caps a thread at 128 VGPRs, 2 at 256.
// Work-groups of up to 2·kSepMaxThreads threads in the 4-waves/SIMD form (rows
// up to 1024 columns, one column per thread), kSepMaxThreads otherwise.
template <int KB, int C, int NV, int OCC, int EP, int VM>
__global__ void __launch_bounds__(OCC >= 4 ? 2 * kSepMaxThreads : kSepMaxThreads, OCC)
    sep_forward_kernel(const SepPassArgs) {
  extern __shared__ __align__(16) float lds[];
  fwd_tile<KB, C, NV, EP, VM>(kargs(), logical_block(), threadIdx.x, blockDim.x, lds);
}

// ---------------------------------------------------------------------------
// Backward pass: VIN ratio planes → ψ' = ψ · Π_v (w_v q_v + 1 − w_v).
// ---------------------------------------------------------------------------
template <int KB, int VIN, int VM, int EB>
__device__ __forceinline__ void bwd_epilogue(KArg *a, const float *buf, const float *tt, const Item &itm, bool vec,
                                             float (&ps)[NX]) {
  // ψ · c_0 · c_1 … applied view by view: the same rounding as one launch per view
#pragma unroll
  for (int v = 0; v < VIN; ++v) {
    float q[NX];
    xconv<KB>(buf + (v * G + itm.g) * lds_pitch(a) + itm.ox, xtab<KB>(tt, v), a->tx[v], q);
    if constexpr (EB & 1) {   // EM normalisation: q / (1 ⊛ X_v) where that exceeds ε
      const float sz = a->nsz[v][itm.z];
      float sx[NX];
      load8<VM>(a->nsx[v] + itm.x, itm.nvalid, vec, sx);
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const float sv = sz * sx[n];
        q[n] = sv > kEps ? q[n] * __builtin_amdgcn_rcpf(sv) : q[n];
      }
    }
    const float w = a->w[v], w1 = 1.f - w;
    if constexpr (EB & 2) {   // per-pixel weights: ω = w · ω_v(pixel)
      float om[NX];
      load8<VM>(a->wpl[v] + itm.off, itm.nvalid, vec, om);
#pragma unroll
      for (int n = 0; n < NX; ++n) {
        const float o = w * om[n];
        ps[n] *= fmaf(o, q[n], 1.f - o);
      }
    } else {
#pragma unroll
      for (int n = 0; n < NX; ++n) ps[n] *= fmaf(w, q[n], w1);
    }
  }
  if (itm.valid) store8<VM>(a->psi_out + itm.off, itm.nvalid, vec, ps);
}

template <int KB, int C, int VIN, int VM, int EB, int u>
__device__ __forceinline__ void bwd_group(KArg *a, const Geo &o, const Cols<C, Shape<KB>::R> &cl,
                                          float *lds, const Loop &st, float (&ring)[VIN][C][Shape<KB>::M],
                                          int i0) {
  constexpr int M = Shape<KB>::M, R = Shape<KB>::R;
  const int i = i0 + u;
  if (i >= o.ngroups) return;
  // column pass on the matrix cores first, then ψ of the first item, then the
  // next group's rows: ψ is not live while the rings are busiest, and since
  // memory loads retire in order the row pass can wait for ψ with the rows
  // still in flight (the prefetched slots are outside this group's window)
  float *buf = lds + (i & 1) * st.bufsz;
#pragma unroll
  for (int v = 0; v < VIN; ++v) {
    float acc[C][G];
    zpass<KB, C, u>(ztab<KB>(st.tt, v), ring[v], acc);
    store_group<KB, C>(buf + v * G * lds_pitch(a), a, cl, acc);
  }
  const Item first = item_at(st.t, st, o, i, a);
  float ps[NX];
  load8<VM>(a->psi_in + first.off, first.nvalid, st.vec, ps);
#pragma unroll
  for (int v = 0; v < VIN; ++v) {
    const float *__restrict__ src = a->in[v] + o.plane_off;
#pragma unroll
    for (int g = 0; g < G; ++g)
      load_row<C, R>(src, st.rbase + (i + 1) * G + KB - 1 + g, a, cl,
                     &ring[v][0][((u + 1) * G + KB - 1 + g) % M], M);
  }
  lds_sync();
  bwd_epilogue<KB, VIN, VM, EB>(a, buf, st.tt, first, st.vec, ps);
  for (int base = st.nt; base < st.nitems; base += st.nt) {
    const Item itm = item_at(base + st.t, st, o, i, a);
    float q[NX];
    load8<VM>(a->psi_in + itm.off, itm.nvalid, st.vec, q);
    bwd_epilogue<KB, VIN, VM, EB>(a, buf, st.tt, itm, st.vec, q);
  }
}

template <int KB, int C, int VIN, int VM, int EB, int... us>
__device__ __forceinline__ void bwd_phases(KArg *a, const Geo &o, const Cols<C, Shape<KB>::R> &cl,
                                           float *lds, const Loop &st, float (&ring)[VIN][C][Shape<KB>::M],
                                           int i0, std::integer_sequence<int, us...>) {
  (bwd_group<KB, C, VIN, VM, EB, us>(a, o, cl, lds, st, ring, i0), ...);
}

// One tile of the backward pass by threads t = 0 … nt−1 with LDS at `lds`
// (barriers as fwd_tile).
template <int KB, int C, int VIN, int VM, int EB>
__device__ __forceinline__ void bwd_tile(KArg *a, int b, int t, int nt, float *lds) {
  using S = Shape<KB>;
  constexpr int R = S::R, M = S::M, U = S::U;
  const Geo o = tile_geo(a, b);
  const Cols<C, R> cl(a, o, t, nt);
  if (a->halo == 0) zero_pads<R>(lds, 2 * VIN * G, a, t, nt);
  const int nxb = (o.xout + NX - 1) / NX;
  float *tt = lds + 2 * VIN * G * a->ldsw;
  fill_tap_table<KB>(tt, a, VIN, t, nt);
  lds_sync();
  const Loop st{t, nt, VIN * G * a->ldsw, o.zs - R, nxb, G * nxb, a->vec != 0, tt};
  float ring[VIN][C][M];
#pragma unroll
  for (int v = 0; v < VIN; ++v) {
    const float *__restrict__ src = a->in[v] + o.plane_off;
#pragma unroll
    for (int m = 0; m < G + KB - 1; ++m) load_row<C, R>(src, st.rbase + m, a, cl, &ring[v][0][m], M);
  }
  for (int i0 = 0; i0 < o.ngroups; i0 += U)
    bwd_phases<KB, C, VIN, VM, EB>(a, o, cl, lds, st, ring, i0, std::make_integer_sequence<int, U>{});
}

template <int KB, int C, int VIN, int OCC, int VM, int EB>
__global__ void __launch_bounds__(OCC >= 4 ? 2 * kSepMaxThreads : kSepMaxThreads, OCC)
    sep_backward_kernel(const SepPassArgs) {
  extern __shared__ __align__(16) float lds[];
  bwd_tile<KB, C, VIN, VM, EB>(kargs(), logical_block(), threadIdx.x, blockDim.x, lds);
}

// Double-buffered column-pass rows and the tap tables of both passes.
template <int KB>
inline size_t lds_bytes(const SepPassArgs &a, int nviews) {
  return sizeof(float) * (2ull * nviews * G * a.ldsw + (size_t)nviews * 8 * Shape<KB>::NK);
}

template <typename K>
inline hipError_t launch_with_lds(K kern, const SepPassArgs &a, int threads, size_t lds,
                                  hipStream_t s) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // 128-bit row-pass accesses need whole 8-column items (checked on the host too)
  if (a.vec && (a.g.X % 8 != 0 || a.x_out % 8 != 0)) return hipErrorInvalidValue;
  // whole-row strips keep zero pad columns: zero boundary only
  if (a.halo == 0 && a.boundary != 0) return hipErrorInvalidValue;
  const unsigned nblocks = (unsigned)a.g.Y * a.nseg * a.nstrip;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int KB, int EP, int VM>
hipError_t forward_bucket_vm(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  const size_t lds = lds_bytes<KB>(a, a.nviews);
  const bool hi = p.occ >= 4;
  // more than kSepMaxThreads threads: the one-column 4-waves/SIMD kernels only
  if (p.threads > kSepMaxThreads && !(hi && p.cols == 1)) return hipErrorInvalidValue;
  if constexpr (KB <= 41) {
    // two columns per thread only where the ring still fits (the planner never asks otherwise)
    if (p.cols == 2) {
      if (a.nviews == 2) return launch_with_lds(sep_forward_kernel<KB, 2, 2, 2, EP, VM>, a, p.threads, lds, s);
      return launch_with_lds(sep_forward_kernel<KB, 2, 1, 2, EP, VM>, a, p.threads, lds, s);
    }
  }
  if (p.cols != 1) return hipErrorInvalidValue;
  if (a.nviews == 2) {
    if (hi) return launch_with_lds(sep_forward_kernel<KB, 1, 2, 4, EP, VM>, a, p.threads, lds, s);
    return launch_with_lds(sep_forward_kernel<KB, 1, 2, 2, EP, VM>, a, p.threads, lds, s);
  }
  if (hi) return launch_with_lds(sep_forward_kernel<KB, 1, 1, 4, EP, VM>, a, p.threads, lds, s);
  return launch_with_lds(sep_forward_kernel<KB, 1, 1, 2, EP, VM>, a, p.threads, lds, s);
}

// 128-bit accesses also need the observations' rows in whole 16-byte units.
inline bool obs_vec_ok(const SepPassArgs &a) {
  const long unit = a.obs_u16 ? 8 : 4;
  bool ok = a.obs_sy % unit == 0 && a.obs_sz % unit == 0;
  for (int v = 0; v < a.nviews; ++v) ok = ok && (uintptr_t)a.obs[v] % 16 == 0;
  return ok;
}

template <int KB>
hipError_t forward_bucket(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  if (a.vec && !obs_vec_ok(a)) return hipErrorInvalidValue;
  if (a.obs_u16)
    return a.vec ? forward_bucket_vm<KB, kEpRatioU16, 1>(a, p, s) : forward_bucket_vm<KB, kEpRatioU16, 0>(a, p, s);
  return a.vec ? forward_bucket_vm<KB, kEpRatio, 1>(a, p, s) : forward_bucket_vm<KB, kEpRatio, 0>(a, p, s);
}

// One-view single-input pass with an adjoint epilogue (kStore, kBR, kBbar, kAccum):
// two columns per thread element-wise or 128-bit (VM 2: chosen at run time),
// one column per thread with the access form fixed at compile time.
template <int KB, int EP>
hipError_t single_ep(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  const size_t lds = lds_bytes<KB>(a, 1);
  if (p.threads > kSepMaxThreads) return hipErrorInvalidValue;
  if constexpr (KB <= 41) {
    if (p.cols == 2) return launch_with_lds(sep_forward_kernel<KB, 2, 1, 2, EP, 2>, a, p.threads, lds, s);
  }
  if (p.cols != 1) return hipErrorInvalidValue;
  if constexpr (KB <= 31) {
    if (a.vec) return launch_with_lds(sep_forward_kernel<KB, 1, 1, 4, EP, 1>, a, p.threads, lds, s);
    return launch_with_lds(sep_forward_kernel<KB, 1, 1, 4, EP, 0>, a, p.threads, lds, s);
  }
  return launch_with_lds(sep_forward_kernel<KB, 1, 1, 2, EP, 2>, a, p.threads, lds, s);
}

// Two terms of one kernel per launch (one column per thread, 128-bit accesses).
template <int KB, int EP>
hipError_t terms_ep(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  if (p.cols != 1 || !a.vec || p.threads > 2 * kSepMaxThreads) return hipErrorInvalidValue;
  if constexpr (KB <= 41) {
    if (p.occ >= 4) return launch_with_lds(sep_forward_kernel<KB, 1, 2, 4, EP, 1>, a, p.threads, lds_bytes<KB>(a, 2), s);
  }
  if (p.threads > kSepMaxThreads) return hipErrorInvalidValue;
  return launch_with_lds(sep_forward_kernel<KB, 1, 2, 2, EP, 1>, a, p.threads, lds_bytes<KB>(a, 2), s);
}

template <int KB>
hipError_t single_bucket(const SepPassArgs &a, const SepPlan &p, int ep, hipStream_t s) {
  if (a.nviews == 2) {
    switch (ep) {
      case kEpTermsSum: return terms_ep<KB, kEpTermsSum>(a, p, s);
      case kEpTermsRatio: return terms_ep<KB, kEpTermsRatio>(a, p, s);
      case kEpTermsUpdate: return terms_ep<KB, kEpTermsUpdate>(a, p, s);
    }
    return hipErrorInvalidValue;
  }
  if (a.nviews != 1) return hipErrorInvalidValue;
  switch (ep) {
    case kEpStore: return single_ep<KB, kEpStore>(a, p, s);
    case kEpBR: return single_ep<KB, kEpBR>(a, p, s);
    case kEpBbar: return single_ep<KB, kEpBbar>(a, p, s);
    case kEpAccum: return single_ep<KB, kEpAccum>(a, p, s);
    case kEpAccumRatio: return single_ep<KB, kEpAccumRatio>(a, p, s);
    case kEpAccumUpdate: return single_ep<KB, kEpAccumUpdate>(a, p, s);
  }
  return hipErrorInvalidValue;
}

template <int KB, int VM, int EB>
hipError_t backward_bucket_vm(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  const size_t lds = lds_bytes<KB>(a, p.vin);
  const bool hi = p.occ >= 4;
  if (p.threads > kSepMaxThreads && !(hi && p.cols == 1 && p.vin == 1)) return hipErrorInvalidValue;
  if constexpr (KB <= 41) {
    if (p.vin == 2) return launch_with_lds(sep_backward_kernel<KB, 1, 2, 2, VM, EB>, a, p.threads, lds, s);
    if (p.cols == 2) return launch_with_lds(sep_backward_kernel<KB, 2, 1, 2, VM, EB>, a, p.threads, lds, s);
  }
  if (p.cols != 1 || p.vin != 1) return hipErrorInvalidValue;
  if (hi) return launch_with_lds(sep_backward_kernel<KB, 1, 1, 4, VM, EB>, a, p.threads, lds, s);
  return launch_with_lds(sep_backward_kernel<KB, 1, 1, 2, VM, EB>, a, p.threads, lds, s);
}

template <int KB, int EB>
hipError_t backward_bucket_eb(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  return a.vec ? backward_bucket_vm<KB, 1, EB>(a, p, s) : backward_bucket_vm<KB, 0, EB>(a, p, s);
}

// EB: bit 0 the EM normalisation (a.nsz set), bit 1 per-pixel weights (a.wpl
// set); separate instances so that the plain passes keep their registers.
template <int KB>
hipError_t backward_bucket(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  switch ((a.nsz[0] ? 1 : 0) | (a.wpl[0] ? 2 : 0)) {
    case 0: return backward_bucket_eb<KB, 0>(a, p, s);
    case 1: return backward_bucket_eb<KB, 1>(a, p, s);
    case 2: return backward_bucket_eb<KB, 2>(a, p, s);
    default: return backward_bucket_eb<KB, 3>(a, p, s);
  }
}

// ---------------------------------------------------------------------------
// Split-view backward pass for two ratio planes: a 1024-thread work-group whose
// first half keeps view 0's ring and second half view 1's, one ring per thread
// (one column each), so it fits 128 VGPRs and runs 4 waves/SIMD.  With 16-row
// groups the row pass has one item per thread covering both views:
// ψ' = ψ · c_0 · c_1 as in the two-plane pass.  Whole rows of X ≤ 512, or
// strips with halo columns whose ring columns fit a half.
// ---------------------------------------------------------------------------
template <int KB, int VM, int EB, int u>
__device__ __forceinline__ void bwd_split_group(KArg *a, const Geo &o, const Cols<1, Shape<KB>::R> &cl, float *lds,
                                                const Loop &st, float (&ring)[1][Shape<KB>::M], int i0, int view) {
  constexpr int M = Shape<KB>::M, R = Shape<KB>::R;
  const int i = i0 + u;
  if (i >= o.ngroups) return;
  float *buf = lds + (i & 1) * st.bufsz;
  {
    float acc[1][G];
    zpass<KB, 1, u>(ztab<KB>(st.tt, view), ring, acc);
    store_group<KB, 1>(buf + view * G * lds_pitch(a), a, cl, acc);
  }
  const Item first = item_at(st.t, st, o, i, a);
  float ps[NX];
  load8<VM>(a->psi_in + first.off, first.nvalid, st.vec, ps);
  const float *__restrict__ src = a->in[view] + o.plane_off;
#pragma unroll
  for (int g = 0; g < G; ++g)
    load_row<1, R>(src, st.rbase + (i + 1) * G + KB - 1 + g, a, cl, &ring[0][((u + 1) * G + KB - 1 + g) % M], M);
  lds_sync();
  bwd_epilogue<KB, 2, VM, EB>(a, buf, st.tt, first, st.vec, ps);
  for (int base = st.nt; base < st.nitems; base += st.nt) {
    const Item itm = item_at(base + st.t, st, o, i, a);
    float q[NX];
    load8<VM>(a->psi_in + itm.off, itm.nvalid, st.vec, q);
    bwd_epilogue<KB, 2, VM, EB>(a, buf, st.tt, itm, st.vec, q);
  }
}

template <int KB, int VM, int EB, int... us>
__device__ __forceinline__ void bwd_split_phases(KArg *a, const Geo &o, const Cols<1, Shape<KB>::R> &cl, float *lds,
                                                 const Loop &st, float (&ring)[1][Shape<KB>::M], int i0, int view,
                                                 std::integer_sequence<int, us...>) {
  (bwd_split_group<KB, VM, EB, us>(a, o, cl, lds, st, ring, i0, view), ...);
}

template <int KB, int VM, int EB>
__global__ void __launch_bounds__(2 * kSepMaxThreads, 4) sep_backward_split_kernel(const SepPassArgs) {
  KArg *a = kargs();
  using S = Shape<KB>;
  constexpr int R = S::R, M = S::M, U = S::U;
  extern __shared__ __align__(16) float lds[];
  const int nt = blockDim.x, t = threadIdx.x, half = nt / 2;
  const int view = t / half, tc = t - view * half;   // wave-uniform view
  const Geo o = tile_geo(a, logical_block());
  const Cols<1, R> cl(a, o, tc, half);
  if (a->halo == 0) zero_pads<R>(lds, 2 * 2 * G, a, t, nt);
  const int nxb = (o.xout + NX - 1) / NX;
  float *tt = lds + 2 * 2 * G * a->ldsw;
  fill_tap_table<KB>(tt, a, 2, t, nt);
  lds_sync();
  const Loop st{t, nt, 2 * G * a->ldsw, o.zs - R, nxb, G * nxb, a->vec != 0, tt};
  const float *__restrict__ src = a->in[view] + o.plane_off;
  float ring[1][M];
#pragma unroll
  for (int m = 0; m < G + KB - 1; ++m) load_row<1, R>(src, st.rbase + m, a, cl, &ring[0][m], M);
  for (int i0 = 0; i0 < o.ngroups; i0 += U)
    bwd_split_phases<KB, VM, EB>(a, o, cl, lds, st, ring, i0, view, std::make_integer_sequence<int, U>{});
}

template <int KB>
hipError_t backward_split_bucket(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  // 128-bit row-pass accesses only (the element-wise form would not fit 128 VGPRs);
  // each half holds one ring column per thread
  if (p.cols != 1 || p.vin != 2 || a.nviews != 2 || !a.vec || a.ncols > (int)(p.threads / 2))
    return hipErrorInvalidValue;
  const size_t lds = lds_bytes<KB>(a, 2);
  // (the plain update only: no registers are left for the epilogue variants)
  if (a.nsz[0] || a.wpl[0]) return hipErrorInvalidValue;
  return launch_with_lds(sep_backward_split_kernel<KB, 1, 0>, a, p.threads, lds, s);
}

}  // namespace MVD_SEP_NS
}  // namespace mvd

#define MVD_SEP_INSTANTIATE_SPLIT(KB)                                                      \
  namespace mvd {                                                                          \
  hipError_t sep_backward_split_kb##KB(const SepPassArgs &a, const SepPlan &p, hipStream_t s) { \
    return MVD_SEP_NS::backward_split_bucket<KB>(a, p, s);                                 \
  }                                                                                        \
  }

#define MVD_SEP_INSTANTIATE(KB)                                                            \
  namespace mvd {                                                                          \
  hipError_t sep_forward_kb##KB(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {  \
    return sepk::forward_bucket<KB>(a, p, s);                                              \
  }                                                                                        \
  hipError_t sep_backward_kb##KB(const SepPassArgs &a, const SepPlan &p, hipStream_t s) { \
    return sepk::backward_bucket<KB>(a, p, s);                                             \
  }                                                                                        \
  hipError_t sep_single_kb##KB(const SepPassArgs &a, const SepPlan &p, int ep, hipStream_t s) { \
    return sepk::single_bucket<KB>(a, p, ep, s);                                           \
  }                                                                                        \
  }
