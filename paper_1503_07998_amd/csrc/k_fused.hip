// One whole iteration of the simultaneous two-view update in one launch
// (Supplementary Note 1 update: ψ' = ψ · Π_v [(φ_v / (ψ ⊛ P_v)) ⊛ X_v]).
//
// The forward and backward separable passes of the two-launch form write the
// ratio planes r_v to memory and read them back: 32 bytes per voxel and
// iteration with uint16 observations.  Here a work-group takes one strip of
// output columns of one plane over the whole plane height and keeps r_v on
// chip: ψ and φ_v are read once and ψ' is written once.
//
// Roles (wave-uniform, 5 waves each):
//   F  threads [0, 320): the forward column pass of both views.  Each thread
//      owns one column of the strip widened by RA + R on both sides (RA: the
//      forward output margin R rounded up to whole 8-column items) and keeps
//      a register ring of ψ rows, loaded one row group ahead.
//   B0 threads [320, 640), B1 [640, 960): the backward column pass of view 0
//      and 1.  Each thread owns one column of the strip widened by R and keeps
//      a register ring of r_v rows, fed from LDS.
// The three roles share one ring declaration, so a thread holds one ring.
//
// Per row group p (G rows), with the backward D groups behind the forward
// (D·G ≥ G + R: the back-projection of a group needs r_v up to R rows below
// it, and rows reach the r ring one group after they are computed):
//   1. F: column pass of group p (both views) → LDS; prefetch group p + 1.
//      B_v: column pass of group p − D → LDS.
//   2. barrier
//   3. forward row pass + ratio of group p, items spread over the F and B0
//      threads → r_v rows in LDS (zero outside the plane);
//      backward row pass + update of group p − D, items on the B1 threads:
//      ψ' = ψ · (w_0 q_0 + 1 − w_0) · (w_1 q_1 + 1 − w_1).
//   4. barrier
//   5. B_v: append group p's r_v rows (own column) to the ring.
// Every output is formed by the same operations in the same order as in the
// two-launch form (column pass, row pass, guarded ratio, product update), so
// results are bitwise the same.  Neighbouring strips read each other's ψ
// columns: ψ' must not overwrite ψ unless the plane is one strip.
#include "k_sep_impl.hpp"

namespace mvd {
namespace sepk {

typedef __attribute__((address_space(4))) const FusedArgs KFArg;

constexpr int kRoleThreads = kFusedThreads / 3;   // threads per role
static_assert(kRoleThreads % 64 == 0, "roles are whole waves");

template <int KB>
struct FShape {
  static constexpr int R = (KB - 1) / 2;
  static constexpr int RA = (R + NX - 1) / NX * NX;   // forward output margin (whole items)
  static constexpr int D = (G + R + G - 1) / G;       // backward lag in row groups
};

// Back-projector tap tables, laid out as fill_tap_table's.
template <int KB>
__device__ __forceinline__ void fill_back_taps(float *TT, KFArg *fa, int t, int nt) {
  constexpr int NK = Shape<KB>::NK;
  for (int e = t; e < 2 * 8 * NK; e += nt) {
    const int v = e / (8 * NK), x = (e / (4 * NK)) & 1, i = (e / NK) % 4, k = e % NK;
    const int j = i + KB - 1 - k;
    TT[e] = (j >= 0 && j < KB) ? (x ? fa->btx[v][j] : fa->btz[v][j]) : 0.f;
  }
}

// Row g and first column of item `it` of a G-row group with `nxb` items per
// row, dealt in pairs of rows as in the separable passes (bank-conflict-free
// 16-byte LDS reads with a pitch of 4 mod 8 floats).
struct FItem {
  int g, ox;
};
__device__ __forceinline__ FItem fitem(int it, int nxb) {
  const int pr = it >> 1;
  const int gp = pr / nxb;
  return FItem{2 * gp + (it & 1), (pr - gp * nxb) * NX};
}

// Per-thread constants of a work-group.  Everything but the item fields is
// the same across a wave (kept in scalar registers).
struct FCtx {
  int role, vb;                // role 0 F, 1 B (view vb)
  int y, x0, ngroups, nphases;
  int pitch;
  size_t plane_off;
  float *bufF, *bufT, *bufB;   // [2][G][pitch] each
  const float *ttF, *ttB;      // tap tables
  // a thread's row-pass item: a forward item (waves with threads < nfi; lanes
  // past nfi compute on item nfi − 1) or a backward item (waves from thread
  // 2·kRoleThreads on, nbi items); never both
  int fwave, bwave;
  bool own;                    // the item is real (else computed on a clamped item, not stored)
  int iv, ig, iox;             // forward: view; row in the group; first column in the LDS row
};

// Row-pass operands of one item, loaded a row group before they are used:
// φ_v for a forward item (uint16 as packed pairs in the first 4 entries) or ψ
// for a backward item (zeros where the item lies outside the plane).
template <int KB, int U16>
__device__ __forceinline__ void load_operands(KFArg *fa, const FCtx &c, int p, float (&o)[NX]) {
  KArg *a = &fa->f;
  const int Z = a->g.Z, X = a->g.X;
  float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
  if (c.fwave) {
    const int z = p * G + c.ig, fx = c.x0 - FShape<KB>::RA + c.iox;   // plane column
    const bool in = c.own && p < c.ngroups && z < Z && fx >= 0 && fx < X;
    const size_t s = (size_t)c.y * a->obs_sy + (size_t)z * a->obs_sz + fx;
    if constexpr (U16) {
      if (in) {
        const uint4 w = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(a->obs[c.iv]) + s);
        lo = make_float4(__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z), __uint_as_float(w.w));
      }
    } else if (in) {
      const float *src = static_cast<const float *>(a->obs[c.iv]) + s;
      lo = *reinterpret_cast<const float4 *>(src);
      hi = *reinterpret_cast<const float4 *>(src + 4);
    }
  }
  o[0] = lo.x; o[1] = lo.y; o[2] = lo.z; o[3] = lo.w;
  o[4] = hi.x; o[5] = hi.y; o[6] = hi.z; o[7] = hi.w;
}

__device__ __forceinline__ void load_psi(KFArg *fa, const FCtx &c, int j, float (&o)[NX]) {
  KArg *a = &fa->f;
  const int Z = a->g.Z, X = a->g.X;
  const int z = j * G + c.ig;
  float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
  const int bx = c.x0 + c.iox;
  if (c.own && j >= 0 && z < Z && bx < X) {
    const float *src = a->psi_in + c.plane_off + (size_t)z * X + bx;
    lo = *reinterpret_cast<const float4 *>(src);
    hi = *reinterpret_cast<const float4 *>(src + 4);
  }
  o[0] = lo.x; o[1] = lo.y; o[2] = lo.z; o[3] = lo.w;
  o[4] = hi.x; o[5] = hi.y; o[6] = hi.z; o[7] = hi.w;
}

template <int U16>
__device__ __forceinline__ float phi_at(const float (&o)[NX], int n) {
  if constexpr (U16)
    return (float)((__float_as_uint(o[n >> 1]) >> (16 * (n & 1))) & 0xffffu);
  else
    return fmaxf(o[n], 0.f);
}

template <int KB, int U16, int u>
__device__ __forceinline__ void fused_phase(KFArg *fa, const FCtx &c, const Cols<1, Shape<KB>::R> &cl,
                                            float (&ring)[1][Shape<KB>::M], float (&opA)[NX], float (&opB)[NX],
                                            int p0) {
  using S = Shape<KB>;
  using FS = FShape<KB>;
  constexpr int M = S::M, R = S::R, U = S::U, RA = FS::RA, D = FS::D;
  // u runs over two ring cycles, so that both the ring phase (u mod U) and the
  // operand arrays' parity (u mod 2) are compile-time constants
  constexpr int ur = u % U;
  constexpr int ub = ((ur - D) % U + U) % U;   // ring phase of the backward group
  KArg *a = &fa->f;
  const int p = p0 + u;
  if (p >= c.nphases) return;   // uniform
  const int j = p - D;
  const bool fon = p < c.ngroups, bon = j >= 0;
  const int Z = a->g.Z, X = a->g.X;

  // this group's row-pass operands were loaded a group ago; the next group's
  // are loaded now (the two arrays swap roles with the phase parity), then the
  // forward ring's next rows
  float(&cur)[NX] = (u & 1) ? opB : opA;
  float(&nxt)[NX] = (u & 1) ? opA : opB;
  const int zf = p * G + c.ig;
  const int fx = c.x0 - RA + c.iox, bx = c.x0 + c.iox;   // plane columns (forward / backward item)
  const bool fin = c.own && fon && zf < Z && fx >= 0 && fx < X;
  const int zb = j * G + c.ig;
  const bool bin = c.own && bon && zb < Z && bx < X;
  if (c.fwave)
    load_operands<KB, U16>(fa, c, p + 1, nxt);
  else if (c.bwave)
    load_psi(fa, c, j + 1, nxt);
  if (c.role == 0 && fon) {
    const float *__restrict__ src = a->psi_in + c.plane_off;
#pragma unroll
    for (int g = 0; g < G; ++g)
      load_row<1, R>(src, -R + (p + 1) * G + KB - 1 + g, a, cl, &ring[0][((ur + 1) * G + KB - 1 + g) % M], M);
  }
  // 2. column passes → LDS
  if (c.role == 0) {
    if (fon) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        float acc[1][G];
        zpass<KB, 1, ur>(ztab<KB>(c.ttF, v), ring, acc);
        store_group<KB, 1>(c.bufF + v * G * c.pitch, a, cl, acc);
      }
    }
  } else if (bon) {
    float acc[1][G];
    zpass<KB, 1, ub>(ztab<KB>(c.ttB, c.vb), ring, acc);
    store_group<KB, 1>(c.bufB + c.vb * G * c.pitch, a, cl, acc);
  }
  lds_sync();
  // 3. row passes
  if (c.fwave) {
    float r[NX];
    if (fon) {
      float b[NX];
      xconv<KB>(c.bufF + (c.iv * G + c.ig) * c.pitch + c.iox, xtab<KB>(c.ttF, c.iv), a->tx[c.iv], b);
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = fin ? guarded_ratio(phi_at<U16>(cur, n), b[n]) : 0.f;
    } else {
#pragma unroll
      for (int n = 0; n < NX; ++n) r[n] = 0.f;   // rows below the plane: r = 0
    }
    if (c.own) {
      float *dst = c.bufT + (c.iv * G + c.ig) * c.pitch + c.iox;
      *reinterpret_cast<float4 *>(dst) = make_float4(r[0], r[1], r[2], r[3]);
      *reinterpret_cast<float4 *>(dst + 4) = make_float4(r[4], r[5], r[6], r[7]);
    }
  }
  if (c.bwave && bon) {
    // ψ · c_0 · c_1, view by view as in the two-plane backward pass
    float ps[NX];
#pragma unroll
    for (int n = 0; n < NX; ++n) ps[n] = cur[n];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      float q[NX];
      xconv<KB>(c.bufB + (v * G + c.ig) * c.pitch + c.iox, xtab<KB>(c.ttB, v), fa->btx[v], q);
      const float w = a->w[v], w1 = 1.f - w;
#pragma unroll
      for (int n = 0; n < NX; ++n) ps[n] *= fmaf(w, q[n], w1);
    }
    if (bin) {
      float *dst = a->psi_out + c.plane_off + (size_t)zb * X + bx;
      *reinterpret_cast<float4 *>(dst) = make_float4(ps[0], ps[1], ps[2], ps[3]);
      *reinterpret_cast<float4 *>(dst + 4) = make_float4(ps[4], ps[5], ps[6], ps[7]);
    }
  }
  lds_sync();
  // 5. group p's ratio rows join the backward rings: r row z sits at ring index z + R
  if (c.role != 0 && cl.act[0]) {
    const float *src = c.bufT + c.vb * G * c.pitch + cl.lcol[0] + (RA - R);
#pragma unroll
    for (int g = 0; g < G; ++g) ring[0][(ur * G + g + R) % M] = src[g * c.pitch];
  }
}

template <int KB, int U16, int... us>
__device__ __forceinline__ void fused_phases(KFArg *fa, const FCtx &c, const Cols<1, Shape<KB>::R> &cl,
                                             float (&ring)[1][Shape<KB>::M], float (&opA)[NX], float (&opB)[NX],
                                             int p0, std::integer_sequence<int, us...>) {
  (fused_phase<KB, U16, us>(fa, c, cl, ring, opA, opB, p0), ...);
}

template <int KB, int U16>
__global__ void __launch_bounds__(1024, 4) fused_kernel(const FusedArgs) {
  using S = Shape<KB>;
  using FS = FShape<KB>;
  constexpr int R = S::R, M = S::M, U = S::U, NK = S::NK, RA = FS::RA, D = FS::D;
  KFArg *fa = (KFArg *)__builtin_amdgcn_kernarg_segment_ptr();
  KArg *a = &fa->f;
  extern __shared__ __align__(16) float lds[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int b = logical_block();
  FCtx c;
  c.role = __builtin_amdgcn_readfirstlane(t < kRoleThreads ? 0 : 1);
  c.vb = __builtin_amdgcn_readfirstlane(t < 2 * kRoleThreads ? 0 : 1);
  const int strip = b % a->nstrip;
  c.y = b / a->nstrip;
  c.x0 = strip * a->x_out;
  c.ngroups = (a->g.Z + G - 1) / G;
  c.nphases = c.ngroups + D;
  c.pitch = a->ldsw;
  c.plane_off = (size_t)c.y * a->g.Z * a->g.X;
  const int setf = 2 * G * c.pitch;
  c.bufF = lds;
  c.bufT = lds + setf;
  c.bufB = lds + 2 * setf;
  float *ttF = lds + 3 * setf;
  float *ttB = ttF + 2 * 8 * NK;
  c.ttF = ttF;
  c.ttB = ttB;
  // row-pass items (the strip width is the compile-time kFusedStrip)
  constexpr int nxbF = (kFusedStrip + 2 * RA) / NX, nfi = 2 * G * nxbF;
  constexpr int nxbB = kFusedStrip / NX, nbi = G * nxbB;
  static_assert(nfi <= 2 * kRoleThreads && nbi <= kRoleThreads, "items fit their threads");
  const int tb = t - 2 * kRoleThreads;
  c.fwave = __builtin_amdgcn_readfirstlane((t & ~63) < nfi ? 1 : 0);
  c.bwave = __builtin_amdgcn_readfirstlane(!c.fwave && tb >= 0 && (tb & ~63) < nbi ? 1 : 0);
  if (c.fwave) {
    const int it = min(t, nfi - 1);
    c.own = t < nfi;
    c.iv = it / (G * nxbF);
    const FItem fi = fitem(it - c.iv * G * nxbF, nxbF);
    c.ig = fi.g;
    c.iox = fi.ox;
  } else {
    const FItem bi = fitem(max(0, min(tb, nbi - 1)), nxbB);
    c.own = tb >= 0 && tb < nbi;
    c.iv = 0;
    c.ig = bi.g;
    c.iox = bi.ox;
  }
  // the columns this thread's ring serves: F the strip ± (RA + R), B_v ± R
  Geo o;
  o.y = c.y;
  o.zs = 0;
  o.ze = a->g.Z;
  o.ngroups = c.ngroups;
  o.plane_off = c.plane_off;
  if (c.role == 0) {
    o.xo0 = c.x0 - RA;
    o.xout = a->x_out + 2 * RA;
  } else {
    o.xo0 = c.x0;
    o.xout = a->x_out;
  }
  const int tr = t - (c.role == 0 ? 0 : (1 + c.vb) * kRoleThreads);
  const Cols<1, R> cl(a, o, tr, kRoleThreads);
  // LDS: zero the column-pass rows past the widest column a ring writes (the
  // row passes read up to NIN4·4 − 1 columns past an item's start)
  {
    const int wf = a->x_out + 2 * RA + 2 * R, wb = a->x_out + 2 * R;
    for (int e = t; e < 2 * G * c.pitch; e += nt) {
      const int col = e % c.pitch;
      if (col >= wf) c.bufF[e] = 0.f;
      if (col >= wb) c.bufB[e] = 0.f;
    }
  }
  fill_tap_table<KB>(ttF, a, 2, t, nt);
  fill_back_taps<KB>(ttB, fa, t, nt);
  float ring[1][M];
  if (c.role == 0) {
    const float *__restrict__ src = a->psi_in + c.plane_off;
#pragma unroll
    for (int m = 0; m < G + KB - 1; ++m) load_row<1, R>(src, -R + m, a, cl, &ring[0][m], M);
  } else {
#pragma unroll
    for (int m = 0; m < R; ++m) ring[0][m] = 0.f;   // r rows above the plane
  }
  // the first group's row-pass operands (phase 0 reads opA)
  float opA[NX], opB[NX];
  if (c.fwave)
    load_operands<KB, U16>(fa, c, 0, opA);
  else if (c.bwave)
    load_psi(fa, c, -D, opA);
  lds_sync();
  for (int p0 = 0; p0 < c.nphases; p0 += 2 * U)
    fused_phases<KB, U16>(fa, c, cl, ring, opA, opB, p0, std::make_integer_sequence<int, 2 * U>{});
}

template <int KB>
hipError_t fused_bucket(const FusedArgs &fa, hipStream_t s) {
  using FS = FShape<KB>;
  const SepPassArgs &a = fa.f;
  constexpr int R = (KB - 1) / 2;
  // the geometry the roles assume: whole 8-column items, rings within their role
  if (a.g.X % NX != 0 || a.x_out != kFusedStrip || a.x_out + 2 * FS::RA + 2 * R > kRoleThreads ||
      a.ldsw < a.x_out + 2 * FS::RA + 2 * R + 4 || a.ldsw % 8 != 4 || a.nviews != 2 || a.boundary != 0 ||
      a.halo != R || a.nstrip != (a.g.X + a.x_out - 1) / a.x_out)
    return hipErrorInvalidValue;
  if (a.nstrip > 1 && a.psi_in == a.psi_out) return hipErrorInvalidValue;
  const size_t lds = fused_lds_bytes(KB, a.ldsw);
  auto kern = a.obs_u16 ? fused_kernel<KB, 1> : fused_kernel<KB, 0>;
  if (lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const unsigned nblocks = (unsigned)a.g.Y * a.nstrip;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kFusedThreads), lds, s, fa);
  return hipGetLastError();
}

}  // namespace sepk

size_t fused_lds_bytes(int kb, int pitch) {
  const size_t nk = (size_t)((kb + 3 + 3) / 4 * 4);
  return sizeof(float) * (3ull * 2 * sepk::G * pitch + 2ull * 2 * 8 * nk);
}

hipError_t launch_fused(const FusedArgs &fa, int kb, hipStream_t s) {
  switch (kb) {
    case 3: return sepk::fused_bucket<3>(fa, s);
    case 7: return sepk::fused_bucket<7>(fa, s);
    case 11: return sepk::fused_bucket<11>(fa, s);
    case 15: return sepk::fused_bucket<15>(fa, s);
    case 21: return sepk::fused_bucket<21>(fa, s);
    case 31: return sepk::fused_bucket<31>(fa, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mvd
