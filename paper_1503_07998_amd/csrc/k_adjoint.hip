// Kernels of the reverse sweep that are not convolution passes.
//
//  * pointwise_sim: from ψ^t, ∂L/∂ψ^{t+1} and q_v (v < V) of the simultaneous
//    update ψ' = ψ · Π_v c_v, c_v = w_v q_v + 1 − w_v:
//        ψ̄  = ψ̄' · Π_v c_v                 (direct term)
//        c̄_v = ψ̄' · ψ · Π_{u≠v} c_u
//        q̄_v = w_v c̄_v  (written over q_v)
//        w̄_v += Σ c̄_v (q_v − 1)           (per-work-group partial sums)
//    With per-pixel weight planes ω_v the tempering weight of a pixel is
//    o_v = w_v ω_v (as in the forward update): c_v = o_v q_v + 1 − o_v,
//    q̄_v = o_v c̄_v, w̄_v += Σ c̄_v (q_v − 1) ω_v and, where asked for,
//    ω̄_v += c̄_v (q_v − 1) w_v pixel by pixel (summed over the iterations in
//    the caller's buffer).  With the EM-normalised back-projection q_v is
//    first divided by s_v = 1 ⊛ X_v where s_v > ε (as in the forward pass),
//    and q̄_v = q̄'_v / s_v, s̄_v = −q̄'_v q_v / s_v are written (s̄_v then
//    feeds the back-projector's tap gradient through s_v).
//  * pointwise_seq: the same for one view of the sequential update.
//  * ratio_plane / bbar_plane: the pointwise ends of the passes of a kernel
//    that is a sum of rank-one terms (the sum formed term by term first):
//    r = φ / b (1 where b ≤ ε) and b̄ = −s · r / b (0 where b ≤ ε); and
//    add_plane, ψ̄ += b̄ ⊛ P^* after a K×K pass stored the convolution.
//  * corr: tap gradient Σ_{y,z,x} ḡ[y][z][x] · ã[y][z+R−j][x+R−i] for every
//    lag (j, i) of a K×K kernel (ã zero or wrapped outside the plane): each
//    thread owns a 4×8 block of lags and slides over 8×64 tiles staged in LDS.
//  * reductions in a fixed order (deterministic) into float64 accumulators.
// (Chain rule of the update of Supplementary Note 1 / Note 2 §1.)
#include "mvd_internal.hpp"
#include <algorithm>

namespace mvd {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ int wrapc(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Sum of one double per thread over the work-group, fixed order; result in thread 0.
__device__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// VW consecutive floats at p + i (one 16-byte access when VW = 4).
template <int VW>
__device__ __forceinline__ void ldv(const float *p, size_t i, float (&o)[VW]) {
  if constexpr (VW == 4) {
    const float4 v = *reinterpret_cast<const float4 *>(p + i);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  } else {
    o[0] = p[i];
  }
}

template <int VW>
__device__ __forceinline__ void stv(float *p, size_t i, const float (&o)[VW]) {
  if constexpr (VW == 4)
    *reinterpret_cast<float4 *>(p + i) = make_float4(o[0], o[1], o[2], o[3]);
  else
    p[i] = o[0];
}

// The normalisation of element i's back-projection: s = nsz[z] · nsx[x] (or
// the sensitivity plane's s[z][x]); q is
// divided by s where s > ε (the forward pass's reciprocal form), and `inv`
// is 1/s there, 0 elsewhere.
__device__ __forceinline__ float norm_of(const AdjPointArgs &a, int v, size_t i, float &inv) {
  const size_t row = i / (size_t)a.X;
  const int x = (int)(i - row * (size_t)a.X);
  const int z = (int)(row % (size_t)a.Z);
  const float sv = a.nsp[v] ? a.nsp[v][(size_t)z * a.X + x] : a.nsz[v][z] * a.nsx[v][x];
  inv = sv > kEps ? __builtin_amdgcn_rcpf(sv) : 0.f;
  return sv;
}

// NV views, VW elements per thread and step (4: every array 16-byte aligned and
// n a multiple of 4).  Π_{u≠v} c_u is formed as (c_0 ⋯ c_{v−1}) · (c_{v+1} ⋯ c_{NV−1}).
// WP: 0 scalar weights only, 1 per-pixel weight planes, 2 weight planes and
// their per-pixel gradients.
template <int NV, int VW, int WP>
__global__ void __launch_bounds__(NT) pointwise_sim_kernel(AdjPointArgs a) {
  __shared__ double sh[NT];
  double wsum[NV];
  float w[NV], w1[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    wsum[v] = 0.0;
    w[v] = a.w[v];
    w1[v] = 1.f - w[v];
  }
  for (size_t i = ((size_t)blockIdx.x * NT + threadIdx.x) * VW; i < a.n; i += (size_t)gridDim.x * NT * VW) {
    float gin[VW], psi[VW], q[NV][VW], gout[VW], inv[NV][VW], sb[NV][VW];
    float om[WP ? NV : 1][VW], gw[WP == 2 ? NV : 1][VW];
    ldv<VW>(a.gbar_in, i, gin);
    ldv<VW>(a.psi, i, psi);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ldv<VW>(a.q[v], i, q[v]);
      if constexpr (WP >= 1) ldv<VW>(a.wpl[v], i, om[v]);
      if constexpr (WP == 2) ldv<VW>(a.gwpl[v], i, gw[v]);
      if (a.nrm) {
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const float sv = norm_of(a, v, i + e, inv[v][e]);
          if (sv > kEps) q[v][e] *= inv[v][e];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      float c[NV], o[NV], pre[NV + 1];
      pre[0] = 1.f;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (WP >= 1) {
          o[v] = w[v] * om[v][e];
          c[v] = fmaf(o[v], q[v][e], 1.f - o[v]);
        } else {
          o[v] = w[v];
          c[v] = fmaf(w[v], q[v][e], w1[v]);
        }
        pre[v + 1] = pre[v] * c[v];
      }
      gout[e] = gin[e] * pre[NV];
      const float gp = gin[e] * psi[e];
      float suf = 1.f;
#pragma unroll
      for (int v = NV - 1; v >= 0; --v) {
        const float cbar = gp * (pre[v] * suf);
        suf *= c[v];
        const float d = q[v][e] - 1.f;
        if constexpr (WP >= 1)
          wsum[v] += (double)cbar * (double)d * (double)om[v][e];
        else
          wsum[v] += (double)cbar * (double)d;
        if constexpr (WP == 2) gw[v][e] += (cbar * d) * w[v];
        const float qb = o[v] * cbar;
        if (a.nrm) {   // q̄ = q̄'/s and s̄ = −q̄' q / s where s > ε (inv = 0 elsewhere)
          sb[v][e] = -(qb * q[v][e]) * inv[v][e];
          q[v][e] = inv[v][e] != 0.f ? qb * inv[v][e] : qb;
        } else {
          q[v][e] = qb;
        }
      }
    }
    stv<VW>(a.gbar_out, i, gout);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      stv<VW>(a.q[v], i, q[v]);
      if constexpr (WP == 2) stv<VW>(a.gwpl[v], i, gw[v]);
      if (a.nrm) stv<VW>(a.sbar[v], i, sb[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double s = block_sum(wsum[v], sh);
    if (threadIdx.x == 0) a.wpart[(size_t)blockIdx.x * NV + v] = s;
  }
}

// Sequential update, view v: ψ_{v+1} = ψ_v · c_v.  gbar holds ∂L/∂ψ_{v+1} on
// entry and the direct term ∂L/∂ψ_v = gbar · c_v on exit; q becomes q̄.
template <int VW, int WP>
__global__ void __launch_bounds__(NT) pointwise_seq_kernel(AdjPointArgs a) {
  __shared__ double sh[NT];
  double wsum = 0.0;
  const float w = a.w[0], w1 = 1.f - w;
  for (size_t i = ((size_t)blockIdx.x * NT + threadIdx.x) * VW; i < a.n; i += (size_t)gridDim.x * NT * VW) {
    float g[VW], q[VW], psi[VW], go[VW], om[VW], gw[VW], inv[VW], sb[VW];
    ldv<VW>(a.gbar_in, i, g);
    ldv<VW>(a.q[0], i, q);
    ldv<VW>(a.psi, i, psi);
    if constexpr (WP >= 1) ldv<VW>(a.wpl[0], i, om);
    if constexpr (WP == 2) ldv<VW>(a.gwpl[0], i, gw);
    if (a.nrm) {
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const float sv = norm_of(a, 0, i + e, inv[e]);
        if (sv > kEps) q[e] *= inv[e];
      }
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const float o = WP >= 1 ? w * om[e] : w;
      const float c = WP >= 1 ? fmaf(o, q[e], 1.f - o) : fmaf(w, q[e], w1);
      const float cbar = g[e] * psi[e];
      const float d = q[e] - 1.f;
      go[e] = g[e] * c;
      if constexpr (WP >= 1)
        wsum += (double)cbar * (double)d * (double)om[e];
      else
        wsum += (double)cbar * (double)d;
      if constexpr (WP == 2) gw[e] += (cbar * d) * w;
      const float qb = o * cbar;
      if (a.nrm) {
        sb[e] = -(qb * q[e]) * inv[e];
        q[e] = inv[e] != 0.f ? qb * inv[e] : qb;
      } else {
        q[e] = qb;
      }
    }
    stv<VW>(a.gbar_out, i, go);
    stv<VW>(a.q[0], i, q);
    if constexpr (WP == 2) stv<VW>(a.gwpl[0], i, gw);
    if (a.nrm) stv<VW>(a.sbar[0], i, sb);
  }
  const double s = block_sum(wsum, sh);
  if (threadIdx.x == 0) a.wpart[blockIdx.x] = s;
}

// r = φ / b, guarded as in the forward pass's epilogue.
__global__ void __launch_bounds__(NT) ratio_plane_kernel(const float *__restrict__ phi, const float *__restrict__ b,
                                                          float *__restrict__ r, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT)
    r[i] = guarded_ratio(phi[i], b[i]);
}

// b ← −s · r / b where b > ε, else 0 (b̄ over b, as the single-term epilogue).
__global__ void __launch_bounds__(NT) bbar_plane_kernel(const float *__restrict__ s, const float *__restrict__ r,
                                                         float *b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const float bb = b[i];
    const float q = nr_quotient(s[i] * r[i], bb);
    b[i] = bb > kEps ? -q : 0.f;
  }
}

// dst += src (ψ̄ += b̄ ⊛ P^* after a K×K pass stored the convolution).
__global__ void __launch_bounds__(NT) add_plane_kernel(float *dst, const float *__restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) dst[i] += src[i];
}

// acc[v] += Σ_b part[b][v]: one work-group per view, fixed order.
__global__ void __launch_bounds__(NT) sum_partials_kernel(const double *__restrict__ part, int nblocks, int nv,
                                                          double *acc) {
  __shared__ double sh[NT];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += NT) s += part[(size_t)b * nv + v];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) acc[v] += s;
}

// ---------------------------------------------------------------------------
// Tap-gradient correlation
// ---------------------------------------------------------------------------
constexpr int CTZ = 8;    // tile rows (one per row group of threads)
constexpr int CTX = 64;   // tile columns
constexpr int LJ = 4;     // lags per thread along z
constexpr int LI = 8;     // lags per thread along x
constexpr int SU = 8;     // window elements staged per thread per step

struct CorrGeo {
  int kzp, kxp, nbj, nbi, nblk, bw, bh;
};

__device__ __forceinline__ CorrGeo corr_geo(const CorrArgs &a) {
  CorrGeo g;
  g.kzp = a.kzp;
  g.kxp = a.kxp;
  g.nbj = g.kzp / LJ;
  g.nbi = g.kxp / LI;
  g.nblk = g.nbj * g.nbi;
  // staged columns: CTX + kxp − 1 used, padded so that the row pitch is 4 (mod 8)
  // floats: tile rows then start 4 banks apart (see the lane mapping below)
  g.bw = CTX + g.kxp + 4;
  g.bh = CTZ + g.kzp - 1;
  return g;
}

__global__ void __launch_bounds__(1024) corr_kernel(CorrArgs a) {
  extern __shared__ __align__(16) float sm[];
  const CorrGeo G = corr_geo(a);
  float *At = sm;                       // [CTZ][CTX]
  float *Bt = sm + CTZ * CTX;           // [bh][bw]
  const int t = threadIdx.x;
  // lane → (x-lag block, tile row, z-lag block), x-lag block fastest: the 8 lanes
  // that share an LDS cycle read windows 8 columns apart in two rows whose
  // pitch is 4 (mod 8) floats, so their 16-byte reads fall in distinct banks
  const int ib = t % G.nbi;
  const int rg = (t / G.nbi) % CTZ;
  const int jb = t / (G.nbi * CTZ);
  const int blk = jb * G.nbi + ib;        // lag block
  const int Z = a.g.Z, X = a.g.X;
  const int ntz = (Z + CTZ - 1) / CTZ, ntx = (X + CTX - 1) / CTX;
  const long ntiles = (long)a.g.Y * ntz * ntx;
  float acc[LJ][LI];
#pragma unroll
  for (int jj = 0; jj < LJ; ++jj)
#pragma unroll
    for (int ii = 0; ii < LI; ++ii) acc[jj][ii] = 0.f;
  // this thread's staging walk over the window, the same for every tile
  const int nt = blockDim.x;
  const int br0 = t / G.bw, bc0 = t % G.bw, dr = nt / G.bw, dc = nt % G.bw;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int txi = (int)(tile % ntx);
    const int tzi = (int)((tile / ntx) % ntz);
    const int y = (int)(tile / ((long)ntx * ntz));
    const int z0 = tzi * CTZ, x0 = txi * CTX;
    const size_t po = (size_t)y * Z * X;
    // stage ḡ (zero outside the plane) and ã rows z0+R−kzp+1 … z0+CTZ−1+R,
    // columns x0+R−kxp+1 … x0+CTX−1+R (zero or wrapped outside)
    for (int e = t; e < CTZ * CTX; e += blockDim.x) {
      const int r = e / CTX, c = e % CTX;
      const int z = z0 + r, x = x0 + c;
      At[e] = (z < Z && x < X) ? a.gbar[po + (size_t)z * X + x] : 0.f;
    }
    // element e = t + k·nt of the [bh][bw] window, walked as (row, column), SU
    // elements at a time: all SU loads are issued (at clamped, valid addresses)
    // before any is stored, so their latencies overlap
    const int zb = z0 + a.rz - G.kzp + 1, xb = x0 + a.rx - G.kxp + 1;
    for (int r = br0, c = bc0, e = t; r < G.bh;) {
      float v[SU];
      int ev[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        int z = zb + r, x = xb + c;
        bool in = r < G.bh;
        if (a.boundary == 0) {
          in = in && z >= 0 && z < Z && x >= 0 && x < X;
          z = min(max(z, 0), Z - 1);
          x = min(max(x, 0), X - 1);
        } else {
          z = wrapc(z, Z);
          x = wrapc(x, X);
        }
        const float w = a.src[po + (size_t)z * X + x];
        v[u] = in ? w : 0.f;
        ev[u] = r < G.bh ? e : -1;
        e += nt;
        r += dr;
        c += dc;
        if (c >= G.bw) {
          c -= G.bw;
          ++r;
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (ev[u] >= 0) Bt[ev[u]] = v[u];
    }
    __syncthreads();
    if (rg < CTZ) {
      const float *Arow = At + rg * CTX;
      for (int xo = 0; xo < CTX; xo += 8) {
        const float4 a0 = *reinterpret_cast<const float4 *>(Arow + xo);
        const float4 a1 = *reinterpret_cast<const float4 *>(Arow + xo + 4);
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        // window start column: xo + kxp − 8 − 8·ib (multiple of 8)
        const int c0 = xo + G.kxp - 8 - LI * ib;
#pragma unroll
        for (int jj = 0; jj < LJ; ++jj) {
          const int j = jb * LJ + jj;
          const float *Br = Bt + (rg + G.kzp - 1 - j) * G.bw + c0;
          float bw16[16];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 f = *reinterpret_cast<const float4 *>(Br + 4 * q);
            bw16[4 * q] = f.x;
            bw16[4 * q + 1] = f.y;
            bw16[4 * q + 2] = f.z;
            bw16[4 * q + 3] = f.w;
          }
#pragma unroll
          for (int xx = 0; xx < 8; ++xx)
#pragma unroll
            for (int ii = 0; ii < LI; ++ii) acc[jj][ii] = fmaf(av[xx], bw16[7 + xx - ii], acc[jj][ii]);
        }
      }
    }
    __syncthreads();
  }
  // reduce the row groups in a fixed order, then one partial per lag
  float *red = sm;   // [CTZ][nblk][LJ*LI] reuses the tile memory
  if (rg < CTZ) {
#pragma unroll
    for (int jj = 0; jj < LJ; ++jj)
#pragma unroll
      for (int ii = 0; ii < LI; ++ii) red[((size_t)rg * G.nblk + blk) * (LJ * LI) + jj * LI + ii] = acc[jj][ii];
  }
  __syncthreads();
  const int nl = G.kzp * G.kxp;
  for (int l = t; l < nl; l += blockDim.x) {
    const int j = l / G.kxp, i = l % G.kxp;
    const int b = (j / LJ) * G.nbi + i / LI;
    const int k = (j % LJ) * LI + (i % LI);
    float s = 0.f;
    for (int r = 0; r < CTZ; ++r) s += red[((size_t)r * G.nblk + b) * (LJ * LI) + k];
    a.part[(size_t)blockIdx.x * nl + l] = s;
  }
}

// ---------------------------------------------------------------------------
// Tap-gradient correlation on the matrix cores.  With x' = x + Rx − i,
//   G[j][i] = Σ_{y,z} Σ_x' ã[y][z + Rz − j][x'] · ḡ[y][z][x' − Rx + i],
// so each row z adds the product of a K × W block of ã rows (A[j][x']) with a
// W × K Toeplitz block of ḡ's row (B[x'][i] = ḡ[z][x' − Rx + i]): a dense
// contraction over x' with no structural zeros.  A tile is 16 rows z × tw
// columns x' (tw ≤ 256, a multiple of 16, chosen on the host so that the tiles
// of a row cover its X + Kx − 1 columns with little excess); the ã rows it
// needs (row pitch ≡ 2 mod 4 floats: the 16 rows × 2 columns that a
// half-wave reads fall in distinct banks) and its ḡ rows (zero outside the
// plane) are staged in LDS.  Wave w takes rows z0 + w, z0 + w + 4, …; each
// step of 4 columns is one v_mfma_f32_16x16x4f32 per 16 × 16 block of G
// (lane l supplies A[16·jb + l % 16][4q + l / 16] and B[4q + l / 16][16·ib + l % 16]).
// A work-group keeps its blocks of G in registers over all its tiles, sums its
// 4 waves in a fixed order and writes one partial, reduced in float64 by the
// same finalize step as the vector form.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MCZ = 16;      // rows z per tile
constexpr int MCXMAX = 256;  // columns x' per tile, at most
constexpr int MCT = 256;     // threads (4 waves)

struct McGeo {
  int kz, kx, xa, ntx, ntz, nzc, nr, pa, pb;
  long nitems;
};

__host__ __device__ inline int mc_pitch(int tw) { return tw + 2; }

__device__ __forceinline__ McGeo mc_geo(const CorrArgs &a) {
  McGeo g;
  g.kz = 2 * a.rz + 1;
  g.kx = 2 * a.rx + 1;
  g.xa = a.rx - g.kx + 1;                          // first column x' that meets a tap
  g.ntx = (a.g.X + g.kx - 1 + a.tw - 1) / a.tw;
  g.ntz = (a.g.Z + MCZ - 1) / MCZ;
  g.nzc = (g.ntz + a.zch - 1) / a.zch;
  g.nr = MCZ + a.kzp - 1;
  g.pa = mc_pitch(a.tw);
  g.pb = a.tw + a.kxp;
  g.nitems = (long)a.g.Y * g.nzc * g.ntx;
  return g;
}

// Stage rows × pitch elements into LDS: element (r, c) comes from src[at(r, c)]
// (at returns a clamped in-plane index and whether the value is kept, else 0)
// and goes to row slot(r).  Each thread walks elements t, t + MCT, … and
// issues MSU loads before it stores any, so that their latencies overlap.
constexpr int MSU = 8;
template <class F, class S>
__device__ __forceinline__ void mc_stage(float *dst, int rows, int pitch, const float *__restrict__ src, F at,
                                         S slot) {
  const int t = threadIdx.x;
  const int dr = MCT / pitch, dc = MCT % pitch;
  int r = t / pitch, c = t % pitch;
  while (r < rows) {
    float v[MSU];
    int ev[MSU];
#pragma unroll
    for (int u = 0; u < MSU; ++u) {
      bool in;
      const size_t i = at(r < rows ? r : rows - 1, c, in);
      const float w = src[i];
      v[u] = in ? w : 0.f;
      ev[u] = r < rows ? slot(r) * pitch + c : -1;
      r += dr;
      c += dc;
      if (c >= pitch) {
        c -= pitch;
        ++r;
      }
    }
#pragma unroll
    for (int u = 0; u < MSU; ++u)
      if (ev[u] >= 0) dst[ev[u]] = v[u];
  }
}

template <int KZB, int KXB>
__global__ void __launch_bounds__(MCT) corr_mfma_kernel(CorrArgs a) {
  extern __shared__ __align__(16) float sm[];
  const McGeo G = mc_geo(a);
  // As: ring of nr rows; window row r of the current tile (ã row z0 + Rz − (kzp − 1) + r,
  // columns x0' + c) sits in slot (ring0 + r) mod nr.  Bs: [MCZ][pb] = ḡ[z0 + r][x0' − Rx + c].
  float *As = sm;
  float *Bs = sm + G.nr * G.pa;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int n = lane & 15, kk = lane >> 4;
  const int Z = a.g.Z, X = a.g.X, tw = a.tw, nr = G.nr;
  const int boundary = a.boundary;
  f32x4 acc[KZB][KXB];
#pragma unroll
  for (int jb = 0; jb < KZB; ++jb)
#pragma unroll
    for (int ib = 0; ib < KXB; ++ib) acc[jb][ib] = f32x4{0.f, 0.f, 0.f, 0.f};
  // item = (plane y, run of zch tiles down z, column tile): the tiles of a run
  // share all but 16 of their ã rows, so each later tile stages only those
  for (long item = blockIdx.x; item < G.nitems; item += gridDim.x) {
    const int tx = (int)(item % G.ntx);
    const int zc = (int)((item / G.ntx) % G.nzc);
    const int y = (int)(item / ((long)G.ntx * G.nzc));
    const int x0 = G.xa + tx * tw, xg = x0 - a.rx;
    const size_t po = (size_t)y * Z * X;
    const int tz0 = zc * a.zch, tz1 = min(G.ntz, tz0 + a.zch);
    int ring0 = 0;
    for (int tz = tz0; tz < tz1; ++tz) {
      const int z0 = tz * MCZ;
      const int za = z0 + a.rz - (a.kzp - 1);
      const int rfirst = tz == tz0 ? 0 : nr - MCZ;   // window rows to stage
      const int rs = ring0 + rfirst;
      mc_stage(
          As, nr - rfirst, G.pa, a.src,
          [&](int r, int c, bool &in) -> size_t {
            int z = za + rfirst + r, x = x0 + c;
            in = c < tw;
            if (boundary == 0) {
              in = in && z >= 0 && z < Z && x >= 0 && x < X;
              z = min(max(z, 0), Z - 1);
              x = min(max(x, 0), X - 1);
            } else {
              z = wrapc(z, Z);
              x = wrapc(x, X);
            }
            return po + (size_t)z * X + x;
          },
          [&](int r) { return rs + r < nr ? rs + r : rs + r - nr; });
      mc_stage(
          Bs, MCZ, G.pb, a.gbar,
          [&](int r, int c, bool &in) -> size_t {
            const int z = z0 + r, x = xg + c;
            in = z < Z && x >= 0 && x < X;
            return po + (size_t)min(z, Z - 1) * X + min(max(x, 0), X - 1);
          },
          [](int r) { return r; });
      __syncthreads();
      for (int zz = w; zz < MCZ && z0 + zz < Z; zz += 4) {
        // A[16·jb + n][4q + kk] = window row zz + kzp − 1 − n − 16·jb, column 4q + kk
        const float *Ar[KZB];
#pragma unroll
        for (int jb = 0; jb < KZB; ++jb) {
          int sl = ring0 + zz + a.kzp - 1 - n - 16 * jb;
          sl = sl < nr ? sl : sl - nr;
          Ar[jb] = As + sl * G.pa + kk;
        }
        const float *Br = Bs + zz * G.pb + kk + n;                  // B[4q + kk][16·ib + n]
        // 4 steps of 4 columns at a time (tw is a multiple of 16), operands of
        // the next 4 loaded before the products of these
        float av[2][4][KZB], bv[2][4][KXB];
        auto load = [&](int buf, int q0) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int jb = 0; jb < KZB; ++jb) av[buf][s][jb] = Ar[jb][4 * (q0 + s)];
#pragma unroll
            for (int ib = 0; ib < KXB; ++ib) bv[buf][s][ib] = Br[4 * (q0 + s) + 16 * ib];
          }
        };
        auto step = [&](int buf) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int jb = 0; jb < KZB; ++jb)
#pragma unroll
              for (int ib = 0; ib < KXB; ++ib)
                acc[jb][ib] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(av[buf][s][jb], bv[buf][s][ib], acc[jb][ib], 0, 0, 0);
        };
        const int nq = tw / 4;
        load(0, 0);
        int q0 = 0;
        for (; q0 + 8 <= nq; q0 += 8) {
          load(1, q0 + 4);
          step(0);
          if (q0 + 8 < nq) load(0, q0 + 8);
          step(1);
        }
        if (q0 < nq) step(0);
      }
      __syncthreads();
      ring0 = ring0 + MCZ < nr ? ring0 + MCZ : ring0 + MCZ - nr;
    }
  }
  // the 4 waves' blocks through LDS, summed in a fixed order; register r of
  // lane l holds row 4·(l / 16) + r, column l % 16 of a block
  float *red = sm;   // [4][kzp][kxp]
  const int nl = a.kzp * a.kxp;
#pragma unroll
  for (int jb = 0; jb < KZB; ++jb)
#pragma unroll
    for (int ib = 0; ib < KXB; ++ib)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[w * nl + (16 * jb + 4 * kk + r) * a.kxp + 16 * ib + n] = acc[jb][ib][r];
  __syncthreads();
  for (int l = t; l < nl; l += MCT)
    a.part[(size_t)blockIdx.x * nl + l] = ((red[l] + red[nl + l]) + red[2 * nl + l]) + red[3 * nl + l];
}

// acc[j][i] += Σ_b part[b][j][i] over lags inside the true kernel: one
// work-group per lag, strided float64 partial sums and a tree in a fixed
// order (bitwise reproducible).
__global__ void __launch_bounds__(NT) corr_finalize_kernel(const float *__restrict__ part, int nblocks, int kzp,
                                                           int kxp, int kz, int kx, double *acc) {
  __shared__ double sh[NT];
  const int l = blockIdx.x;
  const int j = l / kx, i = l % kx;
  const size_t pl = (size_t)j * kxp + i, stride = (size_t)kzp * kxp;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += NT) s += part[(size_t)b * stride + pl];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) acc[l] += s;
}

__global__ void to_f32_kernel(const double *__restrict__ src, float *__restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

__global__ void zero_f64_kernel(double *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = 0.0;
}

}  // namespace

int corr_pad(int k, int unit) {
  int p = unit;
  while (p < k) p *= 2;
  return p;
}

size_t corr_lds_bytes(int kzp, int kxp) {
  const size_t tiles = sizeof(float) * ((size_t)CTZ * CTX + (size_t)(CTZ + kzp - 1) * (CTX + kxp + 4));
  const size_t red = sizeof(float) * (size_t)CTZ * (kzp / LJ) * (kxp / LI) * LJ * LI;
  return tiles > red ? tiles : red;
}

int corr_threads(int kzp, int kxp) { return CTZ * (kzp / LJ) * (kxp / LI); }

bool point_vec(const AdjPointArgs &a, int nv) {
  bool ok = a.n % 4 == 0;
  for (const void *p : {(const void *)a.psi, (const void *)a.gbar_in, (const void *)a.gbar_out})
    ok = ok && (uintptr_t)p % 16 == 0;
  for (int v = 0; v < nv; ++v) {
    ok = ok && (uintptr_t)a.q[v] % 16 == 0;
    if (a.wp >= 1) ok = ok && (uintptr_t)a.wpl[v] % 16 == 0;
    if (a.wp == 2) ok = ok && (uintptr_t)a.gwpl[v] % 16 == 0;
    if (a.nrm) ok = ok && (uintptr_t)a.sbar[v] % 16 == 0;
  }
  return ok;
}

template <int NV, int WP>
hipError_t launch_sim_wp(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  if (point_vec(a, NV))
    hipLaunchKernelGGL((pointwise_sim_kernel<NV, 4, WP>), dim3(nblocks), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((pointwise_sim_kernel<NV, 1, WP>), dim3(nblocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <int NV>
hipError_t launch_sim_nv(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  switch (a.wp) {
    case 0: return launch_sim_wp<NV, 0>(a, nblocks, s);
    case 1: return launch_sim_wp<NV, 1>(a, nblocks, s);
    case 2: return launch_sim_wp<NV, 2>(a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

template <int WP>
hipError_t launch_seq_wp(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  if (point_vec(a, 1))
    hipLaunchKernelGGL((pointwise_seq_kernel<4, WP>), dim3(nblocks), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((pointwise_seq_kernel<1, WP>), dim3(nblocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pointwise_sim(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  switch (a.nv) {
    case 1: return launch_sim_nv<1>(a, nblocks, s);
    case 2: return launch_sim_nv<2>(a, nblocks, s);
    case 3: return launch_sim_nv<3>(a, nblocks, s);
    case 4: return launch_sim_nv<4>(a, nblocks, s);
    case 5: return launch_sim_nv<5>(a, nblocks, s);
    case 6: return launch_sim_nv<6>(a, nblocks, s);
    case 7: return launch_sim_nv<7>(a, nblocks, s);
    case 8: return launch_sim_nv<8>(a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pointwise_seq(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  switch (a.wp) {
    case 0: return launch_seq_wp<0>(a, nblocks, s);
    case 1: return launch_seq_wp<1>(a, nblocks, s);
    case 2: return launch_seq_wp<2>(a, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ratio_plane(const float *phi, const float *b, float *r, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(ratio_plane_kernel, dim3(blocks), dim3(NT), 0, s, phi, b, r, n);
  return hipGetLastError();
}

hipError_t launch_bbar_plane(const float *sum, const float *r, float *b, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bbar_plane_kernel, dim3(blocks), dim3(NT), 0, s, sum, r, b, n);
  return hipGetLastError();
}

hipError_t launch_add_plane(float *dst, const float *src, size_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + NT - 1) / NT, 8192);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(add_plane_kernel, dim3(blocks), dim3(NT), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int nblocks, int nv, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(nv), dim3(NT), 0, s, part, nblocks, nv, acc);
  return hipGetLastError();
}

int corr_mfma_pad(int k) { return (k + 15) / 16 * 16; }

size_t corr_mfma_lds_bytes(int kzp, int kxp, int tw) {
  const size_t tiles = sizeof(float) * ((size_t)(MCZ + kzp - 1) * mc_pitch(tw) + (size_t)MCZ * (tw + kxp));
  const size_t red = sizeof(float) * 4ull * kzp * kxp;
  return tiles > red ? tiles : red;
}

CorrMfmaShape corr_mfma_shape(const PlaneGeom &g, int kz, int kx, int max_blocks) {
  CorrMfmaShape m;
  m.kzp = corr_mfma_pad(kz);
  m.kxp = corr_mfma_pad(kx);
  const int width = g.X + kx - 1;
  const int ntx0 = (width + MCXMAX - 1) / MCXMAX;
  m.tw = (width + 16 * ntx0 - 1) / (16 * ntx0) * 16;
  const int ntx = (width + m.tw - 1) / m.tw;
  const int ntz = (g.Z + MCZ - 1) / MCZ;
  m.lds = corr_mfma_lds_bytes(m.kzp, m.kxp, m.tw);
  // resident work-groups: LDS-bound, at most 4 per CU (registers), 256 CUs
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, 160 * 1024 / m.lds));
  const long slots = std::min<long>(max_blocks, 256L * per_cu);
  // run length down z: fewest tiles on the busiest work-group, then the longest run
  long best = -1;
  m.zch = 1;
  for (int c = 1; c <= ntz; ++c) {
    const long items = (long)g.Y * ntx * ((ntz + c - 1) / c);
    const long span = (items + slots - 1) / slots * c;
    if (best < 0 || span <= best) {
      best = span;
      m.zch = c;
    }
  }
  m.nitems = (long)g.Y * ntx * ((ntz + m.zch - 1) / m.zch);
  m.nblocks = (int)std::min<long>(m.nitems, slots);
  return m;
}

template <int KZB, int KXB>
hipError_t launch_corr_mfma_t(const CorrArgs &a, int nblocks, hipStream_t s) {
  const size_t lds = corr_mfma_lds_bytes(a.kzp, a.kxp, a.tw);
  auto kern = corr_mfma_kernel<KZB, KXB>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(MCT), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_corr_mfma(const CorrArgs &a, int nblocks, hipStream_t s) {
  if (a.kzp % 16 || a.kxp % 16 || a.kzp > 64 || a.kxp > 64 || a.tw <= 0 || a.tw % 16 || a.tw > MCXMAX ||
      a.kzp < 2 * a.rz + 1 || a.kxp < 2 * a.rx + 1 || a.zch < 1)
    return hipErrorInvalidValue;
  const int zb = a.kzp / 16, xb = a.kxp / 16;
#define MVD_CORR_CASE(ZB, XB) \
  if (zb == ZB && xb == XB) return launch_corr_mfma_t<ZB, XB>(a, nblocks, s);
#define MVD_CORR_ROW(ZB) MVD_CORR_CASE(ZB, 1) MVD_CORR_CASE(ZB, 2) MVD_CORR_CASE(ZB, 3) MVD_CORR_CASE(ZB, 4)
  MVD_CORR_ROW(1) MVD_CORR_ROW(2) MVD_CORR_ROW(3) MVD_CORR_ROW(4)
#undef MVD_CORR_ROW
#undef MVD_CORR_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_corr(const CorrArgs &a, int nblocks, hipStream_t s) {
  const size_t lds = corr_lds_bytes(a.kzp, a.kxp);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(corr_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(corr_kernel, dim3(nblocks), dim3(corr_threads(a.kzp, a.kxp)), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_corr_finalize(const float *part, int nblocks, int kzp, int kxp, int kz, int kx, double *acc,
                                hipStream_t s) {
  hipLaunchKernelGGL(corr_finalize_kernel, dim3(kz * kx), dim3(NT), 0, s, part, nblocks, kzp, kxp, kz, kx, acc);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double *src, float *dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double *dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_f64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dst, n);
  return hipGetLastError();
}

}  // namespace mvd
