// Kernels of the reverse sweep that are not convolution passes.
//
//  * pointwise_sim: from ψ^t, ∂L/∂ψ^{t+1} and q_v (v < V) of the simultaneous
//    update ψ' = ψ · Π_v c_v, c_v = w_v q_v + 1 − w_v:
//        ψ̄  = ψ̄' · Π_v c_v                 (direct term)
//        c̄_v = ψ̄' · ψ · Π_{u≠v} c_u
//        q̄_v = w_v c̄_v  (written over q_v)
//        w̄_v += Σ c̄_v (q_v − 1)           (per-work-group partial sums)
//  * pointwise_seq: the same for one view of the sequential update.
//  * corr: tap gradient Σ_{y,z,x} ḡ[y][z][x] · ã[y][z+R−j][x+R−i] for every
//    lag (j, i) of a K×K kernel (ã zero or wrapped outside the plane): each
//    thread owns a 4×8 block of lags and slides over 8×64 tiles staged in LDS.
//  * reductions in a fixed order (deterministic) into float64 accumulators.
// (Chain rule of the update of Supplementary Note 1 / Note 2 §1.)
#include "mvd_internal.hpp"

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

__global__ void __launch_bounds__(NT) pointwise_sim_kernel(AdjPointArgs a) {
  __shared__ double sh[NT];
  double wsum[kMaxViews];
  for (int v = 0; v < kMaxViews; ++v) wsum[v] = 0.0;
  const int nv = a.nv;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < a.n; i += (size_t)gridDim.x * NT) {
    const float gin = a.gbar_in[i];
    const float psi = a.psi[i];
    float q[kMaxViews], c[kMaxViews];
    float prod = 1.f;
    for (int v = 0; v < nv; ++v) {
      q[v] = a.q[v][i];
      c[v] = fmaf(a.w[v], q[v], 1.f - a.w[v]);
      prod *= c[v];
    }
    a.gbar_out[i] = gin * prod;
    const float gp = gin * psi;
    for (int v = 0; v < nv; ++v) {
      float others = 1.f;
      for (int u = 0; u < nv; ++u)
        if (u != v) others *= c[u];
      const float cbar = gp * others;
      wsum[v] += (double)cbar * (double)(q[v] - 1.f);
      a.q[v][i] = a.w[v] * cbar;
    }
  }
  for (int v = 0; v < nv; ++v) {
    const double s = block_sum(wsum[v], sh);
    if (threadIdx.x == 0) a.wpart[(size_t)blockIdx.x * nv + v] = s;
  }
}

// Sequential update, view v: ψ_{v+1} = ψ_v · c_v.  gbar holds ∂L/∂ψ_{v+1} on
// entry and the direct term ∂L/∂ψ_v = gbar · c_v on exit; q becomes q̄.
__global__ void __launch_bounds__(NT) pointwise_seq_kernel(AdjPointArgs a) {
  __shared__ double sh[NT];
  double wsum = 0.0;
  const float w = a.w[0], w1 = 1.f - w;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < a.n; i += (size_t)gridDim.x * NT) {
    const float g = a.gbar_in[i];
    const float q = a.q[0][i];
    const float c = fmaf(w, q, w1);
    const float cbar = g * a.psi[i];
    a.gbar_out[i] = g * c;
    wsum += (double)cbar * (double)(q - 1.f);
    a.q[0][i] = w * cbar;
  }
  const double s = block_sum(wsum, sh);
  if (threadIdx.x == 0) a.wpart[blockIdx.x] = s;
}

// acc[v] += Σ_b part[b][v] (fixed order), one thread per view.
__global__ void sum_partials_kernel(const double *__restrict__ part, int nblocks, int nv, double *acc) {
  const int v = threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * nv + v];
  acc[v] += s;
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

hipError_t launch_pointwise_sim(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(pointwise_sim_kernel, dim3(nblocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pointwise_seq(const AdjPointArgs &a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(pointwise_seq_kernel, dim3(nblocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int nblocks, int nv, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, part, nblocks, nv, acc);
  return hipGetLastError();
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
