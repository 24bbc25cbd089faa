// General (any K×K, not rank-one) forward and backward passes.
//
// Used for PSFs or back-projectors that do not factor into two 1D kernels,
// e.g. compound kernels of views whose PSFs are not axis-aligned.  A
// work-group computes a 16×64 output tile; the input tile plus its K−1 halo is
// staged in LDS (zero or wrapped outside the plane) and every thread computes
// 4 consecutive outputs of one row as a correlation with the point-reflected
// taps, reading 4 new LDS values (one 128-bit read) per 16 FMAs.
// Same epilogues as the separable passes (Supplementary Note 1 update).
#include "mvd_internal.hpp"

namespace mvd {
namespace {

constexpr int TZ = 16;
constexpr int TX = 64;
constexpr int NT = 256;
constexpr int N4 = 4;   // outputs per thread

__device__ __forceinline__ int wrap2(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

struct Tile {
  int y, z0, x0, tw, th;
  size_t plane_off;
};

__device__ __forceinline__ Tile tile_of(const TwoDPassArgs &a) {
  Tile t;
  const int ntx = (a.g.X + TX - 1) / TX;
  const int ntz = (a.g.Z + TZ - 1) / TZ;
  int b = blockIdx.x;
  const int tx = b % ntx;
  b /= ntx;
  const int tz = b % ntz;
  t.y = b / ntz;
  t.z0 = tz * TZ;
  t.x0 = tx * TX;
  const int kxp = (a.kx + 3) & ~3;
  t.tw = TX + kxp + 4;
  t.th = TZ + a.kz - 1;
  t.plane_off = (size_t)t.y * a.g.Z * a.g.X;
  return t;
}

// Stage the input tile: T[r][s] = ã[z0 − Rz + r][x0 − Rx + s] for s < TX + kx − 1,
// zero beyond (those columns only meet zero taps).
__device__ void stage_tile(float *T, const float *__restrict__ src, const TwoDPassArgs &a,
                           const Tile &t) {
  const int rz = (a.kz - 1) / 2, rx = (a.kx - 1) / 2;
  const int used = TX + a.kx - 1;
  for (int e = threadIdx.x; e < t.th * t.tw; e += NT) {
    const int r = e / t.tw, s = e - r * t.tw;
    float v = 0.f;
    if (s < used) {
      int z = t.z0 - rz + r, x = t.x0 - rx + s;
      bool ok;
      if (a.boundary == 0) {
        ok = z >= 0 && z < a.g.Z && x >= 0 && x < a.g.X;
      } else {
        z = wrap2(z, a.g.Z);
        x = wrap2(x, a.g.X);
        ok = true;
      }
      if (ok) v = src[(size_t)z * a.g.X + x];
    }
    T[e] = v;
  }
}

// out[n] = Σ_jj Σ_q ft[jj][q] · T[g + jj][ox + n + q]   (ft = flipped taps, rows padded to kxp)
__device__ __forceinline__ void corr(const float *T, int tw, int g, int ox, const float *__restrict__ ft,
                                     int kz, int kxp, float (&acc)[N4]) {
#pragma unroll
  for (int n = 0; n < N4; ++n) acc[n] = 0.f;
  for (int jj = 0; jj < kz; ++jj) {
    const float *L = T + (g + jj) * tw + ox;
    const float *tr = ft + jj * kxp;
    float4 lo = *reinterpret_cast<const float4 *>(L);
    for (int qb = 0; qb < kxp; qb += 4) {
      const float4 hi = *reinterpret_cast<const float4 *>(L + qb + 4);
      const float w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      const float t0 = tr[qb], t1 = tr[qb + 1], t2 = tr[qb + 2], t3 = tr[qb + 3];
#pragma unroll
      for (int n = 0; n < N4; ++n) {
        acc[n] = fmaf(t0, w[n], acc[n]);
        acc[n] = fmaf(t1, w[n + 1], acc[n]);
        acc[n] = fmaf(t2, w[n + 2], acc[n]);
        acc[n] = fmaf(t3, w[n + 3], acc[n]);
      }
      lo = hi;
    }
  }
}

__global__ void __launch_bounds__(NT) twod_forward_kernel(const TwoDPassArgs a) {
  extern __shared__ __align__(16) float T[];
  const Tile t = tile_of(a);
  const int kxp = (a.kx + 3) & ~3;
  stage_tile(T, a.in[0] + t.plane_off, a, t);
  __syncthreads();
  const int g = threadIdx.x / (TX / N4);
  const int ox = (threadIdx.x % (TX / N4)) * N4;
  const int z = t.z0 + g;
  for (int v = 0; v < a.nviews; ++v) {
    float b[N4];
    corr(T, t.tw, g, ox, a.taps[v], a.kz, kxp, b);
    if (z < a.g.Z) {
      const size_t off = t.plane_off + (size_t)z * a.g.X + t.x0 + ox;
#pragma unroll
      for (int n = 0; n < N4; ++n) {
        if (t.x0 + ox + n < a.g.X) a.out[v][off + n] = a.phi[v] ? guarded_ratio(a.phi[v][off + n], b[n]) : b[n];
      }
    }
  }
}

__global__ void __launch_bounds__(NT) twod_backward_kernel(const TwoDPassArgs a) {
  extern __shared__ __align__(16) float T[];
  const Tile t = tile_of(a);
  const int kxp = (a.kx + 3) & ~3;
  const int g = threadIdx.x / (TX / N4);
  const int ox = (threadIdx.x % (TX / N4)) * N4;
  const int z = t.z0 + g;
  float prod[N4];
#pragma unroll
  for (int n = 0; n < N4; ++n) prod[n] = 1.f;
  for (int v = 0; v < a.nviews; ++v) {
    if (v > 0) __syncthreads();
    stage_tile(T, a.in[v] + t.plane_off, a, t);
    __syncthreads();
    float q[N4];
    corr(T, t.tw, g, ox, a.taps[v], a.kz, kxp, q);
    const float w = a.w[v], w1 = 1.f - w;
#pragma unroll
    for (int n = 0; n < N4; ++n) {
      const float c = fmaf(w, q[n], w1);
      prod[n] = v == 0 ? c : prod[n] * c;
    }
  }
  if (z < a.g.Z) {
    const size_t off = t.plane_off + (size_t)z * a.g.X + t.x0 + ox;
#pragma unroll
    for (int n = 0; n < N4; ++n)
      if (t.x0 + ox + n < a.g.X) a.psi_out[off + n] = a.psi_in[off + n] * prod[n];
  }
}

// ---------------------------------------------------------------------------
// Matrix-core form.  For tap row j, the outputs of 16 rows × 16 columns are a
// matrix product of the input rows (16 × (16 + kx − 1), row m is input row
// m + j) with a banded Toeplitz matrix built from that tap row
// (B[k][n] = ft[j][k − n], zero off the band):  Out += In_j · T_j.  Each step
// of 4 input columns is one v_mfma_f32_16x16x4f32 (float32 products,
// float32 accumulation).  A work-group computes a 32 × 64 output tile with 4
// waves, each 16 rows × 32 columns as two 16 × 16 blocks that share the
// Toeplitz operand.  LDS holds the input tile (row pitch ≡ 2 mod 32 floats:
// the 16 rows × 2 columns a half-wave reads fall in distinct banks) and one
// view's tap rows with 16 leading zeros (so B[k][n] is one load at k − n + 16).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MZ = 32, MX = 64, MNT = 256;

struct MTile {
  int y, z0, x0, th, tw, fl;
  size_t plane_off;
};

template <int NCK>
__device__ __forceinline__ MTile mtile_of(const TwoDPassArgs &a) {
  MTile t;
  const int ntx = (a.g.X + MX - 1) / MX;
  const int ntz = (a.g.Z + MZ - 1) / MZ;
  int b = blockIdx.x;
  const int tx = b % ntx;
  b /= ntx;
  const int tz = b % ntz;
  t.y = b / ntz;
  t.z0 = tz * MZ;
  t.x0 = tx * MX;
  t.th = MZ + a.kz - 1;
  t.tw = mfma_tile_width(NCK);
  t.fl = 4 * NCK + 16;
  t.plane_off = (size_t)t.y * a.g.Z * a.g.X;
  return t;
}

// Input tile T[r][s] = ã[z0 − Rz + r][x0 − Rx + s], r < th, s < tw.
__device__ void mstage_tile(float *T, const float *__restrict__ src, const TwoDPassArgs &a, const MTile &t) {
  const int rz = (a.kz - 1) / 2, rx = (a.kx - 1) / 2;
  for (int e = threadIdx.x; e < t.th * t.tw; e += MNT) {
    const int r = e / t.tw, s = e - r * t.tw;
    int z = t.z0 - rz + r, x = t.x0 - rx + s;
    bool ok;
    if (a.boundary == 0) {
      ok = z >= 0 && z < a.g.Z && x >= 0 && x < a.g.X;
    } else {
      z = wrap2(z, a.g.Z);
      x = wrap2(x, a.g.X);
      ok = true;
    }
    T[e] = ok ? src[(size_t)z * a.g.X + x] : 0.f;
  }
}

// Tap rows F[j][16 + i] = ft[j][i] for i < kx, zero elsewhere in [0, fl).
__device__ void mstage_taps(float *F, const float *__restrict__ ft, const TwoDPassArgs &a, const MTile &t) {
  const int kxp = (a.kx + 3) & ~3;
  for (int e = threadIdx.x; e < a.kz * t.fl; e += MNT) {
    const int j = e / t.fl, i = e - j * t.fl - 16;
    F[e] = (i >= 0 && i < a.kx) ? ft[j * kxp + i] : 0.f;
  }
}

// This wave's two 16 × 16 blocks (rows m0.., columns c0.. and c0+16..).
template <int NCK>
__device__ __forceinline__ void mconv(const float *T, const float *F, const MTile &t, int kz, int m0, int c0,
                                      f32x4 &acc0, f32x4 &acc1) {
  const int lane = threadIdx.x & 63, n = lane & 15, kk = lane >> 4;
  acc0 = f32x4{0.f, 0.f, 0.f, 0.f};
  acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
  const float *Arow = T + (m0 + n) * t.tw + c0 + kk;   // A[m = n][k = kk]: input row m + j
  const float *Frow = F + 16 + kk - n;                 // B[k = kk][n]: ft[j][k − n]
  for (int j = 0; j < kz; ++j) {
    const float *Ar = Arow + j * t.tw;
    const float *Fr = Frow + j * t.fl;
#pragma unroll
    for (int c = 0; c < NCK; ++c) {
      const float b = Fr[4 * c];
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Ar[4 * c], b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Ar[4 * c + 16], b, acc1, 0, 0, 0);
    }
  }
}

template <int NCK>
__global__ void __launch_bounds__(MNT) twod_mfma_forward_kernel(const TwoDPassArgs a) {
  extern __shared__ __align__(16) float sm[];
  const MTile t = mtile_of<NCK>(a);
  float *T = sm;
  float *F = sm + t.th * t.tw;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = 16 * (w >> 1), c0 = 32 * (w & 1);
  mstage_tile(T, a.in[0] + t.plane_off, a, t);
  for (int v = 0; v < a.nviews; ++v) {
    if (v > 0) __syncthreads();   // every wave is done with the previous taps
    mstage_taps(F, a.taps[v], a, t);
    __syncthreads();
    f32x4 acc[2];
    mconv<NCK>(T, F, t, a.kz, m0, c0, acc[0], acc[1]);
    // D[i]: row 4·(lane/16) + i, column lane % 16 of each block
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int x = t.x0 + c0 + 16 * blk + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int z = t.z0 + m0 + 4 * (lane >> 4) + i;
        if (z < a.g.Z && x < a.g.X) {
          const size_t off = t.plane_off + (size_t)z * a.g.X + x;
          a.out[v][off] = a.phi[v] ? guarded_ratio(a.phi[v][off], acc[blk][i]) : acc[blk][i];
        }
      }
    }
  }
}

template <int NCK>
__global__ void __launch_bounds__(MNT) twod_mfma_backward_kernel(const TwoDPassArgs a) {
  extern __shared__ __align__(16) float sm[];
  const MTile t = mtile_of<NCK>(a);
  float *T = sm;
  float *F = sm + t.th * t.tw;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = 16 * (w >> 1), c0 = 32 * (w & 1);
  float prod[2][4];
  for (int v = 0; v < a.nviews; ++v) {
    if (v > 0) __syncthreads();
    mstage_tile(T, a.in[v] + t.plane_off, a, t);
    mstage_taps(F, a.taps[v], a, t);
    __syncthreads();
    f32x4 acc[2];
    mconv<NCK>(T, F, t, a.kz, m0, c0, acc[0], acc[1]);
    const float wv = a.w[v], w1 = 1.f - wv;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float c = fmaf(wv, acc[blk][i], w1);
        prod[blk][i] = v == 0 ? c : prod[blk][i] * c;
      }
  }
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int x = t.x0 + c0 + 16 * blk + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int z = t.z0 + m0 + 4 * (lane >> 4) + i;
      if (z < a.g.Z && x < a.g.X) {
        const size_t off = t.plane_off + (size_t)z * a.g.X + x;
        a.psi_out[off] = a.psi_in[off] * prod[blk][i];
      }
    }
  }
}

size_t tile_lds(const TwoDPassArgs &a) {
  const int kxp = (a.kx + 3) & ~3;
  return sizeof(float) * (size_t)(TZ + a.kz - 1) * (TX + kxp + 4);
}

unsigned tile_count(const TwoDPassArgs &a) {
  return (unsigned)a.g.Y * ((a.g.Z + TZ - 1) / TZ) * ((a.g.X + TX - 1) / TX);
}

template <typename K>
hipError_t launch2d(K kern, const TwoDPassArgs &a, hipStream_t s) {
  const size_t lds = tile_lds(a);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(tile_count(a)), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename K>
hipError_t launch_mfma(K kern, const TwoDPassArgs &a, int nck, hipStream_t s) {
  const size_t lds = mfma_lds_bytes(a.kz, a.kx);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const unsigned tiles = (unsigned)a.g.Y * ((a.g.Z + MZ - 1) / MZ) * ((a.g.X + MX - 1) / MX);
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(MNT), lds, s, a);
  return hipGetLastError();
}

template <int NCK>
hipError_t mfma_pass(const TwoDPassArgs &a, bool fwd, hipStream_t s) {
  return fwd ? launch_mfma(twod_mfma_forward_kernel<NCK>, a, NCK, s)
             : launch_mfma(twod_mfma_backward_kernel<NCK>, a, NCK, s);
}

hipError_t launch_mfma_pass(const TwoDPassArgs &a, bool fwd, hipStream_t s) {
  switch (mfma_chunks(a.kx)) {
    case 6: return mfma_pass<6>(a, fwd, s);
    case 8: return mfma_pass<8>(a, fwd, s);
    case 12: return mfma_pass<12>(a, fwd, s);
    case 16: return mfma_pass<16>(a, fwd, s);
    case 20: return mfma_pass<20>(a, fwd, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

size_t mfma_lds_bytes(int kz, int kx) {
  const int nck = mfma_chunks(kx);
  return sizeof(float) * ((size_t)(MZ + kz - 1) * mfma_tile_width(nck) + (size_t)kz * (4 * nck + 16));
}

hipError_t launch_2d_forward(const TwoDPassArgs &a, hipStream_t s) {
  if (a.mfma) return launch_mfma_pass(a, true, s);
  return launch2d(twod_forward_kernel, a, s);
}

hipError_t launch_2d_backward(const TwoDPassArgs &a, hipStream_t s) {
  if (a.mfma) return launch_mfma_pass(a, false, s);
  return launch2d(twod_backward_kernel, a, s);
}

}  // namespace mvd
