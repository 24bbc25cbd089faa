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

// φ / b for b > ε, else 1: reciprocal refined by one Newton-Raphson correction
// of the quotient (Markstein); within 1 ulp of IEEE, exactly 1 when φ = b.
__device__ __forceinline__ float guarded_ratio(float phi, float b) {
  const float y = __builtin_amdgcn_rcpf(b);
  const float q0 = phi * y;
  const float q = fmaf(fmaf(-b, q0, phi), y, q0);
  return b > kEps ? q : 1.f;
}

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
        if (t.x0 + ox + n < a.g.X) {
          const float p = a.phi[v][off + n];
          a.out[v][off + n] = guarded_ratio(p, b[n]);
        }
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

}  // namespace

hipError_t launch_2d_forward(const TwoDPassArgs &a, hipStream_t s) {
  return launch2d(twod_forward_kernel, a, s);
}

hipError_t launch_2d_backward(const TwoDPassArgs &a, hipStream_t s) {
  return launch2d(twod_backward_kernel, a, s);
}

}  // namespace mvd
