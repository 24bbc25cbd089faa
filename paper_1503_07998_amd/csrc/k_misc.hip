// Element-wise kernels: reslice / convert of the observations, ψ^0, fill, copy,
// the pointwise update from a stored back-projection, calibration kernels.
#include <algorithm>

#include "mvd_internal.hpp"

namespace mvd {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ float obs_value(const void *src, int dtype, size_t i) {
  if (dtype == 1) return (float)static_cast<const uint16_t *>(src)[i];
  return fmaxf(static_cast<const float *>(src)[i], 0.f);   // NaN → 0
}

// dst planes [Y][Z][X] ← src stack [Z][Y][X] (layout 1) or planes (layout 2).
// Each thread moves 4 consecutive elements of one row when X is a multiple of 4.
__global__ void __launch_bounds__(NT) stage_kernel(const void *__restrict__ src, int dtype, int layout,
                                                    PlaneGeom g, float *__restrict__ dst, int vec) {
  const size_t row_elems = (size_t)g.X;
  const size_t total = (size_t)g.Y * g.Z * g.X;
  const size_t step = (size_t)gridDim.x * NT * (vec ? 4 : 1);
  for (size_t e = ((size_t)blockIdx.x * NT + threadIdx.x) * (vec ? 4 : 1); e < total; e += step) {
    const size_t row = e / row_elems;           // = y·Z + z of the destination
    const size_t x = e - row * row_elems;
    const size_t z = row % g.Z, y = row / g.Z;
    const size_t s = layout == 1 ? (z * g.Y + y) * row_elems + x : e;
    if (vec) {
      float4 v;
      if (dtype == 1) {
        const ushort4 u = *reinterpret_cast<const ushort4 *>(static_cast<const uint16_t *>(src) + s);
        v = make_float4((float)u.x, (float)u.y, (float)u.z, (float)u.w);
      } else {
        const float4 f = *reinterpret_cast<const float4 *>(static_cast<const float *>(src) + s);
        v = make_float4(fmaxf(f.x, 0.f), fmaxf(f.y, 0.f), fmaxf(f.z, 0.f), fmaxf(f.w, 0.f));
      }
      *reinterpret_cast<float4 *>(dst + e) = v;
    } else {
      dst[e] = obs_value(src, dtype, s);
    }
  }
}

struct Ptrs {
  const float *p[kMaxViews];
};

struct StageViews {
  const void *src[kMaxViews];
  float *dst[kMaxViews];
  float *mean;   // ψ^0 = (1/V) Σ_v φ_v, or null
  int nv, dtype, layout, vec;
  int ysrc;   // planes of the source stack (its y stride is X, its z stride ysrc·X)
  PlaneGeom g;
};

__device__ __forceinline__ float4 load4(const void *src, int dtype, size_t off) {
  if (dtype == 1) {
    const ushort4 u = *reinterpret_cast<const ushort4 *>(static_cast<const uint16_t *>(src) + off);
    return make_float4((float)u.x, (float)u.y, (float)u.z, (float)u.w);
  }
  const float4 f = *reinterpret_cast<const float4 *>(static_cast<const float *>(src) + off);
  return make_float4(fmaxf(f.x, 0.f), fmaxf(f.y, 0.f), fmaxf(f.z, 0.f), fmaxf(f.w, 0.f));
}

// Every view's observations → float32 planes, and optionally their mean, in
// one pass: one wave per destination row (y, z), lanes along x.
__global__ void __launch_bounds__(NT) stage_views_kernel(StageViews a) {
  const int lane = threadIdx.x & 63;
  const size_t nrows = (size_t)a.g.Y * a.g.Z;
  const size_t X = (size_t)a.g.X;
  const size_t nwaves = (size_t)gridDim.x * (NT / 64);
  const float nvf = (float)a.nv;
  for (size_t rr = (size_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); rr < nrows; rr += nwaves) {
    const size_t y = rr / a.g.Z, z = rr - y * a.g.Z;
    const size_t srow = a.layout == 1 ? (z * a.ysrc + y) * X : rr * X;
    const size_t drow = rr * X;
    if (a.vec) {
      for (size_t x = 4 * (size_t)lane; x < X; x += 256) {
        float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int v = 0; v < a.nv; ++v) {
          const float4 f = load4(a.src[v], a.dtype, srow + x);
          if (a.dst[v]) *reinterpret_cast<float4 *>(a.dst[v] + drow + x) = f;
          sum.x += f.x;
          sum.y += f.y;
          sum.z += f.z;
          sum.w += f.w;
        }
        if (a.mean)
          *reinterpret_cast<float4 *>(a.mean + drow + x) =
              make_float4(sum.x / nvf, sum.y / nvf, sum.z / nvf, sum.w / nvf);
      }
    } else {
      for (size_t x = lane; x < X; x += 64) {
        float sum = 0.f;
        for (int v = 0; v < a.nv; ++v) {
          const float f = obs_value(a.src[v], a.dtype, srow + x);
          if (a.dst[v]) a.dst[v][drow + x] = f;
          sum += f;
        }
        if (a.mean) a.mean[drow + x] = sum / nvf;
      }
    }
  }
}

__global__ void __launch_bounds__(NT) init_mean_kernel(Ptrs ph, int nv, size_t n, float *__restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    float s = 0.f;
    for (int v = 0; v < nv; ++v) s += fmaxf(ph.p[v][i], 0.f);
    dst[i] = s / (float)nv;
  }
}

__global__ void __launch_bounds__(NT) fill_kernel(float *__restrict__ dst, size_t n, float value) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) dst[i] = value;
}

__global__ void __launch_bounds__(NT) copy_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                                   size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) dst[i] = src[i];
}

// Calibration kernels of known traffic (the bandwidth a plain streaming
// kernel reaches, against which the passes are judged): a copy that reads and
// writes every 16-byte unit once, and a read-only sweep whose sums are stored
// only where they hold the all-ones bit pattern (never, for finite data), so it
// writes nothing while the compiler must still load every unit.  Each thread
// moves kProbeU units per step, 16 bytes per lane per access.
constexpr int kProbeU = 4;

__global__ void __launch_bounds__(NT) probe_copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                         size_t n) {
  const size_t step = (size_t)gridDim.x * NT * kProbeU;
  size_t i = (size_t)blockIdx.x * NT * kProbeU + threadIdx.x;
  for (; i + (kProbeU - 1) * NT < n; i += step) {
    float4 v[kProbeU];
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) v[u] = src[i + u * NT];
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) dst[i + u * NT] = v[u];
  }
  for (; i < n; i += NT) dst[i] = src[i];   // the last partial step
}

__global__ void __launch_bounds__(NT) probe_read_kernel(const float4 *__restrict__ src, float *__restrict__ dst,
                                                         size_t n) {
  const size_t step = (size_t)gridDim.x * NT * kProbeU;
  size_t i = (size_t)blockIdx.x * NT * kProbeU + threadIdx.x;
  float s = 0.f;
  for (; i + (kProbeU - 1) * NT < n; i += step) {
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) {
      const float4 v = src[i + u * NT];
      s += (v.x + v.y) + (v.z + v.w);
    }
  }
  for (; i < n; i += NT) {
    const float4 v = src[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (__float_as_uint(s) == 0xffffffffu) dst[blockIdx.x] = s;
}

// ψ_out = ψ_in · (o q' + 1 − o): the update of one view from its stored
// back-projection q (q' = q / s where s > ε with s the view's sensitivity
// plane [Z][X], when given; o = w · ω(pixel) with a weight plane, else w).
// The arithmetic of the separable backward pass's epilogue, element by element.
__global__ void __launch_bounds__(NT) update_plane_kernel(const float *psi_in, float *psi_out,
                                                           const float *__restrict__ q,
                                                           const float *__restrict__ splane, size_t zx,
                                                           const float *__restrict__ wpl, float w, size_t n) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    float qq = q[i];
    if (splane) {
      const float sv = splane[i % zx];
      qq = sv > kEps ? qq * __builtin_amdgcn_rcpf(sv) : qq;
    }
    const float o = wpl ? w * wpl[i] : w;
    psi_out[i] = psi_in[i] * fmaf(o, qq, 1.f - o);
  }
}

unsigned grid_for(size_t work) {
  size_t b = (work + NT - 1) / NT;
  if (b > 65536) b = 65536;   // grid-stride beyond this
  if (b == 0) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_stage_obs(const void *src, int dtype, int layout, PlaneGeom g, float *dst,
                            hipStream_t s) {
  const size_t total = (size_t)g.Y * g.Z * g.X;
  if (total == 0) return hipSuccess;
  const int vec = (g.X % 4 == 0) && ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
  hipLaunchKernelGGL(stage_kernel, dim3(grid_for(vec ? total / 4 : total)), dim3(NT), 0, s, src, dtype,
                     layout, g, dst, vec);
  return hipGetLastError();
}

hipError_t launch_stage_views(const void *const *src, int nv, int dtype, int layout, PlaneGeom g,
                              float *const *dst, float *mean, hipStream_t s, int ysrc) {
  const size_t rows = (size_t)g.Y * g.Z;
  if (rows == 0 || g.X == 0) return hipSuccess;
  if (nv < 1 || nv > kMaxViews) return hipErrorInvalidValue;
  StageViews a{};
  a.nv = nv;
  a.dtype = dtype;
  a.layout = layout;
  a.ysrc = ysrc > 0 ? ysrc : g.Y;
  a.g = g;
  a.mean = mean;
  const uintptr_t sa = dtype == 1 ? 8 : 16;
  int vec = g.X % 4 == 0 && (!mean || (uintptr_t)mean % 16 == 0);
  for (int v = 0; v < nv; ++v) {
    a.src[v] = src[v];
    a.dst[v] = dst ? dst[v] : nullptr;
    vec = vec && (uintptr_t)src[v] % sa == 0 && (uintptr_t)a.dst[v] % 16 == 0;
  }
  a.vec = vec;
  const size_t blocks = std::min<size_t>((rows + NT / 64 - 1) / (NT / 64), 65536);
  hipLaunchKernelGGL(stage_views_kernel, dim3((unsigned)blocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_mean(const float *const *phis, int nv, size_t n, float *dst, hipStream_t s) {
  Ptrs p{};
  for (int v = 0; v < nv && v < kMaxViews; ++v) p.p[v] = phis[v];
  hipLaunchKernelGGL(init_mean_kernel, dim3(grid_for(n)), dim3(NT), 0, s, p, nv, n, dst);
  return hipGetLastError();
}

hipError_t launch_fill(float *dst, size_t n, float value, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(NT), 0, s, dst, n, value);
  return hipGetLastError();
}

hipError_t launch_copy(const float *src, float *dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(NT), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_update_plane(const float *psi_in, float *psi_out, const float *q, const float *splane, size_t zx,
                               const float *wpl, float w, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(update_plane_kernel, dim3(grid_for(n)), dim3(NT), 0, s, psi_in, psi_out, q, splane, zx, wpl, w,
                     n);
  return hipGetLastError();
}

hipError_t launch_stream_probe(int kind, const void *src, void *dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  // 8 work-groups of NT threads per CU (2048 on 256 CUs), grid-stride beyond
  const unsigned blocks = (unsigned)std::min<size_t>((n + (size_t)NT * kProbeU - 1) / ((size_t)NT * kProbeU),
                                                     kProbeBlocks);
  if (kind == 0)
    hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(NT), 0, s, static_cast<const float4 *>(src),
                       static_cast<float4 *>(dst), n);
  else
    hipLaunchKernelGGL(probe_read_kernel, dim3(blocks), dim3(NT), 0, s, static_cast<const float4 *>(src),
                       static_cast<float *>(dst), n);
  return hipGetLastError();
}

}  // namespace mvd
