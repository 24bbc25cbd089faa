// Persistent batched form: one launch works through a queue of tiles of the
// passes of several volumes (Supplementary Note 1 update, every plane on its
// own; Supplementary Note 2 §3 treats planes independently).
//
// A work item is one tile (row segment × column strip) of one plane of one
// volume in one phase: ψ^0, then per iteration the forward passes (blur +
// ratio) and the backward passes (back-projection + update) in the order of
// the volume's update rule.  Items sit in a table in dependency order: an
// item's phase needs every tile of the same plane's previous phase, and those
// items come earlier in the table.  Work-groups take items from an atomic
// head; before running one, a work-group waits until the plane's counter of
// completed tiles reaches the phase's start.  It only ever waits for items
// that running work-groups took before it, so the queue drains whatever the
// number of resident work-groups.  The wait is bounded: after `spin_limit`
// polls the work-group raises the give-up flag, every work-group then skips
// the rest, and the host reports the flag.
//
// Visibility across work-groups (and across the XCDs' separate L2 caches):
// every wave waits until its stores are complete in its XCD's L2, then the
// thread that counts the tile done does so with an agent-scope release (which
// writes that L2 back to memory first), and the waiting thread's agent-scope
// acquire load invalidates the caches its work-group reads through.
#include <algorithm>

#include "k_sep_impl.hpp"

namespace mvd {
namespace {

using namespace sepk;

__device__ __forceinline__ unsigned atomic_load_acq(const unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// ψ^0 of one tile's outputs by threads t = 0 … nt−1: the mean of the views
// (the plain path's arithmetic: a float sum in view order, divided by V) or a
// constant (init 2).
__device__ __forceinline__ void init_tile(const PqJob &j, int b, int t, int nt) {
  const int strip = b % j.nstrip;
  const int t2 = b / j.nstrip;
  const int seg = t2 % j.nseg;
  const int y = t2 / j.nseg;
  const int zs = seg * j.zseg, ze = min(zs + j.zseg, j.g.Z);
  const int x0 = strip * j.x_out, x1 = min(x0 + j.x_out, j.g.X);
  const int w = x1 - x0;
  const long n = (long)(ze - zs) * w;
  const float nvf = (float)j.nv;
  for (long e = t; e < n; e += nt) {
    const int z = zs + (int)(e / w), x = x0 + (int)(e % w);
    float v;
    if (j.init == 2) {
      v = j.init_const;
    } else {
      float sum = 0.f;
      const size_t s = (size_t)y * j.obs_sy + (size_t)z * j.obs_sz + x;
      for (int k = 0; k < j.nv; ++k) {
        const float f = j.obs_u16 ? (float)static_cast<const uint16_t *>(j.obs[k])[s]
                                  : fmaxf(static_cast<const float *>(j.obs[k])[s], 0.f);
        sum += f;
      }
      v = sum / nvf;
    }
    j.est[((size_t)y * j.g.Z + z) * j.g.X + x] = v;
  }
}

// One pass tile: kind 0–3 forward (1 or 2 views, float32 or uint16
// observations), 4 backward (one ratio plane); whole 16-byte row items.  One
// function per kernel-size bucket, called with the pass arguments' address,
// the tile and the threads (t of nt) and LDS that run it: the arguments are
// the same for every lane of a wave, so they are made scalar again on entry
// (the tile code reads its arguments with scalar loads).
template <int KB>
__device__ __noinline__ void pass_tile(int kind, uint64_t aptr, int b, int t, int nt, uint32_t lds_off) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)aptr);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(aptr >> 32));
  KArg *a = (KArg *)(((uint64_t)hi << 32) | lo);
  b = __builtin_amdgcn_readfirstlane(b);
  nt = __builtin_amdgcn_readfirstlane(nt);
  extern __shared__ __align__(16) float lds_all[];
  float *lds = lds_all + __builtin_amdgcn_readfirstlane(lds_off);
  switch (__builtin_amdgcn_readfirstlane(kind)) {
    case 0: fwd_tile<KB, 1, 1, kEpRatio, 1>(a, b, t, nt, lds); break;
    case 1: fwd_tile<KB, 1, 2, kEpRatio, 1>(a, b, t, nt, lds); break;
    case 2: fwd_tile<KB, 1, 1, kEpRatioU16, 1>(a, b, t, nt, lds); break;
    case 3: fwd_tile<KB, 1, 2, kEpRatioU16, 1>(a, b, t, nt, lds); break;
    default: bwd_tile<KB, 1, 1, 1, 0>(a, b, t, nt, lds); break;
  }
}

__device__ __forceinline__ void run_pass(int kb, int kind, const SepPassArgs *a, int b, int t, int nt,
                                         uint32_t lds_off) {
  const uint64_t p = (uint64_t)(uintptr_t)a;
  switch (kb) {
    case 3: pass_tile<3>(kind, p, b, t, nt, lds_off); break;
    case 7: pass_tile<7>(kind, p, b, t, nt, lds_off); break;
    case 11: pass_tile<11>(kind, p, b, t, nt, lds_off); break;
    case 15: pass_tile<15>(kind, p, b, t, nt, lds_off); break;
    case 21: pass_tile<21>(kind, p, b, t, nt, lds_off); break;
    case 31: pass_tile<31>(kind, p, b, t, nt, lds_off); break;
    default: pass_tile<41>(kind, p, b, t, nt, lds_off); break;
  }
}

typedef __attribute__((address_space(4))) const PqJob KJob;

__device__ __forceinline__ bool wait_plane(const PqQueue &q, KJob *j, int y, unsigned need) {
  unsigned polls = 0;
  while (atomic_load_acq(j->done + y) < need) {
    if (__hip_atomic_load(q.giveup, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++polls > q.spin_limit) {
      __hip_atomic_store(q.giveup, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  return true;
}

// Work-groups of kPqThreads threads.  A job whose tiles need at most half of
// them runs two tiles per item, one in each half (the tiles of an item share
// their row segment, so both halves execute the same barriers; a lone tile's
// partner half executes its barriers only); a wider job runs one tile with
// every thread.
__global__ void __launch_bounds__(kPqThreads, 4) pq_kernel(PqQueue q) {
  __shared__ int s_item, s_go;
  extern __shared__ __align__(16) float lds_all[];
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)__hip_atomic_fetch_add(q.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= q.n_items) break;
    const int4 it = q.items[item];   // job, phase, first tile, second tile (−1: none)
    const int jx = __builtin_amdgcn_readfirstlane(it.x);
    KJob *j = (KJob *)(uintptr_t)(q.jobs + jx);   // read-only for the whole launch: scalar loads
    const int phase = __builtin_amdgcn_readfirstlane(it.y);
    const int b0 = __builtin_amdgcn_readfirstlane(it.z);
    const int b1 = __builtin_amdgcn_readfirstlane(it.w);
    const int nt_ = j->ntiles;
    if (threadIdx.x == 0) {
      // every tile of these planes' previous phases must be complete
      const unsigned need = (unsigned)phase * (unsigned)nt_;
      bool go = wait_plane(q, j, b0 / nt_, need);
      if (go && b1 >= 0) go = wait_plane(q, j, b1 / nt_, need);
      s_go = go && __hip_atomic_load(q.giveup, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
    __syncthreads();
    if (s_go) {
      const bool pair = j->pair != 0;
      const int half = pair ? (int)(threadIdx.x / (kPqThreads / 2)) : 0;   // wave-uniform
      const int t = pair ? (int)(threadIdx.x % (kPqThreads / 2)) : (int)threadIdx.x;
      const int nt = pair ? kPqThreads / 2 : kPqThreads;
      const int b = half ? b1 : b0;
      const uint32_t lds_off = (uint32_t)half * (uint32_t)j->lds_floats;
      if (phase == 0) {
        if (j->init != 1 && b >= 0) init_tile(q.jobs[jx], b, t, nt);   // a given ψ^0 is already in place
      } else {
        const int r = (phase - 1) % j->per_iter;
        bool fwd;
        int slot;
        if (j->sim) {
          fwd = r < j->nf;
          slot = fwd ? r : r - j->nf;
        } else {
          fwd = (r & 1) == 0;
          slot = r >> 1;
        }
        const int kind = fwd ? j->fkind[slot] : 4;
        const SepPassArgs *a = fwd ? &q.jobs[jx].f[slot] : &q.jobs[jx].b[slot];
        if (b >= 0) {
          run_pass(j->kb, kind, a, b, t, nt, lds_off);
        } else {   // no second tile: the barriers of the first one
          KArg *ka = fwd ? &j->f[slot] : &j->b[slot];
          const int nb = tile_barriers(ka, b0);
          for (int k = 0; k < nb; ++k) lds_sync();
        }
      }
      // every wave's stores have reached the L2 of this XCD before the barrier;
      // the counting thread's agent-scope release then writes that L2 back
      // (one write-back per item, not one per wave)
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    if (s_go && threadIdx.x == 0) {
      __hip_atomic_fetch_add(j->done + b0 / nt_, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (b1 >= 0) __hip_atomic_fetch_add(j->done + b1 / nt_, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // the last work-group to leave resets the queue and the counters for the next launch
  if (threadIdx.x == 0)
    s_go = __hip_atomic_fetch_add(q.exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (s_go) {
    for (int k = 0; k < q.n_jobs; ++k) {
      unsigned *d = q.jobs[k].done;
      for (int i = threadIdx.x; i < q.jobs[k].g.Y; i += blockDim.x) d[i] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      *q.head = 0u;
      *q.exited = 0u;
    }
  }
}

}  // namespace

size_t pq_lds_bytes(const PqJob &j) {
  // one tile's LDS: the double-buffered column-pass rows and tap tables of
  // its largest pass (floats), rounded to 16 bytes
  const size_t nk = (size_t)((j.kb + 3 + 3) / 4 * 4);
  size_t fl = 0;
  for (int s = 0; s < j.nf; ++s)
    fl = std::max<size_t>(fl, 2ull * j.f[s].nviews * kRowGroup * j.f[s].ldsw + (size_t)j.f[s].nviews * 8 * nk);
  fl = std::max<size_t>(fl, 2ull * kRowGroup * j.b[0].ldsw + 8 * nk);
  return (fl + 3) / 4 * 4 * sizeof(float);
}

hipError_t launch_pq(const PqQueue &q, int nblocks, size_t lds, hipStream_t s) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pq_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(pq_kernel, dim3(nblocks), dim3(kPqThreads), lds, s, q);
  return hipGetLastError();
}

hipError_t pq_occupancy(size_t lds, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pq_kernel, kPqThreads, lds);
}

}  // namespace mvd
