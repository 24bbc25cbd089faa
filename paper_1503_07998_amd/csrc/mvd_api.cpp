// C ABI of the plane-wise MV-RL library: validation, contexts, PSF setup,
// workspace layout and the pass schedule of one deconvolution run.
#include "../../include/mvd.h"
#include "../../include/mvd_testing.h"

#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mvd_internal.hpp"
#include "psf.hpp"

namespace mvd {
static_assert(kMaxPlaneX == MVD_MAX_PLANE_X, "the zero row must cover the widest accepted plane");
hipError_t sep_forward_kb3(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb7(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb11(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb15(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb21(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb31(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb41(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_forward_kb63(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb3(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb7(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb11(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb15(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb21(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb31(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb41(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_kb63(const SepPassArgs &, const SepPlan &, hipStream_t);

hipError_t sep_single_kb3(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb7(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb11(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb15(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb21(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb31(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb41(const SepPassArgs &, const SepPlan &, int, hipStream_t);
hipError_t sep_single_kb63(const SepPassArgs &, const SepPlan &, int, hipStream_t);

hipError_t sep_backward_split_kb3(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_split_kb7(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_split_kb11(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_split_kb15(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_split_kb21(const SepPassArgs &, const SepPlan &, hipStream_t);
hipError_t sep_backward_split_kb31(const SepPassArgs &, const SepPlan &, hipStream_t);

hipError_t launch_sep_backward_split(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  switch (p.bucket) {
    case 3: return sep_backward_split_kb3(a, p, s);
    case 7: return sep_backward_split_kb7(a, p, s);
    case 11: return sep_backward_split_kb11(a, p, s);
    case 15: return sep_backward_split_kb15(a, p, s);
    case 21: return sep_backward_split_kb21(a, p, s);
    case 31: return sep_backward_split_kb31(a, p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sep_single_dispatch(const SepPassArgs &a, const SepPlan &p, int ep, hipStream_t s) {
  switch (p.bucket) {
    case 3: return sep_single_kb3(a, p, ep, s);
    case 7: return sep_single_kb7(a, p, ep, s);
    case 11: return sep_single_kb11(a, p, ep, s);
    case 15: return sep_single_kb15(a, p, ep, s);
    case 21: return sep_single_kb21(a, p, ep, s);
    case 31: return sep_single_kb31(a, p, ep, s);
    case 41: return sep_single_kb41(a, p, ep, s);
    case 63: return sep_single_kb63(a, p, ep, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sep_forward(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  switch (p.bucket) {
    case 3: return sep_forward_kb3(a, p, s);
    case 7: return sep_forward_kb7(a, p, s);
    case 11: return sep_forward_kb11(a, p, s);
    case 15: return sep_forward_kb15(a, p, s);
    case 21: return sep_forward_kb21(a, p, s);
    case 31: return sep_forward_kb31(a, p, s);
    case 41: return sep_forward_kb41(a, p, s);
    case 63: return sep_forward_kb63(a, p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sep_backward(const SepPassArgs &a, const SepPlan &p, hipStream_t s) {
  switch (p.bucket) {
    case 3: return sep_backward_kb3(a, p, s);
    case 7: return sep_backward_kb7(a, p, s);
    case 11: return sep_backward_kb11(a, p, s);
    case 15: return sep_backward_kb15(a, p, s);
    case 21: return sep_backward_kb21(a, p, s);
    case 31: return sep_backward_kb31(a, p, s);
    case 41: return sep_backward_kb41(a, p, s);
    case 63: return sep_backward_kb63(a, p, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace mvd

using namespace mvd;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024;

// Kernels that are not rank one run as sums of rank-one terms when their SVD
// needs at most kLowRankMax terms to reproduce every tap to kLowRankTol of the
// largest (the rank-one test's tolerance); each term costs one 1D pass pair.
constexpr int kLowRankMax = 6;
constexpr double kLowRankTol = 1e-6;

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct ViewPsf {
  bool set = false;
  Kernel psf;               // P_v as given (float32 values in double)
  int back_mode = 0;
  Kernel explicit_back;
  // derived
  Kernel back;              // X_v (float32-rounded values)
  bool sep_p = false, sep_x = false;
  std::vector<float> pz, px, xz, xx;  // 1D factors (z, x) of P_v and X_v
  // kernels that are not rank one but a sum of a few rank-one terms (from
  // their SVD): each term's factors; empty where the K×K passes are taken
  std::vector<std::vector<float>> lpz, lpx, lxz, lxx;
};

thread_local std::string g_noctx_error;

// Live contexts (pointer → serial), so that a batch can tell a context it
// captured from one destroyed since (or a new one at the same address).
std::mutex g_live_mu;
std::map<const mvd_ctx *, uint64_t> g_live;
uint64_t g_next_serial = 1;

// Device scratch of mvd_deconvolve_planes_static: one array per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address (in host code it is only a stand-in for the symbol): each device's
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is passed to kernels.
constexpr size_t kScratchBytes = (size_t)MVD_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

// With `dev` current: this device's scratch address, taken on first use.
hipError_t scratch_setup(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = p;
  *out = p;
  return hipSuccess;
}

}  // namespace

struct mvd_ctx {
  int nv = 0, Z = 0, X = 0, device = MVD_DEVICE_NONE;
  std::vector<ViewPsf> views;
  bool derived = false;
  int kzm = 1, kxm = 1, kxpm = 4;  // common K×K size of the general kernels
  float *d_taps = nullptr;         // [V][2][kzm][kxpm] flipped taps (forward, back), then the
                                   // sensitivity factors [V][2 boundaries][Z + X] (+ pad)
  size_t d_taps_cap = 0;
  std::string err;
  // launch timing (MVD_FLAG_TIMING)
  struct Mark {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  // captured runs (MVD_FLAG_GRAPH)
  struct Graph {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs;
  uint64_t psf_generation = 0;   // bumped by every mvd_set_psf (captured taps change)
  uint64_t serial = 0;           // unique per context of the process (live-context registry)
  // streamed runs: copy-in and copy-out streams and their events
  hipStream_t h2d = nullptr, d2h = nullptr;
  hipEvent_t sev[7] = {};        // start, in[2], done[2], out[2]
  // disk-to-disk runs: page-locked host batches, kept for later calls
  void *fhost = nullptr;
  size_t fhost_bytes = 0;
};

namespace {

mvd_status fail(mvd_ctx *c, mvd_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_noctx_error = buf;
  return s;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old_) != hipSuccess) old_ = -1;
    if (dev >= 0 && dev != old_) ok_ = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (old_ >= 0) (void)hipSetDevice(old_);
  }
  bool ok() const { return ok_; }

 private:
  int old_ = -1;
  bool ok_ = true;
};

bool valid_taps(const float *t, int n) {
  bool any = false;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(t[i]) || t[i] < 0.f) return false;
    if (t[i] > 0.f) any = true;
  }
  return any;
}

Kernel to_kernel(const float *t, int kz, int kx) {
  Kernel k{kz, kx, std::vector<double>((size_t)kz * kx)};
  for (int e = 0; e < kz * kx; ++e) k.t[e] = (double)t[e];
  return k;
}

Kernel round_f32(const Kernel &k) {
  Kernel o = k;
  for (double &e : o.t) e = (double)(float)e;
  return o;
}

std::vector<float> to_f32(const std::vector<double> &v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

// Build X_v, the rank-one factors and the device copy of the flipped taps.
// Floats of the sensitivity factors (padded so that an 8-wide read past a row end
// stays inside the allocation).
// Each [Z] and [X] vector starts on a 16-byte boundary (the passes read 8 at a time).
// Tap sets per view on the device for the K×K passes (P_v, X_v, P_v^*, X_v^*).
constexpr int kTapSets = 4;

size_t norm_stride(const mvd_ctx *c) { return (size_t)((c->Z + 3) / 4 * 4) + (size_t)((c->X + 3) / 4 * 4); }
size_t norm_zlen(const mvd_ctx *c) { return (size_t)((c->Z + 3) / 4 * 4); }
size_t norm_floats(const mvd_ctx *c) { return (size_t)c->nv * 2 * norm_stride(c) + 16; }

mvd_status derive(mvd_ctx *c) {
  std::vector<Kernel> psfs;
  for (auto &v : c->views) psfs.push_back(v.psf);
  c->kzm = 1;
  c->kxm = 1;
  for (int v = 0; v < c->nv; ++v) {
    ViewPsf &w = c->views[v];
    if (w.back_mode == MVD_BACK_FLIPPED) {
      w.back = flip(w.psf);
    } else if (w.back_mode == MVD_BACK_EXPLICIT) {
      w.back = w.explicit_back;
    } else {
      Kernel x;
      if (!compound_back(psfs, v, w.back_mode, &x))
        return fail(c, MVD_ERR_ARG, "view %d: compound back-projector has no positive tap", v);
      w.back = round_f32(x);
    }
    std::vector<double> u, vv;
    w.sep_p = rank_one(w.psf, &u, &vv);
    if (w.sep_p) {
      w.pz = to_f32(u);
      w.px = to_f32(vv);
    }
    w.sep_x = rank_one(w.back, &u, &vv);
    if (w.sep_x) {
      w.xz = to_f32(u);
      w.xx = to_f32(vv);
    }
    // not rank one: a sum of at most kLowRankMax rank-one terms reproducing
    // every tap to kLowRankTol of the largest runs as that many 1D pass pairs
    w.lpz.clear();
    w.lpx.clear();
    w.lxz.clear();
    w.lxx.clear();
    std::vector<std::vector<double>> us, vs;
    if (!w.sep_p && low_rank(w.psf, kLowRankMax, kLowRankTol, &us, &vs))
      for (size_t t = 0; t < us.size(); ++t) {
        w.lpz.push_back(to_f32(us[t]));
        w.lpx.push_back(to_f32(vs[t]));
      }
    if (!w.sep_x && low_rank(w.back, kLowRankMax, kLowRankTol, &us, &vs))
      for (size_t t = 0; t < us.size(); ++t) {
        w.lxz.push_back(to_f32(us[t]));
        w.lxx.push_back(to_f32(vs[t]));
      }
    c->kzm = std::max({c->kzm, w.psf.kz, w.back.kz});
    c->kxm = std::max({c->kxm, w.psf.kx, w.back.kx});
  }
  c->kxpm = (c->kxm + 3) & ~3;
  if (c->device != MVD_DEVICE_NONE) {
    const size_t per = (size_t)c->kzm * c->kxpm;
    const size_t ntaps = (size_t)c->nv * kTapSets * per;
    std::vector<float> host(ntaps + norm_floats(c), 0.f);
    // 1 ⊛ X_v for a rank-one X_v = xz ⊗ xx: (Σ_j xz[j] over rows z + Rz − j inside
    // the plane) · (the same along x); periodic: the full sums
    for (int v = 0; v < c->nv; ++v) {
      const ViewPsf &w = c->views[v];
      if (!w.sep_x) continue;
      for (int bd = 0; bd < 2; ++bd) {
        float *nz = host.data() + ntaps + ((size_t)v * 2 + bd) * norm_stride(c);
        float *nx = nz + norm_zlen(c);
        const int kz = (int)w.xz.size(), kx = (int)w.xx.size(), rz = (kz - 1) / 2, rx = (kx - 1) / 2;
        for (int z = 0; z < c->Z; ++z) {
          double acc = 0.0;
          for (int j = 0; j < kz; ++j)
            if (bd == 1 || (z + rz - j >= 0 && z + rz - j < c->Z)) acc += w.xz[j];
          nz[z] = (float)acc;
        }
        for (int x = 0; x < c->X; ++x) {
          double acc = 0.0;
          for (int i = 0; i < kx; ++i)
            if (bd == 1 || (x + rx - i >= 0 && x + rx - i < c->X)) acc += w.xx[i];
          nx[x] = (float)acc;
        }
      }
    }
    for (int v = 0; v < c->nv; ++v) {
      for (int which = 0; which < kTapSets; ++which) {
        const Kernel &k = which % 2 == 0 ? c->views[v].psf : c->views[v].back;
        float *dst = host.data() + ((size_t)v * kTapSets + which) * per;
        const int oz = (c->kzm - k.kz) / 2, ox = (c->kxm - k.kx) / 2;
        // embedded centred in kzm×kxm; sets 0, 1 point-reflected (ft[jj][q] =
        // k[kzm-1-jj][kxm-1-q]: the passes convolve with k), sets 2, 3 as given
        // (the passes then convolve with k's point reflection)
        for (int j = 0; j < k.kz; ++j)
          for (int i = 0; i < k.kx; ++i) {
            const bool refl = which < 2;
            const int jj = refl ? c->kzm - 1 - (j + oz) : j + oz, q = refl ? c->kxm - 1 - (i + ox) : i + ox;
            dst[(size_t)jj * c->kxpm + q] = (float)k.at(j, i);
          }
      }
    }
    DeviceGuard dg(c->device);
    if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
    const size_t bytes = host.size() * sizeof(float);
    if (bytes > c->d_taps_cap) {
      if (c->d_taps) (void)hipFree(c->d_taps);
      c->d_taps = nullptr;
      c->d_taps_cap = 0;
      if (hipMalloc(&c->d_taps, bytes) != hipSuccess)
        return fail(c, MVD_ERR_ALLOC, "cannot allocate %zu bytes of device taps", bytes);
      c->d_taps_cap = bytes;
    }
    if (hipMemcpy(c->d_taps, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
      return fail(c, MVD_ERR_LAUNCH, "upload of taps failed");
  }
  c->derived = true;
  return MVD_OK;
}

// Device sensitivity factors of view v under `boundary`: [Z] along z, then (at
// norm_zlen) [X].
const float *norm_factors(const mvd_ctx *c, int v, int boundary) {
  const size_t ntaps = (size_t)c->nv * kTapSets * c->kzm * c->kxpm;
  return c->d_taps + ntaps + ((size_t)v * 2 + (boundary == MVD_BOUNDARY_PERIODIC ? 1 : 0)) * norm_stride(c);
}

bool all_set(const mvd_ctx *c) {
  for (auto &v : c->views)
    if (!v.set) return false;
  return true;
}

// Workspace layout of one run: float32 copies of the observations (filled
// only where a K×K forward pass needs them) and the ratio planes.
struct Layout {
  size_t plane_set = 0; // bytes of one [Y][Z][X] float32 set
  size_t phi_off = 0, r_off = 0, acc_off = 0, total = 0;
  int n_ratio = 0;
  bool acc = false;     // a plane set for the partial sums of kernels run as sums of rank-one terms
  size_t sens_off = 0;  // two [Z][X] planes for the sensitivity of the general update, or none
  bool sens = false;
};

// Some pass of the run sums several rank-one terms (a PSF or back-projector
// that is not rank one but of low rank, and K×K passes not forced).
bool uses_low_rank(const mvd_ctx *c, const mvd_run *r) {
  if (!c->derived || (r->flags & MVD_FLAG_FORCE_2D)) return false;
  for (const ViewPsf &w : c->views)
    if ((!w.sep_p && !w.lpz.empty()) || (!w.sep_x && !w.lxz.empty())) return true;
  return false;
}

// Weight planes or the normalised back-projection with a back-projector that
// is not rank one (or with the K×K passes forced): the backward pass stores
// each view's back-projection and updates ψ pointwise.
bool uses_general_update(const mvd_ctx *c, const mvd_run *r) {
  if (!c->derived || !(r->weight_planes || (r->flags & MVD_FLAG_NORMALIZE))) return false;
  if (r->flags & MVD_FLAG_FORCE_2D) return true;
  for (const ViewPsf &w : c->views)
    if (!w.sep_x) return true;
  return false;
}

size_t sens_plane_bytes(const mvd_ctx *c) { return align_up((size_t)c->Z * c->X * sizeof(float)); }

Layout layout_of(const mvd_ctx *c, const mvd_run *r) {
  Layout L;
  L.plane_set = align_up((size_t)r->n_planes * c->Z * c->X * sizeof(float));
  L.n_ratio = r->update == MVD_UPDATE_SIMULTANEOUS ? c->nv : 1;
  size_t off = 0;
  L.phi_off = off;
  off += (size_t)c->nv * L.plane_set;
  L.r_off = off;
  off += (size_t)L.n_ratio * L.plane_set;
  const bool general = uses_general_update(c, r);
  L.acc = uses_low_rank(c, r) || general;
  L.acc_off = off;
  if (L.acc) off += L.plane_set;
  L.sens = general && (r->flags & MVD_FLAG_NORMALIZE);
  L.sens_off = off;
  if (L.sens) off += 2 * sens_plane_bytes(c);
  L.total = r->n_iters > 0 ? off : (size_t)c->nv * L.plane_set;
  return L;
}

mvd_status check_run(mvd_ctx *c, const mvd_run *r) {
  if (!r) return fail(c, MVD_ERR_ARG, "run is NULL");
  if (r->struct_size != sizeof(mvd_run))
    return fail(c, MVD_ERR_ARG, "run->struct_size %u != %zu", r->struct_size, sizeof(mvd_run));
  if (r->n_planes < 1) return fail(c, MVD_ERR_ARG, "n_planes must be >= 1");
  if (r->n_iters < 0) return fail(c, MVD_ERR_ARG, "n_iters must be >= 0");
  if (r->update != MVD_UPDATE_SIMULTANEOUS && r->update != MVD_UPDATE_SEQUENTIAL)
    return fail(c, MVD_ERR_ARG, "unknown update %d", r->update);
  if (r->boundary != MVD_BOUNDARY_ZERO && r->boundary != MVD_BOUNDARY_PERIODIC)
    return fail(c, MVD_ERR_ARG, "unknown boundary %d", r->boundary);
  if (r->init != MVD_INIT_MEAN && r->init != MVD_INIT_GIVEN && r->init != MVD_INIT_CONST)
    return fail(c, MVD_ERR_ARG, "unknown init %d", r->init);
  if (r->init == MVD_INIT_CONST && !(std::isfinite(r->init_const) && r->init_const > 0.f))
    return fail(c, MVD_ERR_ARG, "init_const must be finite and > 0");
  if (r->obs_dtype != MVD_U16 && r->obs_dtype != MVD_F32)
    return fail(c, MVD_ERR_ARG, "unknown obs_dtype %d", r->obs_dtype);
  if (r->obs_layout != MVD_STACK_ZYX && r->obs_layout != MVD_PLANES_YZX)
    return fail(c, MVD_ERR_ARG, "unknown obs_layout %d", r->obs_layout);
  if (r->flags & ~(MVD_FLAG_FORCE_2D | MVD_FLAG_TIMING | MVD_FLAG_GRAPH | MVD_FLAG_TUNE | MVD_FLAG_NORMALIZE))
    return fail(c, MVD_ERR_ARG, "unknown flags 0x%x", r->flags);
  if (r->weight_planes)
    for (int v = 0; v < c->nv; ++v)
      if (!r->weight_planes[v]) return fail(c, MVD_ERR_ARG, "weight_planes[%d] is NULL", v);
  if (r->view_weights)
    for (int v = 0; v < c->nv; ++v) {
      const float w = r->view_weights[v];
      if (!(std::isfinite(w) && w >= 0.f && w <= 1.f))
        return fail(c, MVD_ERR_ARG, "view weight %d = %g outside [0,1]", v, (double)w);
    }
  return MVD_OK;
}

// ---- pass planning -------------------------------------------------------
struct SepGeom {
  SepPlan plan;
  int zseg, nseg, x_out, nstrip, halo, ncols, ldsw;
};

int round_up(int n, int m) { return (n + m - 1) / m * m; }

// Work-groups a separable pass aims for when it splits planes into row
// segments.  Measured at 512 planes of 512×512 with 31 taps: whole-plane
// segments (512 work-groups) run the forward pass in 0.520 ms against 0.592 ms
// for 128-row segments (2048 work-groups), the split-view backward in 0.527
// against 0.563 ms.
constexpr long kSepTargetGroups = 512;

// Launch-shape overrides for tuning experiments, read once from the
// environment: MVD_TUNE="fwd_occ=4,bwd_occ=2,bwd_vin=1,zseg=64" (0 = automatic).
struct Tune {
  int fwd_occ = 0, bwd_occ = 0, bwd_vin = 0, zseg = 0, fwd_views = 0;
  int zseg_scale = 0;   // > 0: segment length × 2^(zseg_scale − 2) of the automatic one (2 = as is)
  int cols = 0;         // 1: one column per thread (strips with halo for rows wider than 512)
  int valu2d = 0;       // 1: general K×K passes on the vector ALUs instead of the matrix cores
  int threads = 0;      // > 0: at most this many threads per work-group (64-multiple ≤ 512;
                        // rows wider than it are split into strips with halos)
  int bwd_threads = 0;  // the same for two-view backward launches only
  int bwd_split = 0;    // two-view backward as one 1024-thread work-group per row segment (half
                        // the threads per view, 16-row groups): 0 where it applies, 2 never
  int valu_corr = 0;    // 1: tap-gradient correlation on the vector ALUs instead of the matrix cores
  int plane_batch = 0;  // > 0: run this many planes through all iterations at a time
  int pq_window = 0;    // persistent batches: planes per window of a volume's items (0: all)
  int pq_zseg_scale = 0;  // persistent batches: segment length × 2^(v − 2) of the planner's (0: × 2)
  int terms = 1;        // kernels of several rank-one terms: two terms per launch (0: one)
  int fused = 0;        // simultaneous two-view runs: one fused launch per iteration where it applies
                        // (a candidate of the tuner, which keeps it where it is faster)
  int wide = 0;         // rows of 513–1024 columns as one column per thread in up to
                        // 1024-thread work-groups (one-ring passes): 0 where it applies, 2 never
};

Tune parse_tune(const char *e) {
  Tune r;
  if (!e) return r;
  const std::string s(e);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t comma = s.find(',', pos);
    if (comma == std::string::npos) comma = s.size();
    const std::string kv = s.substr(pos, comma - pos);
    const size_t eq = kv.find('=');
    if (eq != std::string::npos) {
      const std::string k = kv.substr(0, eq);
      const int v = std::atoi(kv.c_str() + eq + 1);
      if (k == "fwd_occ") r.fwd_occ = v;
      if (k == "bwd_occ") r.bwd_occ = v;
      if (k == "bwd_vin") r.bwd_vin = v;
      if (k == "zseg") r.zseg = v;
      if (k == "fwd_views") r.fwd_views = v;
      if (k == "zseg_scale") r.zseg_scale = v;
      if (k == "cols") r.cols = v;
      if (k == "valu2d") r.valu2d = v;
      if (k == "valu_corr") r.valu_corr = v;
      if (k == "threads") r.threads = v;
      if (k == "bwd_threads") r.bwd_threads = v;
      if (k == "bwd_split") r.bwd_split = v;
      if (k == "plane_batch") r.plane_batch = v;
      if (k == "wide") r.wide = v;
      if (k == "pq_window") r.pq_window = v;
      if (k == "pq_zseg_scale") r.pq_zseg_scale = v;
      if (k == "fused") r.fused = v;
      if (k == "terms") r.terms = v;
    }
    pos = comma + 1;
  }
  return r;
}

Tune &tune_mut() {
  static Tune t = parse_tune(std::getenv("MVD_TUNE"));
  return t;
}

const Tune &tune() { return tune_mut(); }

// Whole rows (no x halo) under the zero boundary; strips with an x halo of R
// columns otherwise.  Periodic runs always take strips: their halo columns are
// read wrapped, so no pass has to copy wrapped values into LDS pad columns.
SepGeom plan_sep(const mvd_ctx *c, int Y, int kb, int boundary, const Tune &tn = tune(), bool one_ring = false) {
  SepGeom s{};
  const int R = (kb - 1) / 2;
  const int X = c->X;
  s.plan.bucket = kb;
  const bool wide_ok = kb <= 41;   // two columns per thread keep the ring in registers
  int maxt = (tn.threads >= 64 && tn.threads <= kSepMaxThreads) ? tn.threads / 64 * 64 : kSepMaxThreads;
  maxt = std::max(maxt, std::min(kSepMaxThreads, round_up(2 * R + 64, 64)));   // a strip keeps ≥ 64 outputs
  const int max_cols = (wide_ok ? 2 : 1) * maxt;
  const bool whole = boundary == MVD_BOUNDARY_ZERO;
  const bool one_col = tn.cols == 1 || !wide_ok || maxt < kSepMaxThreads;
  // whole rows of up to 2·kSepMaxThreads columns, one column per thread: only
  // the one-ring kernels with the 128-VGPR budget accept such work-groups
  const bool wide_rows = one_ring && tn.wide != 2 && whole && wide_ok && tn.threads == 0 && tn.cols == 0 &&
                         X > maxt && X <= 2 * kSepMaxThreads;
  if (wide_rows) maxt = round_up(X, 64);
  if (whole && X <= maxt) {
    s.plan.cols = 1;
    s.nstrip = 1;
    s.x_out = X;
    s.halo = 0;
    s.ncols = X;
  } else if (whole && !one_col && X <= max_cols) {
    s.plan.cols = 2;
    s.nstrip = 1;
    s.x_out = X;
    s.halo = 0;
    s.ncols = X;
  } else {
    s.plan.cols = (X + 2 * R <= maxt || one_col) ? 1 : 2;
    // outputs per strip: the threads' columns minus the halo, rounded down to
    // whole 8-column items so that rounding the strip width up cannot exceed it
    const int per = (s.plan.cols * maxt - 2 * R) / 8 * 8;
    s.nstrip = (X + per - 1) / per;
    s.x_out = round_up((X + s.nstrip - 1) / s.nstrip, 8);
    s.nstrip = (X + s.x_out - 1) / s.x_out;
    s.halo = R;
    s.ncols = s.x_out + 2 * R;
  }
  s.plan.threads = std::min(maxt, round_up((s.ncols + s.plan.cols - 1) / s.plan.cols, 64));
  const int nxb = (s.x_out + 7) / 8;
  // row pitch ≡ 4 (mod 8) floats: the row pass reads pairs of rows whose
  // 16-byte chunks then fall in complementary LDS bank groups
  s.ldsw = round_up(nxb * 8 + kb - 1 + 4, 4);
  if (s.ldsw % 8 == 0) s.ldsw += 4;
  // segments: long ones (each segment refills its ring of K − 1 rows and reads
  // them again from its neighbour), as few as give about 512 work-groups —
  // one or two per CU; segments ≥ 32 rows
  const int Z = c->Z;
  const long tiles = (long)Y * s.nstrip;
  int nseg = (int)std::max(1L, (kSepTargetGroups + tiles - 1) / tiles);
  nseg = std::min(nseg, std::max(1, Z / 32));
  s.zseg = round_up((Z + nseg - 1) / nseg, kRowGroup);
  if (tn.zseg_scale > 0 && tn.zseg_scale != 2) {
    const double f = std::ldexp(1.0, tn.zseg_scale - 2);
    const int want = (int)std::lround(s.zseg * f);
    s.zseg = round_up(std::max(kRowGroup, std::min(round_up(Z, kRowGroup), want)), kRowGroup);
  }
  if (tn.zseg > 0) s.zseg = round_up(tn.zseg, kRowGroup);
  s.nseg = (Z + s.zseg - 1) / s.zseg;
  // one column per thread keeps a K ≤ 41 ring within 128 VGPRs: 4 waves/SIMD
  s.plan.occ = (s.plan.cols == 1 && kb <= 41) ? 4 : 2;
  s.plan.vin = 1;
  return s;
}

// LDS of one view in a separable pass: double-buffered column-pass rows and the
// two passes' [4][NK] tap tables (NK = bucket + 3 rounded up to 4).
size_t sep_lds_per_view(const SepGeom &sg) {
  return sizeof(float) * (2ull * kRowGroup * sg.ldsw + 8ull * ((sg.plan.bucket + 3 + 3) / 4 * 4));
}

// Split-view backward: two views' double-buffered 16-row groups and tap tables.
constexpr int kSplitRows = 16;
size_t split_lds_bytes(const SepGeom &sg) {
  return sizeof(float) * (2ull * 2 * kSplitRows * sg.ldsw + 2ull * 8 * ((sg.plan.bucket + 3 + 3) / 4 * 4));
}

// Geometry of the split-view form from a one-column plan (whole rows, or strips
// with halo columns), or false where it does not apply (several columns per
// thread, > 31 taps, periodic, LDS).
bool split_geom(const SepGeom &sg, PlaneGeom g, int boundary, SepGeom *out) {
  if (sg.plan.cols != 1 || sg.plan.bucket > 31 || boundary != MVD_BOUNDARY_ZERO ||
      sg.plan.threads > kSepMaxThreads || sg.ncols > sg.plan.threads)
    return false;
  SepGeom sp = sg;
  sp.zseg = round_up(sg.zseg, kSplitRows);
  sp.nseg = (g.Z + sp.zseg - 1) / sp.zseg;
  sp.plan.threads = 2 * sg.plan.threads;
  sp.plan.occ = 4;
  sp.plan.vin = 2;
  if (split_lds_bytes(sp) > kLdsLimit) return false;
  *out = sp;
  return true;
}

void fill_sep_common(SepPassArgs &a, const SepGeom &s, PlaneGeom g, int boundary) {
  a.g = g;
  a.boundary = boundary;
  a.zseg = s.zseg;
  a.nseg = s.nseg;
  a.x_out = s.x_out;
  a.nstrip = s.nstrip;
  a.halo = s.halo;
  a.ncols = s.ncols;
  a.ldsw = s.ldsw;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// The row pass moves 8 outputs per item with 128-bit loads and stores only when
// every item is whole: rows and strips are multiples of 8 columns.
bool whole_items(const SepGeom &sg, PlaneGeom g) { return g.X % 8 == 0 && sg.x_out % 8 == 0; }

// centred zero-padding of a 1D factor into kb taps
void put_factor(float *dst, const std::vector<float> &f, int kb) {
  for (int i = 0; i < kb; ++i) dst[i] = 0.f;
  const int off = (kb - (int)f.size()) / 2;
  for (size_t i = 0; i < f.size(); ++i) dst[off + i] = f[i];
}

struct RunState {
  mvd_ctx *c;
  PlaneGeom g;
  int boundary;
  bool force2d;
  hipStream_t s;
  const float *w;  // host weights or nullptr
  bool timing;
  const Tune *tn = &tune();   // launch-shape choices (environment or autotuner)
  bool normalize = false;     // divide back-projections by 1 ⊛ X_v (MVD_FLAG_NORMALIZE)
  const float *const *wpl = nullptr;   // per-pixel weight planes of the whole volume, or null
  size_t wpl_off = 0;                  // elements from their start to this launch's first plane
  float *acc = nullptr;                // partial sums of low-rank kernels' terms (a plane set), or null
  float *sens = nullptr;               // two [Z][X] planes: ones, then a sensitivity 1 ⊛ X_v (general update)
};

hipEvent_t take_event(mvd_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` between two events when timing is on.
template <typename F>
hipError_t timed(const RunState &st, int kind, F &&launch) {
  if (!st.timing) return launch();
  mvd_ctx *c = st.c;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st.s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st.s);
  c->marks.push_back({kind, a, b});
  return e;
}

float weight_of(const RunState &st, int v) { return st.w ? st.w[v] : 1.f; }

// Device taps of view v for the K×K passes: which = 0 convolves with P_v,
// 1 with X_v, 2 with P_v^*, 3 with X_v^* (the point reflections).
const float *dtaps(const mvd_ctx *c, int v, int which) {
  return c->d_taps + ((size_t)v * kTapSets + which) * c->kzm * c->kxpm;
}

// Forward pass over views [v0, v0+n): r[v] = φ_v / (psi ⊛ P_v)
// Observations as the forward pass reads them: the arrays as given (float32 or
// uint16, plane or stack layout, read through strides) for the separable
// passes; float32 planes staged in the workspace for the general passes
// (null where no view needs them).
struct ObsRef {
  const void *const *p;
  bool u16;
  long sy, sz;
  const float *const *staged;
};

ObsRef obs_given(const void *const *obs, int dtype, int layout, const PlaneGeom &g, const float *const *staged) {
  ObsRef o{obs, dtype == MVD_U16, 0, 0, staged};
  if (layout == MVD_STACK_ZYX) {
    o.sy = g.X;
    o.sz = (long)g.Y * g.X;
  } else {
    o.sy = (long)g.Z * g.X;
    o.sz = g.X;
  }
  return o;
}

ObsRef obs_staged(const float *const *staged, const PlaneGeom &g) {
  return ObsRef{reinterpret_cast<const void *const *>(staged), false, (long)g.Z * g.X, g.X, staged};
}

// The forward passes of a run take the general K×K form for some view.
bool run_needs_2d(const RunState &st) {
  if (st.force2d) return true;
  for (int v = 0; v < st.c->nv; ++v)
    if (!st.c->views[v].sep_p) return true;
  return false;
}

hipError_t lowrank_forward(const RunState &st, const float *psi, const float *phi, float *rv, int v);
hipError_t lowrank_backward(const RunState &st, const float *rv, const float *psi_in, float *psi_out, int v);

hipError_t forward_views(const RunState &st, const float *psi, const ObsRef &ob, float *const *r, int v0, int n) {
  mvd_ctx *c = st.c;
  bool sep = !st.force2d;
  int kmax = 1;
  for (int v = v0; v < v0 + n; ++v) {
    sep = sep && c->views[v].sep_p;
    kmax = std::max({kmax, c->views[v].psf.kz, c->views[v].psf.kx});
  }
  // PSFs of low rank: view by view, each as a sum of rank-one terms (the
  // others of the range in their own launches)
  if (!sep && !st.force2d && st.acc) {
    bool lr = false;
    for (int v = v0; v < v0 + n; ++v) lr = lr || (!c->views[v].sep_p && !c->views[v].lpz.empty());
    if (lr) {
      if (n == 1) return lowrank_forward(st, psi, ob.staged ? ob.staged[v0] : nullptr, r[v0], v0);
      for (int v = v0; v < v0 + n; ++v) {
        hipError_t e = forward_views(st, psi, ob, r, v, 1);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
  }
  if (sep) {
    SepGeom sg = plan_sep(c, st.g.Y, sep_bucket(kmax), st.boundary, *st.tn, true);
    // (work-groups beyond kSepMaxThreads exist only in the 128-VGPR form)
    if (st.tn->fwd_occ && sg.plan.threads <= kSepMaxThreads) sg.plan.occ = st.tn->fwd_occ;
    const size_t per_view = sep_lds_per_view(sg);
    int cap = (int)std::max<size_t>(1, std::min<size_t>(kSepFwdViews, kLdsLimit / per_view));
    if (st.tn->fwd_views > 0) cap = std::min(cap, st.tn->fwd_views);
    for (int b = v0; b < v0 + n; b += cap) {
      const int nb = std::min(cap, v0 + n - b);
      SepPassArgs a{};
      fill_sep_common(a, sg, st.g, st.boundary);
      a.nviews = nb;
      a.in[0] = psi;
      a.obs_u16 = ob.u16 ? 1 : 0;
      a.obs_sy = ob.sy;
      a.obs_sz = ob.sz;
      for (int k = 0; k < nb; ++k) {
        const ViewPsf &w = c->views[b + k];
        a.obs[k] = ob.p[b + k];
        a.out[k] = r[b + k];
        put_factor(a.tz[k], w.pz, sg.plan.bucket);
        put_factor(a.tx[k], w.px, sg.plan.bucket);
      }
      const long unit = ob.u16 ? 8 : 4;   // elements per 16 bytes
      a.vec = whole_items(sg, st.g) && aligned16(psi) && ob.sy % unit == 0 && ob.sz % unit == 0;
      for (int k = 0; k < nb; ++k) a.vec = a.vec && aligned16(a.obs[k]) && aligned16(a.out[k]);
      hipError_t e = timed(st, 0, [&] { return launch_sep_forward(a, sg.plan, st.s); });
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (int b = v0; b < v0 + n; b += k2dViews) {
    const int nb = std::min(k2dViews, v0 + n - b);
    TwoDPassArgs a{};
    a.g = st.g;
    a.boundary = st.boundary;
    a.nviews = nb;
    a.kz = c->kzm;
    a.kx = c->kxm;
    a.in[0] = psi;
    a.mfma = st.tn->valu2d ? 0 : 1;
    if (!ob.staged) return hipErrorInvalidValue;
    for (int k = 0; k < nb; ++k) {
      a.phi[k] = ob.staged[b + k];
      a.out[k] = r[b + k];
      a.taps[k] = dtaps(c, b + k, 0);
    }
    hipError_t e = timed(st, 0, [&] { return launch_2d_forward(a, st.s); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Backward pass over views [v0, v0+n): psi_out = psi_in · Π (w q + 1 − w)
hipError_t backward_general(const RunState &st, const float *const *r, const float *psi_in, float *psi_out,
                            int v0, int n);

hipError_t backward_views(const RunState &st, const float *const *r, const float *psi_in, float *psi_out,
                          int v0, int n) {
  mvd_ctx *c = st.c;
  if (st.wpl || st.normalize) {   // weights per pixel or normalisation: rank-one passes, else the general update
    bool general = st.force2d;
    for (int v = v0; v < v0 + n; ++v) general = general || !c->views[v].sep_x;
    if (general) return backward_general(st, r, psi_in, psi_out, v0, n);
  }
  bool sep = !st.force2d;
  int kmax = 1;
  for (int v = v0; v < v0 + n; ++v) {
    sep = sep && c->views[v].sep_x;
    kmax = std::max({kmax, c->views[v].back.kz, c->views[v].back.kx});
  }
  // back-projectors of low rank: view by view in view order (ψ · c_0 · c_1 …)
  if (!sep && !st.force2d && st.acc) {
    bool lr = false;
    for (int v = v0; v < v0 + n; ++v) lr = lr || (!c->views[v].sep_x && !c->views[v].lxz.empty());
    if (lr) {
      if (n == 1) return lowrank_backward(st, r[v0], psi_in, psi_out, v0);
      const float *in = psi_in;
      for (int v = v0; v < v0 + n; ++v) {
        hipError_t e = backward_views(st, r, in, psi_out, v, 1);
        if (e != hipSuccess) return e;
        in = psi_out;
      }
      return hipSuccess;
    }
  }
  const float *cur = psi_in;
  if (sep) {
    SepGeom sg = plan_sep(c, st.g.Y, sep_bucket(kmax), st.boundary, *st.tn);
    const size_t per_view = sep_lds_per_view(sg);
    // Two ratio planes per launch save one read and write of ψ (16 instead of
    // 24 B per voxel for two views) but need two rings (256-VGPR budget, 2
    // waves/SIMD).  With the column pass on the matrix cores the vector ALUs
    // only run the row pass, and the saved traffic wins (vol512: 0.653 ms for
    // both views against 2 × 0.341); the tuner still tries one per launch.
    // Where rows are ≤ 512 wide the split-view form holds one ring per thread
    // in a 1024-thread work-group instead (4 waves/SIMD, 0.616 ms at vol512).
    const bool can_two = n >= 2 && sg.plan.cols == 1 && sg.plan.bucket <= 41 && 2 * per_view <= kLdsLimit;
    bool two = can_two;
    if (st.tn->bwd_vin == 1) two = false;
    if (two && st.tn->bwd_threads > 0) {   // narrower work-groups: more of them per CU
      Tune nt = *st.tn;
      nt.threads = st.tn->bwd_threads;
      sg = plan_sep(c, st.g.Y, sep_bucket(kmax), st.boundary, nt);
    }
    if (!two) {   // one ring per thread: rows up to 1024 wide may take 1024-thread work-groups
      const SepGeom w = plan_sep(c, st.g.Y, sep_bucket(kmax), st.boundary, *st.tn, true);
      if (w.plan.threads > kSepMaxThreads) sg = w;
    }
    sg.plan.vin = two ? 2 : 1;
    if (two) sg.plan.occ = 2;   // two rings: 256-VGPR budget
    if (st.tn->bwd_occ && sg.plan.threads <= kSepMaxThreads) sg.plan.occ = st.tn->bwd_occ;
    // split-view form (two planes per launch in one 1024-thread work-group):
    // rows of ≤ 512 columns, or strips of one ring column per thread, zero
    // boundary, ≤ 31 taps, 128-bit accesses.  Where the pass's own plan takes
    // two columns per thread (rows wider than 512), the split form plans its
    // own one-column strips.
    // (not with the EM normalisation: the split form has no registers left for it)
    SepGeom sp = sg;
    bool split = false;
    if (n >= 2 && !st.normalize && !st.wpl && st.tn->bwd_split != 2 && st.tn->bwd_vin != 1 &&
        (two || sg.plan.cols != 1)) {
      SepGeom base = sg;
      if (!two) {
        Tune t1 = *st.tn;
        t1.cols = 1;
        base = plan_sep(c, st.g.Y, sep_bucket(kmax), st.boundary, t1);
      }
      bool al = aligned16(cur) && aligned16(psi_out);
      for (int v = v0; v < v0 + n; ++v) al = al && aligned16(r[v]);
      split = al && split_geom(base, st.g, st.boundary, &sp) && whole_items(sp, st.g);
    }
    if (split) sg.plan.vin = 2;
    for (int b = v0; b < v0 + n; b += sg.plan.vin) {
      const int nb = std::min(sg.plan.vin, v0 + n - b);
      const bool use_split = split && nb == 2;
      const SepGeom &gm = use_split ? sp : sg;
      SepPlan plan = gm.plan;
      plan.vin = nb;
      SepPassArgs a{};
      fill_sep_common(a, gm, st.g, st.boundary);
      a.nviews = nb;
      for (int k = 0; k < nb; ++k) {
        const ViewPsf &w = c->views[b + k];
        a.in[k] = r[b + k];
        a.w[k] = weight_of(st, b + k);
        put_factor(a.tz[k], w.xz, plan.bucket);
        put_factor(a.tx[k], w.xx, plan.bucket);
        if (st.normalize) {
          a.nsz[k] = norm_factors(c, b + k, st.boundary);
          a.nsx[k] = a.nsz[k] + norm_zlen(c);
        }
        if (st.wpl) a.wpl[k] = st.wpl[b + k] + st.wpl_off;
      }
      a.psi_in = cur;
      a.psi_out = psi_out;
      a.vec = whole_items(gm, st.g) && aligned16(cur) && aligned16(psi_out);
      for (int k = 0; k < nb; ++k) a.vec = a.vec && aligned16(a.in[k]) && (!a.wpl[k] || aligned16(a.wpl[k]));
      hipError_t e = timed(st, 1, [&] {
        return use_split ? launch_sep_backward_split(a, plan, st.s) : launch_sep_backward(a, plan, st.s);
      });
      if (e != hipSuccess) return e;
      cur = psi_out;
    }
    return hipSuccess;
  }
  for (int b = v0; b < v0 + n; b += k2dViews) {
    const int nb = std::min(k2dViews, v0 + n - b);
    TwoDPassArgs a{};
    a.g = st.g;
    a.boundary = st.boundary;
    a.nviews = nb;
    a.kz = c->kzm;
    a.kx = c->kxm;
    a.mfma = st.tn->valu2d ? 0 : 1;
    for (int k = 0; k < nb; ++k) {
      a.in[k] = r[b + k];
      a.w[k] = weight_of(st, b + k);
      a.taps[k] = dtaps(c, b + k, 1);
    }
    a.psi_in = cur;
    a.psi_out = psi_out;
    hipError_t e = timed(st, 1, [&] { return launch_2d_backward(a, st.s); });
    if (e != hipSuccess) return e;
    cur = psi_out;
  }
  return hipSuccess;
}


// ---- reverse sweep (adjoint) ----------------------------------------------
constexpr int kPointBlocks = 1024;
constexpr int kCorrBlocks = 4096;      // vector form: work-groups (partials) at most
constexpr int kCorrMfmaBlocks = 1024;  // matrix-core form

struct BwdLayout {
  size_t plane_set = 0;
  size_t phi_off = 0, b_off = 0, r_off = 0, q_off = 0, g_off = 0, sub_off = 0, rat_off = 0;
  size_t wpart_off = 0, cpart_off = 0, acc_off = 0, total = 0;
  size_t tmp_off = 0;   // a plane set for convolutions finished pointwise (kernels not rank one), else none
  size_t sbar_off = 0, ones_off = 0;   // normalised runs: s̄ per view (or one), a plane set of ones
  size_t sens_off = 0;   // normalised runs with a back-projector not rank one: two scratch [Z][X] planes,
                         // then one sensitivity plane 1 ⊛ X_v per view
  int nsets = 0, nsub = 0;
  bool low_rank = false;   // some view's PSF or back-projector is not rank one
  bool normalize = false;
  bool sens = false;
};

// accumulators: per view [psf kz·kx][back kz·kx], then V weights (doubles)
size_t acc_psf(const mvd_ctx *c, int v) { return (size_t)v * 2 * kMaxK * kMaxK; }
size_t acc_back(const mvd_ctx *c, int v) { return acc_psf(c, v) + kMaxK * kMaxK; }
size_t acc_w(const mvd_ctx *c) { return (size_t)c->nv * 2 * kMaxK * kMaxK; }

BwdLayout bwd_layout_of(const mvd_ctx *c, const mvd_run *r) {
  BwdLayout L;
  const int V = c->nv;
  const bool sim = r->update == MVD_UPDATE_SIMULTANEOUS;
  L.plane_set = align_up((size_t)r->n_planes * c->Z * c->X * sizeof(float));
  L.nsets = sim ? V : 1;
  L.nsub = sim ? 0 : V - 1;
  size_t off = 0;
  L.phi_off = off;
  off += (size_t)V * L.plane_set;   // staged observations
  L.b_off = off;
  off += (size_t)L.nsets * L.plane_set;
  L.r_off = off;
  off += (size_t)L.nsets * L.plane_set;
  L.q_off = off;
  off += (size_t)L.nsets * L.plane_set;
  L.g_off = off;
  off += 2 * L.plane_set;
  L.sub_off = off;
  off += (size_t)L.nsub * L.plane_set;
  L.rat_off = off;
  if (!sim) off += L.plane_set;
  for (const ViewPsf &w : c->views) L.low_rank = L.low_rank || !w.sep_p || !w.sep_x;
  L.tmp_off = off;
  if (L.low_rank) off += L.plane_set;
  L.normalize = (r->flags & MVD_FLAG_NORMALIZE) != 0;
  L.sbar_off = off;
  if (L.normalize) off += (size_t)L.nsets * L.plane_set;
  L.ones_off = off;
  if (L.normalize) off += L.plane_set;
  L.sens = false;
  for (const ViewPsf &w : c->views) L.sens = L.sens || (L.normalize && !w.sep_x);
  L.sens_off = off;
  if (L.sens) off += (size_t)(2 + V) * sens_plane_bytes(c);
  size_t lags = 0;   // padded lags of a partial, either form
  for (auto &w : c->views)
    for (const Kernel *d : {&w.psf, &w.back})
      lags = std::max({lags, (size_t)corr_pad(d->kz, 4) * corr_pad(d->kx, 8),
                       (size_t)corr_mfma_pad(d->kz) * corr_mfma_pad(d->kx)});
  L.wpart_off = off;
  off += align_up(sizeof(double) * kPointBlocks * V);
  L.cpart_off = off;
  off += align_up(sizeof(float) * (size_t)kCorrBlocks * lags);
  L.acc_off = off;
  off += align_up(sizeof(double) * (acc_w(c) + V));
  L.total = off;
  return L;
}

std::vector<float> reversed(const std::vector<float> &f) { return std::vector<float>(f.rbegin(), f.rend()); }

// One view's single-input separable pass with epilogue `ep`.
hipError_t single_pass(const RunState &st, int ep, const float *in, const std::vector<float> &fz,
                       const std::vector<float> &fx, float *out, float *out2, const float *aux0,
                       const float *aux1, const float *phi, float w = 1.f, int kind = 3) {
  const int k = std::max((int)fz.size(), (int)fx.size());
  SepGeom sg = plan_sep(st.c, st.g.Y, sep_bucket(k), st.boundary, *st.tn);
  sg.plan.occ = (sg.plan.cols == 1 && sg.plan.bucket <= 31) ? 4 : 2;
  SepPassArgs a{};
  fill_sep_common(a, sg, st.g, st.boundary);
  a.nviews = 1;
  a.in[0] = in;
  a.out[0] = out;
  a.out2[0] = out2;
  a.aux0[0] = aux0;
  a.aux1[0] = aux1;
  a.phi[0] = phi;
  a.w[0] = w;
  put_factor(a.tz[0], fz, sg.plan.bucket);
  put_factor(a.tx[0], fx, sg.plan.bucket);
  a.vec = whole_items(sg, st.g) && aligned16(in) && aligned16(out);
  for (const void *p : {(const void *)out2, (const void *)aux0, (const void *)aux1, (const void *)phi})
    if (p) a.vec = a.vec && aligned16(p);
  return timed(st, kind, [&] { return launch_sep_single_dispatch(a, sg.plan, ep, st.s); });
}

// Geometry of a pass over two terms of one kernel (one input ring, both terms'
// column and row passes, their sum finishing one output): one column per
// thread and whole 16-byte items, or false (then one term per launch).
bool terms_geom(const RunState &st, int k, SepGeom *out) {
  if (st.tn->terms == 0) return false;
  SepGeom sg = plan_sep(st.c, st.g.Y, sep_bucket(k), st.boundary, *st.tn);
  sg.plan.occ = (sg.plan.cols == 1 && sg.plan.bucket <= 41) ? 4 : 2;
  if (sg.plan.cols != 1 || !whole_items(sg, st.g)) return false;
  if (sg.plan.threads > (sg.plan.occ >= 4 ? 2 * kSepMaxThreads : kSepMaxThreads)) return false;
  if (sizeof(float) * (2ull * 2 * kRowGroup * sg.ldsw + 2ull * 8 * ((sg.plan.bucket + 3 + 3) / 4 * 4)) > kLdsLimit)
    return false;
  *out = sg;
  return true;
}

// Terms t and t + 1 of a kernel in one launch with epilogue `ep` (kEpTermsSum,
// kEpTermsRatio, kEpTermsUpdate): out = finish([aux0 +] conv_t + conv_{t+1}).
hipError_t terms_pass(const RunState &st, const SepGeom &sg, int ep, const float *in,
                      const std::vector<float> *fz, const std::vector<float> *fx, float *out, const float *aux0,
                      const float *aux1, float w, int kind) {
  SepPassArgs a{};
  fill_sep_common(a, sg, st.g, st.boundary);
  a.nviews = 2;
  a.in[0] = in;
  a.out[0] = out;
  a.aux0[0] = aux0;
  a.aux1[0] = aux1;
  a.w[0] = w;
  for (int u = 0; u < 2; ++u) {
    put_factor(a.tz[u], fz[u], sg.plan.bucket);
    put_factor(a.tx[u], fx[u], sg.plan.bucket);
  }
  a.vec = 1;
  return timed(st, kind, [&] { return launch_sep_single_dispatch(a, sg.plan, ep, st.s); });
}

// The terms of one low-rank kernel two per launch, in term order, through the
// partial-sum planes; a last odd term runs alone with `ep_single`.  Returns
// hipErrorNotSupported (before any launch) where the paired form does not apply.
hipError_t lowrank_pairs(const RunState &st, const std::vector<std::vector<float>> &zs,
                         const std::vector<std::vector<float>> &xs, const float *in, float *out, const float *last_op,
                         float w, bool forward) {
  const int R = (int)zs.size();
  int k = 1;
  for (int t = 0; t < R; ++t) k = std::max({k, (int)zs[t].size(), (int)xs[t].size()});
  SepGeom sg;
  if (!terms_geom(st, k, &sg)) return hipErrorNotSupported;
  for (const void *p : {(const void *)in, (const void *)out, (const void *)last_op, (const void *)st.acc})
    if (!aligned16(p)) return hipErrorNotSupported;
  const int kind = forward ? 0 : 1;
  hipError_t e = hipSuccess;
  for (int t = 0; t < R && e == hipSuccess;) {
    const float *aux0 = t == 0 ? nullptr : st.acc;
    if (R - t >= 2) {
      const bool last = R - t == 2;
      const int ep = !last ? kEpTermsSum : (forward ? kEpTermsRatio : kEpTermsUpdate);
      const std::vector<float> fz[2] = {zs[t], zs[t + 1]}, fx[2] = {xs[t], xs[t + 1]};
      e = terms_pass(st, sg, ep, in, fz, fx, last ? out : st.acc, aux0, last ? last_op : nullptr, w, kind);
      t += 2;
    } else {
      e = single_pass(st, forward ? kEpAccumRatio : kEpAccumUpdate, in, zs[t], xs[t], out, nullptr, st.acc, last_op,
                      nullptr, w, kind);
      t += 1;
    }
  }
  return e;
}

// A forward pass of view v whose PSF is a sum of rank-one terms: b = Σ_t ψ ⊛
// (pz_t ⊗ px_t), two terms per launch (or term by term) into the partial-sum
// planes, the last launch finishing r_v = φ_v / b (φ_v from the staged float32
// planes).
hipError_t lowrank_forward(const RunState &st, const float *psi, const float *phi, float *rv, int v) {
  const ViewPsf &w = st.c->views[v];
  const int R = (int)w.lpz.size();
  if (R < 2 || !st.acc || !phi) return hipErrorInvalidValue;
  const hipError_t ep = lowrank_pairs(st, w.lpz, w.lpx, psi, rv, phi, 1.f, true);
  if (ep != hipErrorNotSupported) return ep;
  for (int t = 0; t < R; ++t) {
    const bool last = t == R - 1;
    const int ep = t == 0 ? kEpStore : (last ? kEpAccumRatio : kEpAccum);
    hipError_t e = single_pass(st, ep, psi, w.lpz[t], w.lpx[t], last ? rv : st.acc, nullptr, t > 0 ? st.acc : nullptr,
                               last ? phi : nullptr, nullptr, 1.f, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A backward pass of view v whose back-projector is a sum of rank-one terms:
// q = Σ_t r_v ⊛ (xz_t ⊗ xx_t), two terms per launch (or term by term), the last
// launch finishing ψ_out = ψ_in · (w q + 1 − w).
hipError_t lowrank_backward(const RunState &st, const float *rv, const float *psi_in, float *psi_out, int v) {
  const ViewPsf &w = st.c->views[v];
  const int R = (int)w.lxz.size();
  if (R < 2 || !st.acc) return hipErrorInvalidValue;
  const hipError_t ep = lowrank_pairs(st, w.lxz, w.lxx, rv, psi_out, psi_in, weight_of(st, v), false);
  if (ep != hipErrorNotSupported) return ep;
  for (int t = 0; t < R; ++t) {
    const bool last = t == R - 1;
    const int ep = t == 0 ? kEpStore : (last ? kEpAccumUpdate : kEpAccum);
    hipError_t e = single_pass(st, ep, rv, w.lxz[t], w.lxx[t], last ? psi_out : st.acc, nullptr,
                               t > 0 ? st.acc : nullptr, last ? psi_in : nullptr, nullptr, weight_of(st, v), 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t tap_corr(const RunState &st, const BwdLayout &L, char *ws, const float *gbar, const float *src,
                    int kz, int kx, double *acc) {
  CorrArgs a{};
  a.g = st.g;
  a.boundary = st.boundary;
  a.rz = (kz - 1) / 2;
  a.rx = (kx - 1) / 2;
  a.gbar = gbar;
  a.src = src;
  a.part = reinterpret_cast<float *>(ws + L.cpart_off);
  const bool mfma = !st.tn->valu_corr;
  int nb;
  if (mfma) {
    const CorrMfmaShape m = corr_mfma_shape(st.g, kz, kx, kCorrMfmaBlocks);
    a.kzp = m.kzp;
    a.kxp = m.kxp;
    a.tw = m.tw;
    a.zch = m.zch;
    nb = m.nblocks;
  } else {
    a.kzp = corr_pad(kz, 4);
    a.kxp = corr_pad(kx, 8);
    nb = (int)std::min<long>(kCorrBlocks, (long)st.g.Y * ((st.g.Z + 7) / 8) * ((st.g.X + 63) / 64));
  }
  hipError_t e = timed(st, 4, [&] { return mfma ? launch_corr_mfma(a, nb, st.s) : launch_corr(a, nb, st.s); });
  if (e == hipSuccess)
    e = timed(st, 4, [&] { return launch_corr_finalize(a.part, nb, a.kzp, a.kxp, kz, kx, acc, st.s); });
  return e;
}

// Reverse sweep through view v at estimate psi (b, r, q buffers given):
// gbar_in = ∂L/∂(ψ after the view's factor), gbar_out += the convolution term.
// The pointwise step is done by the caller (it differs between update orders).
struct ViewBufs {
  float *b, *r, *q;
};

// out = Σ_t in ⊛ (fz_t ⊗ fx_t), one term per launch (the first stores, the
// others add in place); `flip` runs every term point-reflected.
hipError_t terms_sum(const RunState &st, const std::vector<std::vector<float>> &fz,
                     const std::vector<std::vector<float>> &fx, const float *in, float *out, bool flip, int kind) {
  hipError_t e = hipSuccess;
  for (size_t t = 0; t < fz.size() && e == hipSuccess; ++t)
    e = single_pass(st, t == 0 ? kEpStore : kEpAccum, in, flip ? reversed(fz[t]) : fz[t],
                    flip ? reversed(fx[t]) : fx[t], out, nullptr, t == 0 ? nullptr : out, nullptr, nullptr, 1.f, kind);
  return e;
}

size_t plane_elems(const RunState &st) { return (size_t)st.g.Y * st.g.Z * st.g.X; }

// out = in ⊛ k on the K×K passes, the convolution itself stored (tap set
// `which` of view v: 0 P_v, 1 X_v, 2 P_v^*, 3 X_v^*).
hipError_t twod_store(const RunState &st, const float *in, int v, int which, float *out, int kind = 3) {
  TwoDPassArgs a{};
  a.g = st.g;
  a.boundary = st.boundary;
  a.nviews = 1;
  a.kz = st.c->kzm;
  a.kx = st.c->kxm;
  a.in[0] = in;
  a.phi[0] = nullptr;
  a.out[0] = out;
  a.taps[0] = dtaps(st.c, v, which);
  a.mfma = st.tn->valu2d ? 0 : 1;
  return timed(st, kind, [&] { return launch_2d_forward(a, st.s); });
}

// q = in ⊛ X_v stored: the rank-one pass, a sum of terms, or the K×K pass
// (forced K×K runs take the K×K pass for every view).
hipError_t back_store(const RunState &st, int v, const float *in, float *out, int kind) {
  const ViewPsf &w = st.c->views[v];
  if (!st.force2d && w.sep_x)
    return single_pass(st, kEpStore, in, w.xz, w.xx, out, nullptr, nullptr, nullptr, nullptr, 1.f, kind);
  if (!st.force2d && !w.lxz.empty()) return terms_sum(st, w.lxz, w.lxx, in, out, false, kind);
  return twod_store(st, in, v, 1, out, kind);
}

// s_v = 1 ⊛ X_v over one plane into out [Z][X] (the same pass as the data's,
// so the same boundary); `ones` is a [Z][X] scratch plane filled here.
hipError_t sens_plane(const RunState &st, int v, float *ones, float *out) {
  RunState one = st;
  one.g.Y = 1;
  hipError_t e = launch_fill(ones, (size_t)st.g.Z * st.g.X, 1.f, st.s);
  if (e == hipSuccess) e = back_store(one, v, ones, out, 2);
  return e;
}

// The backward pass over views [v0, v0+n) view by view: q_v stored (st.acc),
// then ψ_out = ψ_in · (o q'_v + 1 − o) pointwise (ψ · c_0 · c_1 …), with
// q'_v = q_v / s_v under the normalised form (s_v from sens_plane) and
// o = w_v · ω_v(pixel) with weight planes.
hipError_t backward_general(const RunState &st, const float *const *r, const float *psi_in, float *psi_out,
                            int v0, int n) {
  if (!st.acc || (st.normalize && !st.sens)) return hipErrorInvalidValue;
  const size_t zx = (size_t)st.g.Z * st.g.X;
  float *ones = st.sens, *sp = st.sens ? st.sens + sens_plane_bytes(st.c) / sizeof(float) : nullptr;
  const float *in = psi_in;
  for (int v = v0; v < v0 + n; ++v) {
    hipError_t e = back_store(st, v, r[v], st.acc, 1);
    if (e == hipSuccess && st.normalize) e = sens_plane(st, v, ones, sp);
    const float *wp = st.wpl ? st.wpl[v] + st.wpl_off : nullptr;
    if (e == hipSuccess)
      e = timed(st, 1, [&] {
        return launch_update_plane(in, psi_out, st.acc, st.normalize ? sp : nullptr, zx, wp, weight_of(st, v),
                                   plane_elems(st), st.s);
      });
    if (e != hipSuccess) return e;
    in = psi_out;
  }
  return hipSuccess;
}

// b = ψ ⊛ P_v with r = φ / b (guarded), then q = r ⊛ X_v.  Kernels of low
// rank are summed term by term, others run on the K×K passes, and both are
// finished pointwise.
hipError_t view_recompute(const RunState &st, int v, const float *psi, const float *phi, const ViewBufs &vb) {
  const ViewPsf &w = st.c->views[v];
  hipError_t e;
  if (w.sep_p) {
    e = single_pass(st, kEpBR, psi, w.pz, w.px, vb.b, vb.r, nullptr, nullptr, phi);
  } else {
    e = !w.lpz.empty() ? terms_sum(st, w.lpz, w.lpx, psi, vb.b, false, 3) : twod_store(st, psi, v, 0, vb.b);
    if (e == hipSuccess) e = timed(st, 3, [&] { return launch_ratio_plane(phi, vb.b, vb.r, plane_elems(st), st.s); });
  }
  if (e != hipSuccess) return e;
  if (w.sep_x) return single_pass(st, kEpStore, vb.r, w.xz, w.xx, vb.q, nullptr, nullptr, nullptr, nullptr);
  return !w.lxz.empty() ? terms_sum(st, w.lxz, w.lxx, vb.r, vb.q, false, 3) : twod_store(st, vb.r, v, 1, vb.q);
}

hipError_t view_backprop(const RunState &st, const BwdLayout &L, char *ws, int v, const float *psi,
                         const ViewBufs &vb, float *gbar_out, bool want_psf, bool want_back,
                         const float *sbar = nullptr) {
  mvd_ctx *c = st.c;
  const ViewPsf &w = c->views[v];
  double *acc = reinterpret_cast<double *>(ws + L.acc_off);
  hipError_t e = hipSuccess;
  if (want_back) e = tap_corr(st, L, ws, vb.q, vb.r, w.back.kz, w.back.kx, acc + acc_back(c, v));
  // normalised runs: s = 1 ⊛ X_v, so ∂L/∂X_v also gains s̄'s correlation with a plane of ones
  if (e == hipSuccess && want_back && sbar)
    e = tap_corr(st, L, ws, sbar, reinterpret_cast<const float *>(ws + L.ones_off), w.back.kz, w.back.kx,
                 acc + acc_back(c, v));
  // b̄ = −(q̄ ⊛ X^*) · r / b  (written over b; a sum of terms goes through st.acc)
  if (e == hipSuccess) {
    if (w.sep_x) {
      e = single_pass(st, kEpBbar, vb.q, reversed(w.xz), reversed(w.xx), vb.b, nullptr, vb.r, vb.b, nullptr);
    } else {
      e = !w.lxz.empty() ? terms_sum(st, w.lxz, w.lxx, vb.q, st.acc, true, 3) : twod_store(st, vb.q, v, 3, st.acc);
      if (e == hipSuccess)
        e = timed(st, 3, [&] { return launch_bbar_plane(st.acc, vb.r, vb.b, plane_elems(st), st.s); });
    }
  }
  if (e == hipSuccess && want_psf) e = tap_corr(st, L, ws, vb.b, psi, w.psf.kz, w.psf.kx, acc + acc_psf(c, v));
  // ψ̄ += b̄ ⊛ P^*  (term by term for a kernel of low rank)
  if (e == hipSuccess) {
    if (w.sep_p) {
      e = single_pass(st, kEpAccum, vb.b, reversed(w.pz), reversed(w.px), gbar_out, nullptr, gbar_out, nullptr,
                      nullptr);
    } else if (!w.lpz.empty()) {
      for (size_t t = 0; t < w.lpz.size() && e == hipSuccess; ++t)
        e = single_pass(st, kEpAccum, vb.b, reversed(w.lpz[t]), reversed(w.lpx[t]), gbar_out, nullptr, gbar_out,
                        nullptr, nullptr);
    } else {
      e = twod_store(st, vb.b, v, 2, st.acc);
      if (e == hipSuccess)
        e = timed(st, 3, [&] { return launch_add_plane(gbar_out, st.acc, plane_elems(st), st.s); });
    }
  }
  return e;
}


// ---- one run: validation and enqueue ----------------------------------------
mvd_status validate_run(mvd_ctx *c, const void *const *obs, const float *est, const mvd_run *r) {
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  if (!obs) return fail(c, MVD_ERR_ARG, "obs is NULL");
  for (int v = 0; v < c->nv; ++v)
    if (!obs[v]) return fail(c, MVD_ERR_ARG, "obs[%d] is NULL", v);
  if (!est) return fail(c, MVD_ERR_ARG, "est is NULL");
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  if ((r->flags & MVD_FLAG_GRAPH) && (r->flags & MVD_FLAG_TIMING))
    return fail(c, MVD_ERR_ARG, "MVD_FLAG_GRAPH and MVD_FLAG_TIMING exclude each other");
  const Layout L = layout_of(c, r);
  if (L.total > 0 && (!r->workspace || r->workspace_bytes < L.total))
    return fail(c, MVD_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                r->workspace ? r->workspace_bytes : (size_t)0);
  if (r->workspace && ((uintptr_t)r->workspace % kAlign))
    return fail(c, MVD_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  return MVD_OK;
}

// Planes per batch of the plane-blocked schedule (the whole volume: iteration-major).
int plane_batch(const mvd_run *r, const Tune &tn) {
  if (tn.plane_batch > 0) return std::min(tn.plane_batch, r->n_planes);
  return r->n_planes;
}

// Enqueue ψ^0 and every iteration of a validated run on `s`.  Planes are
// independent, so the run may go batch by batch of planes, each batch through
// all T iterations (a batch that fits the last-level cache keeps its working
// set there); the results do not depend on the batch size.
// ---- fused iterations --------------------------------------------------------
// LDS row pitch of the fused iteration's row-group buffers: the widest ring
// (the strip ± (RA + R), RA = R rounded up to whole 8-column items) plus the
// row pass's read-ahead, ≡ 4 (mod 8) floats.
int fused_pitch(int kb) {
  const int R = (kb - 1) / 2, RA = (R + 7) / 8 * 8;
  int pitch = round_up(kFusedStrip + 2 * RA + 2 * R + 4, 4);
  if (pitch % 8 == 0) pitch += 4;
  return pitch;
}

// One launch per iteration (k_fused.hip) for two views updated simultaneously
// under the zero boundary with rank-one PSFs and back-projectors of at most 31
// taps, no normalisation or weight planes, rows of whole 8-column items and
// 16-byte aligned planes and observations.  Returns the common bucket, or 0.
int fused_bucket_of(const RunState &st, const ObsRef &ob) {
  const mvd_ctx *c = st.c;
  if (st.tn->fused == 0 || c->nv != 2 || st.boundary != MVD_BOUNDARY_ZERO || st.force2d || st.normalize || st.wpl)
    return 0;
  if (st.g.X % 8 != 0) return 0;
  const long unit = ob.u16 ? 8 : 4;
  if (ob.sy % unit != 0 || ob.sz % unit != 0) return 0;
  int k = 1;
  for (int v = 0; v < 2; ++v) {
    const ViewPsf &w = c->views[v];
    if (!w.sep_p || !w.sep_x || !w.lpz.empty() || !w.lxz.empty()) return 0;
    k = std::max({k, (int)w.pz.size(), (int)w.px.size(), (int)w.xz.size(), (int)w.xx.size()});
    if (!aligned16(ob.p[v])) return 0;
  }
  const int kb = sep_bucket(k);
  if (kb < 0 || kb > 31) return 0;
  if (fused_lds_bytes(kb, fused_pitch(kb)) > kLdsLimit) return 0;
  return kb;
}

hipError_t fused_iteration(const RunState &st, const ObsRef &ob, int kb, const float *psi_in, float *psi_out) {
  const mvd_ctx *c = st.c;
  FusedArgs fa{};
  SepPassArgs &a = fa.f;
  const int R = (kb - 1) / 2;
  a.g = st.g;
  a.boundary = MVD_BOUNDARY_ZERO;
  a.nviews = 2;
  a.x_out = kFusedStrip;
  a.nstrip = (st.g.X + kFusedStrip - 1) / kFusedStrip;
  a.halo = R;
  a.ncols = kFusedStrip + 2 * R;
  a.ldsw = fused_pitch(kb);
  a.vec = 1;
  a.in[0] = psi_in;
  a.psi_in = psi_in;
  a.psi_out = psi_out;
  a.obs_u16 = ob.u16 ? 1 : 0;
  a.obs_sy = ob.sy;
  a.obs_sz = ob.sz;
  for (int v = 0; v < 2; ++v) {
    const ViewPsf &w = c->views[v];
    a.obs[v] = ob.p[v];
    a.w[v] = weight_of(st, v);
    put_factor(a.tz[v], w.pz, kb);
    put_factor(a.tx[v], w.px, kb);
    put_factor(fa.btz[v], w.xz, kb);
    put_factor(fa.btx[v], w.xx, kb);
  }
  return timed(st, 5, [&] { return launch_fused(fa, kb, st.s); });
}

hipError_t enqueue_run(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, hipStream_t s,
                       const Tune &tn, bool timing_override = false) {
  // a batch of B planes uses the first B planes of every workspace set
  const int B = plane_batch(r, tn);
  mvd_run rl = *r;
  rl.n_planes = B;
  const Layout L = layout_of(c, &rl);
  const PlaneGeom g{r->n_planes, c->Z, c->X};
  const size_t n = (size_t)g.Y * g.Z * g.X;
  char *ws = static_cast<char *>(r->workspace);
  RunState rs{c,  g, r->boundary, (r->flags & MVD_FLAG_FORCE_2D) != 0, s, r->view_weights,
              timing_override || (r->flags & MVD_FLAG_TIMING) != 0, &tn};
  rs.normalize = (r->flags & MVD_FLAG_NORMALIZE) != 0;
  rs.wpl = r->weight_planes;
  if (L.acc) rs.acc = reinterpret_cast<float *>(ws + L.acc_off);
  if (L.sens) rs.sens = reinterpret_cast<float *>(ws + L.sens_off);
  // the separable forward passes read the observations as given; only the
  // general K×K passes need them staged as float32 planes
  const bool need_staged = run_needs_2d(rs);
  std::vector<float *> staged(c->nv);
  for (int v = 0; v < c->nv; ++v) staged[v] = reinterpret_cast<float *>(ws + L.phi_off + (size_t)v * L.plane_set);
  std::vector<float *> rat(L.n_ratio);
  for (int k = 0; k < L.n_ratio; ++k) rat[k] = reinterpret_cast<float *>(ws + L.r_off + (size_t)k * L.plane_set);
  const ObsRef whole = obs_given(obs, r->obs_dtype, r->obs_layout, g, nullptr);
  const size_t esz = r->obs_dtype == MVD_U16 ? 2 : 4;
  const int T = r->n_iters;
  hipError_t e = hipSuccess;
  for (int y0 = 0; y0 < g.Y && e == hipSuccess; y0 += B) {
    const PlaneGeom gb{std::min(B, g.Y - y0), g.Z, g.X};
    const size_t nb = (size_t)gb.Y * g.Z * g.X, off = (size_t)y0 * g.Z * g.X;
    RunState rb = rs;
    rb.g = gb;
    rb.wpl_off = off;
    // this batch's observations: the same strides, starting at plane y0 (the
    // staged planes and ratio planes of a batch are the first planes of their sets)
    std::vector<const void *> ob_p(c->nv);
    for (int v = 0; v < c->nv; ++v) ob_p[v] = static_cast<const char *>(obs[v]) + (size_t)y0 * whole.sy * esz;
    const ObsRef ob{ob_p.data(), whole.u16, whole.sy, whole.sz, need_staged ? staged.data() : nullptr};
    float *est_b = est + off;
    auto slot = [&](int t) { return r->checkpoints + (size_t)t * n + off; };
    float *psi0 = (r->checkpoints && T > 0) ? slot(0) : est_b;
    // one pass over the observations: the staged planes where needed, and ψ^0 = their mean when asked
    float *mean = r->init == MVD_INIT_MEAN ? psi0 : nullptr;
    if (need_staged || mean)
      e = timed(rb, 2, [&] {
        return launch_stage_views(ob_p.data(), c->nv, r->obs_dtype, r->obs_layout, gb,
                                  need_staged ? staged.data() : nullptr, mean, s, g.Y);
      });
    if (e == hipSuccess && r->init == MVD_INIT_CONST)
      e = timed(rb, 2, [&] { return launch_fill(psi0, nb, r->init_const, s); });
    else if (e == hipSuccess && r->init == MVD_INIT_GIVEN && psi0 != est_b)
      e = timed(rb, 2, [&] { return launch_copy(est_b, psi0, nb, s); });
    // fused iterations: ψ^t and ψ^{t+1} in different plane sets where the
    // plane has several strips (a strip reads its neighbours' ψ columns): the
    // checkpoint slots, or the estimate and the first ratio plane set in turn
    // (after an odd count ψ^T is copied back to the estimate)
    const int kbf = r->update == MVD_UPDATE_SIMULTANEOUS && L.n_ratio > 0 && aligned16(est_b) &&
                            aligned16(rat[0]) && (!r->checkpoints || aligned16(r->checkpoints))
                        ? fused_bucket_of(rb, ob)
                        : 0;
    const bool pingpong = kbf && !r->checkpoints && g.X > kFusedStrip;
    for (int t = 0; t < T && e == hipSuccess; ++t) {
      float *cur = r->checkpoints ? slot(t) : est_b;
      float *nxt = r->checkpoints ? (t + 1 < T ? slot(t + 1) : est_b) : est_b;
      if (kbf) {
        if (pingpong) {
          cur = t % 2 ? rat[0] : est_b;
          nxt = t % 2 ? est_b : rat[0];
        }
        e = fused_iteration(rb, ob, kbf, cur, nxt);
        if (e == hipSuccess && pingpong && t == T - 1 && T % 2)
          e = timed(rb, 2, [&] { return launch_copy(rat[0], est_b, nb, s); });
      } else if (r->update == MVD_UPDATE_SIMULTANEOUS) {
        e = forward_views(rb, cur, ob, rat.data(), 0, c->nv);
        if (e == hipSuccess) e = backward_views(rb, rat.data(), cur, nxt, 0, c->nv);
      } else {
        for (int v = 0; v < c->nv && e == hipSuccess; ++v) {
          const float *src = v == 0 ? cur : nxt;
          std::vector<float *> rv(c->nv, rat[0]);
          e = forward_views(rb, src, ob, rv.data(), v, 1);
          if (e == hipSuccess) e = backward_views(rb, rv.data(), src, nxt, v, 1);
        }
      }
    }
  }
  return e;
}

hipError_t autotune(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, hipStream_t s, Tune *out);

// ---- streamed runs --------------------------------------------------------------
// Workspace of a streamed run: `slots` staging slots, each holding V observation
// batches [Z][ys][X] (and, for a host estimate, one float32 batch [ys][Z][X]),
// then the workspace of one batch run.
struct StreamLayout {
  int ys = 0, slots = 0;
  size_t obs_bytes = 0, est_bytes = 0, slot = 0, run_off = 0, run_bytes = 0, total = 0;
};

StreamLayout stream_layout_of(const mvd_ctx *c, const mvd_run *r, int batch, bool est_host) {
  StreamLayout S;
  S.ys = std::min(batch, r->n_planes);
  const size_t s = r->obs_dtype == MVD_U16 ? 2 : 4;
  const size_t vox = (size_t)S.ys * c->Z * c->X;
  S.obs_bytes = align_up(vox * s);
  S.est_bytes = est_host ? align_up(vox * sizeof(float)) : 0;
  S.slot = (size_t)c->nv * S.obs_bytes + S.est_bytes;
  S.slots = (r->n_planes + S.ys - 1) / S.ys > 1 ? 2 : 1;
  S.run_off = (size_t)S.slots * S.slot;
  mvd_run sub = *r;
  sub.n_planes = S.ys;
  S.run_bytes = align_up(layout_of(c, &sub).total);
  S.total = S.run_off + S.run_bytes;
  return S;
}

int memory_kind(const void *p);

mvd_status check_stream_run(mvd_ctx *c, const mvd_run *r, int batch) {
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  if (batch < 1) return fail(c, MVD_ERR_ARG, "batch_planes must be >= 1");
  if (r->obs_layout != MVD_STACK_ZYX) return fail(c, MVD_ERR_ARG, "streamed runs take camera-ordered stacks");
  if (r->checkpoints) return fail(c, MVD_ERR_ARG, "streamed runs keep no checkpoints");
  if (r->flags & MVD_FLAG_GRAPH) return fail(c, MVD_ERR_ARG, "MVD_FLAG_GRAPH is not available for streamed runs");
  return MVD_OK;
}

// Weight planes of a streamed or disk-to-disk run stay on the device (whole
// volume [Y][Z][X] per view; each batch reads its planes in place).
mvd_status check_stream_weights(mvd_ctx *c, const mvd_run *r) {
  if (!r->weight_planes) return MVD_OK;
  for (int v = 0; v < c->nv; ++v)
    if (memory_kind(r->weight_planes[v]) != 2)
      return fail(c, MVD_ERR_ARG, "weight_planes[%d] must be device memory in streamed runs", v);
  return MVD_OK;
}

// 0 pageable/unknown, 1 page-locked host, 2 device (or managed).
int memory_kind(const void *p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (a.type == hipMemoryTypeHost) return 1;
  if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return 2;
  return 0;
}

hipError_t stream_resources(mvd_ctx *c) {
  hipError_t e = hipSuccess;
  if (!c->h2d) e = hipStreamCreateWithFlags(&c->h2d, hipStreamNonBlocking);
  if (e == hipSuccess && !c->d2h) e = hipStreamCreateWithFlags(&c->d2h, hipStreamNonBlocking);
  for (auto &ev : c->sev)
    if (e == hipSuccess && !ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  return e;
}

// Batches b = 0, 1, … of ys planes alternate between two staging slots.
//   copy-in (h2d):  wait until slot's previous batch is computed (and copied
//                   out), copy V observation batches (and ψ^0), record in[k]
//   compute (s):    wait in[k] (and out[k] for a host estimate), run, record done[k]
//   copy-out (d2h): wait done[k], copy ψ^T of the batch to the host, record out[k]
// The streamed form feeds it batches of the caller's stacks; the disk-to-disk
// form feeds it page-locked batches read from files.
struct StreamPipe {
  mvd_ctx *c;
  const mvd_run *r;
  StreamLayout S;
  bool est_host;
  hipStream_t s;
  Tune tn;
  std::vector<const void *> slab;
  hipEvent_t start, *in, *done, *out;

  StreamPipe(mvd_ctx *c_, const mvd_run *r_, int batch, bool est_host_, hipStream_t s_)
      : c(c_), r(r_), S(stream_layout_of(c_, r_, batch, est_host_)), est_host(est_host_), s(s_), tn(tune()),
        slab(c_->nv), start(c_->sev[0]), in(c_->sev + 1), done(c_->sev + 3), out(c_->sev + 5) {}

  int batches() const { return (r->n_planes + S.ys - 1) / S.ys; }

  hipError_t begin() {
    hipError_t e = hipEventRecord(start, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->h2d, start, 0);
    if (e == hipSuccess && est_host) e = hipStreamWaitEvent(c->d2h, start, 0);
    return e;
  }

  // The run of one batch of ny planes from plane y0 (its weight planes, if
  // any, point into the whole volume's: `wb` holds the V pointers).
  mvd_run batch_run(int y0, int ny, std::vector<const float *> &wb) const {
    mvd_run sub = *r;
    sub.n_planes = ny;
    sub.flags &= ~MVD_FLAG_TUNE;
    sub.workspace = static_cast<char *>(r->workspace) + S.run_off;
    sub.workspace_bytes = S.run_bytes;
    if (r->weight_planes) {
      wb.assign(r->weight_planes, r->weight_planes + c->nv);
      for (const float *&p : wb) p += (size_t)y0 * c->Z * c->X;
      sub.weight_planes = wb.data();
    }
    return sub;
  }

  // Batch b: src[v] holds its rows as Z slices of ny·X elements, `pitch` bytes
  // apart; est_b_io is the batch's ψ (host for a host estimate, else device).
  hipError_t batch(int b, const void *const *src, size_t pitch, float *est_b_io) {
    const int Z = c->Z, X = c->X, y0 = b * S.ys, ny = std::min(S.ys, r->n_planes - y0), k = b % S.slots;
    const size_t es = r->obs_dtype == MVD_U16 ? 2 : 4;
    const size_t plane = (size_t)Z * X;
    char *slot = static_cast<char *>(r->workspace) + (size_t)k * S.slot;
    float *est_b = est_host ? reinterpret_cast<float *>(slot + (size_t)c->nv * S.obs_bytes) : est_b_io;
    hipError_t e = hipSuccess;
    if (b >= S.slots) {
      e = hipStreamWaitEvent(c->h2d, done[k], 0);
      if (e == hipSuccess && est_host) e = hipStreamWaitEvent(c->h2d, out[k], 0);
    }
    for (int v = 0; v < c->nv && e == hipSuccess; ++v) {
      char *dst = slot + (size_t)v * S.obs_bytes;
      // rows y0..y0+ny of every slice z: a 2D copy of Z rows of ny·X elements
      e = hipMemcpy2DAsync(dst, (size_t)ny * X * es, src[v], pitch, (size_t)ny * X * es, Z, hipMemcpyDefault,
                           c->h2d);
      slab[v] = dst;
    }
    if (e == hipSuccess && est_host && r->init == MVD_INIT_GIVEN)
      e = hipMemcpyAsync(est_b, est_b_io, (size_t)ny * plane * sizeof(float), hipMemcpyDefault, c->h2d);
    if (e == hipSuccess) e = hipEventRecord(in[k], c->h2d);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, in[k], 0);
    if (e == hipSuccess && est_host && b >= S.slots) e = hipStreamWaitEvent(s, out[k], 0);
    // launch shapes timed on the first batch (full-size batches share its shape)
    std::vector<const float *> wb;
    const mvd_run sub = batch_run(y0, ny, wb);
    if (e == hipSuccess && b == 0 && (r->flags & MVD_FLAG_TUNE) && r->init != MVD_INIT_GIVEN)
      e = autotune(c, slab.data(), est_b, &sub, s, &tn);
    if (e == hipSuccess) e = enqueue_run(c, slab.data(), est_b, &sub, s, tn);
    if (e == hipSuccess) e = hipEventRecord(done[k], s);
    if (e == hipSuccess && est_host) {
      e = hipStreamWaitEvent(c->d2h, done[k], 0);
      if (e == hipSuccess)
        e = hipMemcpyAsync(est_b_io, est_b, (size_t)ny * plane * sizeof(float), hipMemcpyDefault, c->d2h);
      if (e == hipSuccess) e = hipEventRecord(out[k], c->d2h);
    }
    return e;
  }

  // `s` completes only after the last copies
  hipError_t end() {
    hipError_t e = hipSuccess;
    for (int k = 0; k < S.slots && e == hipSuccess && est_host && batches() > 0; ++k)
      e = hipStreamWaitEvent(s, out[k], 0);
    return e;
  }
};

hipError_t enqueue_stream(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, int batch,
                          bool est_host, hipStream_t s) {
  StreamPipe p(c, r, batch, est_host, s);
  const size_t es = r->obs_dtype == MVD_U16 ? 2 : 4;
  const size_t plane = (size_t)c->Z * c->X, row = (size_t)c->X * es;
  std::vector<const void *> src(c->nv);
  hipError_t e = p.begin();
  for (int b = 0; b < p.batches() && e == hipSuccess; ++b) {
    const int y0 = b * p.S.ys;
    for (int v = 0; v < c->nv; ++v) src[v] = static_cast<const char *>(obs[v]) + (size_t)y0 * row;
    e = p.batch(b, src.data(), (size_t)r->n_planes * row, est + (size_t)y0 * plane);
  }
  if (e == hipSuccess) e = p.end();
  return e;
}

// ---- disk-to-disk runs ------------------------------------------------------
// Three actors share a batch counter each: the reader thread (`read`: batches
// in page-locked input slots), the caller's thread (`issued`: batches whose
// copies and iterations are enqueued, with an event per host slot recorded
// after the batch's copy-in and one after its copy-out) and the writer thread
// (`written`).  Host slot k = b mod H serves batch b; the reader refills an
// input slot once the copy-in event of the batch before has completed, and the
// caller reuses an output slot once the writer has written it.
struct FilePipe {
  std::mutex mu;
  std::condition_variable cv;
  int read = 0, issued = 0, written = 0;
  bool failed = false;
  mvd_status st = MVD_OK;
  std::string msg;
  double t_read = 0, t_write = 0, t_wait = 0;

  void fail_with(mvd_status s, const std::string &m) {
    std::lock_guard<std::mutex> lk(mu);
    if (!failed) {
      failed = true;
      st = s;
      msg = m;
    }
    cv.notify_all();
  }
  // wait until pred() or a failure; false on failure
  template <class P>
  bool wait(P pred) {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return failed || pred(); });
    return !failed;
  }
  void bump(int &counter, int value) {
    std::lock_guard<std::mutex> lk(mu);
    counter = value;
    cv.notify_all();
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One piece of a batch read or write.
struct IoPiece {
  int fd;
  int64_t off;
  char *buf;
  size_t len;
};

// Runs the pieces on `threads` threads (pread / pwrite until each piece is
// done); with `drop`, flushes written ranges and drops every range from the
// page cache.  Returns an empty string or the first error.
std::string run_pieces(const std::vector<IoPiece> &pieces, int threads, bool write, bool drop) {
  std::atomic<size_t> next{0};
  std::mutex emu;
  std::string err;
  auto work = [&] {
    for (;;) {
      const size_t i = next.fetch_add(1);
      if (i >= pieces.size()) return;
      const IoPiece &p = pieces[i];
      size_t done = 0;
      while (done < p.len) {
        const ssize_t n = write ? pwrite(p.fd, p.buf + done, p.len - done, (off_t)(p.off + done))
                                : pread(p.fd, p.buf + done, p.len - done, (off_t)(p.off + done));
        if (n < 0 && errno == EINTR) continue;
        if (n <= 0) {
          char m[160];
          snprintf(m, sizeof m, "%s of %zu bytes at offset %lld: %s", write ? "pwrite" : "pread", p.len - done,
                   (long long)(p.off + done), n == 0 ? "end of file" : strerror(errno));
          std::lock_guard<std::mutex> lk(emu);
          if (err.empty()) err = m;
          return;
        }
        done += (size_t)n;
      }
      if (drop) {
        if (write) (void)sync_file_range(p.fd, p.off, (off_t)p.len,
                                         SYNC_FILE_RANGE_WAIT_BEFORE | SYNC_FILE_RANGE_WRITE |
                                             SYNC_FILE_RANGE_WAIT_AFTER);
        (void)posix_fadvise(p.fd, p.off, (off_t)p.len, POSIX_FADV_DONTNEED);
      }
    }
  };
  const int T = (int)std::min<size_t>((size_t)threads, pieces.size());
  std::vector<std::thread> team;
  try {
    for (int t = 1; t < T; ++t) team.emplace_back(work);
  } catch (...) {
    // fewer threads: the caller's thread still drains the list
  }
  work();
  for (auto &t : team) t.join();
  return err;
}

// Cuts [off, off + len) of one file into pieces of about `chunk` bytes.
void add_pieces(std::vector<IoPiece> &out, int fd, int64_t off, char *buf, size_t len, size_t chunk) {
  for (size_t o = 0; o < len; o += chunk) out.push_back(IoPiece{fd, off + (int64_t)o, buf + o, std::min(chunk, len - o)});
}

constexpr size_t kIoChunk = 8u << 20;

mvd_status run_files(mvd_ctx *c, mvd_files *io, const mvd_run *r, int batch, hipStream_t s) {
  const double t0 = now_s();
  const int H = io->host_slots ? io->host_slots : 3;
  const int T = io->io_threads ? io->io_threads : 4;
  const bool drop = io->flags & MVD_FILES_DROP_CACHE;
  const int V = c->nv, Z = c->Z, X = c->X, Y = r->n_planes;
  const size_t es = r->obs_dtype == MVD_U16 ? 2 : 4;
  const size_t plane = (size_t)Z * X;
  StreamPipe p(c, r, batch, true, s);
  const int ys = p.S.ys, nb = p.batches();
  // page-locked batches: H input slots of V compact [Z][ys][X] stacks, then H
  // output slots of [ys][Z][X] float32
  const size_t in_view = align_up((size_t)ys * plane * es), in_slot = (size_t)V * in_view;
  const size_t out_slot = align_up((size_t)ys * plane * sizeof(float));
  const size_t need = (size_t)H * (in_slot + out_slot);
  if (c->fhost_bytes < need) {
    if (c->fhost) (void)hipHostFree(c->fhost);
    c->fhost = nullptr;
    c->fhost_bytes = 0;
    if (hipHostMalloc(&c->fhost, need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c->fhost = nullptr;
      return fail(c, MVD_ERR_ALLOC, "cannot allocate %zu bytes of page-locked host batches", need);
    }
    c->fhost_bytes = need;
  }
  char *hin = static_cast<char *>(c->fhost), *hout = hin + (size_t)H * in_slot;
  std::vector<hipEvent_t> copied(H, nullptr), drained(H, nullptr);
  hipError_t e = hipSuccess;
  for (int k = 0; k < H && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&copied[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&drained[k], hipEventDisableTiming);
  }
  auto destroy_events = [&] {
    for (int k = 0; k < H; ++k) {
      if (copied[k]) (void)hipEventDestroy(copied[k]);
      if (drained[k]) (void)hipEventDestroy(drained[k]);
    }
  };
  if (e != hipSuccess) {
    destroy_events();
    return fail(c, MVD_ERR_ALLOC, "cannot create events: %s", hipGetErrorString(e));
  }
  FilePipe fp;
  int64_t nread = 0, nwritten = 0;
  auto reader = [&] {
    for (int b = 0; b < nb; ++b) {
      const int k = b % H, y0 = b * ys, ny = std::min(ys, Y - y0);
      if (b >= H) {
        if (!fp.wait([&] { return fp.issued > b - H; })) return;
        if (hipEventSynchronize(copied[k]) != hipSuccess) {
          fp.fail_with(MVD_ERR_LAUNCH, "copy-in event failed");
          return;
        }
      }
      const double ta = now_s();
      std::vector<IoPiece> pieces;
      for (int v = 0; v < V; ++v) {
        char *dst = hin + (size_t)k * in_slot + (size_t)v * in_view;
        const size_t run = (size_t)ny * X * es;   // bytes of one slice's rows y0..y0+ny
        if (ny == Y) {
          add_pieces(pieces, io->obs_fd[v], io->obs_offset[v], dst, (size_t)Z * run, kIoChunk);
        } else {
          for (int z = 0; z < Z; ++z)
            add_pieces(pieces, io->obs_fd[v], io->obs_offset[v] + (int64_t)(((size_t)z * Y + y0) * X * es),
                       dst + (size_t)z * run, run, kIoChunk);
        }
      }
      const std::string err = run_pieces(pieces, T, false, drop);
      if (!err.empty()) {
        fp.fail_with(MVD_ERR_IO, "reading batch " + std::to_string(b) + ": " + err);
        return;
      }
      for (const auto &q : pieces) nread += (int64_t)q.len;
      fp.t_read += now_s() - ta;
      fp.bump(fp.read, b + 1);
    }
  };
  auto writer = [&] {
    for (int b = 0; b < nb; ++b) {
      const int k = b % H, y0 = b * ys, ny = std::min(ys, Y - y0);
      if (!fp.wait([&] { return fp.issued > b; })) return;
      if (hipEventSynchronize(drained[k]) != hipSuccess) {
        fp.fail_with(MVD_ERR_LAUNCH, "copy-out event failed");
        return;
      }
      const double ta = now_s();
      std::vector<IoPiece> pieces;
      add_pieces(pieces, io->est_fd, io->est_offset + (int64_t)((size_t)y0 * plane * sizeof(float)),
                 hout + (size_t)k * out_slot, (size_t)ny * plane * sizeof(float), kIoChunk);
      const std::string err = run_pieces(pieces, T, true, drop);
      if (!err.empty()) {
        fp.fail_with(MVD_ERR_IO, "writing batch " + std::to_string(b) + ": " + err);
        return;
      }
      nwritten += (int64_t)((size_t)ny * plane * sizeof(float));
      fp.t_write += now_s() - ta;
      fp.bump(fp.written, b + 1);
    }
    if ((io->flags & MVD_FILES_SYNC) && nb > 0) {
      const double ta = now_s();
      if (fdatasync(io->est_fd) != 0) {
        fp.fail_with(MVD_ERR_IO, std::string("fdatasync: ") + strerror(errno));
        return;
      }
      fp.t_write += now_s() - ta;
    }
  };
  std::thread tr, tw;
  try {
    tr = std::thread(reader);
    tw = std::thread(writer);
  } catch (...) {
    fp.fail_with(MVD_ERR_ALLOC, "cannot start the reader and writer threads");
  }
  std::vector<const void *> src(V);
  e = fp.failed ? hipSuccess : p.begin();
  for (int b = 0; b < nb && e == hipSuccess; ++b) {
    const int k = b % H, ny = std::min(ys, Y - b * ys);
    const double ta = now_s();
    if (!fp.wait([&] { return fp.read > b && (b < H || fp.written > b - H); })) break;
    fp.t_wait += now_s() - ta;
    for (int v = 0; v < V; ++v) src[v] = hin + (size_t)k * in_slot + (size_t)v * in_view;
    e = p.batch(b, src.data(), (size_t)ny * X * es, reinterpret_cast<float *>(hout + (size_t)k * out_slot));
    if (e == hipSuccess) e = hipEventRecord(copied[k], c->h2d);
    if (e == hipSuccess) e = hipEventRecord(drained[k], c->d2h);
    if (e == hipSuccess) fp.bump(fp.issued, b + 1);
  }
  if (e == hipSuccess) e = p.end();
  if (e != hipSuccess) fp.fail_with(MVD_ERR_LAUNCH, std::string("streamed batch failed: ") + hipGetErrorString(e));
  fp.wait([&] { return fp.written == nb; });
  if (tr.joinable()) tr.join();
  if (tw.joinable()) tw.join();
  // nothing may still use the host batches or the events when the call returns
  hipError_t es1 = hipStreamSynchronize(s);
  hipError_t es2 = hipStreamSynchronize(c->h2d);
  hipError_t es3 = hipStreamSynchronize(c->d2h);
  destroy_events();
  if (fp.failed) return fail(c, fp.st, "%s", fp.msg.c_str());
  if (es1 != hipSuccess || es2 != hipSuccess || es3 != hipSuccess)
    return fail(c, MVD_ERR_LAUNCH, "stream synchronisation failed");
  io->seconds[0] = fp.t_read;
  io->seconds[1] = fp.t_write;
  io->seconds[2] = fp.t_wait;
  io->seconds[3] = now_s() - t0;
  io->bytes[0] = nread;
  io->bytes[1] = nwritten;
  return MVD_OK;
}

// ---- graph capture ----------------------------------------------------------
// A captured run is reused when every pointer and parameter is the same.
std::vector<uint64_t> run_key(const mvd_ctx *c, const void *const *obs, const float *est, const mvd_run *r) {
  std::vector<uint64_t> k;
  for (int v = 0; v < c->nv; ++v) k.push_back((uint64_t)(uintptr_t)obs[v]);
  k.push_back((uint64_t)(uintptr_t)est);
  k.push_back((uint64_t)(uintptr_t)r->checkpoints);
  k.push_back((uint64_t)(uintptr_t)r->workspace);
  k.push_back(r->workspace_bytes);
  const int32_t fields[] = {(int32_t)r->flags, r->n_planes, r->n_iters, r->update, r->boundary, r->init,
                            r->obs_dtype, r->obs_layout};
  for (int32_t f : fields) k.push_back((uint64_t)(uint32_t)f);
  uint32_t ic;
  std::memcpy(&ic, &r->init_const, 4);
  k.push_back(ic);
  for (int v = 0; v < c->nv; ++v) {
    uint32_t w = 0x3f800000u;
    if (r->view_weights) std::memcpy(&w, &r->view_weights[v], 4);
    k.push_back(w);
    k.push_back(r->weight_planes ? (uint64_t)(uintptr_t)r->weight_planes[v] : 0);
  }
  k.push_back(c->psf_generation);
  return k;
}

// Capture `launch(stream)` into an executable graph.
template <typename F>
hipError_t capture(F &&launch, hipGraph_t *graph, hipGraphExec_t *exec) {
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch(cs);
    hipGraph_t gph = nullptr;
    e = hipStreamEndCapture(cs, &gph);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, gph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
      *graph = gph;
    } else if (gph) {
      (void)hipGraphDestroy(gph);
    }
  }
  (void)hipStreamDestroy(cs);
  return e;
}

hipError_t cached_graph(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, const Tune &tn,
                        hipGraphExec_t *out) {
  const std::vector<uint64_t> key = run_key(c, obs, est, r);
  for (auto &g : c->graphs)
    if (g.key == key) {
      *out = g.exec;
      return hipSuccess;
    }
  mvd_ctx::Graph g;
  g.key = key;
  hipError_t e = capture([&](hipStream_t cs) { return enqueue_run(c, obs, est, r, cs, tn); }, &g.graph,
                         &g.exec);
  if (e != hipSuccess) return e;
  if (c->graphs.size() >= 8) {   // keep the cache small: drop the oldest
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    (void)hipGraphDestroy(c->graphs.front().graph);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back(g);
  *out = g.exec;
  return hipSuccess;
}


// ---- autotuner ----------------------------------------------------------------
// Launch-shape candidates timed per workload (kernel sizes, plane shape, planes,
// views, update order, boundary); the fastest is cached for the process.  Each
// candidate starts from the process-wide overrides.
std::vector<Tune> tune_candidates() {
  std::vector<Tune> c(12, tune());
  for (Tune &t : c) t.fused = 0;
  c[11].fused = 1;       // one fused launch per iteration (where it applies)
  c[1].fwd_occ = 2;
  c[2].fwd_views = 1;
  c[3].bwd_vin = 1;      // one ratio plane per backward launch
  c[4].zseg_scale = 1;   // segments × 1/2, × 2, × 4, × 8
  c[5].zseg_scale = 3;
  c[6].zseg_scale = 4;
  c[7].zseg_scale = 5;
  c[8].cols = 1;
  c[9].bwd_split = 2;    // two-plane backward without the split-view form
  c[10].wide = 2;        // rows wider than 512 as two columns per thread
  return c;
}

std::string tune_key(const mvd_ctx *c, const mvd_run *r) {
  std::string k = "Z" + std::to_string(c->Z) + "X" + std::to_string(c->X) + "Y" + std::to_string(r->n_planes) +
                  "V" + std::to_string(c->nv) + "u" + std::to_string(r->update) + "b" + std::to_string(r->boundary) +
                  "f" + std::to_string(r->flags & (MVD_FLAG_FORCE_2D | MVD_FLAG_NORMALIZE)) +
                  (r->weight_planes ? "w" : "") + "K";
  for (auto &w : c->views)
    k += std::to_string(w.psf.kz) + "x" + std::to_string(w.psf.kx) + (w.sep_p ? "s" : "g") +
         std::to_string(w.back.kz) + "x" + std::to_string(w.back.kx) + (w.sep_x ? "s" : "g") + ",";
  return k;
}

std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune_cache;

// Pass launch time (ms: forward, backward and fused launches) of the marks
// recorded since the last drain: the cost of an iteration.  (The one-iteration
// probe ends a fused run with the copy back of an odd count, a cost paid once
// per run, which is left out.)
double drain_marks(mvd_ctx *c) {
  double ms = 0.0;
  for (auto &m : c->marks) {
    float t = 0.f;
    if ((m.kind == 0 || m.kind == 1 || m.kind == 5) && hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) ms += t;
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  c->marks.clear();
  return ms;
}

// Time every candidate on one iteration of the item's own run (the item's
// estimate is overwritten, so items that start from a given estimate are not
// tuned) and return the fastest.
// A probe runs one iteration, so it needs the workspace of a run with
// n_iters ≥ 1; a run without iterations has no passes to tune and makes none.
bool tune_probe(const mvd_run *r, mvd_run *probe) {
  if (r->n_iters < 1) return false;
  *probe = *r;
  probe->n_iters = 1;
  probe->checkpoints = nullptr;
  probe->flags &= ~(MVD_FLAG_GRAPH | MVD_FLAG_TIMING | MVD_FLAG_TUNE);
  return true;
}

hipError_t autotune(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, hipStream_t s, Tune *out) {
  mvd_run probe;
  if (!tune_probe(r, &probe)) {
    *out = Tune{};
    return hipSuccess;
  }
  const std::string key = tune_key(c, r);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *out = it->second;
      return hipSuccess;
    }
  }
  // the caller's timing records are kept aside while the candidates are timed
  std::vector<mvd_ctx::Mark> kept;
  kept.swap(c->marks);
  struct Restore {
    mvd_ctx *c;
    std::vector<mvd_ctx::Mark> &kept;
    ~Restore() {
      (void)drain_marks(c);
      c->marks.swap(kept);
    }
  } restore{c, kept};
  hipError_t e = enqueue_run(c, obs, est, &probe, s, Tune{});   // warm-up
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const std::vector<Tune> cand = tune_candidates();
  double best = 1e30;
  Tune pick{};
  for (const Tune &t : cand) {
    if (e != hipSuccess) break;
    double ms = 0.0;
    // the first run of a candidate is not counted: it pays the first launch of
    // kernels the others did not use (code loading, attributes)
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = enqueue_run(c, obs, est, &probe, s, t, true);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess) {
        const double m = drain_marks(c);
        if (rep > 0) ms += m;
      }
    }
    if (e == hipSuccess && ms < best) {
      best = ms;
      pick = t;
    }
  }
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = pick;
  *out = pick;
  return hipSuccess;
}

}  // namespace

// ---- persistent batched form ----------------------------------------------
// Whether a run can go through the persistent queue kernel: rank-one passes
// of at most 41 taps, the plain update (no normalisation, no per-pixel
// weights), no checkpoints, and whole 16-byte row items.
bool pq_eligible(const mvd_ctx *c, const void *const *obs, const float *est, const mvd_run *r, std::string *why) {
  auto no = [&](const char *m) {
    if (why) *why = m;
    return false;
  };
  if (r->flags & (MVD_FLAG_FORCE_2D | MVD_FLAG_NORMALIZE)) return no("K×K or normalised passes");
  if (r->weight_planes) return no("per-pixel weights");
  if (r->checkpoints) return no("checkpoints");
  int kmax = 1;
  for (int v = 0; v < c->nv; ++v) {
    const ViewPsf &w = c->views[v];
    if (!w.sep_p || !w.sep_x) return no("a PSF or back-projector that is not rank one");
    kmax = std::max({kmax, w.psf.kz, w.psf.kx, w.back.kz, w.back.kx});
  }
  if (sep_bucket(kmax) > 41) return no("more than 41 taps");
  if (c->X % 8) return no("rows not a multiple of 8 columns");
  const ObsRef ob = obs_given(obs, r->obs_dtype, r->obs_layout, PlaneGeom{r->n_planes, c->Z, c->X}, nullptr);
  const long unit = ob.u16 ? 8 : 4;
  if (ob.sy % unit || ob.sz % unit) return no("observation rows not in whole 16-byte units");
  for (int v = 0; v < c->nv; ++v)
    if (!aligned16(obs[v])) return no("observations not 16-byte aligned");
  if (!aligned16(est)) return no("estimate not 16-byte aligned");
  return true;
}

// The launch shapes of the persistent form: one column per thread, at most
// kSepMaxThreads columns per tile (wider rows in strips with halos).
Tune pq_tune() {
  Tune t;
  t.threads = kSepMaxThreads;
  t.cols = 1;
  return t;
}

// The job of one volume: its tiling and the arguments of every pass.
bool pq_job(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r, unsigned *done, PqJob *out) {
  const PlaneGeom g{r->n_planes, c->Z, c->X};
  int kmax = 1;
  for (int v = 0; v < c->nv; ++v)
    kmax = std::max({kmax, c->views[v].psf.kz, c->views[v].psf.kx, c->views[v].back.kz, c->views[v].back.kx});
  // rows of 513–1024 columns: one whole-row tile per work-group (every thread
  // a column); otherwise tiles of at most kSepMaxThreads columns, two per item
  // segments twice the planner's length: fewer items, each with a fixed cost
  // (dequeue, dependency check, ring fill); measured on the three-volume mix:
  // 64.9 ms per step against 70.1 ms with the planner's segments
  Tune tw{}, tp = pq_tune();
  tw.zseg_scale = tp.zseg_scale = tune().pq_zseg_scale > 0 ? tune().pq_zseg_scale : 3;
  const SepGeom wide = plan_sep(c, g.Y, sep_bucket(kmax), r->boundary, tw, true);
  const bool one = wide.plan.threads > kSepMaxThreads && wide.plan.threads <= kPqThreads && wide.halo == 0 &&
                   wide.plan.cols == 1;
  const SepGeom sg = one ? wide : plan_sep(c, g.Y, sep_bucket(kmax), r->boundary, tp);
  if (sg.plan.cols != 1 || !whole_items(sg, g)) return false;
  if (!one && sg.plan.threads > kPqThreads / 2) return false;
  PqJob j{};
  j.g = g;
  j.kb = sg.plan.bucket;
  j.pair = one ? 0 : 1;
  j.nseg = sg.nseg;
  j.nstrip = sg.nstrip;
  j.zseg = sg.zseg;
  j.x_out = sg.x_out;
  j.ntiles = sg.nseg * sg.nstrip;
  j.sim = r->update == MVD_UPDATE_SIMULTANEOUS;
  const int V = c->nv;
  j.nf = j.sim ? (V + 1) / 2 : V;
  j.per_iter = j.sim ? j.nf + V : 2 * V;
  j.init = r->init == MVD_INIT_MEAN ? 0 : (r->init == MVD_INIT_GIVEN ? 1 : 2);
  j.init_const = r->init_const;
  j.nv = V;
  const ObsRef ob = obs_given(obs, r->obs_dtype, r->obs_layout, g, nullptr);
  j.obs_u16 = ob.u16 ? 1 : 0;
  j.obs_sy = ob.sy;
  j.obs_sz = ob.sz;
  for (int v = 0; v < V; ++v) j.obs[v] = obs[v];
  j.est = est;
  j.done = done;
  const Layout L = layout_of(c, r);
  char *ws = static_cast<char *>(r->workspace);
  auto ratio = [&](int v) { return reinterpret_cast<float *>(ws + L.r_off + (size_t)(j.sim ? v : 0) * L.plane_set); };
  for (int s = 0; s < j.nf; ++s) {
    SepPassArgs &a = j.f[s];
    fill_sep_common(a, sg, g, r->boundary);
    const int v0 = j.sim ? 2 * s : s;
    a.nviews = j.sim ? std::min(2, V - v0) : 1;
    a.in[0] = est;
    a.obs_u16 = j.obs_u16;
    a.obs_sy = ob.sy;
    a.obs_sz = ob.sz;
    for (int k = 0; k < a.nviews; ++k) {
      const ViewPsf &w = c->views[v0 + k];
      a.obs[k] = obs[v0 + k];
      a.out[k] = ratio(v0 + k);
      put_factor(a.tz[k], w.pz, j.kb);
      put_factor(a.tx[k], w.px, j.kb);
      if (!aligned16(a.out[k])) return false;
    }
    a.vec = 1;
    j.fkind[s] = (ob.u16 ? 2 : 0) + (a.nviews == 2 ? 1 : 0);
  }
  for (int v = 0; v < V; ++v) {
    SepPassArgs &a = j.b[v];
    fill_sep_common(a, sg, g, r->boundary);
    a.nviews = 1;
    a.in[0] = ratio(v);
    a.w[0] = r->view_weights ? r->view_weights[v] : 1.f;
    put_factor(a.tz[0], c->views[v].xz, j.kb);
    put_factor(a.tx[0], c->views[v].xx, j.kb);
    a.psi_in = est;
    a.psi_out = est;
    a.vec = 1;
  }
  j.lds_floats = (int)(pq_lds_bytes(j) / sizeof(float));
  *out = j;
  return true;
}

// Items of all jobs in dependency order.  Each job's tiles go window by
// window (`win` planes), a window's tiles by (phase, plane, tile); a job with
// paired tiles takes them two at a time (consecutive tiles of one phase and
// row segment: the same barriers).  Then the jobs' lists are merged so that
// every job advances in proportion to its length (all finish together).  A
// phase of a plane needs only the plane's earlier phases, and each job's own
// order is kept, so those come earlier.
std::vector<int4> pq_items(const std::vector<PqJob> &jobs, const std::vector<int> &win,
                           const std::vector<int> &iters) {
  std::vector<std::vector<int4>> per(jobs.size());
  for (size_t k = 0; k < jobs.size(); ++k) {
    const PqJob &j = jobs[k];
    const int nphase = 1 + iters[k] * j.per_iter;
    for (int y0 = 0; y0 < j.g.Y; y0 += win[k]) {
      const int y1 = std::min(j.g.Y, y0 + win[k]);
      for (int p = 0; p < nphase; ++p) {
        if (!j.pair) {
          for (int b = y0 * j.ntiles; b < y1 * j.ntiles; ++b) per[k].push_back(make_int4((int)k, p, b, -1));
          continue;
        }
        // pair tiles of the same row segment: within a segment, consecutive (plane, strip)
        for (int seg = 0; seg < j.nseg; ++seg) {
          int pend = -1;
          for (int y = y0; y < y1; ++y)
            for (int st = 0; st < j.nstrip; ++st) {
              const int b = (y * j.nseg + seg) * j.nstrip + st;
              if (pend < 0) {
                pend = b;
              } else {
                per[k].push_back(make_int4((int)k, p, pend, b));
                pend = -1;
              }
            }
          if (pend >= 0) per[k].push_back(make_int4((int)k, p, pend, -1));
        }
      }
    }
  }
  std::vector<int4> out;
  std::vector<size_t> pos(jobs.size(), 0);
  for (;;) {   // next: the job whose next item sits earliest in its own list, relatively
    int best = -1;
    double key = 2.0;
    for (size_t k = 0; k < per.size(); ++k) {
      if (pos[k] >= per[k].size()) continue;
      const double f = (pos[k] + 0.5) / per[k].size();
      if (f < key) {
        key = f;
        best = (int)k;
      }
    }
    if (best < 0) break;
    out.push_back(per[best][pos[best]++]);
  }
  return out;
}

// Polls before a wait gives up (test hook; 0 = the default).
std::atomic<unsigned> g_pq_spin{0};
constexpr unsigned kPqSpinDefault = 1u << 24;

struct PqState {
  void *dmem = nullptr;         // jobs, items, counters
  PqQueue q{};
  int nblocks = 0;
  size_t lds = 0;
};

struct mvd_batch {
  int device = -1;
  struct Item {
    mvd_ctx *ctx;
    uint64_t serial, psf_generation;   // the context's identity and taps at capture
    std::vector<const void *> obs;
    float *est;
    mvd_run run;
    std::vector<float> weights;
    std::vector<const float *> wplanes;
    Tune tn;
  };
  std::vector<Item> items;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool persistent = false;   // one persistent queue launch instead of the graph
  PqState pq;
  std::string why_graph;      // why the graph form was taken
  double form_ms[2] = {0.0, 0.0};   // tuned batches: persistent and graph form, ms per launch (0: not timed)
};

namespace {

// Build the persistent form of a batch: job table, item table and counters in
// one device allocation made here (at creation; launches allocate nothing).
hipError_t pq_setup(mvd_batch *b, int window) {
  std::vector<PqJob> jobs(b->items.size());
  std::vector<int> win(b->items.size());
  std::vector<size_t> done_off(b->items.size());
  std::vector<int> iters(b->items.size());
  size_t ndone = 0;
  for (size_t k = 0; k < b->items.size(); ++k) {
    const auto &it = b->items[k];
    iters[k] = it.run.n_iters;
    done_off[k] = ndone;
    ndone += (size_t)it.run.n_planes;
  }
  // jobs, then items, then counters (per plane, then head / exited / give-up)
  const size_t jobs_bytes = align_up(jobs.size() * sizeof(PqJob));
  for (size_t k = 0; k < b->items.size(); ++k) {
    auto &it = b->items[k];
    if (!pq_job(it.ctx, it.obs.data(), it.est, &it.run, nullptr, &jobs[k])) return hipErrorInvalidValue;
    // planes per window (0: the whole volume, iteration-major as the plain path)
    win[k] = window > 0 ? std::min(window, jobs[k].g.Y) : jobs[k].g.Y;
  }
  const std::vector<int4> items = pq_items(jobs, win, iters);
  const size_t items_bytes = align_up(items.size() * sizeof(int4));
  const size_t done_bytes = align_up((ndone + 3) * sizeof(unsigned));
  hipError_t e = hipMalloc(&b->pq.dmem, jobs_bytes + items_bytes + done_bytes);
  if (e != hipSuccess) return e;
  char *base = static_cast<char *>(b->pq.dmem);
  unsigned *done = reinterpret_cast<unsigned *>(base + jobs_bytes + items_bytes);
  for (size_t k = 0; k < jobs.size(); ++k) jobs[k].done = done + done_off[k];
  e = hipMemcpy(base, jobs.data(), jobs.size() * sizeof(PqJob), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + jobs_bytes, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(done, 0, (ndone + 3) * sizeof(unsigned));
  if (e != hipSuccess) return e;
  PqQueue &q = b->pq.q;
  q.items = reinterpret_cast<const int4 *>(base + jobs_bytes);
  q.n_items = (int)items.size();
  q.n_jobs = (int)jobs.size();
  q.jobs = reinterpret_cast<const PqJob *>(base);
  q.head = done + ndone;
  q.exited = done + ndone + 1;
  q.giveup = done + ndone + 2;
  size_t lds = 0;
  for (const PqJob &j : jobs) lds = std::max(lds, (j.pair ? 2 : 1) * (size_t)j.lds_floats * sizeof(float));
  if (lds > kLdsLimit) return hipErrorInvalidValue;
  b->pq.lds = lds;
  int per_cu = 0, cus = 0;
  e = pq_occupancy(lds, &per_cu);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  b->pq.nblocks = per_cu * cus;
  return hipSuccess;
}

}  // namespace

// One warm-up launch and two timed launches of a batch in its current form on
// `s`: the mean duration (HIP events) in *ms.
static mvd_status batch_time_launches(mvd_batch *b, hipStream_t s, double *ms) {
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  mvd_status st = e == hipSuccess ? MVD_OK : MVD_ERR_LAUNCH;
  if (st == MVD_OK) st = mvd_batch_launch(b, s);
  if (st == MVD_OK) st = mvd_batch_wait(b, s);
  if (st == MVD_OK && hipEventRecord(t0, s) != hipSuccess) st = MVD_ERR_LAUNCH;
  for (int k = 0; k < 2 && st == MVD_OK; ++k) st = mvd_batch_launch(b, s);
  if (st == MVD_OK && hipEventRecord(t1, s) != hipSuccess) st = MVD_ERR_LAUNCH;
  if (st == MVD_OK) st = mvd_batch_wait(b, s);
  float f = 0.f;
  if (st == MVD_OK && hipEventElapsedTime(&f, t0, t1) != hipSuccess) st = MVD_ERR_LAUNCH;
  *ms = f / 2.0;
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  return st;
}

// ===========================================================================
extern "C" {

int mvd_version(void) { return MVD_ABI_VERSION; }

const char *mvd_status_string(mvd_status s) {
  switch (s) {
    case MVD_OK: return "ok";
    case MVD_ERR_ARG: return "invalid argument";
    case MVD_ERR_STATE: return "invalid state";
    case MVD_ERR_WORKSPACE: return "workspace too small";
    case MVD_ERR_DEVICE: return "device unavailable";
    case MVD_ERR_LAUNCH: return "launch failed";
    case MVD_ERR_UNSUPPORTED: return "unsupported";
    case MVD_ERR_ALLOC: return "allocation failed";
    case MVD_ERR_IO: return "file read or write failed";
  }
  return "unknown status";
}

mvd_status mvd_create(mvd_ctx **out, int n_views, int n_z, int n_x, int device) {
  if (!out) return fail(nullptr, MVD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_views < 1 || n_views > MVD_MAX_VIEWS)
    return fail(nullptr, MVD_ERR_ARG, "n_views %d outside [1, %d]", n_views, MVD_MAX_VIEWS);
  if (n_z < 1 || n_x < 1) return fail(nullptr, MVD_ERR_ARG, "plane %d x %d is empty", n_z, n_x);
  if ((long long)n_z * n_x > (1LL << 31))
    return fail(nullptr, MVD_ERR_ARG, "plane %d x %d too large", n_z, n_x);
  // rows outside the plane are read from a static row of kMaxPlaneX zeros
  if (n_x > MVD_MAX_PLANE_X)
    return fail(nullptr, MVD_ERR_ARG, "plane width %d above MVD_MAX_PLANE_X = %d", n_x, MVD_MAX_PLANE_X);
  if (device != MVD_DEVICE_NONE) {
    int n = 0;
    if (device < 0 || hipGetDeviceCount(&n) != hipSuccess || device >= n)
      return fail(nullptr, MVD_ERR_DEVICE, "HIP device %d not available", device);
  }
  if (device != MVD_DEVICE_NONE) {
    // the static entry point's scratch address on this device (once per device)
    DeviceGuard dg(device);
    void *p = nullptr;
    if (!dg.ok()) return fail(nullptr, MVD_ERR_DEVICE, "cannot select device %d", device);
    const hipError_t e = scratch_setup(device, &p);
    if (e != hipSuccess)
      return fail(nullptr, MVD_ERR_DEVICE, "device %d: scratch address unavailable: %s", device, hipGetErrorString(e));
  }
  mvd_ctx *c = new (std::nothrow) mvd_ctx;
  if (!c) return fail(nullptr, MVD_ERR_ALLOC, "out of host memory");
  c->nv = n_views;
  c->Z = n_z;
  c->X = n_x;
  c->device = device;
  c->views.resize(n_views);
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    c->serial = g_next_serial++;
    g_live[c] = c->serial;
  }
  *out = c;
  g_noctx_error.clear();
  return MVD_OK;
}

void mvd_destroy(mvd_ctx *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(ctx);
  }
  if (ctx->device != MVD_DEVICE_NONE) {
    DeviceGuard dg(ctx->device);
    for (auto &m : ctx->marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    for (auto &g : ctx->graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    if (ctx->d_taps) (void)hipFree(ctx->d_taps);
    for (auto e : ctx->sev)
      if (e) (void)hipEventDestroy(e);
    if (ctx->h2d) (void)hipStreamDestroy(ctx->h2d);
    if (ctx->d2h) (void)hipStreamDestroy(ctx->d2h);
    if (ctx->fhost) (void)hipHostFree(ctx->fhost);
  }
  delete ctx;
}

mvd_status mvd_get_timing(mvd_ctx *c, mvd_timing *out, int reset) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!out || out->struct_size != sizeof(mvd_timing))
    return fail(c, MVD_ERR_ARG, "out is NULL or has a wrong struct_size");
  for (int k = 0; k < MVD_TIMING_KINDS; ++k) {
    out->count[k] = 0;
    out->ms[k] = 0.0;
  }
  if (c->marks.empty()) return MVD_OK;
  DeviceGuard dg(c->device);
  if (hipEventSynchronize(c->marks.back().b) != hipSuccess)
    return fail(c, MVD_ERR_LAUNCH, "event synchronisation failed");
  for (auto &m : c->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess)
      return fail(c, MVD_ERR_LAUNCH, "event timing failed");
    out->count[m.kind] += 1;
    out->ms[m.kind] += ms;
  }
  if (reset) {
    for (auto &m : c->marks) {
      c->pool.push_back(m.a);
      c->pool.push_back(m.b);
    }
    c->marks.clear();
  }
  return MVD_OK;
}

mvd_status mvd_set_psf(mvd_ctx *c, int view, const float *taps, int kz, int kx, int back_mode,
                       const float *back_taps) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (view < 0 || view >= c->nv) return fail(c, MVD_ERR_ARG, "view %d outside [0, %d)", view, c->nv);
  if (kz < 1 || kx < 1 || kz > MVD_MAX_K || kx > MVD_MAX_K || kz % 2 == 0 || kx % 2 == 0)
    return fail(c, MVD_ERR_ARG, "PSF %d x %d: sides must be odd and in [1, %d]", kz, kx, MVD_MAX_K);
  if (!taps) return fail(c, MVD_ERR_ARG, "taps is NULL");
  if (!valid_taps(taps, kz * kx))
    return fail(c, MVD_ERR_ARG, "taps must be finite, >= 0 and not all zero");
  if (back_mode < MVD_BACK_FLIPPED || back_mode > MVD_BACK_EXPLICIT)
    return fail(c, MVD_ERR_ARG, "unknown back-projector mode %d", back_mode);
  if (back_mode == MVD_BACK_EXPLICIT) {
    if (!back_taps) return fail(c, MVD_ERR_ARG, "explicit back-projector needs back_taps");
    if (!valid_taps(back_taps, kz * kx))
      return fail(c, MVD_ERR_ARG, "back_taps must be finite, >= 0 and not all zero");
  }
  ViewPsf &w = c->views[view];
  w.psf = to_kernel(taps, kz, kx);
  w.back_mode = back_mode;
  w.explicit_back = back_mode == MVD_BACK_EXPLICIT ? to_kernel(back_taps, kz, kx) : Kernel{};
  w.set = true;
  c->derived = false;
  c->psf_generation += 1;
  if (all_set(c)) return derive(c);
  return MVD_OK;
}

mvd_status mvd_get_back_taps(mvd_ctx *c, int view, float *out) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (view < 0 || view >= c->nv) return fail(c, MVD_ERR_ARG, "view %d outside [0, %d)", view, c->nv);
  if (!out) return fail(c, MVD_ERR_ARG, "out is NULL");
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  const Kernel &b = c->views[view].back;
  for (size_t e = 0; e < b.t.size(); ++e) out[e] = (float)b.t[e];
  return MVD_OK;
}

mvd_status mvd_psf_info(mvd_ctx *c, int view, int *sp, int *sx) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (view < 0 || view >= c->nv) return fail(c, MVD_ERR_ARG, "view %d outside [0, %d)", view, c->nv);
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  const ViewPsf &w = c->views[view];
  if (sp) *sp = w.sep_p ? 1 : (int)w.lpz.size();
  if (sx) *sx = w.sep_x ? 1 : (int)w.lxz.size();
  return MVD_OK;
}

mvd_status mvd_workspace_bytes(const mvd_ctx *cc, const mvd_run *r, size_t *bytes) {
  mvd_ctx *c = const_cast<mvd_ctx *>(cc);
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!bytes) return fail(c, MVD_ERR_ARG, "bytes is NULL");
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  *bytes = layout_of(c, r).total;
  return MVD_OK;
}

mvd_status mvd_reslice(mvd_ctx *c, const void *stack, int dtype, int n_planes, float *planes,
                       void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!stack || !planes) return fail(c, MVD_ERR_ARG, "null buffer");
  if (dtype != MVD_U16 && dtype != MVD_F32) return fail(c, MVD_ERR_ARG, "unknown dtype %d", dtype);
  if (n_planes < 1) return fail(c, MVD_ERR_ARG, "n_planes must be >= 1");
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
  PlaneGeom g{n_planes, c->Z, c->X};
  hipError_t e = launch_stage_obs(stack, dtype, MVD_STACK_ZYX, g, planes, (hipStream_t)stream);
  if (e != hipSuccess) return fail(c, MVD_ERR_LAUNCH, "reslice launch: %s", hipGetErrorString(e));
  return MVD_OK;
}

mvd_status mvd_deconvolve_planes(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r,
                                 void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  mvd_status st = validate_run(c, obs, est, r);
  if (st != MVD_OK) return st;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
  hipError_t e = hipSuccess;
  Tune tn = tune();
  if ((r->flags & MVD_FLAG_TUNE) && r->init != MVD_INIT_GIVEN)
    e = autotune(c, obs, est, r, (hipStream_t)stream, &tn);
  if (e != hipSuccess) {
  } else if (r->flags & MVD_FLAG_GRAPH) {
    hipGraphExec_t exec = nullptr;
    e = cached_graph(c, obs, est, r, tn, &exec);
    if (e == hipSuccess) e = hipGraphLaunch(exec, (hipStream_t)stream);
  } else {
    e = enqueue_run(c, obs, est, r, (hipStream_t)stream, tn);
  }
  if (e != hipSuccess) return fail(c, MVD_ERR_LAUNCH, "launch failed: %s", hipGetErrorString(e));
  return MVD_OK;
}

mvd_status mvd_deconvolve_planes_static(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r,
                                        void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  if (r->flags & (MVD_FLAG_TIMING | MVD_FLAG_GRAPH | MVD_FLAG_TUNE))
    return fail(c, MVD_ERR_ARG, "timing, graph and tuning flags create events or graphs: not in the static form");
  if (r->workspace || r->workspace_bytes)
    return fail(c, MVD_ERR_ARG, "the static form uses the library's scratch: pass no workspace");
  if (!obs) return fail(c, MVD_ERR_ARG, "obs is NULL");
  for (int v = 0; v < c->nv; ++v)
    if (!obs[v]) return fail(c, MVD_ERR_ARG, "obs[%d] is NULL", v);
  if (!est) return fail(c, MVD_ERR_ARG, "est is NULL");
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  // the largest batch of planes whose workspace fits the scratch; each batch
  // goes through all iterations (planes are independent)
  auto need = [&](int planes) {
    mvd_run one = *r;
    one.n_planes = planes;
    return layout_of(c, &one).total;
  };
  if (need(1) > kScratchBytes)
    return fail(c, MVD_ERR_WORKSPACE, "one plane needs %zu bytes of workspace; the static scratch holds %zu",
                need(1), kScratchBytes);
  int B = (int)std::min<size_t>((size_t)r->n_planes, std::max<size_t>(1, kScratchBytes / need(1)));
  while (B > 1 && need(B) > kScratchBytes) --B;
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
  void *ptr = nullptr;
  hipError_t e = scratch_setup(c->device, &ptr);
  if (e != hipSuccess) return fail(c, MVD_ERR_DEVICE, "scratch address unavailable: %s", hipGetErrorString(e));
  mvd_run rr = *r;
  rr.workspace = ptr;
  rr.workspace_bytes = kScratchBytes;
  Tune tn = tune();
  tn.plane_batch = tn.plane_batch > 0 ? std::min(tn.plane_batch, B) : B;
  e = enqueue_run(c, obs, est, &rr, (hipStream_t)stream, tn);
  if (e != hipSuccess) return fail(c, MVD_ERR_LAUNCH, "launch failed: %s", hipGetErrorString(e));
  return MVD_OK;
}

mvd_status mvd_stream_workspace_bytes(const mvd_ctx *cc, const mvd_run *r, int batch_planes, int est_on_host,
                                      size_t *bytes) {
  mvd_ctx *c = const_cast<mvd_ctx *>(cc);
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!bytes) return fail(c, MVD_ERR_ARG, "bytes is NULL");
  mvd_status st = check_stream_run(c, r, batch_planes);
  if (st != MVD_OK) return st;
  *bytes = stream_layout_of(c, r, batch_planes, est_on_host != 0).total;
  return MVD_OK;
}

mvd_status mvd_deconvolve_stream(mvd_ctx *c, const void *const *obs, float *est, const mvd_run *r,
                                 int batch_planes, void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  mvd_status st = check_stream_run(c, r, batch_planes);
  if (st != MVD_OK) return st;
  if (!obs) return fail(c, MVD_ERR_ARG, "obs is NULL");
  for (int v = 0; v < c->nv; ++v)
    if (!obs[v]) return fail(c, MVD_ERR_ARG, "obs[%d] is NULL", v);
  if (!est) return fail(c, MVD_ERR_ARG, "est is NULL");
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  if (r->workspace && ((uintptr_t)r->workspace % kAlign))
    return fail(c, MVD_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
  for (int v = 0; v < c->nv; ++v)
    if (memory_kind(obs[v]) == 0)
      return fail(c, MVD_ERR_ARG, "obs[%d] is pageable host memory: use page-locked or device memory", v);
  const int ek = memory_kind(est);
  if (ek == 0) return fail(c, MVD_ERR_ARG, "est is pageable host memory: use page-locked or device memory");
  st = check_stream_weights(c, r);
  if (st != MVD_OK) return st;
  const bool est_host = ek == 1;
  const StreamLayout S = stream_layout_of(c, r, batch_planes, est_host);
  if (!r->workspace || r->workspace_bytes < S.total)
    return fail(c, MVD_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", S.total,
                r->workspace ? r->workspace_bytes : (size_t)0);
  if (stream_resources(c) != hipSuccess) return fail(c, MVD_ERR_ALLOC, "cannot create copy streams or events");
  hipError_t e = enqueue_stream(c, obs, est, r, batch_planes, est_host, (hipStream_t)stream);
  if (e != hipSuccess) return fail(c, MVD_ERR_LAUNCH, "streamed run failed: %s", hipGetErrorString(e));
  return MVD_OK;
}

mvd_status mvd_deconvolve_files(mvd_ctx *c, mvd_files *io, const mvd_run *r, int batch_planes, void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!io || io->struct_size != sizeof(mvd_files)) return fail(c, MVD_ERR_ARG, "io is NULL or has a wrong struct_size");
  mvd_status st = check_stream_run(c, r, batch_planes);
  if (st != MVD_OK) return st;
  if (r->init == MVD_INIT_GIVEN) return fail(c, MVD_ERR_ARG, "the disk-to-disk form reads no initial estimate");
  if (io->flags & ~(uint32_t)(MVD_FILES_SYNC | MVD_FILES_DROP_CACHE))
    return fail(c, MVD_ERR_ARG, "unknown flags 0x%x", io->flags);
  if (io->host_slots != 0 && (io->host_slots < 2 || io->host_slots > 8))
    return fail(c, MVD_ERR_ARG, "host_slots %d outside {0} and [2, 8]", io->host_slots);
  if (io->io_threads < 0 || io->io_threads > 64) return fail(c, MVD_ERR_ARG, "io_threads %d outside [0, 64]", io->io_threads);
  const size_t es = r->obs_dtype == MVD_U16 ? 2 : 4;
  const int64_t stack = (int64_t)((size_t)c->Z * r->n_planes * c->X * es);
  for (int v = 0; v < c->nv; ++v) {
    struct stat sb;
    if (io->obs_fd[v] < 0 || fstat(io->obs_fd[v], &sb) != 0)
      return fail(c, MVD_ERR_ARG, "obs_fd[%d] = %d is not an open descriptor", v, io->obs_fd[v]);
    if (!S_ISREG(sb.st_mode)) return fail(c, MVD_ERR_ARG, "obs_fd[%d] is not a regular file", v);
    if (io->obs_offset[v] < 0) return fail(c, MVD_ERR_ARG, "obs_offset[%d] is negative", v);
    if ((int64_t)sb.st_size < io->obs_offset[v] + stack)
      return fail(c, MVD_ERR_ARG, "view %d: file of %lld bytes holds no %lld-byte stack at offset %lld", v,
                  (long long)sb.st_size, (long long)stack, (long long)io->obs_offset[v]);
    if (fcntl(io->obs_fd[v], F_GETFL) & O_WRONLY) return fail(c, MVD_ERR_ARG, "obs_fd[%d] is write-only", v);
  }
  {
    struct stat sb;
    if (io->est_fd < 0 || fstat(io->est_fd, &sb) != 0)
      return fail(c, MVD_ERR_ARG, "est_fd = %d is not an open descriptor", io->est_fd);
    if (!S_ISREG(sb.st_mode)) return fail(c, MVD_ERR_ARG, "est_fd is not a regular file");
    if (io->est_offset < 0) return fail(c, MVD_ERR_ARG, "est_offset is negative");
    const int fl = fcntl(io->est_fd, F_GETFL);
    if ((fl & O_ACCMODE) == O_RDONLY) return fail(c, MVD_ERR_ARG, "est_fd is not open for writing");
    if (fl & O_APPEND) return fail(c, MVD_ERR_ARG, "est_fd is in append mode (positioned writes needed)");
  }
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  if (r->workspace && ((uintptr_t)r->workspace % kAlign))
    return fail(c, MVD_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
  const StreamLayout S = stream_layout_of(c, r, batch_planes, true);
  if (!r->workspace || r->workspace_bytes < S.total)
    return fail(c, MVD_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", S.total,
                r->workspace ? r->workspace_bytes : (size_t)0);
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);
  st = check_stream_weights(c, r);
  if (st != MVD_OK) return st;
  if (stream_resources(c) != hipSuccess) return fail(c, MVD_ERR_ALLOC, "cannot create copy streams or events");
  return run_files(c, io, r, batch_planes, (hipStream_t)stream);
}

// Test hook (mvd_testing.h): the launch geometry the planner picks for
// a separable pass over `n_planes` planes with kernel size k, so host-side tests
// can check every access of the kernels' index arithmetic against its buffer.
// out[16]: bucket, cols, threads, occ, zseg, nseg, x_out, nstrip, halo, ncols,
// ldsw, vec (for 16-byte aligned buffers), lds bytes per view.
// k < 0: the plan of a one-ring pass for kernel size −k (the forward pass and
// the one-plane backward, which may take rows up to 1024 wide in one work-group).
int mvd_internal_sep_plan(const mvd_ctx *c, int n_planes, int k, int boundary, int *out) {
  const bool one_ring = k < 0;
  k = one_ring ? -k : k;
  if (!c || !out || n_planes < 1 || k < 1 || k > MVD_MAX_K) return MVD_ERR_ARG;
  if (boundary != MVD_BOUNDARY_ZERO && boundary != MVD_BOUNDARY_PERIODIC) return MVD_ERR_ARG;
  const SepGeom sg = plan_sep(c, n_planes, sep_bucket(k), boundary, tune(), one_ring);
  out[0] = sg.plan.bucket;
  out[1] = sg.plan.cols;
  out[2] = sg.plan.threads;
  out[3] = sg.plan.occ;
  out[4] = sg.zseg;
  out[5] = sg.nseg;
  out[6] = sg.x_out;
  out[7] = sg.nstrip;
  out[8] = sg.halo;
  out[9] = sg.ncols;
  out[10] = sg.ldsw;
  out[11] = whole_items(sg, PlaneGeom{n_planes, c->Z, c->X}) ? 1 : 0;
  out[12] = (int)sep_lds_per_view(sg);
  return MVD_OK;
}


// Test hook (mvd_testing.h): the matrix-core general pass's plan for a
// kz × kx kernel, for the host-side bounds model.  out[3]: column steps, input
// tile row pitch, LDS bytes.
int mvd_internal_mfma_plan(int kz, int kx, int *out) {
  if (!out || kz < 1 || kx < 1 || kz > MVD_MAX_K || kx > MVD_MAX_K) return MVD_ERR_ARG;
  out[0] = mfma_chunks(kx);
  out[1] = mfma_tile_width(out[0]);
  out[2] = (int)mfma_lds_bytes(kz, kx);
  return MVD_OK;
}

int mvd_internal_version(void) { return MVD_TESTING_VERSION; }

int mvd_internal_fused_plan(const mvd_ctx *c, int kb, int *out) {
  if (!c || !out) return MVD_ERR_ARG;
  if (kb != 3 && kb != 7 && kb != 11 && kb != 15 && kb != 21 && kb != 31) return MVD_ERR_UNSUPPORTED;
  const int R = (kb - 1) / 2, RA = (R + 7) / 8 * 8;
  out[0] = kb;
  out[1] = kFusedStrip;
  out[2] = (c->X + kFusedStrip - 1) / kFusedStrip;
  out[3] = R;
  out[4] = RA;
  out[5] = fused_pitch(kb);
  out[6] = (int)fused_lds_bytes(kb, out[5]);
  out[7] = kFusedThreads;
  return MVD_OK;
}

int mvd_internal_psf_terms(mvd_ctx *c, int view, int which, float *out, int cap) {
  if (!c || view < 0 || view >= c->nv || !c->derived || (which != 0 && which != 1)) return MVD_ERR_ARG;
  const ViewPsf &w = c->views[view];
  const bool one = which == 0 ? w.sep_p : w.sep_x;
  const auto &zs = which == 0 ? w.lpz : w.lxz;
  const auto &xs = which == 0 ? w.lpx : w.lxx;
  const int R = one ? 1 : (int)zs.size();
  if (out) {
    const Kernel &k = which == 0 ? w.psf : w.back;
    long o = 0;
    for (int t = 0; t < R && t < cap; ++t) {
      const std::vector<float> &fz = one ? (which == 0 ? w.pz : w.xz) : zs[t];
      const std::vector<float> &fx = one ? (which == 0 ? w.px : w.xx) : xs[t];
      for (int j = 0; j < k.kz; ++j) out[o++] = fz[j];
      for (int i = 0; i < k.kx; ++i) out[o++] = fx[i];
    }
  }
  return R;
}

int mvd_internal_set_pq_spin(unsigned polls) {
  g_pq_spin.store(polls);
  return MVD_OK;
}

int mvd_internal_batch_raise_giveup(mvd_batch *b) {
  if (!b || !b->persistent) return MVD_ERR_ARG;
  DeviceGuard dg(b->device);
  return hipMemset(b->pq.q.giveup, 1, sizeof(unsigned)) == hipSuccess ? MVD_OK : MVD_ERR_LAUNCH;
}

long mvd_internal_pq_order(int n_jobs, const int *n_planes, const int *nseg, const int *nstrip, const int *pair,
                           const int *per_iter, const int *iters, int window, int *out, long cap) {
  if (n_jobs < 1 || !n_planes || !nseg || !nstrip || !pair || !per_iter || !iters) return MVD_ERR_ARG;
  std::vector<PqJob> jobs(n_jobs);
  std::vector<int> win(n_jobs), it(iters, iters + n_jobs);
  for (int k = 0; k < n_jobs; ++k) {
    if (n_planes[k] < 1 || nseg[k] < 1 || nstrip[k] < 1 || per_iter[k] < 1 || iters[k] < 0) return MVD_ERR_ARG;
    jobs[k].g = PlaneGeom{n_planes[k], 1, 1};
    jobs[k].nseg = nseg[k];
    jobs[k].nstrip = nstrip[k];
    jobs[k].ntiles = nseg[k] * nstrip[k];
    jobs[k].pair = pair[k] ? 1 : 0;
    jobs[k].per_iter = per_iter[k];
    win[k] = window > 0 ? std::min(window, n_planes[k]) : n_planes[k];
  }
  const std::vector<int4> items = pq_items(jobs, win, it);
  if (out)
    for (long i = 0; i < (long)items.size() && i < cap; ++i) {
      out[4 * i] = items[i].x;
      out[4 * i + 1] = items[i].y;
      out[4 * i + 2] = items[i].z;
      out[4 * i + 3] = items[i].w;
    }
  return (long)items.size();
}

int mvd_internal_tune_probe_bytes(const mvd_ctx *c, const mvd_run *r, size_t *bytes) {
  if (!c || !r || !bytes || r->struct_size != sizeof(mvd_run) || r->n_planes < 1 || r->n_iters < 0)
    return MVD_ERR_ARG;
  mvd_run probe;
  *bytes = tune_probe(r, &probe) ? layout_of(c, &probe).total : 0;
  return MVD_OK;
}

// Calibration hook (mvd_testing.h): a copy (kind 0) or read-only sweep (kind 1)
// of `bytes` on the caller's stream.
int mvd_internal_stream_probe(int kind, const void *src, void *dst, size_t bytes, void *stream) {
  if ((kind != 0 && kind != 1) || !src || !dst || bytes % 16 != 0 || !aligned16(src) || !aligned16(dst))
    return MVD_ERR_ARG;
  return launch_stream_probe(kind, src, dst, bytes, static_cast<hipStream_t>(stream)) == hipSuccess
             ? MVD_OK
             : MVD_ERR_LAUNCH;
}

// Test hook (mvd_testing.h): replace the process-wide launch-shape overrides (the MVD_TUNE
// syntax; NULL: re-read the environment).  Lets one process compare the
// alternative forms of a pass; not thread-safe against running calls.
int mvd_internal_set_tune(const char *spec) {
  tune_mut() = parse_tune(spec ? spec : std::getenv("MVD_TUNE"));
  return MVD_OK;
}

// Test hook (mvd_testing.h): the matrix-core tap-gradient correlation's launch for a volume of
// n_planes × Z × X and a kz × kx kernel.  out[7]: kzp, kxp, tile width, tiles
// per z run, work items, work-groups, LDS bytes.
int mvd_internal_corr_plan(int n_planes, int Z, int X, int kz, int kx, long *out) {
  if (!out || n_planes < 1 || Z < 1 || X < 1 || kz < 1 || kx < 1 || kz > MVD_MAX_K || kx > MVD_MAX_K)
    return MVD_ERR_ARG;
  const CorrMfmaShape m = corr_mfma_shape(PlaneGeom{n_planes, Z, X}, kz, kx, kCorrMfmaBlocks);
  const long v[7] = {m.kzp, m.kxp, m.tw, m.zch, m.nitems, m.nblocks, (long)m.lds};
  for (int i = 0; i < 7; ++i) out[i] = v[i];
  return MVD_OK;
}

// Test hook (mvd_testing.h): the split-view backward plan (same out[] layout as the separable
// plan; returns MVD_ERR_UNSUPPORTED where the form does not apply).
int mvd_internal_split_plan(const mvd_ctx *c, int n_planes, int k, int *out) {
  if (!c || !out || n_planes < 1 || k < 1 || k > MVD_MAX_K) return MVD_ERR_ARG;
  SepGeom sg = plan_sep(c, n_planes, sep_bucket(k), MVD_BOUNDARY_ZERO);
  if (sg.plan.cols != 1) {   // the split form's own one-column strips
    Tune t1 = tune();
    t1.cols = 1;
    sg = plan_sep(c, n_planes, sep_bucket(k), MVD_BOUNDARY_ZERO, t1);
  }
  SepGeom sp;
  if (!split_geom(sg, PlaneGeom{n_planes, c->Z, c->X}, MVD_BOUNDARY_ZERO, &sp)) return MVD_ERR_UNSUPPORTED;
  const int v[13] = {sp.plan.bucket, sp.plan.cols, sp.plan.threads, sp.plan.occ, sp.zseg, sp.nseg, sp.x_out,
                     sp.nstrip, sp.halo, sp.ncols, sp.ldsw, whole_items(sp, PlaneGeom{n_planes, c->Z, c->X}) ? 1 : 0,
                     (int)split_lds_bytes(sp)};
  for (int i = 0; i < 13; ++i) out[i] = v[i];
  return MVD_OK;
}

mvd_status mvd_backward_workspace_bytes(const mvd_ctx *cc, const mvd_run *r, size_t *bytes) {
  mvd_ctx *c = const_cast<mvd_ctx *>(cc);
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!bytes) return fail(c, MVD_ERR_ARG, "bytes is NULL");
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  *bytes = bwd_layout_of(c, r).total;
  return MVD_OK;
}

mvd_status mvd_backward(mvd_ctx *c, const void *const *obs, const float *grad_est, const mvd_run *r,
                        float *const *grad_psf, float *const *grad_back, float *grad_weights,
                        float *grad_init, void *stream) {
  mvd_grads out{};
  out.struct_size = sizeof(mvd_grads);
  out.grad_psf = grad_psf;
  out.grad_back = grad_back;
  out.grad_weights = grad_weights;
  out.grad_init = grad_init;
  return mvd_backward_grads(c, obs, grad_est, r, &out, stream);
}

mvd_status mvd_backward_grads(mvd_ctx *c, const void *const *obs, const float *grad_est, const mvd_run *r,
                              const mvd_grads *out, void *stream) {
  if (!c) return fail(nullptr, MVD_ERR_ARG, "ctx is NULL");
  c->err.clear();
  if (!out || out->struct_size != sizeof(mvd_grads))
    return fail(c, MVD_ERR_ARG, "out is NULL or its struct_size is not sizeof(mvd_grads)");
  float *const *grad_psf = out->grad_psf;
  float *const *grad_back = out->grad_back;
  float *grad_weights = out->grad_weights;
  float *grad_init = out->grad_init;
  float *const *grad_wpl = out->grad_weight_planes;
  mvd_status st = check_run(c, r);
  if (st != MVD_OK) return st;
  if (grad_wpl) {
    if (!r->weight_planes) return fail(c, MVD_ERR_ARG, "grad_weight_planes needs run->weight_planes");
    for (int v = 0; v < c->nv; ++v)
      if (!grad_wpl[v]) return fail(c, MVD_ERR_ARG, "grad_weight_planes[%d] is NULL", v);
  }
  if (!obs || !grad_est) return fail(c, MVD_ERR_ARG, "obs or grad_est is NULL");
  for (int v = 0; v < c->nv; ++v)
    if (!obs[v]) return fail(c, MVD_ERR_ARG, "obs[%d] is NULL", v);
  if (r->n_iters < 1) return fail(c, MVD_ERR_ARG, "n_iters must be >= 1 for the reverse sweep");
  if (!r->checkpoints) return fail(c, MVD_ERR_ARG, "run->checkpoints must hold psi^0..psi^{T-1}");
  if (!c->derived) return fail(c, MVD_ERR_STATE, "not every view has a PSF");
  const BwdLayout L = bwd_layout_of(c, r);
  if (!r->workspace || r->workspace_bytes < L.total)
    return fail(c, MVD_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                r->workspace ? r->workspace_bytes : (size_t)0);
  if ((uintptr_t)r->workspace % kAlign) return fail(c, MVD_ERR_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (c->device == MVD_DEVICE_NONE) return fail(c, MVD_ERR_DEVICE, "host-only context");
  DeviceGuard dg(c->device);
  if (!dg.ok()) return fail(c, MVD_ERR_DEVICE, "cannot select device %d", c->device);

  hipStream_t s = (hipStream_t)stream;
  const PlaneGeom g{r->n_planes, c->Z, c->X};
  const size_t n = (size_t)g.Y * g.Z * g.X;
  char *ws = static_cast<char *>(r->workspace);
  // launch shapes: those the autotuner chose for the forward run of the same
  // workload, if it ran (the reverse sweep's passes have the same shapes)
  Tune tn = tune();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(c, r));
    if (it != g_tune_cache.end()) tn = it->second;
  }
  RunState rs{c, g, r->boundary, false, s, r->view_weights, (r->flags & MVD_FLAG_TIMING) != 0, &tn};
  rs.wpl = r->weight_planes;   // the sequential sub-states are tempered as in the forward call
  rs.normalize = L.normalize;  // and normalised
  if (L.low_rank) rs.acc = reinterpret_cast<float *>(ws + L.tmp_off);   // partial sums of terms
  const int V = c->nv;
  const bool sim = r->update == MVD_UPDATE_SIMULTANEOUS;
  const int wp = !r->weight_planes ? 0 : (grad_wpl ? 2 : 1);
  auto plane = [&](size_t off, int k) { return reinterpret_cast<float *>(ws + off + (size_t)k * L.plane_set); };
  double *acc = reinterpret_cast<double *>(ws + L.acc_off);
  double *wpart = reinterpret_cast<double *>(ws + L.wpart_off);
  const bool want_psf = grad_psf != nullptr, want_back = grad_back != nullptr;

  std::vector<const float *> phi(V);
  std::vector<float *> staged(V);
  for (int v = 0; v < V; ++v) {
    staged[v] = plane(L.phi_off, v);
    phi[v] = staged[v];
  }
  hipError_t e = launch_zero_f64(acc, (int)(acc_w(c) + V), s);
  if (e == hipSuccess) e = launch_stage_views(obs, V, r->obs_dtype, r->obs_layout, g, staged.data(), nullptr, s);
  int cur = 0;
  if (e == hipSuccess) e = launch_copy(grad_est, plane(L.g_off, 0), n, s);
  for (int v = 0; v < V && e == hipSuccess && grad_wpl; ++v) e = launch_fill(grad_wpl[v], n, 0.f, s);
  if (e == hipSuccess && L.normalize) e = launch_fill(plane(L.ones_off, 0), n, 1.f, s);
  // sensitivity planes 1 ⊛ X_v of back-projectors that are not rank one (the
  // others have separable factors); the first two planes are the sequential
  // sub-states' scratch
  auto sens_of = [&](int v) {
    return reinterpret_cast<float *>(ws + L.sens_off + (size_t)(2 + v) * sens_plane_bytes(c));
  };
  if (L.sens) {
    rs.sens = reinterpret_cast<float *>(ws + L.sens_off);
    for (int v = 0; v < V && e == hipSuccess; ++v)
      if (!c->views[v].sep_x) e = sens_plane(rs, v, rs.sens, sens_of(v));
  }
  // the normalisation's factors as the pointwise kernels read them
  auto set_norm = [&](AdjPointArgs &pa, int slot, int v) {
    pa.nrm = L.normalize ? 1 : 0;
    pa.Z = c->Z;
    pa.X = c->X;
    if (!L.normalize) return;
    if (c->views[v].sep_x) {
      pa.nsz[slot] = norm_factors(c, v, r->boundary);
      pa.nsx[slot] = pa.nsz[slot] + norm_zlen(c);
    } else {
      pa.nsp[slot] = sens_of(v);
    }
    pa.sbar[slot] = plane(L.sbar_off, L.nsets > 1 ? v : 0);
  };
  const int T = r->n_iters;
  for (int t = T - 1; t >= 0 && e == hipSuccess; --t) {
    const float *psi = r->checkpoints + (size_t)t * n;
    if (sim) {
      std::vector<ViewBufs> vb(V);
      for (int v = 0; v < V && e == hipSuccess; ++v) {
        vb[v] = ViewBufs{plane(L.b_off, v), plane(L.r_off, v), plane(L.q_off, v)};
        e = view_recompute(rs, v, psi, phi[v], vb[v]);
      }
      if (e != hipSuccess) break;
      AdjPointArgs pa{};
      pa.n = n;
      pa.nv = V;
      pa.psi = psi;
      pa.gbar_in = plane(L.g_off, cur);
      pa.gbar_out = plane(L.g_off, 1 - cur);
      for (int v = 0; v < V; ++v) {
        pa.q[v] = vb[v].q;
        pa.w[v] = weight_of(rs, v);
        if (wp >= 1) pa.wpl[v] = r->weight_planes[v];
        if (wp == 2) pa.gwpl[v] = grad_wpl[v];
        set_norm(pa, v, v);
      }
      pa.wp = wp;
      pa.wpart = wpart;
      e = timed(rs, 3, [&] { return launch_pointwise_sim(pa, kPointBlocks, s); });
      if (e == hipSuccess) e = launch_sum_partials(wpart, kPointBlocks, V, acc + acc_w(c), s);
      for (int v = 0; v < V && e == hipSuccess; ++v)
        e = view_backprop(rs, L, ws, v, psi, vb[v], plane(L.g_off, 1 - cur), want_psf, want_back,
                          L.normalize ? plane(L.sbar_off, v) : nullptr);
      cur = 1 - cur;
    } else {
      // sub-states ψ_v of the sequential sweep: ψ_0 = ψ^t, ψ_{v+1} = ψ_v · c_v(ψ_v)
      std::vector<const float *> sub(V);
      sub[0] = psi;
      float *rat = plane(L.rat_off, 0);
      for (int v = 0; v + 1 < V && e == hipSuccess; ++v) {
        float *dst = plane(L.sub_off, v);
        std::vector<float *> rv(V, rat);
        e = forward_views(rs, sub[v], obs_staged(staged.data(), g), rv.data(), v, 1);
        if (e == hipSuccess) e = backward_views(rs, rv.data(), sub[v], dst, v, 1);
        sub[v + 1] = dst;
      }
      const ViewBufs vb{plane(L.b_off, 0), plane(L.r_off, 0), plane(L.q_off, 0)};
      for (int v = V - 1; v >= 0 && e == hipSuccess; --v) {
        e = view_recompute(rs, v, sub[v], phi[v], vb);
        if (e != hipSuccess) break;
        AdjPointArgs pa{};
        pa.n = n;
        pa.nv = 1;
        pa.psi = sub[v];
        pa.gbar_in = plane(L.g_off, cur);
        pa.gbar_out = plane(L.g_off, 1 - cur);
        pa.q[0] = vb.q;
        pa.w[0] = weight_of(rs, v);
        pa.wp = wp;
        if (wp >= 1) pa.wpl[0] = r->weight_planes[v];
        if (wp == 2) pa.gwpl[0] = grad_wpl[v];
        set_norm(pa, 0, v);
        pa.wpart = wpart;
        e = timed(rs, 3, [&] { return launch_pointwise_seq(pa, kPointBlocks, s); });
        if (e == hipSuccess) e = launch_sum_partials(wpart, kPointBlocks, 1, acc + acc_w(c) + v, s);
        if (e == hipSuccess)
          e = view_backprop(rs, L, ws, v, sub[v], vb, plane(L.g_off, 1 - cur), want_psf, want_back,
                            L.normalize ? plane(L.sbar_off, 0) : nullptr);
        cur = 1 - cur;
      }
    }
  }
  for (int v = 0; v < V && e == hipSuccess; ++v) {
    const ViewPsf &w = c->views[v];
    if (want_psf && grad_psf[v]) e = launch_to_f32(acc + acc_psf(c, v), grad_psf[v], w.psf.kz * w.psf.kx, s);
    if (e == hipSuccess && want_back && grad_back[v])
      e = launch_to_f32(acc + acc_back(c, v), grad_back[v], w.back.kz * w.back.kx, s);
  }
  if (e == hipSuccess && grad_weights) e = launch_to_f32(acc + acc_w(c), grad_weights, V, s);
  if (e == hipSuccess && grad_init) e = launch_copy(plane(L.g_off, cur), grad_init, n, s);
  if (e != hipSuccess) return fail(c, MVD_ERR_LAUNCH, "launch failed: %s", hipGetErrorString(e));
  return MVD_OK;
}


mvd_status mvd_batch_create(mvd_batch **out, const mvd_item *items, int n_items, uint32_t flags, void *stream) {
  if (!out) return fail(nullptr, MVD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!items || n_items < 1 || n_items > 64) return fail(nullptr, MVD_ERR_ARG, "need 1..64 items");
  if (flags & ~(MVD_BATCH_TUNE | MVD_BATCH_GRAPH)) return fail(nullptr, MVD_ERR_ARG, "unknown batch flags 0x%x", flags);
  const int dev = items[0].ctx ? items[0].ctx->device : -1;
  for (int i = 0; i < n_items; ++i) {
    mvd_ctx *c = items[i].ctx;
    if (!c) return fail(nullptr, MVD_ERR_ARG, "item %d: ctx is NULL", i);
    c->err.clear();
    mvd_status st = validate_run(c, items[i].obs, items[i].est, items[i].run);
    if (st != MVD_OK) return fail(nullptr, st, "item %d: %s", i, c->err.c_str());
    if (items[i].run->flags & (MVD_FLAG_TIMING | MVD_FLAG_GRAPH))
      return fail(nullptr, MVD_ERR_ARG, "item %d: timing and graph flags are not batch item flags", i);
    if (c->device != dev) return fail(nullptr, MVD_ERR_ARG, "item %d: all items must share one device", i);
  }
  DeviceGuard dg(dev);
  if (!dg.ok()) return fail(nullptr, MVD_ERR_DEVICE, "cannot select device %d", dev);
  mvd_batch *b = new (std::nothrow) mvd_batch;
  if (!b) return fail(nullptr, MVD_ERR_ALLOC, "out of host memory");
  b->device = dev;
  for (int i = 0; i < n_items; ++i) {
    mvd_batch::Item it;
    it.ctx = items[i].ctx;
    it.serial = it.ctx->serial;
    it.psf_generation = it.ctx->psf_generation;
    it.obs.assign(items[i].obs, items[i].obs + it.ctx->nv);
    it.est = items[i].est;
    it.run = *items[i].run;
    if (it.run.view_weights) {
      it.weights.assign(it.run.view_weights, it.run.view_weights + it.ctx->nv);
      it.run.view_weights = it.weights.data();
    }
    if (it.run.weight_planes) {
      it.wplanes.assign(it.run.weight_planes, it.run.weight_planes + it.ctx->nv);
      it.run.weight_planes = it.wplanes.data();
    }
    b->items.push_back(std::move(it));
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  // the persistent queue form where every item allows it, else the graph form
  bool pq = !(flags & MVD_BATCH_GRAPH);
  for (size_t i = 0; i < b->items.size() && pq; ++i) {
    const auto &it = b->items[i];
    std::string why;
    if (!pq_eligible(it.ctx, it.obs.data(), it.est, &it.run, &why)) {
      pq = false;
      b->why_graph = "item " + std::to_string(i) + ": " + why;
    }
  }
  // with MVD_BATCH_TUNE both forms are built and timed (unless an item's given
  // ψ^0 would be overwritten by the timing launches)
  bool both = (flags & MVD_BATCH_TUNE) != 0;
  for (const auto &it : b->items) both = both && it.run.init != MVD_INIT_GIVEN;
  if (pq) {
    e = pq_setup(b, tune().pq_window);
    if (e == hipSuccess) {
      b->persistent = true;
      if (!both) {
        *out = b;
        return MVD_OK;
      }
    } else {
      // a batch the persistent form cannot take runs as a graph
      b->why_graph = std::string("persistent setup: ") + hipGetErrorString(e);
      if (b->pq.dmem) (void)hipFree(b->pq.dmem);
      b->pq = PqState{};
      (void)hipGetLastError();
      e = hipSuccess;
    }
  }
  if (flags & MVD_BATCH_TUNE) {
    for (auto &it : b->items) {
      if (e != hipSuccess) break;
      if (it.run.init == MVD_INIT_GIVEN) continue;   // tuning would overwrite the given estimate
      e = autotune(it.ctx, it.obs.data(), it.est, &it.run, s, &it.tn);
    }
  }
  // one graph, one branch per item: fork from the capture stream, join back
  std::vector<hipStream_t> br(b->items.size(), nullptr);
  std::vector<hipEvent_t> join(b->items.size(), nullptr);
  hipEvent_t fork = nullptr;
  for (size_t i = 0; i < br.size() && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) {
    e = capture(
        [&](hipStream_t cs) {
          hipError_t ce = hipEventRecord(fork, cs);
          for (size_t i = 0; i < b->items.size() && ce == hipSuccess; ++i) {
            auto &it = b->items[i];
            ce = hipStreamWaitEvent(br[i], fork, 0);
            if (ce == hipSuccess) ce = enqueue_run(it.ctx, it.obs.data(), it.est, &it.run, br[i], it.tn);
            if (ce == hipSuccess) ce = hipEventRecord(join[i], br[i]);
            if (ce == hipSuccess) ce = hipStreamWaitEvent(cs, join[i], 0);
          }
          return ce;
        },
        &b->graph, &b->exec);
  }
  for (size_t i = 0; i < br.size(); ++i) {
    if (br[i]) (void)hipStreamDestroy(br[i]);
    if (join[i]) (void)hipEventDestroy(join[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (e != hipSuccess) {
    mvd_batch_destroy(b);
    return fail(nullptr, MVD_ERR_LAUNCH, "batch setup failed: %s", hipGetErrorString(e));
  }
  if (b->persistent) {
    // both forms exist: time each (one warm-up and two timed launches) and keep the faster
    double ms[2] = {0.0, 0.0};
    mvd_status st = MVD_OK;
    for (int form = 0; form < 2 && st == MVD_OK; ++form) {
      b->persistent = form == 0;
      st = batch_time_launches(b, s, &ms[form]);
    }
    if (st != MVD_OK) {
      const std::string msg = mvd_last_error(nullptr);
      mvd_batch_destroy(b);
      return fail(nullptr, st, "batch form timing failed: %s", msg.c_str());
    }
    b->form_ms[0] = ms[0];
    b->form_ms[1] = ms[1];
    b->persistent = ms[0] <= ms[1];
    if (b->persistent) {
      (void)hipGraphExecDestroy(b->exec);
      (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
    } else {
      (void)hipFree(b->pq.dmem);
      b->pq = PqState{};
      b->why_graph = "tuned: the graph form was faster";
    }
  }
  *out = b;
  return MVD_OK;
}

mvd_status mvd_batch_launch(mvd_batch *b, void *stream) {
  if (!b || (!b->exec && !b->persistent)) return fail(nullptr, MVD_ERR_ARG, "batch is NULL");
  {
    // the captured launches hold the items' taps and tap buffers: a context
    // destroyed or given new PSFs since capture invalidates the batch
    std::lock_guard<std::mutex> lk(g_live_mu);
    for (size_t i = 0; i < b->items.size(); ++i) {
      const auto &it = b->items[i];
      auto f = g_live.find(it.ctx);
      if (f == g_live.end() || f->second != it.serial)
        return fail(nullptr, MVD_ERR_STATE, "item %zu: its context was destroyed after the batch was created", i);
      if (it.ctx->psf_generation != it.psf_generation)
        return fail(nullptr, MVD_ERR_STATE, "item %zu: mvd_set_psf was called after the batch was created", i);
    }
  }
  DeviceGuard dg(b->device);
  if (b->persistent) {
    PqQueue q = b->pq.q;
    const unsigned lim = g_pq_spin.load();
    q.spin_limit = lim ? lim : kPqSpinDefault;
    hipError_t e = launch_pq(q, b->pq.nblocks, b->pq.lds, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, MVD_ERR_LAUNCH, "persistent launch failed: %s", hipGetErrorString(e));
    return MVD_OK;
  }
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, MVD_ERR_LAUNCH, "graph launch failed: %s", hipGetErrorString(e));
  return MVD_OK;
}

mvd_status mvd_batch_wait(mvd_batch *b, void *stream) {
  if (!b) return fail(nullptr, MVD_ERR_ARG, "batch is NULL");
  DeviceGuard dg(b->device);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, MVD_ERR_LAUNCH, "batch execution failed: %s", hipGetErrorString(e));
  if (b->persistent) {
    unsigned flag = 0;
    e = hipMemcpy(&flag, b->pq.q.giveup, sizeof(flag), hipMemcpyDeviceToHost);
    if (e == hipSuccess && flag) e = hipMemset(b->pq.q.giveup, 0, sizeof(unsigned));
    if (e != hipSuccess) return fail(nullptr, MVD_ERR_LAUNCH, "batch status read failed: %s", hipGetErrorString(e));
    if (flag) return fail(nullptr, MVD_ERR_LAUNCH, "persistent batch: a work-group gave up waiting for a dependency");
  }
  return MVD_OK;
}

mvd_status mvd_batch_info(const mvd_batch *b, int *out) {
  if (!b || !out) return fail(nullptr, MVD_ERR_ARG, "batch or out is NULL");
  out[0] = b->persistent ? 1 : 0;
  out[1] = b->persistent ? b->pq.q.n_items : 0;
  out[2] = b->persistent ? b->pq.nblocks : 0;
  out[3] = b->persistent ? (int)b->pq.lds : 0;
  return MVD_OK;
}

mvd_status mvd_batch_form_times(const mvd_batch *b, double *out) {
  if (!b || !out) return fail(nullptr, MVD_ERR_ARG, "batch or out is NULL");
  out[0] = b->form_ms[0];
  out[1] = b->form_ms[1];
  return MVD_OK;
}

mvd_status mvd_batch_tuning(const mvd_batch *b, int item, int *out) {
  if (!b || !out || item < 0 || item >= (int)b->items.size()) return fail(nullptr, MVD_ERR_ARG, "bad batch item");
  const Tune &t = b->items[item].tn;
  out[0] = t.fwd_occ;
  out[1] = t.fwd_views;
  out[2] = t.bwd_vin;
  out[3] = t.zseg_scale;
  out[4] = t.cols;
  return MVD_OK;
}

void mvd_batch_destroy(mvd_batch *b) {
  if (!b) return;
  DeviceGuard dg(b->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->pq.dmem) (void)hipFree(b->pq.dmem);
  delete b;
}

mvd_status mvd_batch_run(const mvd_item *items, int n_items, void *stream) {
  mvd_batch *b = nullptr;
  mvd_status st = mvd_batch_create(&b, items, n_items, 0, stream);
  if (st != MVD_OK) return st;
  st = mvd_batch_launch(b, stream);
  const mvd_status w = mvd_batch_wait(b, stream);
  if (st == MVD_OK) st = w;
  mvd_batch_destroy(b);
  return st;
}

const char *mvd_last_error(const mvd_ctx *c) {
  if (!c) return g_noctx_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
