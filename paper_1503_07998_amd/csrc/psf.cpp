// Host-side PSF algebra in float64: point reflection, compound back-projectors
// (Supplementary Note 2 §1) and the rank-one test that decides whether a kernel
// runs as two 1D passes.
#include "psf.hpp"

#include <algorithm>
#include <cmath>

namespace mvd {

Kernel flip(const Kernel &k) {
  Kernel o{k.kz, k.kx, std::vector<double>(k.t.size())};
  for (int j = 0; j < k.kz; ++j)
    for (int i = 0; i < k.kx; ++i) o.at(j, i) = k.at(k.kz - 1 - j, k.kx - 1 - i);
  return o;
}

Kernel conv_full(const Kernel &a, const Kernel &b) {
  Kernel o{a.kz + b.kz - 1, a.kx + b.kx - 1, {}};
  o.t.assign((size_t)o.kz * o.kx, 0.0);
  for (int j = 0; j < a.kz; ++j)
    for (int i = 0; i < a.kx; ++i) {
      const double w = a.at(j, i);
      if (w == 0.0) continue;
      for (int q = 0; q < b.kz; ++q)
        for (int p = 0; p < b.kx; ++p) o.at(j + q, i + p) += w * b.at(q, p);
    }
  return o;
}

Kernel crop_center(const Kernel &a, int kz, int kx) {
  Kernel o{kz, kx, std::vector<double>((size_t)kz * kx, 0.0)};
  const int cz = (a.kz - 1) / 2, cx = (a.kx - 1) / 2;
  const int rz = (kz - 1) / 2, rx = (kx - 1) / 2;
  for (int j = 0; j < kz; ++j) {
    const int sj = cz - rz + j;
    if (sj < 0 || sj >= a.kz) continue;
    for (int i = 0; i < kx; ++i) {
      const int si = cx - rx + i;
      if (si < 0 || si >= a.kx) continue;
      o.at(j, i) = a.at(sj, si);
    }
  }
  return o;
}

// X_v for the compound modes.  W_v = all views except v; ⊙ is the pixel-wise
// product, C the centred crop to P_v's size, N the division by the sum.
bool compound_back(const std::vector<Kernel> &psfs, int v, int mode, Kernel *out) {
  const Kernel fv = flip(psfs[v]);
  const int nv = (int)psfs.size();
  Kernel x = fv;
  if (mode == 3) {  // Optimization II: (P_v^*)^{⊙V}
    for (double &e : x.t) e = std::pow(e, (double)nv);
  } else if (mode == 1 || mode == 2) {  // Efficient Bayesian / Optimization I
    for (int w = 0; w < nv; ++w) {
      if (w == v) continue;
      Kernel c = conv_full(fv, psfs[w]);
      if (mode == 1) c = conv_full(c, flip(psfs[w]));
      const Kernel cc = crop_center(c, fv.kz, fv.kx);
      for (size_t e = 0; e < x.t.size(); ++e) x.t[e] *= cc.t[e];
    }
  } else {
    return false;
  }
  double s = 0.0;
  for (double e : x.t) s += e;
  if (!(s > 0.0) || !std::isfinite(s)) return false;
  for (double &e : x.t) e /= s;
  *out = x;
  return true;
}

// Rank-one test: pivot on the largest tap a[p][q]; u_j = a[j][q],
// v_i = a[p][i] / a[p][q].  Accept when every tap is reproduced to 1e-6
// relative (plus 1e-12 of the largest tap), then balance the two factors to
// equal sums.
bool rank_one(const Kernel &k, std::vector<double> *u, std::vector<double> *v) {
  int p = 0, q = 0;
  double amax = -1.0;
  for (int j = 0; j < k.kz; ++j)
    for (int i = 0; i < k.kx; ++i)
      if (k.at(j, i) > amax) {
        amax = k.at(j, i);
        p = j;
        q = i;
      }
  if (!(amax > 0.0)) return false;
  std::vector<double> uu(k.kz), vv(k.kx);
  for (int j = 0; j < k.kz; ++j) uu[j] = k.at(j, q);
  for (int i = 0; i < k.kx; ++i) vv[i] = k.at(p, i) / amax;
  for (int j = 0; j < k.kz; ++j)
    for (int i = 0; i < k.kx; ++i) {
      const double a = k.at(j, i), r = uu[j] * vv[i];
      if (std::fabs(a - r) > 1e-6 * std::fabs(a) + 1e-12 * amax) return false;
    }
  double su = 0.0, sv = 0.0;
  for (double e : uu) su += e;
  for (double e : vv) sv += e;
  const double s = std::sqrt(su / sv);
  for (double &e : uu) e /= s;
  for (double &e : vv) e *= s;
  *u = uu;
  *v = vv;
  return true;
}

}  // namespace mvd
