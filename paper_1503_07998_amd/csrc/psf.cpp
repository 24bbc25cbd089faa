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

// Singular value decomposition of k (kz × kx) by one-sided Jacobi rotations
// (Hestenes): columns of A = k are rotated pairwise until orthogonal; then
// σ_i = |a_i|, v_i = the accumulated rotations' column i, u_i = a_i / σ_i.
// Small matrices (at most 63 × 63), float64, converged to 1e-15.
static void jacobi_svd(const Kernel &k, std::vector<double> *sv, std::vector<std::vector<double>> *U,
                       std::vector<std::vector<double>> *V) {
  const int m = k.kz, n = k.kx;
  std::vector<std::vector<double>> a(n, std::vector<double>(m)), v(n, std::vector<double>(n, 0.0));
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < m; ++j) a[i][j] = k.at(j, i);
    v[i][i] = 1.0;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int j = 0; j < m; ++j) {
          alpha += a[p][j] * a[p][j];
          beta += a[q][j] * a[q][j];
          gamma += a[p][j] * a[q][j];
        }
        if (gamma == 0.0 || std::fabs(gamma) <= 1e-15 * std::sqrt(alpha * beta)) continue;
        off = std::max(off, std::fabs(gamma) / std::sqrt(alpha * beta));
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int j = 0; j < m; ++j) {
          const double x = a[p][j], y = a[q][j];
          a[p][j] = c * x - s * y;
          a[q][j] = s * x + c * y;
        }
        for (int j = 0; j < n; ++j) {
          const double x = v[p][j], y = v[q][j];
          v[p][j] = c * x - s * y;
          v[q][j] = s * x + c * y;
        }
      }
    if (off <= 1e-15) break;
  }
  std::vector<int> order(n);
  std::vector<double> norm(n);
  for (int i = 0; i < n; ++i) {
    double s2 = 0.0;
    for (int j = 0; j < m; ++j) s2 += a[i][j] * a[i][j];
    norm[i] = std::sqrt(s2);
    order[i] = i;
  }
  std::sort(order.begin(), order.end(), [&](int x, int y) { return norm[x] > norm[y]; });
  sv->clear();
  U->clear();
  V->clear();
  for (int i : order) {
    sv->push_back(norm[i]);
    std::vector<double> u(m, 0.0);
    if (norm[i] > 0.0)
      for (int j = 0; j < m; ++j) u[j] = a[i][j] / norm[i];
    U->push_back(u);
    V->push_back(v[i]);
  }
}

// The fewest rank-one terms Σ_t u_t ⊗ v_t (from the SVD, each term's factors
// scaled by √σ_t) that reproduce every tap to tol · max|k|, at most rmax of
// them; false if more are needed.
bool low_rank(const Kernel &k, int rmax, double tol, std::vector<std::vector<double>> *us,
              std::vector<std::vector<double>> *vs) {
  double amax = 0.0;
  for (double e : k.t) amax = std::max(amax, std::fabs(e));
  if (!(amax > 0.0)) return false;
  std::vector<double> sv;
  std::vector<std::vector<double>> U, V;
  jacobi_svd(k, &sv, &U, &V);
  std::vector<double> approx(k.t.size(), 0.0);
  us->clear();
  vs->clear();
  for (int r = 0; r < rmax && r < (int)sv.size(); ++r) {
    const double sq = std::sqrt(sv[r]);
    std::vector<double> u(U[r]), v(V[r]);
    for (double &e : u) e *= sq;
    for (double &e : v) e *= sq;
    us->push_back(u);
    vs->push_back(v);
    double err = 0.0;
    for (int j = 0; j < k.kz; ++j)
      for (int i = 0; i < k.kx; ++i) {
        double &ap = approx[(size_t)j * k.kx + i];
        ap += u[j] * v[i];
        err = std::max(err, std::fabs(ap - k.at(j, i)));
      }
    if (err <= tol * amax) return true;
  }
  return false;
}

}  // namespace mvd
