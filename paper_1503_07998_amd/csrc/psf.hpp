// Host-side PSF algebra (float64).  Internal.
#pragma once

#include <vector>

namespace mvd {

struct Kernel {
  int kz = 0, kx = 0;
  std::vector<double> t;  // [kz][kx]
  double &at(int j, int i) { return t[(size_t)j * kx + i]; }
  double at(int j, int i) const { return t[(size_t)j * kx + i]; }
};

Kernel flip(const Kernel &k);
Kernel conv_full(const Kernel &a, const Kernel &b);
Kernel crop_center(const Kernel &a, int kz, int kx);
// mode: 1 efficient Bayesian, 2 optimization I, 3 optimization II
bool compound_back(const std::vector<Kernel> &psfs, int v, int mode, Kernel *out);
bool rank_one(const Kernel &k, std::vector<double> *u, std::vector<double> *v);
// The fewest rank-one terms u_t ⊗ v_t from k's SVD reproducing every tap to
// tol · max|k| (at most rmax; false if more are needed).
bool low_rank(const Kernel &k, int rmax, double tol, std::vector<std::vector<double>> *us,
              std::vector<std::vector<double>> *vs);

}  // namespace mvd
