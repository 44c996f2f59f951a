// Host CSR matrices and the smoothed-aggregation setup (amg.cpp).
#pragma once

#include <vector>

#include "dgnp_impl.hpp"

namespace dgnp {

struct Csr {
  int n = 0, m = 0;  // rows, columns
  std::vector<int> rp, ci;
  std::vector<double> v;
};

struct AmgHierarchy {
  std::vector<Csr> A;      // A[0] = finest scalar level
  std::vector<Csr> P, R;   // P[l]: level l+1 -> level l, R[l] = P[l]^T
  std::vector<std::vector<double>> dinv;
  std::vector<double> lmax;   // largest eigenvalue estimate of D^{-1} A per level
  std::vector<double> coarse_inv;  // dense row-major inverse of A.back()
};

Csr csr_transpose(const Csr& A);
Csr csr_matmul(const Csr& A, const Csr& B);
double lmax_dinvA(const Csr& A, const std::vector<double>& dinv, int iters);
AmgHierarchy sa_setup(const Csr& A1, int max_levels, int coarse_size, double theta);

}  // namespace dgnp
