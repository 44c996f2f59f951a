// Host CSR matrices and the smoothed-aggregation setup (amg.cpp).
#pragma once

#include <functional>
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
  std::vector<Csr> work;  // the products A_l P_l, kept for the next set-up
};

// fn(first row, end row) over chunks of rows [0, n) on the host worker pool
// (row-independent work only)
void host_parallel_rows(int n, const std::function<void(int, int)>& fn);
Csr csr_transpose(const Csr& A);
// the same built in the arrays of `storage` (any earlier matrix)
Csr csr_transpose(const Csr& A, Csr&& storage);
Csr csr_matmul(const Csr& A, const Csr& B);
// the same product built in the arrays of `storage` (any earlier matrix)
Csr csr_matmul(const Csr& A, const Csr& B, Csr&& storage);
// inverse of a square CSR matrix as a dense row-major array: Cholesky when it is
// positive definite (banded when its entries lie within a third of the order of
// the diagonal), else Gauss-Jordan with partial pivoting; throws when singular
std::vector<double> dense_inverse(const Csr& A);
// power iterations for the largest eigenvalue of D^{-1} A; x_io (may be null):
// start vector in (used when its size matches), last vector out
double lmax_dinvA(const Csr& A, const std::vector<double>& dinv, int iters, std::vector<double>* x_io = nullptr);
// x0 (may be null) receives the finest level's last power-iteration vector;
// recycle (may be null) lends the arrays of an earlier hierarchy, which is
// left without a usable hierarchy (the result does not depend on it)
AmgHierarchy sa_setup(Csr A1, int max_levels, int coarse_size, double theta,
                      std::vector<double>* x0 = nullptr, AmgHierarchy* recycle = nullptr);
// the same hierarchy shape for a new finest matrix with the aggregates and
// prolongators of prev kept: only the Galerkin products, smoother data and
// coarse inverse are recomputed; the finest estimate warm-starts from x0
AmgHierarchy sa_setup_reuse(Csr A1, const AmgHierarchy& prev, std::vector<double>* x0);
// the same, taking prev's prolongators and product arrays instead of copying
// them (prev is left without a usable hierarchy)
AmgHierarchy sa_setup_reuse(Csr A1, AmgHierarchy&& prev, std::vector<double>* x0);

}  // namespace dgnp
