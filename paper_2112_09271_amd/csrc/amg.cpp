// Host setup of the smoothed-aggregation algebraic multigrid hierarchy used
// for the potential block (the paper applies AMG to A_phiphi, Sec. 4.1; this is
// smoothed aggregation in the sense of Vanek, Mandel and Brezina, 1996):
// symmetric strength of connection, greedy three-phase aggregation, piecewise
// constant tentative prolongator, damped-Jacobi smoothing of the prolongator
// with the filtered matrix, Galerkin coarse operators R A P with R = P^T, and a
// dense inverse on the coarsest level.
#include "amg.hpp"

#include <algorithm>
#include <cmath>

namespace dgnp {

Csr csr_transpose(const Csr& A) {
  Csr T;
  T.n = A.m;
  T.m = A.n;
  T.rp.assign(size_t(T.n) + 1, 0);
  for (int k = 0; k < A.rp[A.n]; ++k) T.rp[A.ci[k] + 1]++;
  for (int i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int p = pos[A.ci[k]]++;
      T.ci[p] = i;
      T.v[p] = A.v[k];
    }
  return T;
}

// Gustavson row-by-row product with a dense accumulator; columns sorted.
Csr csr_matmul(const Csr& A, const Csr& B) {
  Csr C;
  C.n = A.n;
  C.m = B.m;
  C.rp.assign(size_t(C.n) + 1, 0);
  std::vector<double> acc(static_cast<size_t>(B.m), 0.0);
  std::vector<int> mark(static_cast<size_t>(B.m), -1), cols;
  for (int i = 0; i < A.n; ++i) {
    cols.clear();
    for (int ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
      const int j = A.ci[ka];
      const double a = A.v[ka];
      for (int kb = B.rp[j]; kb < B.rp[j + 1]; ++kb) {
        const int c = B.ci[kb];
        if (mark[c] != i) {
          mark[c] = i;
          acc[c] = 0.0;
          cols.push_back(c);
        }
        acc[c] += a * B.v[kb];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int c : cols) {
      C.ci.push_back(c);
      C.v.push_back(acc[c]);
    }
    C.rp[i + 1] = int(C.ci.size());
  }
  return C;
}

static std::vector<double> diag_of(const Csr& A) {
  std::vector<double> d(static_cast<size_t>(A.n), 0.0);
  for (int i = 0; i < A.n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] = A.v[k];
  return d;
}

double lmax_dinvA(const Csr& A, const std::vector<double>& dinv, int iters) {
  const int n = A.n;
  std::vector<double> x(static_cast<size_t>(n)), y(static_cast<size_t>(n));
  uint64_t s = 0x9E3779B97F4A7C15ull;
  for (int i = 0; i < n; ++i) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    x[i] = double(s % 1000003) / 1000003.0 + 0.5;
  }
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    double nx = 0.0, ny = 0.0;
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) acc += A.v[k] * x[A.ci[k]];
      y[i] = dinv[i] * acc;
      nx += x[i] * x[i];
      ny += y[i] * y[i];
    }
    if (ny == 0.0) return 1.0;
    lam = std::sqrt(ny / nx);
    const double inv = 1.0 / std::sqrt(ny);
    for (int i = 0; i < n; ++i) x[i] = y[i] * inv;
  }
  return lam;
}

static std::vector<double> dense_inverse(const Csr& A) {
  const int n = A.n;
  std::vector<double> a(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) a[size_t(i) * n + A.ci[k]] += A.v[k];
  std::vector<int> piv(static_cast<size_t>(n));
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + k]) > std::fabs(a[size_t(p) * n + k])) p = r;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(a[size_t(k) * n + c], a[size_t(p) * n + c]);
    const double d = a[size_t(k) * n + k];
    if (d == 0.0) throw Error(DGNP_E_BREAKDOWN, "singular coarsest AMG matrix");
    const double inv = 1.0 / d;
    a[size_t(k) * n + k] = 1.0;
    for (int c = 0; c < n; ++c) a[size_t(k) * n + c] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      const double f = a[size_t(r) * n + k];
      if (f == 0.0) continue;
      a[size_t(r) * n + k] = 0.0;
      for (int c = 0; c < n; ++c) a[size_t(r) * n + c] -= f * a[size_t(k) * n + c];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k)
      for (int r = 0; r < n; ++r) std::swap(a[size_t(r) * n + k], a[size_t(r) * n + piv[k]]);
  return a;
}

// one coarsening step: returns the smoothed prolongator
static Csr sa_prolongator(const Csr& A, double theta) {
  const int n = A.n;
  const std::vector<double> d = diag_of(A);
  // strength of connection
  std::vector<char> strong(A.v.size(), 0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j != i && std::fabs(A.v[k]) >= theta * std::sqrt(std::fabs(d[i] * d[j]))) strong[k] = 1;
    }
  // aggregation
  std::vector<int> agg(static_cast<size_t>(n), -1);
  int na = 0;
  for (int i = 0; i < n; ++i) {  // phase 1: whole strong neighbourhoods
    if (agg[i] >= 0) continue;
    bool free_nbhd = true;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong[k] && agg[A.ci[k]] >= 0) {
        free_nbhd = false;
        break;
      }
    if (!free_nbhd) continue;
    agg[i] = na;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong[k]) agg[A.ci[k]] = na;
    ++na;
  }
  std::vector<int> agg1 = agg;  // phase 2: join the most strongly connected phase-1 aggregate
  for (int i = 0; i < n; ++i) {
    if (agg1[i] >= 0) continue;
    double best = 0.0;
    int ba = -1;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong[k] && agg1[A.ci[k]] >= 0 && std::fabs(A.v[k]) > best) {
        best = std::fabs(A.v[k]);
        ba = agg1[A.ci[k]];
      }
    if (ba >= 0) agg[i] = ba;
  }
  for (int i = 0; i < n; ++i) {  // phase 3: leftovers with their free neighbours
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong[k] && agg[A.ci[k]] < 0) agg[A.ci[k]] = na;
    ++na;
  }
  Csr Pt;
  Pt.n = n;
  Pt.m = na;
  Pt.rp.resize(size_t(n) + 1);
  Pt.ci.resize(size_t(n));
  Pt.v.assign(size_t(n), 1.0);
  for (int i = 0; i < n; ++i) {
    Pt.rp[i] = i;
    Pt.ci[i] = agg[i];
  }
  Pt.rp[n] = n;
  // filtered matrix: weak connections lumped onto the diagonal
  Csr Af;
  Af.n = Af.m = n;
  Af.rp.assign(size_t(n) + 1, 0);
  for (int i = 0; i < n; ++i) {
    double lump = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) continue;
      if (strong[k]) {
        Af.ci.push_back(j);
        Af.v.push_back(A.v[k]);
      } else {
        lump += A.v[k];
      }
    }
    Af.ci.push_back(i);
    Af.v.push_back(d[i] + lump);
    Af.rp[i + 1] = int(Af.ci.size());
  }
  std::vector<double> dinv(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) dinv[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
  const double lam = lmax_dinvA(Af, dinv, 20);
  const double omega = (4.0 / 3.0) / lam;
  Csr AP = csr_matmul(Af, Pt);
  for (int i = 0; i < n; ++i)
    for (int k = AP.rp[i]; k < AP.rp[i + 1]; ++k) AP.v[k] *= -omega * dinv[i];
  // P = Pt - omega D^{-1} Af Pt
  Csr P;
  P.n = n;
  P.m = na;
  P.rp.assign(size_t(n) + 1, 0);
  for (int i = 0; i < n; ++i) {
    bool own = false;
    for (int k = AP.rp[i]; k < AP.rp[i + 1]; ++k) {
      double v = AP.v[k];
      if (AP.ci[k] == agg[i]) {
        v += 1.0;
        own = true;
      }
      P.ci.push_back(AP.ci[k]);
      P.v.push_back(v);
    }
    if (!own) {
      // keep columns sorted
      auto it = std::lower_bound(P.ci.begin() + P.rp[i], P.ci.end(), agg[i]);
      const size_t pos = size_t(it - P.ci.begin());
      P.ci.insert(it, agg[i]);
      P.v.insert(P.v.begin() + long(pos), 1.0);
    }
    P.rp[i + 1] = int(P.ci.size());
  }
  return P;
}

AmgHierarchy sa_setup(const Csr& A1, int max_levels, int coarse_size, double theta) {
  AmgHierarchy H;
  H.A.push_back(A1);
  while (int(H.A.size()) < max_levels && H.A.back().n > coarse_size) {
    const Csr& A = H.A.back();
    Csr P = sa_prolongator(A, theta);
    if (P.m >= A.n * 0.9 || P.m == 0) break;  // stalled coarsening
    Csr R = csr_transpose(P);
    Csr Ac = csr_matmul(R, csr_matmul(A, P));
    H.P.push_back(std::move(P));
    H.R.push_back(std::move(R));
    H.A.push_back(std::move(Ac));
  }
  if (H.A.back().n > 4096)
    throw Error(DGNP_E_BREAKDOWN, "algebraic multigrid coarsening stalled at " + std::to_string(H.A.back().n) +
                                      " unknowns");
  for (const Csr& A : H.A) {
    std::vector<double> d = diag_of(A), dinv(d.size());
    for (size_t i = 0; i < d.size(); ++i) dinv[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
    H.lmax.push_back(lmax_dinvA(A, dinv, 20));
    H.dinv.push_back(std::move(dinv));
  }
  H.coarse_inv = dense_inverse(H.A.back());
  return H;
}

}  // namespace dgnp
