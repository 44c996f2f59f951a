// Host check of the smoothed-aggregation set-up (amg.cpp) on the 7-point
// Laplacian of an n^3 grid: SpGEMM and transpose against dense products,
// every node aggregated, symmetric Galerkin operators, the coarsest inverse,
// bitwise-identical hierarchies across repeated runs, and the set-up that
// keeps an earlier hierarchy's prolongators.  Prints "ok" and
// returns 0, or names the failed check and returns 1.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "amg.hpp"

using dgnp::Csr;

static Csr laplace3d(int n) {
  Csr A;
  A.n = A.m = n * n * n;
  A.rp.push_back(0);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int r = i + n * (j + n * k);
        const int off[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (auto& o : off) {
          const int ii = i + o[0], jj = j + o[1], kk = k + o[2];
          if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) continue;
          A.ci.push_back(ii + n * (jj + n * kk));
          A.v.push_back(o[0] == 0 && o[1] == 0 && o[2] == 0 ? 6.0 + 0.01 * (r % 7) : -1.0);
        }
        A.rp.push_back(int(A.ci.size()));
      }
  return A;
}

static std::vector<double> dense(const Csr& A) {
  std::vector<double> d(size_t(A.n) * A.m, 0.0);
  for (int i = 0; i < A.n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) d[size_t(i) * A.m + A.ci[k]] += A.v[k];
  return d;
}

static int fail(const char* what) {
  printf("FAILED: %s\n", what);
  return 1;
}

int main() {
  // SpGEMM and transpose on a small case against dense arithmetic
  {
    Csr A = laplace3d(5), B = dgnp::csr_transpose(laplace3d(5));
    Csr C = dgnp::csr_matmul(A, B);
    std::vector<double> a = dense(A), b = dense(B), c = dense(C);
    const int n = A.n;
    double err = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += a[size_t(i) * n + k] * b[size_t(k) * n + j];
        err = std::fmax(err, std::fabs(s - c[size_t(i) * n + j]));
      }
    if (err > 1e-12) return fail("csr_matmul differs from the dense product");
    for (int i = 0; i < C.n; ++i)
      for (int k = C.rp[i] + 1; k < C.rp[i + 1]; ++k)
        if (C.ci[k] <= C.ci[k - 1]) return fail("csr_matmul columns not sorted");
  }
  // hierarchy on a grid large enough for several chunks of rows
  Csr A = laplace3d(30);
  dgnp::AmgHierarchy H = dgnp::sa_setup(A, 12, 256, 0.0);
  if (H.A.size() < 2) return fail("no coarsening");
  for (size_t l = 0; l + 1 < H.A.size(); ++l) {
    const Csr& P = H.P[l];
    if (P.n != H.A[l].n || P.m != H.A[l + 1].n) return fail("prolongator shape");
    if (P.m >= P.n / 4) return fail("weak coarsening");
    for (int i = 0; i < P.n; ++i)
      if (P.rp[i + 1] == P.rp[i]) return fail("row of P without an aggregate");
    // Galerkin operator symmetric
    const Csr& Ac = H.A[l + 1];
    std::vector<double> d = dense(Ac);
    for (int i = 0; i < Ac.n; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(d[size_t(i) * Ac.n + j] - d[size_t(j) * Ac.n + i]) > 1e-10 * std::fabs(d[size_t(i) * Ac.n + i]))
          return fail("coarse operator not symmetric");
    if (!(H.lmax[l] > 1.0 && H.lmax[l] < 2.0)) return fail("lambda_max of D^-1 A outside (1, 2)");
  }
  // the coarsest inverse
  {
    const Csr& Ac = H.A.back();
    std::vector<double> d = dense(Ac);
    const int n = Ac.n;
    double err = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += H.coarse_inv[size_t(i) * n + k] * d[size_t(k) * n + j];
        err = std::fmax(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
      }
    if (err > 1e-10) return fail("coarsest inverse");
  }
  // a second set-up (worker pool already running) gives the same hierarchy bit for bit
  dgnp::AmgHierarchy H2 = dgnp::sa_setup(A, 12, 256, 0.0);
  if (H2.A.size() != H.A.size()) return fail("repeat: level count");
  for (size_t l = 0; l < H.A.size(); ++l)
    if (H2.A[l].v != H.A[l].v || H2.A[l].ci != H.A[l].ci || H2.lmax[l] != H.lmax[l])
      return fail("repeat: hierarchy differs");
  // reuse of the prolongators: for the same matrix the Galerkin levels are
  // those of the fresh set-up bit for bit; the finest lambda_max estimate
  // continues the power iteration from its last vector, so it can only grow
  // towards the true value, which the Gershgorin bound 2 caps (row sums of
  // |D^{-1} A| are at most 1 + 6/6 here); coarser levels repeat the cold
  // estimate exactly.  For 2 A every Galerkin level doubles and D^{-1} A, hence
  // lambda_max, is unchanged.
  {
    std::vector<double> x0;
    dgnp::AmgHierarchy Hc = dgnp::sa_setup(A, 12, 256, 0.0, &x0);
    if (x0.size() != size_t(A.n)) return fail("reuse: no start vector kept");
    dgnp::AmgHierarchy Hr = dgnp::sa_setup_reuse(A, Hc, &x0);
    if (Hr.A.size() != Hc.A.size()) return fail("reuse: level count");
    for (size_t l = 0; l < Hc.A.size(); ++l) {
      if (Hr.A[l].v != Hc.A[l].v || Hr.A[l].ci != Hc.A[l].ci) return fail("reuse: Galerkin level differs");
      if (l > 0 && Hr.lmax[l] != Hc.lmax[l]) return fail("reuse: coarse lambda_max differs");
    }
    if (!(Hr.lmax[0] >= Hc.lmax[0] * (1.0 - 1e-12) && Hr.lmax[0] <= 2.0))
      return fail("reuse: warm lambda_max not between the cold estimate and the Gershgorin bound");
    if (Hr.coarse_inv != Hc.coarse_inv) return fail("reuse: coarsest inverse differs");
    Csr A2 = A;
    for (double& v : A2.v) v *= 2.0;
    dgnp::AmgHierarchy H2r = dgnp::sa_setup_reuse(A2, Hc, &x0);
    for (size_t l = 1; l < Hc.A.size(); ++l)
      for (size_t k = 0; k < Hc.A[l].v.size(); ++k)
        if (std::fabs(H2r.A[l].v[k] - 2.0 * Hc.A[l].v[k]) > 1e-12 * std::fabs(Hc.A[l].v[k]) + 1e-14)
          return fail("reuse: rescaled Galerkin level");
    if (!(H2r.lmax[0] >= Hc.lmax[0] * (1.0 - 1e-12) && H2r.lmax[0] <= 2.0)) return fail("reuse: rescaled lambda_max");
    Csr B = laplace3d(29);
    bool threw = false;
    try {
      (void)dgnp::sa_setup_reuse(B, Hc, &x0);
    } catch (const dgnp::Error&) {
      threw = true;
    }
    if (!threw) return fail("reuse: a vertex level of another size must be refused");
  }
  // the reuse that takes over the previous hierarchy (prolongators moved, the
  // products formed into its arrays, values only while the patterns agree)
  // gives the copying reuse's hierarchy, kept products included, bit for bit:
  // twice in a row, then for a matrix of a smaller pattern (one symmetric pair
  // of entries removed: a row of A P loses a column) and back (it gains one),
  // where its products are rebuilt
  {
    auto same = [](const dgnp::AmgHierarchy& a, const dgnp::AmgHierarchy& b) {
      if (a.A.size() != b.A.size() || a.lmax != b.lmax || a.coarse_inv != b.coarse_inv) return false;
      for (size_t l = 0; l < a.A.size(); ++l)
        if (a.A[l].v != b.A[l].v || a.A[l].ci != b.A[l].ci || a.A[l].rp != b.A[l].rp) return false;
      if (a.work.size() != b.work.size()) return false;
      for (size_t l = 0; l < a.work.size(); ++l)
        if (a.work[l].v != b.work[l].v || a.work[l].ci != b.work[l].ci || a.work[l].rp != b.work[l].rp)
          return false;
      return true;
    };
    Csr A2 = A, A3 = A, A4;
    for (double& v : A2.v) v *= 2.0;
    for (int i = 0; i < A3.n; ++i)
      for (int k = A3.rp[i]; k < A3.rp[i + 1]; ++k)
        if (A3.ci[k] == i) A3.v[k] += 0.5;
    {
      const int r0 = 0, r1 = 1;  // drop the coupling of rows 0 and 1
      A4.n = A4.m = A.n;
      A4.rp.push_back(0);
      for (int i = 0; i < A.n; ++i) {
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int j = A.ci[k];
          if ((i == r0 && j == r1) || (i == r1 && j == r0)) continue;
          A4.ci.push_back(j);
          A4.v.push_back(A.v[k]);
        }
        A4.rp.push_back(int(A4.ci.size()));
      }
    }
    std::vector<double> xa, xb;
    dgnp::AmgHierarchy Hc = dgnp::sa_setup(A, 12, 256, 0.0, &xa);
    xb = xa;
    dgnp::AmgHierarchy Hm = Hc;
    dgnp::AmgHierarchy R1 = dgnp::sa_setup_reuse(A2, Hc, &xa);
    dgnp::AmgHierarchy M1 = dgnp::sa_setup_reuse(A2, std::move(Hm), &xb);
    if (!same(R1, M1) || xa != xb) return fail("consuming reuse differs (first call)");
    dgnp::AmgHierarchy R2 = dgnp::sa_setup_reuse(A3, R1, &xa);
    dgnp::AmgHierarchy M2 = dgnp::sa_setup_reuse(A3, std::move(M1), &xb);
    if (!same(R2, M2) || xa != xb) return fail("consuming reuse differs (second call)");
    dgnp::AmgHierarchy R3 = dgnp::sa_setup_reuse(A4, R2, &xa);
    dgnp::AmgHierarchy M3 = dgnp::sa_setup_reuse(A4, std::move(M2), &xb);
    if (!same(R3, M3) || xa != xb) return fail("consuming reuse differs (pattern changed)");
    if (R3.A[0].rp[R3.A[0].n] != A.rp[A.n] - 2) return fail("pattern change not taken");
    if (R3.work[0].rp[R3.work[0].n] == R2.work[0].rp[R2.work[0].n]) return fail("A P kept its pattern");
    dgnp::AmgHierarchy R4 = dgnp::sa_setup_reuse(A, R3, &xa);
    dgnp::AmgHierarchy M4 = dgnp::sa_setup_reuse(A, std::move(M3), &xb);
    if (!same(R4, M4) || xa != xb) return fail("consuming reuse differs (pattern restored)");
  }
  // the inverse of the coarsest level: banded Cholesky (entries within a third
  // of the order of the diagonal: the 7-point Laplacian of a 7^3 grid plus a
  // shift, bandwidth 49 of 343), the dense Cholesky for the same matrix with
  // its unknowns reversed in pairs of halves (a band of about the order), and
  // Gauss-Jordan for an indefinite banded matrix; each A^{-1} A = I to 1e-12,
  // and the two Cholesky routes give the same inverse up to the renumbering
  {
    Csr L = laplace3d(7);
    for (int i = 0; i < L.n; ++i)
      for (int k = L.rp[i]; k < L.rp[i + 1]; ++k)
        if (L.ci[k] == i) L.v[k] += 0.25;
    const int n = L.n, h = n / 2;
    auto perm = [&](int i) { return i < h ? h - 1 - i + (n - h) : i - h; };  // a bijection of 0..n-1
    Csr Lp;
    Lp.n = Lp.m = n;
    {
      std::vector<std::vector<std::pair<int, double>>> rows(static_cast<size_t>(n));
      for (int i = 0; i < n; ++i)
        for (int k = L.rp[i]; k < L.rp[i + 1]; ++k) rows[size_t(perm(i))].push_back({perm(L.ci[k]), L.v[k]});
      Lp.rp.push_back(0);
      for (auto& r : rows) {
        std::sort(r.begin(), r.end());
        for (auto& e : r) {
          Lp.ci.push_back(e.first);
          Lp.v.push_back(e.second);
        }
        Lp.rp.push_back(int(Lp.ci.size()));
      }
    }
    Csr Li = L;  // indefinite: a large negative shift
    for (int i = 0; i < n; ++i)
      for (int k = Li.rp[i]; k < Li.rp[i + 1]; ++k)
        if (Li.ci[k] == i) Li.v[k] -= 6.0;
    auto identity_err = [](const Csr& M, const std::vector<double>& inv) {
      const int n = M.n;
      std::vector<double> d = dense(M);
      double err = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double s = 0.0;
          for (int k = 0; k < n; ++k) s += inv[size_t(i) * n + k] * d[size_t(k) * n + j];
          err = std::fmax(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
        }
      return err;
    };
    std::vector<double> ib = dgnp::dense_inverse(L), id = dgnp::dense_inverse(Lp), ii = dgnp::dense_inverse(Li);
    if (identity_err(L, ib) > 1e-12) return fail("banded Cholesky inverse");
    if (identity_err(Lp, id) > 1e-12) return fail("dense Cholesky inverse");
    if (identity_err(Li, ii) > 1e-12) return fail("Gauss-Jordan inverse of an indefinite matrix");
    double dmax = 0.0, imax = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        dmax = std::fmax(dmax, std::fabs(ib[size_t(i) * n + j] - id[size_t(perm(i)) * n + perm(j)]));
        imax = std::fmax(imax, std::fabs(ib[size_t(i) * n + j]));
      }
    if (dmax > 1e-13 * imax) return fail("banded and dense Cholesky inverses differ");
  }
  // a fresh set-up that recycles an earlier hierarchy's arrays (values-only
  // products where the patterns agree) builds bitwise the same hierarchy as
  // one without: recycling a hierarchy of the same matrix, of a matrix of
  // another pattern, and of another size
  {
    auto same_levels = [](const dgnp::AmgHierarchy& a, const dgnp::AmgHierarchy& b) {
      if (a.A.size() != b.A.size() || a.lmax != b.lmax || a.coarse_inv != b.coarse_inv) return false;
      for (size_t l = 0; l < a.A.size(); ++l)
        if (a.A[l].v != b.A[l].v || a.A[l].ci != b.A[l].ci || a.A[l].rp != b.A[l].rp) return false;
      for (size_t l = 0; l < a.P.size(); ++l)
        if (a.P[l].v != b.P[l].v || a.P[l].ci != b.P[l].ci || a.R[l].v != b.R[l].v || a.R[l].ci != b.R[l].ci)
          return false;
      return true;
    };
    std::vector<double> xa, xb;
    const dgnp::AmgHierarchy ref = dgnp::sa_setup(A, 12, 256, 0.0, &xa);
    Csr Ad = A;  // another pattern: the coupling of rows 0 and 1 dropped
    {
      Csr B;
      B.n = B.m = A.n;
      B.rp.push_back(0);
      for (int i = 0; i < A.n; ++i) {
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
          if (!((i == 0 && A.ci[k] == 1) || (i == 1 && A.ci[k] == 0))) {
            B.ci.push_back(A.ci[k]);
            B.v.push_back(A.v[k]);
          }
        B.rp.push_back(int(B.ci.size()));
      }
      Ad = B;
    }
    const Csr* donors[3] = {&A, &Ad, nullptr};
    Csr small = laplace3d(12);
    donors[2] = &small;
    for (const Csr* dm : donors) {
      dgnp::AmgHierarchy donor = dgnp::sa_setup(*dm, 12, 256, 0.0);
      dgnp::AmgHierarchy H1 = dgnp::sa_setup(A, 12, 256, 0.0, &xb, &donor);
      if (!same_levels(H1, ref) || xa != xb) return fail("recycled fresh set-up differs");
    }
  }
  // checksum of every value of the hierarchy (bit patterns), to compare runs
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](double x) {
    uint64_t b;
    std::memcpy(&b, &x, sizeof b);
    h = (h ^ b) * 1099511628211ull;
  };
  for (size_t l = 0; l < H.A.size(); ++l) {
    for (double x : H.A[l].v) mix(x);
    mix(H.lmax[l]);
  }
  for (const Csr& P : H.P)
    for (double x : P.v) mix(x);
  for (double x : H.coarse_inv) mix(x);
  printf("ok levels %zu sizes", H.A.size());
  for (auto& L : H.A) printf(" %d", L.n);
  printf(" checksum %016llx\n", static_cast<unsigned long long>(h));
  return 0;
}
