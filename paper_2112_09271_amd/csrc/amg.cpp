// Host setup of the smoothed-aggregation algebraic multigrid hierarchy used
// for the potential block (the paper applies AMG to A_phiphi, Sec. 4.1; this is
// smoothed aggregation in the sense of Vanek, Mandel and Brezina, 1996):
// symmetric strength of connection, greedy three-phase aggregation, piecewise
// constant tentative prolongator, damped-Jacobi smoothing of the prolongator
// with the filtered matrix, Galerkin coarse operators R A P with R = P^T, and a
// dense inverse on the coarsest level.
#include "amg.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <type_traits>

namespace dgnp {

// Rows are processed in fixed chunks of CH rows on up to 16 host threads;
// every reduction is formed per chunk and combined in chunk order, so results
// do not depend on the number of threads.
static constexpr int CH = 2048;
// Sparse products compute every row on its own (no cross-row reduction), so
// they take finer chunks (the result does not depend on the chunking); so do
// the independent columns / rows of the coarsest inverse.
static constexpr int CHM = 64, CHD = 8;

// A persistent pool of host workers (created on first use, joined at exit):
// a job is a chunk count and a function; the workers and the caller take
// chunks from a shared counter.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool;
    return pool;
  }
  int size() const { return int(workers_.size()) + 1; }
  // calls fn(thread, chunk) for every chunk in [0, nch)
  void run(int nch, const std::function<void(int, int)>& fn) {
    if (nch < 4 || workers_.empty()) {  // a few chunks: waking the workers costs more than it saves
      for (int c = 0; c < nch; ++c) fn(0, c);
      return;
    }
    std::lock_guard<std::mutex> one_job(run_m_);  // contexts on several host threads take turns
    std::unique_lock<std::mutex> lk(m_);
    job_ = &fn;
    nch_ = nch;
    next_.store(0);
    helpers_ = std::min(int(workers_.size()), nch - 1);  // workers 1..helpers_ take part
    active_ = helpers_;
    ++gen_;
    cv_.notify_all();
    lk.unlock();
    work(0);
    lk.lock();
    done_cv_.wait(lk, [&] { return active_ == 0; });
    job_ = nullptr;
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  HostPool() {
    int nt = int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
    if (const char* e = getenv("DGNP_HOST_THREADS")) nt = std::max(1, std::min(64, atoi(e)));
    for (int t = 1; t < nt; ++t)
      workers_.emplace_back([this, t]() {
        uint64_t seen = 0;
        while (true) {
          std::unique_lock<std::mutex> lk(m_);
          cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
          if (stop_) return;
          seen = gen_;
          if (t > helpers_) continue;
          lk.unlock();
          work(t);
          lk.lock();
          if (--active_ == 0) done_cv_.notify_all();
        }
      });
  }
  void work(int t) {
    for (int c = next_.fetch_add(1); c < nch_; c = next_.fetch_add(1)) (*job_)(t, c);
  }
  std::vector<std::thread> workers_;
  std::mutex run_m_, m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int, int)>* job_ = nullptr;
  int nch_ = 0, active_ = 0, helpers_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

static int host_threads(int) { return HostPool::get().size(); }

// fn(thread, chunk, first row, end row); thread < host_threads(#chunks)
template <typename F>
static void parallel_chunks_t(int n, F&& fn) {
  const int nch = (n + CH - 1) / CH;
  const std::function<void(int, int)> job = [&](int t, int c) { fn(t, c, c * CH, std::min(n, (c + 1) * CH)); };
  HostPool::get().run(nch, job);
}

template <typename F>
static void parallel_chunks(int n, F&& fn) {
  parallel_chunks_t(n, [&](int, int c, int r0, int r1) { fn(c, r0, r1); });
}

// fn(thread, chunk, first, end) over chunks of `ch` indices (row-independent work only)
template <typename F>
static void parallel_rows(int n, int ch, F&& fn) {
  const int nch = (n + ch - 1) / ch;
  const std::function<void(int, int)> job = [&](int t, int c) { fn(t, c, c * ch, std::min(n, (c + 1) * ch)); };
  HostPool::get().run(nch, job);
}

void host_parallel_rows(int n, const std::function<void(int, int)>& fn) {
  parallel_rows(n, CH, [&](int, int, int r0, int r1) { fn(r0, r1); });
}

Csr csr_transpose(const Csr& A) { return csr_transpose(A, Csr()); }

Csr csr_transpose(const Csr& A, Csr&& storage) {
  Csr T = std::move(storage);
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

// Gustavson row-by-row product with a dense accumulator per host thread, in
// two passes over the rows: the number of distinct columns of every row, then,
// after a prefix sum, its sorted columns and values written in place.  Every
// entry is summed over A's row in order and, within it, over B's row in order,
// so the result does not depend on the chunking.  `storage` lends its arrays
// (kept between set-ups, so that a large product does not pay the page faults
// of fresh memory every time).
Csr csr_matmul(const Csr& A, const Csr& B, Csr&& storage) {
  if (A.n >= (1 << 30)) throw Error(DGNP_E_ARG, "sparse product: 2^30 rows or more");  // marks 2 i + 1
  Csr C = std::move(storage);
  C.n = A.n;
  C.m = B.m;
  C.rp.assign(size_t(C.n) + 1, 0);
  const int nt = host_threads(0);
  std::vector<std::vector<double>> accs(static_cast<size_t>(nt));
  std::vector<std::vector<int>> marks(static_cast<size_t>(nt)), colss(static_cast<size_t>(nt));
  auto scratch = [&](int t) {
    if (marks[size_t(t)].size() != size_t(B.m)) {
      accs[size_t(t)].assign(size_t(B.m), 0.0);
      marks[size_t(t)].assign(size_t(B.m), -1);
    }
  };
  // pass 1: row i of the product marks its columns with 2 i
  parallel_rows(A.n, CHM, [&](int t, int, int r0, int r1) {
    scratch(t);
    int* mark = marks[size_t(t)].data();
    for (int i = r0; i < r1; ++i) {
      int cnt = 0;
      for (int ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int j = A.ci[ka];
        for (int kb = B.rp[j]; kb < B.rp[j + 1]; ++kb) {
          const int c = B.ci[kb];
          if (mark[c] != 2 * i) {
            mark[c] = 2 * i;
            ++cnt;
          }
        }
      }
      C.rp[i + 1] = cnt;
    }
  });
  for (int i = 0; i < C.n; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(size_t(C.rp[C.n]));
  C.v.resize(size_t(C.rp[C.n]));
  // pass 2: the values, marks 2 i + 1
  parallel_rows(A.n, CHM, [&](int t, int, int r0, int r1) {
    scratch(t);
    double* acc = accs[size_t(t)].data();
    int* mark = marks[size_t(t)].data();
    std::vector<int>& cols = colss[size_t(t)];
    for (int i = r0; i < r1; ++i) {
      cols.clear();
      for (int ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int j = A.ci[ka];
        const double a = A.v[ka];
        for (int kb = B.rp[j]; kb < B.rp[j + 1]; ++kb) {
          const int c = B.ci[kb];
          if (mark[c] != 2 * i + 1) {
            mark[c] = 2 * i + 1;
            acc[c] = 0.0;
            cols.push_back(c);
          }
          acc[c] += a * B.v[kb];
        }
      }
      std::sort(cols.begin(), cols.end());
      int* ci = C.ci.data() + C.rp[i];
      double* cv = C.v.data() + C.rp[i];
      for (size_t k = 0; k < cols.size(); ++k) {
        ci[k] = cols[k];
        cv[k] = acc[cols[k]];
      }
    }
  });
  return C;
}

Csr csr_matmul(const Csr& A, const Csr& B) { return csr_matmul(A, B, Csr()); }

// C = A B into the rows and columns C already holds (the product of matrices
// with the same patterns, formed earlier): only the values, in the order of
// csr_matmul, so they equal its result bit for bit.  Returns false (C's values
// then undefined) when C has another shape, a term of the product falls
// outside C's row, or one of C's columns receives none.
static bool csr_matmul_values(const Csr& A, const Csr& B, Csr& C) {
  if (A.n >= (1 << 30) || C.n != A.n || C.m != B.m || C.rp.size() != size_t(A.n) + 1 || C.ci.size() != size_t(C.rp[C.n]) ||
      C.v.size() != C.ci.size())
    return false;
  const int nt = host_threads(0);
  std::vector<std::vector<double>> accs(static_cast<size_t>(nt));
  std::vector<std::vector<int>> marks(static_cast<size_t>(nt));
  std::atomic<bool> ok{true};
  parallel_rows(A.n, CHM, [&](int t, int, int r0, int r1) {
    if (marks[size_t(t)].size() != size_t(B.m)) {
      accs[size_t(t)].assign(size_t(B.m), 0.0);
      marks[size_t(t)].assign(size_t(B.m), -1);
    }
    double* acc = accs[size_t(t)].data();
    int* mark = marks[size_t(t)].data();
    for (int i = r0; i < r1 && ok.load(std::memory_order_relaxed); ++i) {
      const int c0 = C.rp[i], c1 = C.rp[i + 1];
      for (int k = c0; k < c1; ++k) mark[C.ci[k]] = 2 * i;  // column of the row, not yet reached
      int reached = 0;
      for (int ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int j = A.ci[ka];
        const double a = A.v[ka];
        for (int kb = B.rp[j]; kb < B.rp[j + 1]; ++kb) {
          const int c = B.ci[kb];
          if (mark[c] != 2 * i + 1) {
            if (mark[c] != 2 * i) {
              ok.store(false, std::memory_order_relaxed);
              return;
            }
            mark[c] = 2 * i + 1;
            acc[c] = 0.0;
            ++reached;
          }
          acc[c] += a * B.v[kb];
        }
      }
      if (reached != c1 - c0) {
        ok.store(false, std::memory_order_relaxed);
        return;
      }
      for (int k = c0; k < c1; ++k) C.v[k] = acc[C.ci[k]];
    }
  });
  return ok.load();
}

static std::vector<double> diag_of(const Csr& A) {
  std::vector<double> d(static_cast<size_t>(A.n), 0.0);
  parallel_rows(A.n, CH, [&](int, int, int r0, int r1) {
    for (int i = r0; i < r1; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] == i) d[i] = A.v[k];
  });
  return d;
}

double lmax_dinvA(const Csr& A, const std::vector<double>& dinv, int iters, std::vector<double>* x_io) {
  const int n = A.n;
  std::vector<double> x(static_cast<size_t>(n)), y(static_cast<size_t>(n));
  if (x_io && x_io->size() == size_t(n)) {
    x = *x_io;  // warm start from an earlier estimate's last vector
  } else {
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < n; ++i) {
      s ^= s << 13;
      s ^= s >> 7;
      s ^= s << 17;
      x[i] = double(s % 1000003) / 1000003.0 + 0.5;
    }
  }
  const int nch = (n + CH - 1) / CH;
  std::vector<double> px(static_cast<size_t>(nch)), py(static_cast<size_t>(nch));
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    parallel_chunks(n, [&](int ch, int r0, int r1) {
      double sx = 0.0, sy = 0.0;
      for (int i = r0; i < r1; ++i) {
        double acc = 0.0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) acc += A.v[k] * x[A.ci[k]];
        y[i] = dinv[i] * acc;
        sx += x[i] * x[i];
        sy += y[i] * y[i];
      }
      px[size_t(ch)] = sx;
      py[size_t(ch)] = sy;
    });
    double nx = 0.0, ny = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      nx += px[size_t(ch)];
      ny += py[size_t(ch)];
    }
    if (ny == 0.0) return 1.0;
    lam = std::sqrt(ny / nx);
    const double inv = 1.0 / std::sqrt(ny);
    parallel_chunks(n, [&](int, int r0, int r1) {
      for (int i = r0; i < r1; ++i) x[i] = y[i] * inv;
    });
  }
  if (x_io) *x_io = std::move(x);
  return lam;
}

// dot product with four independent partial sums (a fixed order)
static inline double dot4(const double* x, const double* y, int n) {
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    t0 += x[k] * y[k];
    t1 += x[k + 1] * y[k + 1];
    t2 += x[k + 2] * y[k + 2];
    t3 += x[k + 3] * y[k + 3];
  }
  for (; k < n; ++k) t0 += x[k] * y[k];
  return (t0 + t1) + (t2 + t3);
}

// Inverse of the symmetric positive definite coarsest matrix by Cholesky:
// A = L L^T (lower triangle of the row-major array), M = L^{-1}, then
// A^{-1} = M^T M; about n^3 flops, every inner loop a contiguous dot product.
// Returns false at a pivot that is not positive.
static bool cholesky_inverse(std::vector<double>& a, int n) {
  auto at = [&](int i, int j) -> double& { return a[size_t(i) * n + j]; };
  for (int j = 0; j < n; ++j) {
    const double* rj = &a[size_t(j) * n];
    double d = at(j, j) - dot4(rj, rj, j);
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    at(j, j) = d;
    const double id = 1.0 / d;
    for (int i = j + 1; i < n; ++i) at(i, j) = (at(i, j) - dot4(&a[size_t(i) * n], rj, j)) * id;
  }
  // m[j * n + i] = M_ij: column j of M contiguous; M_ij = -(sum_{k=j}^{i-1} L_ik M_kj) / L_ii.
  // Each column is its own triangular solve: columns run on the worker pool.
  std::vector<double> m(size_t(n) * n, 0.0);
  parallel_rows(n, CHD, [&](int, int, int j0, int j1) {
    for (int j = j0; j < j1; ++j) {
      double* mj = &m[size_t(j) * n];
      mj[j] = 1.0 / at(j, j);
      for (int i = j + 1; i < n; ++i) mj[i] = -dot4(&a[size_t(i) * n] + j, mj + j, i - j) * (1.0 / at(i, i));
    }
  });
  // (A^{-1})_ij = sum_{k >= max(i, j)} M_ki M_kj; rows i on the pool, each
  // entry written by the row that owns its lower-triangle position
  std::vector<double> inv(size_t(n) * n);
  parallel_rows(n, CHD, [&](int, int, int i0, int i1) {
    for (int i = i0; i < i1; ++i)
      for (int j = 0; j <= i; ++j) {
        const double t = dot4(&m[size_t(i) * n + i], &m[size_t(j) * n + i], n - i);
        inv[size_t(i) * n + j] = t;
        inv[size_t(j) * n + i] = t;
      }
  });
  a.swap(inv);
  return true;
}

// The same for a matrix whose entries lie within bw of the diagonal: the
// Cholesky factor stays inside that band, so the factorisation costs about
// n bw^2 / 2 flops; then, column by column on the worker pool, M = L^{-1} e_j
// (a banded forward substitution from row j on) and the part i >= j of
// column j of A^{-1} = L^{-T} M by a banded back substitution stopped at row j
// (about n^2 bw flops in all, against n^3 for the dense route).
static bool band_cholesky_inverse(std::vector<double>& a, int n, int bw) {
  auto at = [&](int i, int j) -> double& { return a[size_t(i) * n + j]; };
  for (int j = 0; j < n; ++j) {
    const double* rj = &a[size_t(j) * n];
    const int k0 = std::max(0, j - bw);
    double d = at(j, j) - dot4(rj + k0, rj + k0, j - k0);
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    at(j, j) = d;
    const double id = 1.0 / d;
    const int i1 = std::min(n - 1, j + bw);
    for (int i = j + 1; i <= i1; ++i) {
      const int ki = std::max(0, i - bw);  // row i of L starts at column i - bw
      at(i, j) = (at(i, j) - dot4(&a[size_t(i) * n] + ki, rj + ki, j - ki)) * id;
    }
  }
  // lt[i][t] = L_{i+t, i}: the band of L^T row by row; rd[i] = 1 / L_ii
  const int W = bw + 1;
  std::vector<double> lt(size_t(n) * W, 0.0), rd(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) {
    rd[i] = 1.0 / at(i, i);
    for (int t = 0; t < W && i + t < n; ++t) lt[size_t(i) * W + t] = at(i + t, i);
  }
  std::vector<double> m(size_t(n) * n, 0.0), inv(size_t(n) * n);
  parallel_rows(n, CHD, [&](int, int, int j0, int j1) {
    for (int j = j0; j < j1; ++j) {
      double* mj = &m[size_t(j) * n];  // column j of M, rows j .. n-1
      mj[j] = rd[j];
      for (int i = j + 1; i < n; ++i) {
        const int k0 = std::max(j, i - bw);
        mj[i] = -dot4(&a[size_t(i) * n] + k0, mj + k0, i - k0) * rd[i];
      }
      // (A^{-1})_{ij} for i >= j, kept in row j (symmetry) and mirrored into
      // column j (rows below j: not written by their own row)
      double* xj = &inv[size_t(j) * n];
      for (int i = n - 1; i >= j; --i) {
        const int len = std::min(bw, n - 1 - i);
        xj[i] = (mj[i] - dot4(&lt[size_t(i) * W + 1], xj + i + 1, len)) * rd[i];
      }
      for (int i = j + 1; i < n; ++i) inv[size_t(i) * n + j] = xj[i];
    }
  });
  a.swap(inv);
  return true;
}

std::vector<double> dense_inverse(const Csr& A) {
  const int n = A.n;
  std::vector<double> a(static_cast<size_t>(n) * n, 0.0);
  int bw = 0;
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      a[size_t(i) * n + A.ci[k]] += A.v[k];
      bw = std::max(bw, std::abs(A.ci[k] - i));
    }
  {
    std::vector<double> c = a;
    if (3 * bw <= n ? band_cholesky_inverse(c, n, bw) : cholesky_inverse(c, n)) return c;
  }
  // not positive definite: Gauss-Jordan with partial pivoting
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
static Csr sa_prolongator(const Csr& A, double theta, double lam_A, Csr&& storage) {
  const int n = A.n;
  const std::vector<double> d = diag_of(A);
  // strength of connection
  std::vector<char> strong(A.v.size(), 0);
  parallel_rows(n, CH, [&](int, int, int r0, int r1) {
    for (int i = r0; i < r1; ++i)
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int j = A.ci[k];
        if (j != i && (theta == 0.0 || std::fabs(A.v[k]) >= theta * std::sqrt(std::fabs(d[i] * d[j]))))
          strong[k] = 1;
      }
  });
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
  // filtered matrix: weak connections lumped onto the diagonal (with theta = 0
  // every connection is strong and the filtered matrix is A itself)
  Csr Afb;
  const Csr& Af = theta == 0.0 ? A : Afb;
  if (theta != 0.0) {
    Afb.n = Afb.m = n;
    Afb.rp.assign(size_t(n) + 1, 0);
  }
  for (int i = 0; i < n && theta != 0.0; ++i) {
    double lump = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) continue;
      if (strong[k]) {
        Afb.ci.push_back(j);
        Afb.v.push_back(A.v[k]);
      } else {
        lump += A.v[k];
      }
    }
    Afb.ci.push_back(i);
    Afb.v.push_back(d[i] + lump);
    Afb.rp[i + 1] = int(Afb.ci.size());
  }
  std::vector<double> dinv(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) dinv[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
  // with theta = 0 every connection is strong and the filtered matrix is A itself
  const double lam = theta == 0.0 && lam_A > 0.0 ? lam_A : lmax_dinvA(Af, dinv, 20, nullptr);
  const double omega = (4.0 / 3.0) / lam;
  Csr AP = csr_matmul(Af, Pt);
  // P = Pt - omega D^{-1} Af Pt, in two passes over the rows on the worker
  // pool: the row lengths (the own aggregate's column is added when Af Pt
  // lacks it), then the columns in order with the values
  Csr P = std::move(storage);
  P.n = n;
  P.m = na;
  P.rp.assign(size_t(n) + 1, 0);
  auto has_own = [&](int i) {
    for (int k = AP.rp[i]; k < AP.rp[i + 1]; ++k)
      if (AP.ci[k] == agg[i]) return true;
    return false;
  };
  parallel_rows(n, CH, [&](int, int, int r0, int r1) {
    for (int i = r0; i < r1; ++i) P.rp[i + 1] = AP.rp[i + 1] - AP.rp[i] + (has_own(i) ? 0 : 1);
  });
  for (int i = 0; i < n; ++i) P.rp[i + 1] += P.rp[i];
  P.ci.resize(size_t(P.rp[n]));
  P.v.resize(size_t(P.rp[n]));
  parallel_rows(n, CH, [&](int, int, int r0, int r1) {
    for (int i = r0; i < r1; ++i) {
      const int a = agg[i];
      bool pending = !has_own(i);  // the own column still to be placed (value 1)
      int o = P.rp[i];
      for (int k = AP.rp[i]; k < AP.rp[i + 1]; ++k) {
        const int c = AP.ci[k];
        if (pending && a < c) {
          P.ci[o] = a;
          P.v[o++] = 1.0;
          pending = false;
        }
        double v = AP.v[k];
        v *= -omega * dinv[i];
        if (c == a) v += 1.0;
        P.ci[o] = c;
        P.v[o++] = v;
      }
      if (pending) {
        P.ci[o] = a;
        P.v[o] = 1.0;
      }
    }
  });
  return P;
}

static void sa_mark(std::chrono::steady_clock::time_point& t0, const char* what) {
  static const bool trace = getenv("DGNP_TRACE_SETUP") != nullptr;
  if (!trace) return;
  const auto t1 = std::chrono::steady_clock::now();
  fprintf(stderr, "[setup]   sa %-18s %8.3f ms\n", what, 1e3 * std::chrono::duration<double>(t1 - t0).count());
  t0 = t1;
}

// Jacobi diagonal and the largest eigenvalue estimate of D^{-1} A of a level;
// x0 (finest level only, may be null): start vector in, last vector out, with
// `iters` power steps
static void smoother_data(AmgHierarchy& H, const Csr& A, int iters, std::vector<double>* x0) {
  std::vector<double> d = diag_of(A), dinv(d.size());
  for (size_t i = 0; i < d.size(); ++i) dinv[i] = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
  H.lmax.push_back(lmax_dinvA(A, dinv, iters, x0));
  H.dinv.push_back(std::move(dinv));
}

AmgHierarchy sa_setup(Csr A1, int max_levels, int coarse_size, double theta, std::vector<double>* x0,
                      AmgHierarchy* recycle) {
  auto t0 = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) { sa_mark(t0, what); };
  AmgHierarchy H;
  H.A.push_back(std::move(A1));
  if (x0) x0->clear();  // cold: the estimate does not depend on earlier set-ups
  smoother_data(H, H.A.back(), 20, x0);
  mark("lmax");
  while (int(H.A.size()) < max_levels && H.A.back().n > coarse_size) {
    const Csr& A = H.A.back();
    // arrays lent by the recycled hierarchy (empty when it has no such level)
    const size_t l = H.A.size() - 1;
    auto lend = [&](std::vector<Csr>* v, size_t i) {
      return recycle && v && i < v->size() ? std::move((*v)[i]) : Csr();
    };
    Csr P = sa_prolongator(A, theta, H.lmax.back(), lend(recycle ? &recycle->P : nullptr, l));
    mark("prolongator");
    if (P.m >= A.n * 0.9 || P.m == 0) break;  // stalled coarsening
    Csr R = csr_transpose(P, lend(recycle ? &recycle->R : nullptr, l));
    // the products values-only into the lent arrays when their patterns agree
    Csr AP = lend(recycle ? &recycle->work : nullptr, l);
    if (!csr_matmul_values(A, P, AP)) AP = csr_matmul(A, P, std::move(AP));
    Csr Ac = lend(recycle ? &recycle->A : nullptr, l + 1);
    if (!csr_matmul_values(R, AP, Ac)) Ac = csr_matmul(R, AP, std::move(Ac));
    H.work.push_back(std::move(AP));
    mark("RAP");
    H.P.push_back(std::move(P));
    H.R.push_back(std::move(R));
    H.A.push_back(std::move(Ac));
    smoother_data(H, H.A.back(), 20, nullptr);
    mark("lmax");
  }
  if (H.A.back().n > 4096)
    throw Error(DGNP_E_BREAKDOWN, "algebraic multigrid coarsening stalled at " + std::to_string(H.A.back().n) +
                                      " unknowns");
  H.coarse_inv = dense_inverse(H.A.back());
  mark("coarse inverse");
  return H;
}

// a non-const prev gives up its prolongators, restrictions and product arrays
// (moved, not copied); a const one is copied from
template <typename Prev>
static AmgHierarchy reuse_impl(Csr A1, Prev& prev, std::vector<double>* x0) {
  constexpr bool consume = !std::is_const<Prev>::value;
  auto t0 = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) { sa_mark(t0, what); };
  if (prev.A.empty() || prev.A[0].n != A1.n || prev.P.size() + 1 != prev.A.size() ||
      prev.R.size() != prev.P.size())
    throw Error(DGNP_E_STATE, "aggregation reuse: the vertex level changed size");
  for (size_t l = 0; l < prev.P.size(); ++l) {
    const Csr &P = prev.P[l], &R = prev.R[l];
    if (P.n != prev.A[l].n || P.m != prev.A[l + 1].n || P.rp.size() != size_t(P.n) + 1 || R.n != P.m ||
        R.m != P.n || R.rp.size() != size_t(R.n) + 1)
      throw Error(DGNP_E_STATE, "aggregation reuse: the kept hierarchy is incomplete");
  }
  AmgHierarchy H;
  H.A.push_back(std::move(A1));
  smoother_data(H, H.A.back(), x0 && x0->size() == size_t(H.A[0].n) ? 8 : 20, x0);
  mark("lmax (warm)");
  // the products A_l P_l and R_l (A_l P_l): values only, into the previous
  // set-up's arrays, while the vertex graph and with it every pattern is the
  // same; built afresh otherwise
  H.work.resize(prev.P.size());
  for (size_t l = 0; l < prev.P.size(); ++l) {
    Csr store;
    if constexpr (consume) {
      H.P.push_back(std::move(prev.P[l]));
      H.R.push_back(std::move(prev.R[l]));
      store = std::move(prev.A[l + 1]);
      if (l < prev.work.size()) H.work[l] = std::move(prev.work[l]);
    } else {
      H.P.push_back(prev.P[l]);
      H.R.push_back(prev.R[l]);
    }
    Csr& AP = H.work[l];
    if (!csr_matmul_values(H.A[l], H.P.back(), AP)) AP = csr_matmul(H.A[l], H.P.back(), std::move(AP));
    if (!csr_matmul_values(H.R.back(), AP, store)) store = csr_matmul(H.R.back(), AP, std::move(store));
    H.A.push_back(std::move(store));
    smoother_data(H, H.A.back(), 20, nullptr);
  }
  mark("RAP (kept P)");
  H.coarse_inv = dense_inverse(H.A.back());
  mark("coarse inverse");
  return H;
}

AmgHierarchy sa_setup_reuse(Csr A1, const AmgHierarchy& prev, std::vector<double>* x0) {
  return reuse_impl(std::move(A1), prev, x0);
}

AmgHierarchy sa_setup_reuse(Csr A1, AmgHierarchy&& prev, std::vector<double>* x0) {
  return reuse_impl(std::move(A1), prev, x0);
}

}  // namespace dgnp
