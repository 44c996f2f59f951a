// Block-triangular preconditioner (paper Sec. 4.1 Eq. P1 and Sec. 4.2 Eq. P2):
//   concentration blocks A_ckck  -> one element-block ILU(0) solve each
//   potential block A_phiphi     -> one multigrid V-cycle: Chebyshev-accelerated
//                                   element-block Jacobi on the DG level, the
//                                   Galerkin projection onto the continuous Q1
//                                   vertex space, and a smoothed-aggregation
//                                   AMG hierarchy below it
//   off-diagonal coupling blocks -> matrix-free Jacobian applies
// One application of each inner solver makes P a fixed linear operator, so its
// exact transpose exists (used by the adjoint).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <thread>
#include <type_traits>

#include "amg.hpp"
#include "blas.hpp"
#include "kernels_block.hpp"
#include "kernels_gmg.hpp"
#include "kernels_phi.hpp"
#include "solver.hpp"

namespace dgnp {

// A device CSR matrix; its row pointers and column indices may be another
// matrix's (rpx, cix not null: the single-precision copy of a level shares the
// double copy's index arrays)
template <typename T>
struct DevCsr {
  int n = 0;
  DevBuf<int> rp, ci;
  DevBuf<T> v;
  const int* rpx = nullptr;
  const int* cix = nullptr;
  const int* rptr() const { return rpx ? rpx : rp.p; }
  const int* cptr() const { return cix ? cix : ci.p; }
};

struct MgLevel {  // scalar levels (index >= 1 in the V-cycle)
  int n = 0;
  DevCsr<double> A, P, R;  // P: next level -> this level
  DevCsr<float> A32, P32, R32;
  DevBuf<double> dinv;
  DevBuf<float> dinv32;
  double lmax = 1.0;
};

template <typename T>
struct Work {  // per-level work vectors
  std::vector<DevBuf<T>*> x, b, r, d, z;
};

// Host-to-device uploads of the set-up without a host wait per array: each
// array is converted into pinned staging memory and copied asynchronously.
// The staging memory is reused from the next set-up on (the set-up ends with
// a stream synchronisation); chunks grow as needed and live with the context.
struct PinnedStage {
  struct Chunk {
    char* p;
    size_t size;
  };
  std::vector<Chunk> chunks;
  size_t cur = 0, used = 0;
  PinnedStage() = default;
  PinnedStage(const PinnedStage&) = delete;
  PinnedStage& operator=(const PinnedStage&) = delete;
  ~PinnedStage() {
    for (auto& ch : chunks) (void)hipHostFree(ch.p);
  }
  void reset() { cur = used = 0; }
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    while (cur < chunks.size() && used + bytes > chunks[cur].size) {
      ++cur;
      used = 0;
    }
    if (cur == chunks.size()) {
      Chunk ch{nullptr, std::max(bytes, size_t(8) << 20)};
      DGNP_HIP(hipHostMalloc(reinterpret_cast<void**>(&ch.p), ch.size, hipHostMallocDefault));
      chunks.push_back(ch);
      used = 0;
    }
    void* r = chunks[cur].p + used;
    used += bytes;
    return r;
  }
  // dst = (T) src[0..n), asynchronously on s (large arrays are staged by row
  // chunks on the host worker pool)
  template <typename T, typename S>
  void upload(DevBuf<T>& dst, const S* src, size_t n, hipStream_t s) {
    dst.fit(n);
    if (n == 0) return;
    T* h = static_cast<T*>(take(n * sizeof(T)));
    if (n >= (size_t(1) << 20) && n < (size_t(1) << 31)) {
      host_parallel_rows(int(n), [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i) h[i] = T(src[i]);
      });
    } else {
      for (size_t i = 0; i < n; ++i) h[i] = T(src[i]);
    }
    DGNP_HIP(hipMemcpyAsync(dst.p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// Three side streams (default priority) of the concentration set-up and a pool
// of events for the fork / join hand-offs between them and the caller's
// stream.  An event is recorded once per set-up; a wait takes the record that
// precedes it, so reusing the pool in the next set-up is safe.
struct SideStreams {
  hipStream_t st[3] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> ev;
  size_t next = 0;
  SideStreams() = default;
  SideStreams(const SideStreams&) = delete;
  SideStreams& operator=(const SideStreams&) = delete;
  ~SideStreams() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t q : st)
      if (q) (void)hipStreamDestroy(q);
  }
  hipStream_t stream(int i) {
    if (!st[i]) DGNP_HIP(hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking));
    return st[i];
  }
  // work queued on `to` after this call waits for the work queued on `from` before it
  void order(hipStream_t from, hipStream_t to) {
    if (next == ev.size()) {
      hipEvent_t e = nullptr;
      DGNP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ev.push_back(e);
    }
    hipEvent_t e = ev[next++];
    DGNP_HIP(hipEventRecord(e, from));
    DGNP_HIP(hipStreamWaitEvent(to, e, 0));
  }
};

struct Precond {
  SideStreams side;
  int nslot = 0;
  int64_t bsz = 0;                  // doubles per block = nb * nb
  DevBuf<double> blk;               // [m][E][nslot][nb][nb]
  DevBuf<float> blk32;              // concentration fields only: [m-1][E][nslot][nb][nb]
  // host aggregation hierarchy of the last set-up and the vertex level's last
  // power-iteration vector: later set-ups of the same Newton solve keep its
  // aggregates and prolongators
  AmgHierarchy sa_prev;
  std::vector<double> sa_x0;
  DevBuf<float> phi32;              // potential field: [E][nslot][nb][ld32], ld32 = pot_ld(nb, true)
  bool phi32_blocks = false;        // phi32 holds the current blocks (with p-multigrid only on request)
  DevBuf<double> dinv_phi;          // [E][nb][nb]
  DevBuf<float> dinv_phi32;         // [E][nb][ld32]
  double lmax0 = 1.0;
  // last power-iteration vector of each precision: later estimates (the next
  // linearisation points) start from it with fewer steps
  DevBuf<double> lvec64;
  DevBuf<float> lvec32;
  // p-multigrid on the potential: the order-p level is applied matrix-free
  // (its inverse diagonal blocks above); the next level is the potential block
  // re-discretised at p = 1 (nb1 = 2^d nodes per element) at the corner values
  // x1 of the state, and its Q1 Galerkin operator starts the vertex hierarchy
  bool pmg = false;
  bool pmg_galerkin = false;         // p = 1 level: Galerkin product instead of re-discretisation
  int nb1 = 0;
  DevBuf<double> x1;                // [m][E][nb1]
  DevBuf<double> blk1, dinv1;       // [E][nslot][nb1][nb1], [E][nb1][nb1]
  DevBuf<float> blk1_32, dinv1_32;
  double lmax1 = 1.0;
  DevBuf<double> lvec1_64;
  DevBuf<float> lvec1_32;
  DevBuf<double> mf64;              // order-p operator output [Nf]
  DevBuf<float> mf32;
  // kappa tables of the matrix-free potential operator (3-D): volume [E][nqv]
  // and own-trace face [E][6][nqf] Gauss points, with the quadrature weights
  DevBuf<double> kv64, kf64;
  DevBuf<float> kv32, kf32;
  // hyperplane levels of the lexicographic element order
  std::vector<int64_t> lev_ptr;
  DevBuf<int> lev_elems;
  // Q1 vertex space
  int nvx[3] = {1, 1, 1};
  int64_t nvert = 0;
  DevBuf<double> gal;
  DevBuf<double> vst;               // [nvert][3^d] vertex stencil of the Galerkin operator
  std::vector<MgLevel> mg;          // mg[0] = vertex level
  DevBuf<double> cinv;
  DevBuf<float> cinv32;
  int nc = 0;
  // work
  std::vector<std::unique_ptr<DevBuf<double>>> wd;
  std::vector<std::unique_ptr<DevBuf<float>>> wf;
  DevBuf<double> vN, yN, tN;
  DevBuf<float> vN32, yN32, tN32;
  DevBuf<double> red;
  PinnedStage stage;
  // dataflow sweeps: packed (value, count) words [forward / backward][field][Nf * W]
  // (W = 1 in single, 2 in double precision), timeout flag
  DevBuf<uint64_t> df_wp, df_wp64;
  DevBuf<int> df_err;
  int df_grid[2] = {0, 0};  // double, float
  int df_spin = 1 << 22;
  bool df_on = true;
  // single-precision line sweeps: lines along axis line_ax (the longest), one
  // first element per line in level order
  bool lines_on = false;
  DevBuf<int> line_first;
  int nline = 0, line_len = 0, line_ax = 0, line_grid = 0;
  int64_t line_stride = 1;
  // geometric multigrid on the concentration blocks (instead of one BILU(0)
  // solve): level 0 is the fine grid (its unfactored blocks in A; its factors
  // are blk / blk32 above), levels 1.. the coarsened boxes with their Galerkin
  // operators and factors; the last level is solved with its dense inverse
  struct GLevel {
    int n[3] = {1, 1, 1};
    int64_t E = 0;
    DevBuf<int> nbr;
    std::vector<int64_t> lev_ptr;
    DevBuf<int> lev_elems;
    DevBuf<double> A, F;  // [m-1][E][nslot][bsz]: operator, BILU(0) factors
    DevBuf<float> A32, F32;  // A32 with rows of pot_ld(nb, true) floats (the block SpMV's layout)
    DevBuf<double> x, b, r, z, aux;  // [m-1][E nb] work vectors
    DevBuf<float> x32, b32, r32, z32, aux32;
    // dataflow sweeps of the level (as the fine level's): packed words and grids
    DevBuf<uint64_t> wp, wp64;
    int df_grid[2] = {0, 0};  // double, float
  };
  bool gmg = false;
  bool gmg_df = true;  // coarse-level sweeps as dataflow launches
  int gmg_nu = 2;
  std::vector<GLevel> gl;
  DevBuf<double> gmg_pi;  // [2^d][nb][nb] child prolongations
  DevBuf<float> gmg_pi32;
  int gmg_nc = 0;         // unknowns per field of the coarsest level
  DevBuf<double> gmg_cinv, gmg_cinvT;  // [m-1][nc][nc] coarsest inverse and its transpose
  DevBuf<float> gmg_cinv32, gmg_cinvT32;
  DevBuf<int> gmg_err;    // set when the coarsest level is singular (its inverse is then NaN)
  // numeric state: potential part (phi block, its inverse blocks, multigrid
  // hierarchy, lambda_max) and concentration part (BILU(0) factors), in double
  // and, for the mixed path, single precision
  bool phi_ok = false, phi32_ok = false, conc_ok = false, conc32_ok = false, assembled = false;
  bool ready() const { return phi_ok && conc_ok; }
  bool ready32() const { return phi32_ok && conc32_ok; }
};

void precond_destroy(Precond* p) { delete p; }

// ---- typed accessors -------------------------------------------------------------
template <typename T> struct Sel;
template <> struct Sel<double> {
  static double* blk(Precond& P) { return P.blk.p; }
  static double* dinv(Precond& P) { return P.dinv_phi.p; }
  static double* cblk(Precond& P, int64_t fstride) { return P.blk.p + fstride; }
  static double* blk1(Precond& P) { return P.blk1.p; }
  static double* dinv1(Precond& P) { return P.dinv1.p; }
  static double* mf(Precond& P) { return P.mf64.p; }
  static DevBuf<double>& lvec(Precond& P) { return P.lvec64; }
  static DevBuf<double>& lvec1(Precond& P) { return P.lvec1_64; }
  static DevCsr<double>& A(MgLevel& L) { return L.A; }
  static DevCsr<double>& Pm(MgLevel& L) { return L.P; }
  static DevCsr<double>& R(MgLevel& L) { return L.R; }
  static double* ldinv(MgLevel& L) { return L.dinv.p; }
  static double* cinv(Precond& P) { return P.cinv.p; }
  static double* w(Precond& P, size_t i) { return P.wd[i]->p; }
  static double* vN(Precond& P) { return P.vN.p; }
  static double* yN(Precond& P) { return P.yN.p; }
  static double* tN(Precond& P) { return P.tN.p; }
};
template <> struct Sel<float> {
  static float* blk(Precond& P) { return P.phi32.p; }
  static float* cblk(Precond& P, int64_t) { return P.blk32.p; }
  static float* blk1(Precond& P) { return P.blk1_32.p; }
  static float* dinv1(Precond& P) { return P.dinv1_32.p; }
  static float* mf(Precond& P) { return P.mf32.p; }
  static DevBuf<float>& lvec(Precond& P) { return P.lvec32; }
  static DevBuf<float>& lvec1(Precond& P) { return P.lvec1_32; }
  static float* dinv(Precond& P) { return P.dinv_phi32.p; }
  static DevCsr<float>& A(MgLevel& L) { return L.A32; }
  static DevCsr<float>& Pm(MgLevel& L) { return L.P32; }
  static DevCsr<float>& R(MgLevel& L) { return L.R32; }
  static float* ldinv(MgLevel& L) { return L.dinv32.p; }
  static float* cinv(Precond& P) { return P.cinv32.p; }
  static float* w(Precond& P, size_t i) { return P.wf[i]->p; }
  static float* vN(Precond& P) { return P.vN32.p; }
  static float* yN(Precond& P) { return P.yN32.p; }
  static float* tN(Precond& P) { return P.tN32.p; }
};


// ---- concentration-block multigrid: host set-up ----------------------------------
// hyperplane levels ix + iy + iz of the lexicographic elements of an n grid
static void hyperplane_order(int dim, const int* n, std::vector<int64_t>& ptr, std::vector<int>& flat) {
  const int nz = dim == 3 ? n[2] : 1;
  const int64_t E = int64_t(n[0]) * n[1] * nz;
  std::vector<std::vector<int>> lv(size_t(n[0] + n[1] + nz - 2));
  for (int64_t e = 0; e < E; ++e) {
    const int x = int(e % n[0]), y = int((e / n[0]) % n[1]), z = int(e / (int64_t(n[0]) * n[1]));
    lv[size_t(x + y + z)].push_back(int(e));
  }
  ptr.assign(1, 0);
  flat.clear();
  for (auto& v : lv) {
    flat.insert(flat.end(), v.begin(), v.end());
    ptr.push_back(int64_t(flat.size()));
  }
}

// slot-ordered neighbours (-x, +x, -y, +y, -z, +z), -1 on the boundary
static std::vector<int> grid_neighbours(int dim, const int* n) {
  const int nz = dim == 3 ? n[2] : 1;
  const int64_t E = int64_t(n[0]) * n[1] * nz;
  const int64_t stride[3] = {1, n[0], int64_t(n[0]) * n[1]};
  std::vector<int> nbr(size_t(E) * 2 * dim, -1);
  for (int64_t e = 0; e < E; ++e) {
    const int id[3] = {int(e % n[0]), int((e / n[0]) % n[1]), int(e / stride[2])};
    for (int a = 0; a < dim; ++a) {
      if (id[a] > 0) nbr[size_t(e * 2 * dim + 2 * a)] = int(e - stride[a]);
      if (id[a] < n[a] - 1) nbr[size_t(e * 2 * dim + 2 * a + 1)] = int(e + stride[a]);
    }
  }
  return nbr;
}

// Pi[c][k][i]: the coarse nodal basis function i at fine node k of child c
// (bit a of c: upper half along axis a), the tensor product of the 1-D Lagrange
// interpolants of the p + 1 coarse nodes at the child's nodes
static std::vector<double> child_prolongations(int p, int dim) {
  const RefTables R = make_ref_tables(p);
  const int nn = p + 1, nb = dim == 3 ? nn * nn * nn : nn * nn;
  double V[2][4][4];  // V[s][k][i] = l_i((x_k + 2 s - 1) / 2)
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < nn; ++k) {
      const double x = 0.5 * (R.xn[size_t(k)] + 2.0 * s - 1.0);
      for (int i = 0; i < nn; ++i) {
        double l = 1.0;
        for (int j = 0; j < nn; ++j)
          if (j != i) l *= (x - R.xn[size_t(j)]) / (R.xn[size_t(i)] - R.xn[size_t(j)]);
        V[s][k][i] = l;
      }
    }
  std::vector<double> Pi(size_t(1 << dim) * nb * nb);
  for (int c = 0; c < (1 << dim); ++c)
    for (int k = 0; k < nb; ++k)
      for (int i = 0; i < nb; ++i) {
        double v = 1.0;
        int kk = k, ii = i;
        for (int a = 0; a < dim; ++a) {
          v *= V[(c >> a) & 1][kk % nn][ii % nn];
          kk /= nn;
          ii /= nn;
        }
        Pi[(size_t(c) * nb + k) * nb + i] = v;
      }
  return Pi;
}

static void gmg_symbolic(dgnp_ctx& c, Precond& P) {
  P.gmg = true;
  P.gmg_nu = c.gmg_nu;
  P.gl.clear();
  P.gl.emplace_back();
  {
    Precond::GLevel& g = P.gl.back();
    for (int a = 0; a < 3; ++a) g.n[a] = c.n[a];
    g.E = c.E;
  }
  // coarsen by 2 along every axis while every count is even (down to a
  // single element where the counts allow)
  for (;;) {
    const Precond::GLevel& f = P.gl.back();
    bool even = true;
    for (int a = 0; a < c.dim; ++a) even = even && f.n[a] % 2 == 0;
    if (!even || f.E <= 1) break;
    Precond::GLevel g;
    for (int a = 0; a < 3; ++a) g.n[a] = a < c.dim ? f.n[a] / 2 : 1;
    g.E = int64_t(g.n[0]) * g.n[1] * g.n[2];
    P.gl.push_back(std::move(g));
  }
  const int64_t nc = P.gl.back().E * c.nb;
  DGNP_REQUIRE(nc <= 1024, DGNP_E_ARG,
               "the coarsest multigrid level has " + std::to_string(nc) +
                   " unknowns per field (at most 1024): the element counts need more factors of 2");
  P.gmg_nc = int(nc);
  P.gmg_df = getenv("DGNP_NO_DATAFLOW") == nullptr;
  const int nf = c.m - 1;
  for (size_t l = 1; l < P.gl.size(); ++l) {
    Precond::GLevel& g = P.gl[l];
    g.nbr.upload(grid_neighbours(c.dim, g.n), c.stream);
    std::vector<int> flat;
    hyperplane_order(c.dim, g.n, g.lev_ptr, flat);
    g.lev_elems.upload(flat, c.stream);
    if (P.gmg_df && l + 1 < P.gl.size()) {
      // packed (value, count) words of the forward and backward sweeps, all
      // fields: one word per float entry, two per double entry
      const size_t ne = size_t(nf) * size_t(g.E) * c.nb;
      g.wp.alloc(2 * ne);
      g.wp64.alloc(4 * ne);
      DGNP_HIP(hipMemset(g.wp.p, 0, g.wp.n * sizeof(uint64_t)));
      DGNP_HIP(hipMemset(g.wp64.p, 0, g.wp64.n * sizeof(uint64_t)));
      g.df_grid[0] = ilu_dataflow_grid<double>(c.nb, c.dim, g.E, nf);
      g.df_grid[1] = ilu_dataflow_grid<float>(c.nb, c.dim, g.E, nf);
    }
  }
  const std::vector<double> Pi = child_prolongations(c.p, c.dim);
  P.gmg_pi.upload(Pi, c.stream);
  std::vector<float> Pi32(Pi.begin(), Pi.end());
  P.gmg_pi32.upload(Pi32, c.stream);
  DGNP_HIP(hipStreamSynchronize(c.stream));
}

void precond_symbolic(dgnp_ctx& c) {
  if (!c.pc) c.pc = new Precond();
  Precond& P = *c.pc;
  P.nslot = 2 * c.dim + 1;
  P.bsz = int64_t(c.nb) * c.nb;
  P.pmg = c.phi_mg == DGNP_PHIMG_P || c.phi_mg == DGNP_PHIMG_PG;
  P.pmg_galerkin = c.phi_mg == DGNP_PHIMG_PG;
  P.nb1 = 1 << c.dim;
  // hyperplane levels ix + iy + iz
  const int L = c.n[0] + c.n[1] + (c.dim == 3 ? c.n[2] : 1) - (c.dim == 3 ? 2 : 1);
  std::vector<std::vector<int>> lv(static_cast<size_t>(L));
  for (int64_t e = 0; e < c.E; ++e) {
    int id[3] = {int(e % c.n[0]), int((e / c.n[0]) % c.n[1]),
                 c.dim == 3 ? int(e / (int64_t(c.n[0]) * c.n[1])) : 0};
    lv[size_t(id[0] + id[1] + id[2])].push_back(int(e));
  }
  P.lev_ptr.assign(1, 0);
  std::vector<int> flat;
  flat.reserve(size_t(c.E));
  for (auto& v : lv) {
    flat.insert(flat.end(), v.begin(), v.end());
    P.lev_ptr.push_back(int64_t(flat.size()));
  }
  P.lev_elems.upload(flat, c.stream);
  P.nvert = 1;
  for (int d = 0; d < 3; ++d) {
    P.nvx[d] = d < c.dim ? c.n[d] + 1 : 1;
    P.nvert *= P.nvx[d];
  }
  RefTables all[3] = {make_ref_tables(1), make_ref_tables(2), make_ref_tables(3)};
  upload_ref_tables_block(all, 3);
  upload_ref_tables_phi(all, 3);
  upload_gll_nodes(all, 3);
  P.red.alloc(size_t(reduce_scratch_size()));
  const int nf = c.m - 1;
  // The dataflow sweep pays off where the levels are narrow and the level
  // launches are latency-bound; with wide levels (several hundred elements on
  // average) the level-scheduled sweep streams the factor at higher bandwidth.
  const double width = double(c.E) / double(P.lev_ptr.size() - 1);
  P.df_on = getenv("DGNP_NO_DATAFLOW") == nullptr && (width < 256.0 || getenv("DGNP_DATAFLOW") != nullptr);
  if (const char* sl = getenv("DGNP_DATAFLOW_SPIN")) P.df_spin = std::max(0, atoi(sl));
  P.df_wp.alloc(size_t(2) * nf * c.Nf);
  P.df_wp64.alloc(size_t(4) * nf * c.Nf);
  P.df_err.alloc(1);
  DGNP_HIP(hipMemsetAsync(P.df_wp.p, 0, P.df_wp.n * sizeof(uint64_t), c.stream));
  DGNP_HIP(hipMemsetAsync(P.df_wp64.p, 0, P.df_wp64.n * sizeof(uint64_t), c.stream));
  DGNP_HIP(hipMemsetAsync(P.df_err.p, 0, sizeof(int), c.stream));
  DGNP_HIP(hipStreamSynchronize(c.stream));
  P.df_grid[0] = ilu_dataflow_grid<double>(c.nb, c.dim, c.E, nf);
  P.df_grid[1] = ilu_dataflow_grid<float>(c.nb, c.dim, c.E, nf);
  // lines along the longest axis, ordered by the level of their first element
  {
    int ax = 0;
    for (int d = 1; d < c.dim; ++d)
      if (c.n[d] > c.n[ax]) ax = d;
    const int n3[3] = {c.n[0], c.n[1], c.dim == 3 ? c.n[2] : 1};
    const int64_t stride[3] = {1, n3[0], int64_t(n3[0]) * n3[1]};
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    std::vector<std::vector<int>> bylev(size_t(n3[o1] + n3[o2] - 1));
    for (int b = 0; b < n3[o2]; ++b)
      for (int a = 0; a < n3[o1]; ++a) bylev[size_t(a + b)].push_back(int(a * stride[o1] + b * stride[o2]));
    std::vector<int> first;
    for (auto& v : bylev) first.insert(first.end(), v.begin(), v.end());
    P.line_first.upload(first, c.stream);
    P.nline = int(first.size());
    P.line_len = n3[ax];
    P.line_ax = ax;
    P.line_stride = stride[ax];
    P.line_grid = ilu_lines_grid(c.nb, c.dim, P.nline, nf);
    // 64-row blocks (p = 3) go by lines at any level width: with every line
    // resident the sweep streams the factors (64x16x8 channel 531 -> 296 us,
    // 128x32x16 channel 2.0 -> 1.84 ms per forward sweep, against the element
    // order and the level launches).  Smaller blocks go by lines where the
    // levels are wide (256x64x32 channel at p = 1: 350 level launches per
    // sweep; Krylov part of the solve 1.15 -> 0.85 s) and keep the element
    // order where they are narrow (16^3 cube, p = 2: 68 against 81 us).
    P.lines_on = (c.nb >= 64 || width >= 256.0) && getenv("DGNP_DATAFLOW") == nullptr &&
                 getenv("DGNP_NO_DATAFLOW") == nullptr;
    const char* sw = getenv("DGNP_ILU_SWEEP");  // "line", "element" or "level"
    if (sw && std::string(sw) == "line") {
      P.lines_on = true;
    } else if (sw && std::string(sw) == "element") {
      P.lines_on = false;
      P.df_on = true;
    } else if (sw && std::string(sw) == "level") {
      P.lines_on = false;
      P.df_on = false;
    }
  }
  if (c.conc_pc == DGNP_CPC_GMG) gmg_symbolic(c, P);
}

// Reports (and clears) a dataflow sweep that ended at its wait limit; the
// counters are reset so that later sweeps start consistent.  Synchronises.
// A new linearisation point clears such a state silently (the failed solve has
// reported it already, possibly as a non-finite vector).
void precond_check(dgnp_ctx& c, bool report) {
  if (!c.pc || !c.pc->df_err.p) return;
  Precond& P = *c.pc;
  int h = 0;
  DGNP_HIP(hipDeviceSynchronize());
  DGNP_HIP(hipMemcpy(&h, P.df_err.p, sizeof(int), hipMemcpyDeviceToHost));
  if (h == 0) return;
  DGNP_HIP(hipMemset(P.df_wp.p, 0, P.df_wp.n * sizeof(uint64_t)));
  DGNP_HIP(hipMemset(P.df_wp64.p, 0, P.df_wp64.n * sizeof(uint64_t)));
  for (auto& g : P.gl) {
    if (g.wp.p) DGNP_HIP(hipMemset(g.wp.p, 0, g.wp.n * sizeof(uint64_t)));
    if (g.wp64.p) DGNP_HIP(hipMemset(g.wp64.p, 0, g.wp64.n * sizeof(uint64_t)));
  }
  DGNP_HIP(hipMemset(P.df_err.p, 0, sizeof(int)));
  DGNP_HIP(hipDeviceSynchronize());
  if (report) throw Error(DGNP_E_BREAKDOWN, "ILU dataflow sweep exceeded its wait limit");
}

// ---- vertex matrix from the per-element Galerkin blocks ----------------------
// CSR of the Galerkin vertex operator from its dense per-vertex stencil
// st[r][o] (o over {-1, 0, 1}^d, first axis fastest); exact zeros are dropped
// the vertex operator as CSR from its stencil st (exact zeros left out): row
// lengths, their prefix sums, then the entries, row chunks on the host pool
// (small operators in one serial pass).
// storage (may be empty): a matrix of the same order whose arrays are reused,
// so that a new set-up writes into memory that is already mapped
static Csr vertex_matrix(const dgnp_ctx& c, const Precond& P, const double* st, Csr&& storage) {
  const int d = c.dim;
  const int ns = d == 3 ? 27 : 9;
  const int n = int(P.nvert);
  Csr A;
  if (storage.n == n) {
    A.rp = std::move(storage.rp);
    A.ci = std::move(storage.ci);
    A.v = std::move(storage.v);
  }
  A.n = A.m = n;
  A.rp.resize(size_t(n) + 1);
  A.rp[0] = 0;
  // columns of the ns stencil entries of row r (-1 outside the grid): the
  // entry off couples vertex r to r + delta[off] when every coordinate moved
  // stays inside the grid
  int delta[27];
  for (int off = 0; off < ns; ++off)
    delta[off] = (off % 3 - 1) + (d > 1 ? ((off / 3) % 3 - 1) * P.nvx[0] : 0) +
                 (d > 2 ? (off / 9 - 1) * P.nvx[0] * P.nvx[1] : 0);
  auto columns = [&](int r, int* col) {
    const int rc[3] = {r % P.nvx[0], (r / P.nvx[0]) % P.nvx[1], r / (P.nvx[0] * P.nvx[1])};
    bool in[3][3];  // in[a][o]: coordinate a moved by o - 1 stays inside
    for (int a = 0; a < 3; ++a)
      for (int o = 0; o < 3; ++o) in[a][o] = a >= d ? o == 1 : (rc[a] + o - 1 >= 0 && rc[a] + o - 1 < P.nvx[a]);
    for (int off = 0; off < ns; ++off) {
      const bool ok = in[0][off % 3] && in[1][(off / 3) % 3] && (d < 3 || in[2][off / 9]);
      col[off] = ok ? r + delta[off] : -1;
    }
  };
  if (n < 8192) {  // small: one serial pass (the pool would run it serially anyway)
    A.ci.clear();
    A.v.clear();
    int col[27];
    for (int r = 0; r < n; ++r) {
      columns(r, col);
      for (int off = 0; off < ns; ++off) {
        const double val = st[size_t(r) * ns + off];
        if (val == 0.0 || col[off] < 0) continue;
        A.ci.push_back(col[off]);
        A.v.push_back(val);
      }
      A.rp[size_t(r) + 1] = int(A.ci.size());
    }
    return A;
  }
  host_parallel_rows(n, [&](int r0, int r1) {
    int col[27];
    for (int r = r0; r < r1; ++r) {
      columns(r, col);
      int k = 0;
      for (int off = 0; off < ns; ++off)
        if (st[size_t(r) * ns + off] != 0.0 && col[off] >= 0) ++k;
      A.rp[size_t(r) + 1] = k;
    }
  });
  for (int r = 0; r < n; ++r) A.rp[size_t(r) + 1] += A.rp[size_t(r)];
  A.ci.resize(size_t(A.rp[size_t(n)]));
  A.v.resize(A.ci.size());
  host_parallel_rows(n, [&](int r0, int r1) {
    int col[27];
    for (int r = r0; r < r1; ++r) {
      columns(r, col);
      int k = A.rp[size_t(r)];
      for (int off = 0; off < ns; ++off) {
        const double val = st[size_t(r) * ns + off];
        if (val == 0.0 || col[off] < 0) continue;
        A.ci[size_t(k)] = col[off];
        A.v[size_t(k)] = val;
        ++k;
      }
    }
  });
  return A;
}

static void upload_csr(DevCsr<double>& D, const Csr& A, PinnedStage& st, hipStream_t s) {
  D.n = A.n;
  st.upload(D.rp, A.rp.data(), A.rp.size(), s);
  st.upload(D.ci, A.ci.data(), A.ci.size(), s);
  st.upload(D.v, A.v.data(), A.v.size(), s);
}

// single-precision copy of a device matrix: its values converted on the
// device, its index arrays those of the double copy
static void copy_csr32(DevCsr<float>& D, const DevCsr<double>& A, hipStream_t s) {
  D.n = A.n;
  D.rp.release();
  D.ci.release();
  D.rpx = A.rptr();
  D.cix = A.cptr();
  D.v.alloc(A.v.n);
  cvt_d2f(A.v.p, D.v.p, int64_t(A.v.n), s);
}

// per V-cycle level: 5 vectors (x, b, r, d, z) for each precision; arrays of
// unchanged size are kept.  Levels: the order-p DG level, with p-multigrid the
// p = 1 DG level, then the vertex / aggregation levels.
static int64_t level_size(const dgnp_ctx& c, const Precond& P, size_t l) {
  if (l == 0) return c.Nf;
  if (P.pmg && l == 1) return c.E * P.nb1;
  return P.mg[l - (P.pmg ? 2 : 1)].n;
}
static size_t level_count(const Precond& P) { return 1 + (P.pmg ? 1 : 0) + P.mg.size(); }

static void ensure_work(dgnp_ctx& c, Precond& P) {
  const size_t nlev = level_count(P);
  while (P.wd.size() < 5 * nlev) {
    P.wd.emplace_back(new DevBuf<double>());
    P.wf.emplace_back(new DevBuf<float>());
  }
  P.wd.resize(5 * nlev);
  P.wf.resize(5 * nlev);
  for (size_t l = 0; l < nlev; ++l)
    for (int k = 0; k < 5; ++k) P.wd[l * 5 + k]->alloc(size_t(level_size(c, P, l)));
  P.vN.alloc(size_t(c.N));
  P.yN.alloc(size_t(c.N));
  P.tN.alloc(size_t(c.N));
  if (P.pmg) P.mf64.alloc(size_t(c.Nf));
}

// work vectors of the element levels only (order p and, with p-multigrid,
// p = 1): their sizes do not depend on the host hierarchy
static void ensure_work_elem(dgnp_ctx& c, Precond& P, bool f32) {
  const size_t ne = P.pmg ? 2 : 1;
  while (P.wd.size() < 5 * ne) {
    P.wd.emplace_back(new DevBuf<double>());
    P.wf.emplace_back(new DevBuf<float>());
  }
  for (size_t l = 0; l < ne; ++l)
    for (int k = 0; k < 5; ++k) {
      P.wd[l * 5 + k]->alloc(size_t(level_size(c, P, l)));
      if (f32) P.wf[l * 5 + k]->alloc(size_t(level_size(c, P, l)));
    }
  if (P.pmg) {
    P.mf64.alloc(size_t(c.Nf));
    if (f32) P.mf32.alloc(size_t(c.Nf));
  }
}

static void ensure_work32(dgnp_ctx& c, Precond& P) {
  const size_t nlev = level_count(P);
  for (size_t l = 0; l < nlev; ++l)
    for (int k = 0; k < 5; ++k) P.wf[l * 5 + k]->alloc(size_t(level_size(c, P, l)));
  P.vN32.alloc(size_t(c.N));
  P.yN32.alloc(size_t(c.N));
  P.tN32.alloc(size_t(c.N));
  if (P.pmg) P.mf32.alloc(size_t(c.Nf));
}

// potential rows of J applied to a potential-only vector: y = A_phiphi x at
// order p, matrix-free (the Jacobian operator with only the potential input
// read and only the potential rows formed)
template <typename T>
static void phi_mf_apply(dgnp_ctx& c, const T* x, T* y, hipStream_t s) {
  const bool f32 = std::is_same<T, float>::value;
  ScopeTimer tm(c, f32 ? "phi_apply_f32" : "phi_apply", s);
  KArgs A = c.kargs();
  Precond& P = *c.pc;
  if (c.dim == 3) {  // SIPG with tabulated kappa (kernels_phi.hip)
    const size_t nqv = size_t(c.nq) * c.nq * c.nq, nqf = size_t(c.nq) * c.nq;
    if constexpr (std::is_same<T, float>::value) {
      DGNP_REQUIRE(P.kv32.p && P.kf32.p && P.kv32.n == size_t(c.E) * nqv && P.kf32.n == size_t(c.E) * 6 * nqf,
                   DGNP_E_STATE, "single-precision potential operator tables not set up");
      launch_phi_op<float>(c.p, A, x, P.kv32.p, P.kf32.p, y, s);
    } else {
      DGNP_REQUIRE(P.kv64.p && P.kf64.p && P.kv64.n == size_t(c.E) * nqv && P.kf64.n == size_t(c.E) * 6 * nqf,
                   DGNP_E_STATE, "potential operator tables not set up");
      launch_phi_op<double>(c.p, A, x, P.kv64.p, P.kf64.p, y, s);
    }
    return;
  }
  A.vin_mask = 1u;
  const void* xs = f32 ? static_cast<const void*>(c.d_x32.p) : static_cast<const void*>(c.d_x.p);
  launch_dg(c.dim, c.p, c.m, f32, M_JACP, A, xs, x, y, nullptr, s);
}

// largest eigenvalue of D_b^{-1} A on a potential level by power iteration on the device, in
// the arithmetic of the smoother that uses it: from a hashed start vector 20
// steps, from the previous linearisation point's last vector 8 steps
// (renormalised every 4 steps; the estimate is the growth of the last step).
// The norms stay on the device until the end (one host wait).
// op(x, y): x <- D^{-1} A x with y as work space (n entries).
template <typename T, typename Op>
static double power_lmax(dgnp_ctx& c, Precond& P, hipStream_t s, int64_t n, Op op, T* x, T* y, DevBuf<T>& keep) {
  double* sq = P.red.p;            // [0]: |x|^2 before the last step, [1]: after, [2]: start
  double* part = P.red.p + MAXV;   // block partials
  auto norm2 = [&](const T* v, double* out) {
    if constexpr (std::is_same<T, float>::value)
      vsq_into(v, n, out, part, s);
    else
      vdots_into(v, 0, 1, v, n, out, part, s);
  };
  const bool warm = keep.n == size_t(n);
  if (warm)
    vcopy<T>(keep.p, x, n, s);
  else
    vfill_hash<T>(x, n, s);
  norm2(x, sq + 2);
  vscale_rsqrt_inplace<T>(sq + 2, x, n, s);
  const int groups = warm ? 2 : 5;
  for (int g = 0; g < groups; ++g) {
    for (int it = 0; it < 4; ++it) {
      if (it == 3) norm2(x, sq);
      op(x, y);
    }
    norm2(x, sq + 1);
    vscale_rsqrt_inplace<T>(sq + 1, x, n, s);
  }
  keep.alloc(size_t(n));
  vcopy<T>(x, keep.p, n, s);
  double h[2] = {0.0, 0.0};
  DGNP_HIP(hipMemcpyAsync(h, sq, sizeof(h), hipMemcpyDeviceToHost, s));
  DGNP_HIP(hipStreamSynchronize(s));
  const double lam = std::sqrt(h[1]) / std::sqrt(h[0]);
  if (!(lam > 0.0) || !std::isfinite(lam)) {
    keep.release();
    throw Error(DGNP_E_NONFINITE, "power iteration failed");
  }
  return lam;
}

// x <- D_b^{-1} A x on an element-block level (nb rows per block)
template <typename T>
static auto block_op(dgnp_ctx& c, int nb, const T* blk, const T* dinv, hipStream_t s) {
  return [&c, nb, blk, dinv, s](T* x, T* y) {
    launch_bspmv<T>(nb, c.dim, c.E, blk, c.d_nbr.p, x, nullptr, T(1), T(0), y, s);
    launch_bdiag<T>(nb, c.E, dinv, y, x, s);
  };
}

static bool trace_setup() {
  static const bool on = getenv("DGNP_TRACE_SETUP") != nullptr;
  return on;
}

struct PhaseClock {
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  hipStream_t s;
  explicit PhaseClock(hipStream_t st) : s(st) {}
  void mark(const char* what) {
    if (!trace_setup()) return;
    (void)hipStreamSynchronize(s);
    const auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "[setup] %-22s %8.3f ms\n", what, 1e3 * std::chrono::duration<double>(now - t).count());
    t = now;
  }
};

// Concentration multigrid, numeric part (see gmg_symbolic): the fine level's
// unfactored blocks are kept (gmg_copy_fine, before the fine blocks are
// factorised in place), every coarser level gets its Galerkin operator and
// (all but the coarsest) its BILU(0) factors, the coarsest its dense inverse
// (Gauss-Jordan on the device, in double); nothing waits for the host, so the
// set-up stays queued behind the assembly.  The Galerkin chain runs on s, each
// level's factorisation on side stream 1 as soon as its operator exists; s
// waits for them at the end.  Single-precision copies with f32.
static void gmg_copy_fine(dgnp_ctx& c, Precond& P, bool f32, hipStream_t s) {
  const int nf = c.m - 1, nb = c.nb;
  Precond::GLevel& g0 = P.gl[0];
  const int64_t per0 = g0.E * P.nslot * P.bsz;
  g0.A.alloc(size_t(nf * per0));
  ScopeTimer tm(c, "gmg_copy", s);
  DGNP_HIP(hipMemcpyAsync(g0.A.p, P.blk.p + per0, size_t(nf * per0) * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (f32) {
    g0.A32.alloc(g0.A.n / nb * pot_ld(nb, true));
    cvt_d2f_rows(g0.A.p, g0.A32.p, int64_t(g0.A.n / nb), nb, pot_ld(nb, true), s);
  }
}

static void gmg_numeric(dgnp_ctx& c, Precond& P, bool f32, hipStream_t s) {
  const int nf = c.m - 1, ns = P.nslot, nb = c.nb;
  auto per = [&](const Precond::GLevel& g) { return g.E * ns * P.bsz; };
  hipStream_t fs = P.side.stream(1);
  bool forked = false;
  for (size_t l = 1; l < P.gl.size(); ++l) {
    Precond::GLevel& f = P.gl[l - 1];
    Precond::GLevel& g = P.gl[l];
    g.A.alloc(size_t(nf * per(g)));
    {
      ScopeTimer tm(c, "gmg_galerkin", s);
      launch_gmg_galerkin(nb, c.dim, nf, f.A.p, per(f), l == 1 ? c.d_nbr.p : f.nbr.p, f.n, P.gmg_pi.p, g.A.p,
                          per(g), g.E, s);
    }
    if (l + 1 < P.gl.size()) {
      g.F.alloc(g.A.n);
      DGNP_HIP(hipMemcpyAsync(g.F.p, g.A.p, g.A.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      float* b32 = nullptr;
      if (f32) {
        g.F32.alloc(g.A.n);
        b32 = g.F32.p;
      }
      P.side.order(s, fs);
      forked = true;
      ScopeTimer tm(c, "gmg_factor", fs);
      for (size_t lv = 0; lv + 1 < g.lev_ptr.size(); ++lv)
        launch_ilu_factor(nb, c.dim, nf, per(g), g.F.p, g.nbr.p, g.lev_elems.p, g.lev_ptr[lv],
                          g.lev_ptr[lv + 1] - g.lev_ptr[lv], fs, b32);
    }
    if (f32) {
      g.A32.alloc(g.A.n / nb * pot_ld(nb, true));
      cvt_d2f_rows(g.A.p, g.A32.p, int64_t(g.A.n / nb), nb, pot_ld(nb, true), s);
    }
  }
  // work vectors of every level
  for (size_t l = 0; l < P.gl.size(); ++l) {
    Precond::GLevel& g = P.gl[l];
    const size_t n = size_t(nf * g.E * nb);
    g.r.alloc(n);
    g.z.alloc(n);
    if (l > 0) {
      g.x.alloc(n);
      g.b.alloc(n);
      g.aux.alloc(n);
    }
    if (f32) {
      g.r32.alloc(n);
      g.z32.alloc(n);
      if (l > 0) {
        g.x32.alloc(n);
        g.b32.alloc(n);
        g.aux32.alloc(n);
      }
    }
  }
  // coarsest level: dense inverse per field, on the device
  Precond::GLevel& gc = P.gl.back();
  const int64_t n = P.gmg_nc;
  P.gmg_cinv.alloc(size_t(nf * n * n));
  P.gmg_cinvT.alloc(size_t(nf * n * n));
  P.gmg_err.alloc(1);
  {
    ScopeTimer tm(c, "gmg_coarse_inverse", s);
    launch_gmg_dense_inverse(nb, c.dim, nf, gc.A.p, per(gc), P.gl.size() == 1 ? c.d_nbr.p : gc.nbr.p, gc.E,
                             P.gmg_cinv.p, P.gmg_cinvT.p, P.gmg_err.p, s);
  }
  if (f32) {
    P.gmg_cinv32.alloc(P.gmg_cinv.n);
    P.gmg_cinvT32.alloc(P.gmg_cinvT.n);
    cvt_d2f(P.gmg_cinv.p, P.gmg_cinv32.p, int64_t(P.gmg_cinv.n), s);
    cvt_d2f(P.gmg_cinvT.p, P.gmg_cinvT32.p, int64_t(P.gmg_cinvT.n), s);
  }
  if (forked) P.side.order(fs, s);
}

void precond_numeric(dgnp_ctx& c, bool f32, hipStream_t s, bool assemble_only, int parts) {
  precond_check(c, false);
  Precond& P = *c.pc;
  P.stage.reset();  // precond_check has synchronised the device: earlier copies are complete
  P.side.next = 0;
  PhaseClock clk(s);
  const int64_t per_field = c.E * P.nslot * P.bsz;
  const bool phi = (parts & PC_PHI) != 0, conc = (parts & PC_CONC) != 0;
  if ((parts & PC_WARM) == 0) {  // cold power iterations: results do not depend on earlier solves
    P.lvec32.release();
    P.lvec64.release();
    P.lvec1_32.release();
    P.lvec1_64.release();
  }
  P.blk.alloc(size_t(c.m * per_field));
  // with both parts the potential field is assembled on s and the
  // concentration fields by the concentration part on a side stream, so that
  // their factorisation runs beside the potential's set-up.  Both assemblies
  // fill the device, so they are ordered: the potential first (its hierarchy
  // is then built on the host beside the factorisation), except with 64-row
  // blocks, whose factorisation chain is the longest part of the set-up and
  // starts first
  const bool split = phi && conc && !assemble_only;
  const bool conc_first = split && c.nb >= 64;
  // with a large vertex grid the host hierarchy is the longest part of the
  // set-up: the concentration part is then queued behind the kernels of the
  // vertex stencil the host waits for (DGNP_CONC_LATE=0 / 1 forces the choice;
  // the order changes no result)
  const char* late_env = getenv("DGNP_CONC_LATE");
  const bool conc_late =
      split && !conc_first && (late_env ? atoi(late_env) != 0 : P.nvert >= (int64_t(1) << 16));
  if (!split) {
    ScopeTimer tm(c, "assemble", s);
    const int f0 = phi ? 0 : 1, f1 = conc ? c.m : 1;
    launch_assemble(c.dim, c.p, c.m, f0, f1 - f0, c.kargs(), c.d_x.p, P.blk.p, s);
  }
  clk.mark("assemble");
  if (phi) P.phi_ok = P.phi32_ok = P.phi32_blocks = false;
  if (conc) P.conc_ok = P.conc32_ok = false;
  if (assemble_only) {
    DGNP_HIP(hipStreamSynchronize(s));
    P.assembled = true;
    return;
  }
  // concentration blocks: BILU(0) level by level, then their single copy; all
  // of it is queued without a host wait on side streams (the fine chain, the
  // multigrid levels), so that with both parts it runs on the device beside
  // the potential's device work while the host builds the potential
  // hierarchy; s waits for the side streams at the end of the set-up
  hipStream_t conc_streams[2] = {nullptr, nullptr};
  auto join_conc = [&]() {
    for (hipStream_t& q : conc_streams)
      if (q) {
        P.side.order(q, s);
        q = nullptr;
      }
  };
  auto conc_part = [&]() {
    hipStream_t fs = P.side.stream(0);
    P.side.order(s, fs);
    conc_streams[0] = fs;
    if (split) {
      ScopeTimer tm(c, "assemble", fs);
      launch_assemble(c.dim, c.p, c.m, 1, c.m - 1, c.kargs(), c.d_x.p, P.blk.p, fs);
    }
    if (conc_first) P.side.order(fs, s);
    // the single-precision copies are written by the factorisation kernels
    // themselves, block by block as each is finished
    float* b32 = nullptr;
    if (f32) {
      P.blk32.alloc(size_t((c.m - 1) * per_field));
      b32 = P.blk32.p;
    }
    // the fine factorisation runs on side stream 0; with the multigrid its
    // fine level first keeps a copy of the unfactored blocks, and the coarse
    // levels run beside the fine factorisation (Galerkin chain on side
    // stream 2, their factorisations on side stream 1)
    if (P.gmg) {
      gmg_copy_fine(c, P, f32, fs);
      conc_streams[1] = P.side.stream(2);
      P.side.order(fs, conc_streams[1]);
      gmg_numeric(c, P, f32, conc_streams[1]);
    }
    for (size_t l = 0; l + 1 < P.lev_ptr.size(); ++l) {
      ScopeTimer tm(c, "ilu_factor", fs);
      launch_ilu_factor(c.nb, c.dim, c.m - 1, per_field, P.blk.p + per_field, c.d_nbr.p, P.lev_elems.p,
                        P.lev_ptr[l], P.lev_ptr[l + 1] - P.lev_ptr[l], fs, b32);
    }
    if (trace_setup()) {
      join_conc();
      clk.mark("concentration factors (fine level, multigrid levels)");
    }
  };
  if (split) {
    if (conc_first) conc_part();
    {
      ScopeTimer tm(c, "assemble", s);
      launch_assemble(c.dim, c.p, c.m, 0, 1, c.kargs(), c.d_x.p, P.blk.p, s);
    }
    if (!conc_first && !conc_late) conc_part();
  }
  if (phi) {
    // potential block: element-diagonal inverses (block-Jacobi smoother)
    P.dinv_phi.alloc(size_t(c.E * P.bsz));
    {
      ScopeTimer tm(c, "block_inverse", s);
      launch_block_inverse(c.nb, c.E, P.blk.p, P.nslot, P.dinv_phi.p, s);
    }
    clk.mark("block inverse");
    // p-multigrid: the potential block at p = 1, re-discretised (interior
    // penalty for p = 1, at the state's corner values) or as the Galerkin
    // product of the order-p block, and its inverse blocks
    const double* gal_blk = P.blk.p;
    int gal_p = c.p;
    if (P.pmg && c.dim == 3) {
      // kappa tables of the matrix-free potential operator: double always (the
      // double V-cycle is usable after either set-up), single with f32
      const int nqv = c.nq * c.nq * c.nq, nqf = c.nq * c.nq;
      P.kv64.alloc(size_t(c.E) * nqv);
      P.kf64.alloc(size_t(c.E) * 6 * nqf);
      launch_phi_kappa<double>(c.p, c.m, c.kargs(), c.d_x.p, P.kv64.p, P.kf64.p, s);
      if (f32) {
        P.kv32.alloc(size_t(c.E) * nqv);
        P.kf32.alloc(size_t(c.E) * 6 * nqf);
        launch_phi_kappa<float>(c.p, c.m, c.kargs(), c.d_x.p, P.kv32.p, P.kf32.p, s);
      }
    }
    if (P.pmg) {
      P.x1.alloc(size_t(c.m) * c.E * P.nb1);
      launch_p1_inject(c.dim, c.p, c.d_x.p, P.x1.p, c.m, c.E, s);
      KArgs A1 = c.kargs();
      A1.delta = c.delta / double(c.p * c.p);
      P.blk1.alloc(size_t(c.E) * P.nslot * P.nb1 * P.nb1);
      if (P.pmg_galerkin) {
        // P^T A_p P block by block (P: the element-local p = 1 -> p interpolation)
        launch_q1_galerkin(c.dim, c.p, c.E, P.blk.p, P.blk1.p, s);
      } else {
        ScopeTimer tm(c, "assemble", s);
        launch_assemble(c.dim, 1, c.m, 0, 1, A1, P.x1.p, P.blk1.p, s);
      }
      P.dinv1.alloc(size_t(c.E) * P.nb1 * P.nb1);
      launch_block_inverse(P.nb1, c.E, P.blk1.p, P.nslot, P.dinv1.p, s);
      gal_blk = P.blk1.p;
      gal_p = 1;
      clk.mark("p = 1 level");
    }
    // Galerkin projection onto Q1 vertices (of the order-p block, or of the
    // p = 1 block with p-multigrid), then host SA setup
    const int NV = 1 << c.dim;
    P.gal.alloc(size_t(c.E) * P.nslot * NV * NV);
    launch_q1_galerkin(c.dim, gal_p, c.E, gal_blk, P.gal.p, s);
    P.vst.alloc(size_t(P.nvert) * (c.dim == 3 ? 27 : 9));
    launch_vertex_stencil(c.dim, P.gal.p, c.d_nbr.p, c.n, P.nvert, P.vst.p, s);
    if (conc_late) conc_part();
    // the stencil comes back into the pinned staging memory (kept between
    // set-ups: a copy into pageable memory goes through the runtime's bounce
    // buffer, and a fresh array of this size costs its page faults every time)
    double* st = static_cast<double*>(P.stage.take(P.vst.n * sizeof(double)));
    DGNP_HIP(hipMemcpyAsync(st, P.vst.p, P.vst.n * sizeof(double), hipMemcpyDeviceToHost, s));
    DGNP_HIP(hipStreamSynchronize(s));
    clk.mark("galerkin + stencil");
    // The vertex matrix and its aggregation hierarchy are built on a helper
    // host thread, after this thread has queued the single-precision
    // potential blocks (the concentration part is already queued on its side
    // streams); this thread then runs the element levels' lambda_max
    // estimates on the device.
    // Within one Newton solve the aggregates and smoothed prolongators of the
    // first set-up are kept (only R A P is recomputed): the potential block
    // changes with the concentrations, its vertex graph does not.
    const bool no_reuse = getenv("DGNP_NO_AMG_REUSE") != nullptr;
    const bool reuse =
        !no_reuse && (parts & PC_WARM) != 0 && !P.sa_prev.A.empty() && P.sa_prev.A[0].n == int(P.nvert);
    if (f32) {
      // single-precision potential blocks: they do not depend on the host
      // hierarchy, so they too run while the host builds it
      // (the assembled blocks only without p-multigrid: its order-p level is
      // applied matrix-free and needs the inverse diagonal blocks alone)
      const int ld32 = pot_ld(c.nb, true);
      if (!P.pmg) {
        P.phi32.alloc(size_t(c.E) * P.nslot * c.nb * ld32);
        cvt_d2f_rows(P.blk.p, P.phi32.p, c.E * P.nslot * c.nb, c.nb, ld32, s);
        P.phi32_blocks = true;
      }
      P.dinv_phi32.alloc(size_t(c.E) * c.nb * ld32);
      cvt_d2f_rows(P.dinv_phi.p, P.dinv_phi32.p, c.E * c.nb, c.nb, ld32, s);
      if (P.pmg) {
        P.blk1_32.alloc(P.blk1.n);
        cvt_d2f(P.blk1.p, P.blk1_32.p, int64_t(P.blk1.n), s);
        P.dinv1_32.alloc(P.dinv1.n);
        cvt_d2f(P.dinv1.p, P.dinv1_32.p, int64_t(P.dinv1.n), s);
      }
    }
    // the host hierarchy starts once the device work above is queued (its
    // worker pool would otherwise compete with the launches)
    AmgHierarchy H;
    std::exception_ptr sa_err;
    std::thread sa_thread([&]() {
      try {
        // the previous set-up's vertex matrix lends its arrays (only its order is
        // read afterwards, by the reuse check)
        Csr storage;
        if (!P.sa_prev.A.empty() && P.sa_prev.A[0].n == int(P.nvert)) {
          storage.n = P.sa_prev.A[0].n;
          storage.rp = std::move(P.sa_prev.A[0].rp);
          storage.ci = std::move(P.sa_prev.A[0].ci);
          storage.v = std::move(P.sa_prev.A[0].v);
        }
        Csr A1 = vertex_matrix(c, P, st, std::move(storage));
        // the kept hierarchy gives up its prolongators and product arrays
        H = reuse ? sa_setup_reuse(std::move(A1), std::move(P.sa_prev), &P.sa_x0)
                  : sa_setup(std::move(A1), 12, 256, 0.0, &P.sa_x0, &P.sa_prev);  // lends its arrays
      } catch (...) {
        sa_err = std::current_exception();
        P.sa_prev = AmgHierarchy();  // possibly taken apart: the next set-up starts afresh
      }
    });
    struct Joiner {
      std::thread& t;
      ~Joiner() {
        if (t.joinable()) t.join();
      }
    } joiner{sa_thread};
    // lambda_max of the smoothers' D^{-1} A on the element levels, in the
    // arithmetic of the smoother
    ensure_work_elem(c, P, f32);
    auto lmax_levels = [&](auto tag) {
      using T = decltype(tag);
      T* x0 = Sel<T>::w(P, 0);
      T* y0 = Sel<T>::w(P, 1);
      DevBuf<T>& keep0 = Sel<T>::lvec(P);
      if (P.pmg) {
        const T* dv = Sel<T>::dinv(P);
        auto op0 = [&](T* x, T* y) {
          phi_mf_apply<T>(c, x, y, s);
          launch_bdiag<T>(c.nb, c.E, dv, y, x, s);
        };
        P.lmax0 = power_lmax<T>(c, P, s, c.Nf, op0, x0, y0, keep0);
        DevBuf<T>& keep1 = Sel<T>::lvec1(P);
        P.lmax1 = power_lmax<T>(c, P, s, c.E * P.nb1, block_op<T>(c, P.nb1, Sel<T>::blk1(P), Sel<T>::dinv1(P), s),
                                Sel<T>::w(P, 5), Sel<T>::w(P, 6), keep1);
      } else {
        P.lmax0 = power_lmax<T>(c, P, s, c.Nf, block_op<T>(c, c.nb, Sel<T>::blk(P), Sel<T>::dinv(P), s), x0, y0,
                                keep0);
      }
    };
    if (f32)
      lmax_levels(float(0));
    else
      lmax_levels(double(0));
    clk.mark("lmax level 0");
    sa_thread.join();
    if (sa_err) std::rethrow_exception(sa_err);
    // kept again only once this hierarchy's uploads are queued: a set-up that
    // fails from here on leaves none, and the next one starts afresh
    P.sa_prev = AmgHierarchy();
    clk.mark(reuse ? "vertex matrix + sa setup (prolongators kept)" : "vertex matrix + sa setup");
    if (trace_setup()) {
      fprintf(stderr, "[setup] hierarchy: DG %lld", (long long)c.Nf);
      for (auto& A : H.A) fprintf(stderr, " -> %d (nnz %zu)", A.n, A.v.size());
      fprintf(stderr, "\n");
    }
    // with the prolongators kept, the device already holds them: the
    // hierarchy they came from was uploaded in full by the previous set-up
    // (it is kept only once its uploads are queued)
    const bool keep_pr = reuse && P.mg.size() == H.A.size();
    P.mg.resize(H.A.size());  // device arrays of equal size are reused
    for (size_t l = 0; l < H.A.size(); ++l) {
      MgLevel& L = P.mg[l];
      L.n = H.A[l].n;
      upload_csr(L.A, H.A[l], P.stage, s);
      if (l + 1 < H.A.size() && !keep_pr) {
        upload_csr(L.P, H.P[l], P.stage, s);
        upload_csr(L.R, H.R[l], P.stage, s);
      }
      P.stage.upload(L.dinv, H.dinv[l].data(), H.dinv[l].size(), s);
      L.lmax = H.lmax[l];
    }
    P.nc = H.A.back().n;
    P.stage.upload(P.cinv, H.coarse_inv.data(), H.coarse_inv.size(), s);
    clk.mark("upload hierarchy");
    ensure_work(c, P);
    clk.mark("work vectors");
    if (f32) {
      // single-precision copies converted on the device from the double ones
      for (size_t l = 0; l < H.A.size(); ++l) {
        MgLevel& L = P.mg[l];
        copy_csr32(L.A32, L.A, s);
        if (l + 1 < H.A.size()) {
          copy_csr32(L.P32, L.P, s);
          copy_csr32(L.R32, L.R, s);
        }
        L.dinv32.alloc(L.dinv.n);
        cvt_d2f(L.dinv.p, L.dinv32.p, int64_t(L.dinv.n), s);
      }
      P.cinv32.alloc(P.cinv.n);
      cvt_d2f(P.cinv.p, P.cinv32.p, int64_t(P.cinv.n), s);
      ensure_work32(c, P);
      clk.mark("float copies (phi)");
    }
    P.sa_prev = std::move(H);  // the staged uploads above copied what they need
    P.phi_ok = true;
    P.phi32_ok = f32;
  }
  if (conc && !phi) {
    conc_part();
    if (f32) {
      ensure_work(c, P);
      ensure_work32(c, P);
    }
  }
  join_conc();
  if (conc) {
    P.conc_ok = true;
    P.conc32_ok = f32;
  }
  P.assembled = true;
  DGNP_HIP(hipStreamSynchronize(s));
}

void precond_invalidate(dgnp_ctx& c) {
  if (c.pc) c.pc->phi_ok = c.pc->phi32_ok = c.pc->phi32_blocks = c.pc->conc_ok = c.pc->conc32_ok = c.pc->assembled = false;
}

void get_block(dgnp_ctx& c, int field, int64_t elem, int slot, double* out) {
  DGNP_REQUIRE(c.pc && c.pc->assembled, DGNP_E_STATE, "no assembled blocks before set_state");
  Precond& P = *c.pc;
  const int64_t off = ((int64_t(field) * c.E + elem) * P.nslot + slot) * P.bsz;
  DGNP_HIP(hipMemcpy(out, P.blk.p + off, size_t(P.bsz) * sizeof(double), hipMemcpyDeviceToHost));
}

// ---- V-cycle -----------------------------------------------------------------------
// Levels: 0 = the order-p DG space; with p-multigrid 0 is applied matrix-free
// and 1 is the p = 1 DG space (element blocks); the element-block level is
// followed by the vertex (Q1) and aggregation levels (CSR), the last of which
// is solved with its dense inverse.
template <typename T>
struct Mg {
  dgnp_ctx& c;
  Precond& P;
  hipStream_t s;
  static constexpr bool F32 = std::is_same<T, float>::value;
  int top() const { return P.pmg ? 1 : 0; }  // index of the element-block level
  bool mf(int l) const { return P.pmg && l == 0; }
  MgLevel& csr(int l) const { return P.mg[size_t(l - top() - 1)]; }
  int64_t size(int l) const { return level_size(c, P, size_t(l)); }
  // element-block level data
  int bnb() const { return P.pmg ? P.nb1 : c.nb; }
  int bp() const { return P.pmg ? 1 : c.p; }
  const T* bblk() const { return P.pmg ? Sel<T>::blk1(P) : Sel<T>::blk(P); }
  const T* bdinv() const { return P.pmg ? Sel<T>::dinv1(P) : Sel<T>::dinv(P); }
  double lmax(int l) const {
    if (l == 0) return P.lmax0;
    if (P.pmg && l == 1) return P.lmax1;
    return csr(l).lmax;
  }
  // rc = R (b - A x): the residual of level l restricted to level l + 1
  void residual_restrict(int l, const T* x, const T* b, T* r, T* rc) {
    if (mf(l)) {
      phi_mf_apply<T>(c, x, r, s);
      launch_p1<T>(false, c.dim, c.p, b, r, rc, T(0), c.E, s);
      return;
    }
    if (l == top()) {
      launch_bspmv<T>(bnb(), c.dim, c.E, bblk(), c.d_nbr.p, x, b, T(-1), T(1), r, s);
      if (l + 1 < last()) {
        // the vertex level smooths: its first Chebyshev step rides on the restriction
        launch_q1<T>(false, c.dim, bp(), c.n, r, rc, T(0), c.E, P.nvert, s, Sel<T>::ldinv(csr(l + 1)),
                     T(cheb_c1(l + 1)), Sel<T>::w(P, size_t(l + 1) * 5 + 3));
        first_done = l + 1;
      } else {
        launch_q1<T>(false, c.dim, bp(), c.n, r, rc, T(0), c.E, P.nvert, s);
      }
    } else {
      DevCsr<T>& M = Sel<T>::A(csr(l));
      launch_csr_spmv<T>(M.n, M.rptr(), M.cptr(), M.v.p, x, b, T(-1), T(1), r, s);
      DevCsr<T>& R = Sel<T>::R(csr(l));
      launch_csr_spmv<T>(R.n, R.rptr(), R.cptr(), R.v.p, r, nullptr, T(1), T(0), rc, s, int64_t(R.v.n));
    }
  }
  void prolong_add(int l, const T* xc, T* x) {
    if (mf(l)) {
      launch_p1<T>(true, c.dim, c.p, xc, nullptr, x, T(1), c.E, s);
    } else if (l == top()) {
      launch_q1<T>(true, c.dim, bp(), c.n, xc, x, T(1), c.E, P.nvert, s);
    } else {
      DevCsr<T>& Pm = Sel<T>::Pm(csr(l));
      launch_csr_spmv<T>(Pm.n, Pm.rptr(), Pm.cptr(), Pm.v.p, xc, x, T(1), T(1), x, s);
    }
  }
  // one fused Chebyshev step on level l (see launch_cheb_blk)
  void step(int l, const T* u, const T* base, const T* dprev, const T* x_in, double c1, double c2, T* r_out,
            T* d_out, T* x_out) {
    if (mf(l)) {
      // r = base - A u with the matrix-free product, then the block-diagonal step
      T* y = nullptr;
      if (u) {
        y = Sel<T>::mf(P);
        phi_mf_apply<T>(c, u, y, s);
      }
      ScopeTimer tm(c, F32 ? "cheb_mf_f32" : "cheb_mf", s);
      launch_cheb_blk<T>(c.nb, c.dim, c.E, Sel<T>::blk(P), c.d_nbr.p, Sel<T>::dinv(P), nullptr, base, y, dprev, x_in,
                         T(c1), T(c2), r_out, d_out, x_out, s);
    } else if (l == top()) {
      ScopeTimer tm(c, P.pmg ? (F32 ? "cheb_blk1_f32" : "cheb_blk1") : (F32 ? "cheb_blk_f32" : "cheb_blk"), s);
      launch_cheb_blk<T>(bnb(), c.dim, c.E, bblk(), c.d_nbr.p, bdinv(), u, base, nullptr, dprev, x_in, T(c1),
                         T(c2), r_out, d_out, x_out, s);
    } else {
      DevCsr<T>& M = Sel<T>::A(csr(l));
      launch_cheb_csr<T>(M.n, M.rptr(), M.cptr(), M.v.p, Sel<T>::ldinv(csr(l)), u, base, dprev, x_in, T(c1), T(c2),
                         r_out, d_out, x_out, s);
    }
  }
  // Chebyshev smoothing of degree 2 on [0.1, 1.1] * lmax(D^{-1} A):
  //   d_1 = D^{-1} r_0 / theta,  x_1 = x_0 + d_1,  r_1 = r_0 - A d_1,
  //   d_2 = (2 rho_1 / delta) D^{-1} r_1 + rho_1 rho_0 d_1,  x_2 = x_1 + d_2,
  // rho_0 = delta / theta, rho_1 = 1 / (2 theta / delta - rho_0); two fused
  // launches per sweep.  Zero initial guess: r_0 = b; otherwise r_0 = b - A x_0.
  int last() const { return top() + int(P.mg.size()); }
  // level whose first zero-guess Chebyshev step the restriction already wrote
  int first_done = -1;
  double cheb_c1(int l) const {
    const double lm = lmax(l), lo = 0.1 * lm, hi = 1.1 * lm;
    return 1.0 / (0.5 * (hi + lo));
  }
  void cheb(int l, const T* b, T* x, bool zero_init) {
    T* r1 = Sel<T>::w(P, size_t(l) * 5 + 2);
    T* d1 = Sel<T>::w(P, size_t(l) * 5 + 3);
    T* x1 = Sel<T>::w(P, size_t(l) * 5 + 4);
    const double lm = lmax(l), lo = 0.1 * lm, hi = 1.1 * lm;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    const double a2 = 2.0 * rho1 / delta, b2 = rho1 * rho0;
    if (zero_init) {
      if (first_done == l)
        first_done = -1;  // d_1 written by the restriction into this level
      else
        step(l, nullptr, b, nullptr, nullptr, cheb_c1(l), 0.0, nullptr, nullptr, d1);  // x_1 = d_1
      step(l, d1, b, d1, d1, a2, b2, nullptr, nullptr, x);
    } else {
      step(l, x, b, nullptr, x, 1.0 / theta, 0.0, r1, d1, x1);
      step(l, d1, r1, d1, x1, a2, b2, nullptr, nullptr, x);
    }
  }
  void vcycle(int l, const T* b, T* x) {
    if (l == last()) {
      launch_dense_gemv<T>(P.nc, Sel<T>::cinv(P), b, x, s);
      return;
    }
    cheb(l, b, x, true);
    T* r = Sel<T>::w(P, size_t(l) * 5 + 2);
    T* bc = Sel<T>::w(P, size_t(l + 1) * 5 + 1);
    T* xc = Sel<T>::w(P, size_t(l + 1) * 5 + 0);
    residual_restrict(l, x, b, r, bc);
    vcycle(l + 1, bc, xc);
    prolong_add(l, xc, x);
    cheb(l, b, x, false);
  }
};

bool precond_sweeps_resident(const dgnp_ctx& c, bool f32, bool transpose) {
  if (!c.pc || transpose) return false;
  const Precond& P = *c.pc;
  return (P.lines_on && f32) || P.df_on;
}

// ILU solves of all concentration blocks at once (one launch per level covers
// every field): in/out point at the first concentration field (field 1).
template <typename T>
static void ilu_solve(dgnp_ctx& c, Precond& P, bool transpose, const T* in, T* out, hipStream_t s) {
  const int64_t fstride = c.E * P.nslot * P.bsz;
  const T* blk = Sel<T>::cblk(P, fstride);
  const int L = int(P.lev_ptr.size()) - 1;
  const int nf = c.m - 1;
  const bool f32 = std::is_same<T, float>::value;
  static const char* names[4][2] = {{"ilu_fwd", "ilu_fwd_f32"}, {"ilu_bwd", "ilu_bwd_f32"},
                                    {"ilu_fwdT", "ilu_fwdT_f32"}, {"ilu_bwdT", "ilu_bwdT_f32"}};
  const int k0 = transpose ? 2 : 0;
  if (!transpose && P.lines_on && f32) {
    uint64_t* wp = P.df_wp.p;
    const float* bf = reinterpret_cast<const float*>(blk);
    {
      ScopeTimer tm(c, names[0][1], s);
      launch_ilu_lines(0, c.nb, c.dim, bf, c.d_nbr.p, P.line_first.p, P.nline, P.line_len, P.line_stride, P.line_ax,
                       nf, fstride, c.Nf, reinterpret_cast<const float*>(in), reinterpret_cast<float*>(out), wp,
                       P.df_err.p, P.df_spin, P.line_grid, s);
    }
    {
      ScopeTimer tm(c, names[1][1], s);
      launch_ilu_lines(1, c.nb, c.dim, bf, c.d_nbr.p, P.line_first.p, P.nline, P.line_len, P.line_stride, P.line_ax,
                       nf, fstride, c.Nf, reinterpret_cast<const float*>(out), reinterpret_cast<float*>(out),
                       wp + int64_t(nf) * c.Nf, P.df_err.p, P.df_spin, P.line_grid, s);
    }
    return;
  }
  if (!transpose && P.df_on) {
    // packed words: one per entry in single precision, two in double
    uint64_t* wp = f32 ? P.df_wp.p : P.df_wp64.p;
    const int64_t half = int64_t(nf) * c.Nf * (f32 ? 1 : 2);
    {
      ScopeTimer tm(c, names[0][f32], s);
      launch_ilu_dataflow<T>(0, c.nb, c.dim, blk, c.d_nbr.p, P.lev_elems.p, c.E, nf, fstride, c.Nf, in, out, wp,
                             P.df_err.p, P.df_spin, P.df_grid[f32], s);
    }
    {
      ScopeTimer tm(c, names[1][f32], s);
      launch_ilu_dataflow<T>(1, c.nb, c.dim, blk, c.d_nbr.p, P.lev_elems.p, c.E, nf, fstride, c.Nf, out, out,
                             wp + half, P.df_err.p, P.df_spin, P.df_grid[f32], s);
    }
    return;
  }
  T* aux = transpose ? Sel<T>::vN(P) + c.Nf : nullptr;  // concentration part of a work vector
  // timed per level launch (one event pair per kernel) when profiling is on
  for (int l = 0; l < L; ++l) {
    ScopeTimer tm(c, names[k0][f32], s);
    launch_ilu_solve<T>(k0, c.nb, c.dim, blk, c.d_nbr.p, P.lev_elems.p, P.lev_ptr[l],
                        P.lev_ptr[l + 1] - P.lev_ptr[l], nf, fstride, c.Nf, in, transpose ? aux : out, nullptr,
                        s);
  }
  for (int l = L - 1; l >= 0; --l) {
    ScopeTimer tm(c, names[k0 + 1][f32], s);
    launch_ilu_solve<T>(k0 + 1, c.nb, c.dim, blk, c.d_nbr.p, P.lev_elems.p, P.lev_ptr[l],
                        P.lev_ptr[l + 1] - P.lev_ptr[l], nf, fstride, c.Nf, transpose ? nullptr : out, out, aux,
                        s);
  }
}

// ---- concentration multigrid: the V-cycle -----------------------------------------
template <typename T> struct GSel;
template <> struct GSel<double> {
  using L = Precond::GLevel;
  static const double* A(L& g) { return g.A.p; }
  static const double* F(L& g) { return g.F.p; }
  static double* x(L& g) { return g.x.p; }
  static double* b(L& g) { return g.b.p; }
  static double* r(L& g) { return g.r.p; }
  static double* z(L& g) { return g.z.p; }
  static double* aux(L& g) { return g.aux.p; }
  static const double* pi(Precond& P) { return P.gmg_pi.p; }
  static const double* cinv(Precond& P, bool tr) { return tr ? P.gmg_cinvT.p : P.gmg_cinv.p; }
};
template <> struct GSel<float> {
  using L = Precond::GLevel;
  static const float* A(L& g) { return g.A32.p; }
  static const float* F(L& g) { return g.F32.p; }
  static float* x(L& g) { return g.x32.p; }
  static float* b(L& g) { return g.b32.p; }
  static float* r(L& g) { return g.r32.p; }
  static float* z(L& g) { return g.z32.p; }
  static float* aux(L& g) { return g.aux32.p; }
  static const float* pi(Precond& P) { return P.gmg_pi32.p; }
  static const float* cinv(Precond& P, bool tr) { return tr ? P.gmg_cinvT32.p : P.gmg_cinv32.p; }
};

// BILU(0) solve (or its transpose) of every concentration field on level l:
// the fine level through ilu_solve (dataflow or line sweeps where they run),
// the coarser ones level-scheduled
template <typename T>
static void gmg_ilu(dgnp_ctx& c, Precond& P, int l, bool tr, const T* in, T* out, hipStream_t s) {
  if (l == 0) return ilu_solve<T>(c, P, tr, in, out, s);
  Precond::GLevel& g = P.gl[size_t(l)];
  const int nf = c.m - 1;
  const int64_t fs = g.E * P.nslot * P.bsz, vs = g.E * c.nb;
  const T* blk = GSel<T>::F(g);
  if (!tr && g.wp.p) {
    // one dataflow launch per sweep, as on the fine level
    const bool f32 = std::is_same<T, float>::value;
    uint64_t* wp = f32 ? g.wp.p : g.wp64.p;
    const int64_t half = int64_t(nf) * vs * (f32 ? 1 : 2);
    launch_ilu_dataflow<T>(0, c.nb, c.dim, blk, g.nbr.p, g.lev_elems.p, g.E, nf, fs, vs, in, out, wp, P.df_err.p,
                           P.df_spin, g.df_grid[f32], s);
    launch_ilu_dataflow<T>(1, c.nb, c.dim, blk, g.nbr.p, g.lev_elems.p, g.E, nf, fs, vs, out, out, wp + half,
                           P.df_err.p, P.df_spin, g.df_grid[f32], s);
    return;
  }
  const int L = int(g.lev_ptr.size()) - 1;
  T* aux = tr ? GSel<T>::aux(g) : nullptr;
  const int k0 = tr ? 2 : 0;
  for (int lv = 0; lv < L; ++lv)
    launch_ilu_solve<T>(k0, c.nb, c.dim, blk, g.nbr.p, g.lev_elems.p, g.lev_ptr[lv], g.lev_ptr[lv + 1] - g.lev_ptr[lv],
                        nf, fs, vs, in, tr ? aux : out, nullptr, s);
  for (int lv = L - 1; lv >= 0; --lv)
    launch_ilu_solve<T>(k0 + 1, c.nb, c.dim, blk, g.nbr.p, g.lev_elems.p, g.lev_ptr[lv],
                        g.lev_ptr[lv + 1] - g.lev_ptr[lv], nf, fs, vs, tr ? nullptr : out, out, aux, s);
}

// One V-cycle from a zero initial guess on level l for every concentration
// field: nu Richardson steps x <- x + M^{-1} (b - A x) with the level's BILU(0)
// M, the coarse correction x <- x + P V_{l+1}(P^T (b - A x)), nu more steps; the
// coarsest level multiplies by its dense inverse.  tr: the same cycle with A^T,
// M^{-T} and the transposed coarsest inverse, which is the cycle's transpose
// (restriction and prolongation are each other's transposes).
template <typename T>
static void gmg_vcycle(dgnp_ctx& c, Precond& P, bool tr, int l, const T* b, T* x, hipStream_t s) {
  const int nf = c.m - 1, last = int(P.gl.size()) - 1;
  Precond::GLevel& g = P.gl[size_t(l)];
  const int64_t nfl = g.E * c.nb;
  if (l == last) {
    const int n = P.gmg_nc;
    launch_dense_gemv<T>(n, GSel<T>::cinv(P, tr), b, x, s, nf, nfl);
    return;
  }
  const T* A = GSel<T>::A(g);
  const int* nbr = l == 0 ? c.d_nbr.p : g.nbr.p;
  const int ld = pot_ld(c.nb, std::is_same<T, float>::value);
  const int64_t fs = g.E * P.nslot * c.nb * ld;
  T* r = GSel<T>::r(g);
  T* z = GSel<T>::z(g);
  // r = b - A x (forward: the block SpMV of the potential block, all fields in one launch)
  auto resid = [&]() {
    if (tr)
      launch_gmg_resid<T>(c.nb, c.dim, nf, true, A, fs, ld, nbr, g.E, x, b, r, s);
    else
      launch_bspmv<T>(c.nb, c.dim, g.E, A, nbr, x, b, T(-1), T(1), r, s, nf, fs, nfl);
  };
  auto richardson = [&]() {
    resid();
    gmg_ilu<T>(c, P, l, tr, r, z, s);
    vaxpy<T>(T(1), z, x, nf * nfl, s);
  };
  gmg_ilu<T>(c, P, l, tr, b, x, s);  // first step from x = 0
  for (int k = 1; k < P.gmg_nu; ++k) richardson();
  Precond::GLevel& gc = P.gl[size_t(l + 1)];
  const int64_t nfc = gc.E * c.nb;
  resid();
  launch_gmg_restrict<T>(c.nb, c.dim, nf, GSel<T>::pi(P), g.n, r, nfl, GSel<T>::b(gc), nfc, s);
  gmg_vcycle<T>(c, P, tr, l + 1, GSel<T>::b(gc), GSel<T>::x(gc), s);
  launch_gmg_prolong<T>(c.nb, c.dim, nf, GSel<T>::pi(P), g.n, GSel<T>::x(gc), nfc, x, nfl, s);
  for (int k = 0; k < P.gmg_nu; ++k) richardson();
}

// the concentration blocks' solve of the block-triangular preconditioner
template <typename T>
static void conc_solve(dgnp_ctx& c, Precond& P, bool transpose, const T* in, T* out, hipStream_t s) {
  if (!P.gmg) return ilu_solve<T>(c, P, transpose, in, out, s);
  ScopeTimer tm(c, std::is_same<T, float>::value ? "gmg_f32" : "gmg", s);
  gmg_vcycle<T>(c, P, transpose, 0, in, out, s);
}

template <typename T>
static void apply_t(dgnp_ctx& c, const T* r, T* z, bool transpose, int kind, hipStream_t s) {
  Precond& P = *c.pc;
  Mg<T> mg{c, P, s};
  const int64_t Nf = c.Nf;
  const bool f32 = std::is_same<T, float>::value;
  T* y = Sel<T>::yN(P);
  T* t = Sel<T>::tN(P);
  // kinds: "c first" (P2, or P1 transposed) and "phi first" (P1, or P2 transposed)
  const bool c_first = (kind == DGNP_PC_P2) != transpose;
  // the coupling applies read z with the other part masked out (counted as zero)
  const unsigned phi_only = 1u, conc_only = ~1u;
  if (c_first) {
    conc_solve<T>(c, P, transpose, r + Nf, z + Nf, s);
    if (!transpose) {
      jac_apply(c, z, t, f32, false, s, conc_only, true, r);  // t = r - A_phic z_c, potential rows only
    } else {
      jac_apply(c, z, y, f32, true, s, conc_only);
      vsub<T>(r, y, t, Nf, s);
    }
    ScopeTimer tm(c, f32 ? "vcycle_f32" : "vcycle", s);
    mg.vcycle(0, t, z);
  } else {
    {
      ScopeTimer tm(c, f32 ? "vcycle_f32" : "vcycle", s);
      mg.vcycle(0, r, z);
    }
    jac_apply(c, z, y, f32, transpose, s, phi_only);
    vsub<T>(r + Nf, y + Nf, t + Nf, (c.m - 1) * Nf, s);
    conc_solve<T>(c, P, transpose, t + Nf, z + Nf, s);
  }
}

void precond_apply(dgnp_ctx& c, const void* r, void* z, bool f32, bool transpose, int kind, hipStream_t s) {
  DGNP_REQUIRE(c.pc && c.pc->ready(), DGNP_E_STATE, "precond_apply before set_state");
  if (f32) {
    DGNP_REQUIRE(c.pc->ready32(), DGNP_E_STATE, "float preconditioner needs set_state with DGNP_F32");
    apply_t<float>(c, static_cast<const float*>(r), static_cast<float*>(z), transpose, kind, s);
  } else {
    apply_t<double>(c, static_cast<const double*>(r), static_cast<double*>(z), transpose, kind, s);
  }
}

// y = A_phiphi x with the assembled potential block
void phi_block_apply(dgnp_ctx& c, const double* x, double* y, hipStream_t s) {
  DGNP_REQUIRE(c.pc && c.pc->phi_ok, DGNP_E_STATE, "potential block not set up");
  launch_bspmv<double>(c.nb, c.dim, c.E, c.pc->blk.p, c.d_nbr.p, x, nullptr, 1.0, 0.0, y, s);
}
void phi_block_apply(dgnp_ctx& c, const float* x, float* y, hipStream_t s) {
  DGNP_REQUIRE(c.pc && c.pc->phi32_ok, DGNP_E_STATE, "single-precision potential block not set up");
  Precond& P = *c.pc;
  if (!P.phi32_blocks) {  // set-ups with p-multigrid leave the copy to the first request
    const int ld32 = pot_ld(c.nb, true);
    P.phi32.alloc(size_t(c.E) * P.nslot * c.nb * ld32);
    cvt_d2f_rows(P.blk.p, P.phi32.p, c.E * P.nslot * c.nb, c.nb, ld32, s);
    P.phi32_blocks = true;
  }
  launch_bspmv<float>(c.nb, c.dim, c.E, P.phi32.p, c.d_nbr.p, x, nullptr, 1.0f, 0.0f, y, s);
}

void phi_apply(dgnp_ctx& c, const void* x, void* y, bool f32, bool matfree, hipStream_t s) {
  DGNP_REQUIRE(c.pc && (f32 ? c.pc->phi32_ok : c.pc->phi_ok), DGNP_E_STATE,
               "potential block not set up in this precision");
  if (!matfree) {
    if (f32)
      phi_block_apply(c, static_cast<const float*>(x), static_cast<float*>(y), s);
    else
      phi_block_apply(c, static_cast<const double*>(x), static_cast<double*>(y), s);
    return;
  }
  DGNP_REQUIRE(c.pc->pmg && c.dim == 3, DGNP_E_ARG, "matrix-free potential block: 3-D with p-multigrid");
  if (f32)
    phi_mf_apply<float>(c, static_cast<const float*>(x), static_cast<float*>(y), s);
  else
    phi_mf_apply<double>(c, static_cast<const double*>(x), static_cast<double*>(y), s);
}

// potential-block V-cycle alone (used for the initial potential solve)
void vcycle_phi(dgnp_ctx& c, const double* b, double* x, hipStream_t s) {
  DGNP_REQUIRE(c.pc && c.pc->phi_ok, DGNP_E_STATE, "potential hierarchy not set up");
  Mg<double> mg{c, *c.pc, s};
  mg.vcycle(0, b, x);
}
void vcycle_phi(dgnp_ctx& c, const float* b, float* x, hipStream_t s) {
  DGNP_REQUIRE(c.pc && c.pc->phi32_ok, DGNP_E_STATE, "single-precision potential hierarchy not set up");
  Mg<float> mg{c, *c.pc, s};
  mg.vcycle(0, b, x);
}

}  // namespace dgnp
