// Host drivers: linearisation state, matrix-free Jacobian applies, flexible
// GMRES with FP64 classical Gram-Schmidt (twice), Newton with backtracking
// line search (paper Sec. 4), mixed precision by iterative refinement, and the
// adjoint of the outflow-flux objective.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "blas.hpp"
#include "kernels_jac.hpp"
#include "solver.hpp"

namespace dgnp {

using clk = std::chrono::steady_clock;
static double since(clk::time_point t0) { return std::chrono::duration<double>(clk::now() - t0).count(); }

void set_state(dgnp_ctx& c, const double* x, int prec, hipStream_t s, bool assemble_only, bool apply_only,
               int parts) {
  ++c.state_epoch;
  c.d_x.alloc(size_t(c.N));
  if (x != c.d_x.p) vcopy<double>(x, c.d_x.p, c.N, s);
  c.has_state = true;
  c.has_state32 = false;
  if (prec == DGNP_F32) {
    c.d_x32.alloc(size_t(c.N));
    cvt_d2f(c.d_x.p, c.d_x32.p, c.N, s);
    c.has_state32 = true;
  }
  if (c.dim == 3 && c.jac_tab) {
    size_t nf = 0;
    const size_t nv = jlin_table_sizes(c.p, c.m, c.E, c.n, &nf);
    const KArgs A = c.kargs();
    c.d_jtv.alloc(nv);
    c.d_jtf.alloc(nf);
    launch_jlin_tables<double>(c.p, c.m, A, c.d_x.p, c.d_jtv.p, c.d_jtf.p, s);
    if (prec == DGNP_F32) {
      c.d_jtv32.alloc(nv);
      c.d_jtf32.alloc(nf);
      launch_jlin_tables<float>(c.p, c.m, A, c.d_x.p, c.d_jtv32.p, c.d_jtf32.p, s);
    }
  }
  if (apply_only)
    precond_invalidate(c);
  else
    precond_numeric(c, prec == DGNP_F32, s, assemble_only, parts);
  DGNP_HIP(hipStreamSynchronize(s));
}

void jac_apply(dgnp_ctx& c, const void* v, void* y, bool f32, bool transpose, hipStream_t s, unsigned vmask,
               bool phi_rows, const void* base) {
  DGNP_REQUIRE(c.has_state, DGNP_E_STATE, "jacobian_apply before set_state");
  DGNP_REQUIRE(!f32 || c.has_state32, DGNP_E_STATE, "float apply needs set_state with DGNP_F32");
  const void* xs = f32 ? static_cast<const void*>(c.d_x32.p) : static_cast<const void*>(c.d_x.p);
  static const char* names[2][2] = {{"jac_apply", "jac_apply_f32"}, {"jacT_apply", "jacT_apply_f32"}};
  ScopeTimer tm(c, names[transpose ? 1 : 0][f32 ? 1 : 0], s);
  KArgs A = c.kargs();
  A.vin_mask = vmask;
  DGNP_REQUIRE(!base || (phi_rows && !transpose), DGNP_E_ARG, "base needs the potential-rows apply");
  A.jbase = base;
  // forward applies in 3-D read the tabulated linearisation data; the coupling
  // form (potential rows) assumes that the potential part of v is masked out
  if (c.dim == 3 && c.jac_tab && !transpose && (!phi_rows || (vmask & 1u) == 0)) {
    if (f32)
      launch_jlin<float>(c.p, c.m, phi_rows, A, static_cast<const float*>(v), c.d_jtv32.p, c.d_jtf32.p,
                         static_cast<float*>(y), s);
    else
      launch_jlin<double>(c.p, c.m, phi_rows, A, static_cast<const double*>(v), c.d_jtv.p, c.d_jtf.p,
                          static_cast<double*>(y), s);
    return;
  }
  launch_dg(c.dim, c.p, c.m, f32, transpose ? M_JACT : (phi_rows ? M_JACP : M_JAC), A, xs, v, y, nullptr, s);
}

dgnp_solve_opts default_solve_opts() {
  dgnp_solve_opts o{};
  o.rtol = 1e-8;
  o.atol = 0.0;
  o.max_newton = 30;
  o.prec = DGNP_F64;
  o.lin_rtol = 1e-3;
  o.restart = 120;
  o.max_lin_it = 600;
  o.pc_kind = DGNP_PC_P2;
  o.verbose = 0;
  return o;
}

// ---------------------------------------------------------------------------
// Flexible GMRES (right preconditioning) for Op x = b with Op = J or J^T and
// preconditioner P or P^T.  Arnoldi basis, orthogonalisation and all inner
// products in FP64.  With f32 the operator and preconditioner are applied in
// FP32 (the Krylov relation then holds for the FP32 operator); every restart
// recomputes the true FP64 residual b - Op x, which makes the restarts the
// steps of an iterative refinement.
// ---------------------------------------------------------------------------
struct Krylov {
  DevBuf<double> V, Z, w, r, hd, vt, zt;
  DevBuf<float> Z32, v32, w32, zt32;
  int restart = 0;
  int64_t n = 0;
  // captured "preconditioner + Jacobian" graphs, keyed by (f32, transpose)
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  uint64_t gepoch[2][2] = {{0, 0}, {0, 0}};
  int gpc[2][2] = {{-1, -1}, {-1, -1}};
  // pinned host slots for the coefficient blocks of two consecutive Arnoldi
  // steps
  static constexpr size_t HSLOT = DCGS_COEF;
  double* hpin = nullptr;      // host view
  double* hpin_dev = nullptr;  // the same memory as the device addresses it
  // sequence numbers: the coefficient kernel of a step stores its number into
  // the slot last, which tells the host that the slot is complete
  unsigned long long seq = 0, slot_seq[2] = {0, 0};
  ~Krylov() {
    for (auto& row : gexec)
      for (auto& g : row)
        if (g) (void)hipGraphExecDestroy(g);
    if (hpin) (void)hipHostFree(hpin);
  }
};

void krylov_destroy(Krylov* k) { delete k; }

static bool graphs_enabled(const dgnp_ctx& c) {
  const char* e = getenv("DGNP_NO_GRAPHS");
  return !c.profiling && !(e && e[0] && e[0] != '0');
}

// Graph capture pays for sequences of many short launches (level-scheduled
// sweeps: one launch per hyperplane level).  With the resident-grid sweeps the
// sequence is about twenty launches, which the host queues well ahead of the
// device, and direct launches avoid the graph's entry and exit gaps (16^3 cube
// 0.139 -> 0.137 s).  DGNP_GRAPHS=1 captures in every case.
static bool use_graph(const dgnp_ctx& c, bool f32, bool transpose) {
  if (!graphs_enabled(c)) return false;
  const char* f = getenv("DGNP_GRAPHS");
  if (f && f[0] == '1') return true;
  return !precond_sweeps_resident(c, f32, transpose);
}

// z_stage = P in_stage; w = J z_stage, either captured once per linearisation
// point as a HIP graph (the sequence of ~10^2 small level-scheduled kernels
// then launches as one unit) or issued directly.
static void pc_then_jac(dgnp_ctx& c, Krylov& K, bool f32, bool transpose, int pc_kind, hipStream_t s) {
  const void* in = f32 ? static_cast<const void*>(K.v32.p) : static_cast<const void*>(K.vt.p);
  void* zs = f32 ? static_cast<void*>(K.zt32.p) : static_cast<void*>(K.zt.p);
  void* w = f32 ? static_cast<void*>(K.w32.p) : static_cast<void*>(K.w.p);
  if (!use_graph(c, f32, transpose)) {
    precond_apply(c, in, zs, f32, transpose, pc_kind, s);
    jac_apply(c, zs, w, f32, transpose, s);
    return;
  }
  const int a = f32 ? 1 : 0, b = transpose ? 1 : 0;
  if (!K.gexec[a][b] || K.gepoch[a][b] != c.state_epoch || K.gpc[a][b] != pc_kind) {
    if (K.gexec[a][b]) DGNP_HIP(hipGraphExecDestroy(K.gexec[a][b]));
    K.gexec[a][b] = nullptr;
    hipGraph_t g = nullptr;
    DGNP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      precond_apply(c, in, zs, f32, transpose, pc_kind, s);
      jac_apply(c, zs, w, f32, transpose, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    DGNP_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DGNP_HIP(e);
    K.gexec[a][b] = ex;
    K.gepoch[a][b] = c.state_epoch;
    K.gpc[a][b] = pc_kind;
  }
  DGNP_HIP(hipGraphLaunch(K.gexec[a][b], s));
}

static Krylov& krylov(dgnp_ctx& c, int restart, bool f32) {
  if (!c.kry) c.kry = new Krylov();
  Krylov* K = c.kry;
  if (K->restart != restart || K->n != c.N) {
    K->V.alloc(size_t(restart + 1) * c.N);
    K->w.alloc(size_t(c.N));
    K->r.alloc(size_t(c.N));
    K->hd.alloc(size_t(std::max(reduce_scratch_size(), dcgs_partial_size())) + DCGS_COEF + MAXV + 8);
    DGNP_HIP(hipMemset(K->hd.p, 0, K->hd.n * sizeof(double)));  // includes the reduction's counter
    K->Z.release();
    K->Z32.release();
    K->restart = restart;
    K->n = c.N;
  }
  if (!K->hpin) {
    // coherent host memory: the coefficient kernel stores into it directly
    DGNP_HIP(hipHostMalloc(reinterpret_cast<void**>(&K->hpin), 2 * Krylov::HSLOT * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    for (size_t i = 0; i < 2 * Krylov::HSLOT; ++i) K->hpin[i] = 0.0;
    DGNP_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&K->hpin_dev), K->hpin, 0));
  }
  if (f32 && !K->Z32.p) {
    K->Z32.alloc(size_t(restart) * c.N);
    K->v32.alloc(size_t(c.N));
    K->w32.alloc(size_t(c.N));
    K->zt32.alloc(size_t(c.N));
  }
  if (!f32 && !K->Z.p) {
    K->Z.alloc(size_t(restart) * c.N);
    K->vt.alloc(size_t(c.N));
    K->zt.alloc(size_t(c.N));
  }
  return *K;
}

struct LinResult {
  int its = 0, refinements = 0;
  double res = 0.0;
  bool converged = false;
};

static void op_apply64(dgnp_ctx& c, const double* v, double* y, bool transpose, hipStream_t s) {
  jac_apply(c, v, y, false, transpose, s);
}

static LinResult fgmres(dgnp_ctx& c, const double* b, double* x, double target, int restart, int maxit,
                        bool f32, bool transpose, int pc_kind, bool x_is_zero, int verbose, hipStream_t s) {
  Krylov& K = krylov(c, restart, f32);
  const int64_t N = c.N;
  LinResult out;
  const size_t rs = static_cast<size_t>(restart);
  std::vector<double> H((rs + 1) * rs), g(rs + 1), cs(rs), sn(rs), y(rs);
  bool first = true;
  while (true) {
    // true FP64 residual
    if (first && x_is_zero) {
      vcopy<double>(b, K.r.p, N, s);
    } else {
      op_apply64(c, x, K.r.p, transpose, s);
      vaxpby<double>(1.0, b, -1.0, K.r.p, N, s);
      ++out.refinements;
    }
    first = false;
    const double beta = vnorm2(K.r.p, N, K.hd.p, s);
    out.res = beta;
    if (!std::isfinite(beta)) {
      precond_check(c);  // an ended dataflow sweep is reported as such
      throw Error(DGNP_E_NONFINITE, "non-finite linear residual");
    }
    if (verbose > 1) fprintf(stderr, "  fgmres restart: |r| = %.3e (target %.3e)\n", beta, target);
    if (beta <= target) {
      out.converged = true;
      break;
    }
    if (out.its >= maxit) break;
    // u = r / beta (kept in K.r) and its copy for the preconditioner input
    if (f32) {
      vscale_dual(1.0 / beta, K.r.p, K.r.p, K.v32.p, N, s);
    } else {
      vscale<double>(1.0 / beta, K.r.p, N, s);
      vcopy<double>(K.r.p, K.vt.p, N, s);
    }
    std::fill(g.begin(), g.end(), 0.0);
    // Arnoldi with delayed classical Gram-Schmidt: step q applies P and the
    // operator to u_q (the direction left by step q - 1 after one projection
    // pass), and one reduction both reorthogonalises u_q against the basis (its
    // coefficients complete column q - 1 of H) and projects the new w once (the
    // first part of column q).  The basis is read twice per step instead of
    // four times.  Step q + 1 is queued before the host reads step q, so the
    // device does not wait for the host's rotations; steps queued past
    // convergence are discarded.
    double* part = K.hd.p;
    double* coef = K.hd.p + dcgs_partial_size();
    // the coefficient kernel of step q stores the entries the host reads into
    // pinned slot q % 2 (free again: the host has read step q - 2 before step
    // q is queued) and then the step's sequence number; no event is recorded
    // between steps, so the device runs them back to back
    auto slot = [&](int q) { return K.hpin_dev + size_t(q % 2) * Krylov::HSLOT; };
    auto next_seq = [&](int q) { return K.slot_seq[q % 2] = ++K.seq; };
    auto issue_step = [&](int q) {
      pc_then_jac(c, K, f32, transpose, pc_kind, s);
      {
        // the update pass also stores z_q into Z (preconditioner output column)
        ScopeTimer tm(c, "cgs2", s);
        if (f32) {
          dcgs_reduce(K.V.p, N, q, K.r.p, K.w32.p, true, K.w.p, N, part, coef, s, slot(q), next_seq(q));
          dcgs_update<float>(K.V.p, N, q, coef, K.r.p, K.w.p, K.v32.p, K.zt32.p, K.Z32.p + int64_t(q) * N, N, s);
        } else {
          dcgs_reduce(K.V.p, N, q, K.r.p, K.w.p, false, nullptr, N, part, coef, s, slot(q), next_seq(q));
          dcgs_update<double>(K.V.p, N, q, coef, K.r.p, K.w.p, K.vt.p, K.zt.p, K.Z.p + int64_t(q) * N, N, s);
        }
      }
    };
    auto issue_final = [&](int q) {  // reorthogonalisation of u_q only: completes column q - 1
      {
        ScopeTimer tm(c, "cgs2", s);
        dcgs_reduce(K.V.p, N, q, K.r.p, nullptr, false, nullptr, N, part, coef, s, slot(q), next_seq(q));
      }
    };
    auto read = [&](int q) -> const double* {
      const double* hb = K.hpin + size_t(q % 2) * Krylov::HSLOT;
      const unsigned long long want = K.slot_seq[q % 2];
      const unsigned long long* flag = reinterpret_cast<const unsigned long long*>(hb + DCGS_FLAG);
      // wait for the slot's sequence number; the stream is queried now and
      // then, so that a failed stream raises its error and a finished stream
      // without the number (not expected) does not leave the host waiting
      for (unsigned n = 1; __atomic_load_n(flag, __ATOMIC_ACQUIRE) != want; ++n) {
        if ((n & 1023u) != 0) continue;
        const hipError_t e = hipStreamQuery(s);
        if (e == hipErrorNotReady) continue;
        DGNP_HIP(e);
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != want)
          throw Error(DGNP_E_BREAKDOWN, "Arnoldi coefficients did not arrive");
      }
      if (!std::isfinite(hb[DCGS_ALPHA]) || !std::isfinite(hb[DCGS_HJJ]) || !std::isfinite(hb[DCGS_RHO])) {
        DGNP_HIP(hipStreamSynchronize(s));
        precond_check(c);  // a dataflow sweep that ended at its wait limit left NaN rows
        throw Error(DGNP_E_NONFINITE, "non-finite Arnoldi vector");
      }
      return hb;
    };
    // column jc of H is complete: add the reorthogonalisation s (scaled by the
    // direction's scale rho), set h_{jc+1,jc}, rotate; true when converged
    auto finish_column = [&](int jc, const double* hb, double rho) -> bool {
      double* col = H.data() + size_t(jc) * (restart + 1);
      for (int i = 0; i <= jc; ++i) col[i] += rho * hb[i];
      const double hn = rho * hb[DCGS_ALPHA];
      col[jc + 1] = hn;
      ++out.its;
      for (int i = 0; i < jc; ++i) {
        const double t = cs[size_t(i)] * col[i] + sn[size_t(i)] * col[i + 1];
        col[i + 1] = -sn[size_t(i)] * col[i] + cs[size_t(i)] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[jc], col[jc + 1]);
      if (den == 0.0) {
        DGNP_HIP(hipStreamSynchronize(s));
        throw Error(DGNP_E_BREAKDOWN, "FGMRES breakdown");
      }
      cs[size_t(jc)] = col[jc] / den;
      sn[size_t(jc)] = col[jc + 1] / den;
      col[jc] = den;
      col[jc + 1] = 0.0;
      g[size_t(jc + 1)] = -sn[size_t(jc)] * g[size_t(jc)];
      g[size_t(jc)] = cs[size_t(jc)] * g[size_t(jc)];
      const double est = std::fabs(g[size_t(jc + 1)]);
      if (verbose > 2) fprintf(stderr, "    it %d: est %.3e\n", out.its, est);
      return est <= target || hn == 0.0;
    };
    const int jmax = std::min(restart, maxit - out.its);
    int k = 0;  // columns used for the update
    bool done = false;
    double rho_prev = 1.0;
    issue_step(0);
    for (int q = 0; q < jmax; ++q) {
      if (q + 1 < jmax)
        issue_step(q + 1);
      else
        issue_final(q + 1);
      const double* hb = read(q);
      if (q == 0) {
        g[0] = beta * hb[DCGS_ALPHA];  // r = beta u_0 = beta alpha_0 v_0
      } else if (finish_column(q - 1, hb, rho_prev)) {
        k = q;
        done = true;
        break;
      }
      double* col = H.data() + size_t(q) * (restart + 1);
      for (int i = 0; i < q; ++i) col[i] = hb[MAXV + i];
      col[q] = hb[DCGS_HJJ];
      rho_prev = hb[DCGS_RHO];
    }
    if (!done && jmax > 0) {
      const double* hb = read(jmax);
      finish_column(jmax - 1, hb, rho_prev);
      k = jmax;
    }
    // back substitution and update x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[size_t(i)];
      for (int l = i + 1; l < k; ++l) acc -= H[size_t(l) * (restart + 1) + i] * y[size_t(l)];
      y[size_t(i)] = acc / H[size_t(i) * (restart + 1) + i];
    }
    double* yd = coef + DCGS_COEF;
    DGNP_HIP(hipMemcpyAsync(yd, y.data(), sizeof(double) * size_t(k), hipMemcpyHostToDevice, s));
    if (f32)
      vcombine<float>(K.Z32.p, N, k, yd, x, N, s);
    else
      vcombine<double>(K.Z.p, N, k, yd, x, N, s);
    DGNP_HIP(hipStreamSynchronize(s));
  }
  return out;
}

// ---------------------------------------------------------------------------
// Initial guess (paper Sec. 4.3): constant concentrations equal to the mean
// of the inflow / Dirichlet data, and the potential from the charge equation
// at those concentrations, R_phi(c0, phi) = 0, which is linear in phi; solved
// with conjugate gradients preconditioned by the potential V-cycle.
// ---------------------------------------------------------------------------
static void initial_guess(dgnp_ctx& c, double* x, hipStream_t s, int prec, int verbose) {
  const int64_t Nf = c.Nf;
  vfill<double>(x, 0.0, Nf, s);
  for (int k = 1; k < c.m; ++k) {
    double mean = 1.0;
    if (!c.dir_face.empty()) {
      // caller face data: the mean over the Gauss points of the data-carrying faces
      double sum = 0.0;
      int64_t cnt = 0;
      for (int t = 0; t < 2 * c.dim; ++t) {
        if (c.c_bc[t] != DGNP_C_DIRICHLET && c.c_bc[t] != DGNP_C_INFLOW) continue;
        const int64_t f0 = c.btag_off[t], f1 = t + 1 < 2 * c.dim ? c.btag_off[t + 1] : c.n_bface;
        for (int64_t bf = f0; bf < f1; ++bf)
          for (int q = 0; q < c.nqf; ++q, ++cnt) sum += c.dir_face[(size_t(k) * c.n_bface + bf) * c.nqf + q];
      }
      if (cnt > 0) mean = sum / double(cnt);
    } else if (!c.mms && c.n_bnode > 0) {
      mean = 0.0;
      for (int64_t j = 0; j < c.n_bnode; ++j) mean += c.bc_conc[size_t(k - 1) * c.n_bnode + j];
      mean /= double(c.n_bnode);
    }
    vfill<double>(x + k * Nf, mean, Nf, s);
  }
  // only the potential part of the preconditioner is needed here; with the
  // single-precision path the operator and the V-cycle run in single precision
  // inside the double-precision conjugate gradient iteration
  const bool f32 = prec == DGNP_F32;
  set_state(c, x, prec, s, false, false, PC_PHI);
  DevBuf<double> r, z, p, q, phi;
  r.alloc(size_t(c.N));
  z.alloc(size_t(Nf));
  p.alloc(size_t(Nf));
  q.alloc(size_t(Nf));
  phi.alloc(size_t(Nf));
  DevBuf<float> a32, b32;
  if (f32) {
    a32.alloc(size_t(Nf));
    b32.alloc(size_t(Nf));
  }
  auto precond = [&](const double* rin, double* zout) {
    if (f32) {
      cvt_d2f(rin, a32.p, Nf, s);
      vcycle_phi(c, a32.p, b32.p, s);
      cvt_f2d(b32.p, zout, Nf, s);
    } else {
      vcycle_phi(c, rin, zout, s);
    }
  };
  auto matvec = [&](const double* xin, double* yout) {
    if (f32) {
      cvt_d2f(xin, a32.p, Nf, s);
      phi_block_apply(c, a32.p, b32.p, s);
      cvt_f2d(b32.p, yout, Nf, s);
    } else {
      phi_block_apply(c, xin, yout, s);
    }
  };
  DevBuf<double> red;
  red.alloc(size_t(reduce_scratch_size()));
  launch_dg(c.dim, c.p, c.m, false, M_RES, c.kargs(), x, nullptr, r.p, nullptr, s);
  vscale<double>(-1.0, r.p, Nf, s);  // right-hand side -R_phi(c0, 0), kept in r[0:Nf]
  const double bn = vnorm2(r.p, Nf, red.p, s);
  vfill<double>(phi.p, 0.0, Nf, s);
  if (bn > 0.0) {
    precond(r.p, z.p);
    vcopy<double>(z.p, p.p, Nf, s);
    double rz = vdot(r.p, z.p, Nf, red.p, s);
    for (int it = 0; it < 500; ++it) {
      matvec(p.p, q.p);
      const double pq = vdot(p.p, q.p, Nf, red.p, s);
      const double alpha = rz / pq;
      vaxpy<double>(alpha, p.p, phi.p, Nf, s);
      vaxpy<double>(-alpha, q.p, r.p, Nf, s);
      const double rn = vnorm2(r.p, Nf, red.p, s);
      if (verbose > 1) fprintf(stderr, "  initial potential CG %d: %.3e\n", it, rn / bn);
      if (rn <= 1e-6 * bn) break;
      precond(r.p, z.p);
      const double rz_new = vdot(r.p, z.p, Nf, red.p, s);
      vaxpby<double>(1.0, z.p, rz_new / rz, p.p, Nf, s);
      rz = rz_new;
    }
  }
  vcopy<double>(phi.p, x, Nf, s);
  DGNP_HIP(hipStreamSynchronize(s));
}

struct NewtonWork {
  DevBuf<double> r, rt, xt, dx, b, red;
};

int newton_solve(dgnp_ctx& c, double* x, const dgnp_solve_opts& o, dgnp_solve_stats& st) {
  const auto t0 = clk::now();
  hipStream_t s = c.work;
  const int64_t N = c.N;
  NewtonWork W;
  W.r.alloc(size_t(N));
  W.rt.alloc(size_t(N));
  W.xt.alloc(size_t(N));
  W.dx.alloc(size_t(N));
  W.b.alloc(size_t(N));
  W.red.alloc(size_t(reduce_scratch_size()));
  st = dgnp_solve_stats{};
  DGNP_REQUIRE(o.restart >= 1 && o.restart <= MAXV - 8, DGNP_E_ARG, "restart must be 1..120");
  DGNP_REQUIRE(o.prec == DGNP_F64 || o.prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
  double x0;
  DGNP_HIP(hipMemcpy(&x0, x, sizeof(double), hipMemcpyDeviceToHost));
  // The potential block depends on the concentrations only; right after the
  // initial guess (which changes the potential alone) the first linearisation
  // keeps its potential hierarchy and sets up the concentration part.
  bool phi_current = false;
  if (std::isnan(x0)) {
    const auto ts = clk::now();
    initial_guess(c, x, s, o.prec, o.verbose);
    st.t_setup += since(ts);
    phi_current = true;
  }
  const bool f32 = o.prec == DGNP_F32;
  auto resid = [&](const double* xv, double* rv) {
    {
      ScopeTimer tm(c, "residual", s);
      launch_dg(c.dim, c.p, c.m, false, M_RES, c.kargs(), xv, nullptr, rv, nullptr, s);
    }
    return vnorm2(rv, N, W.red.p, s);
  };
  double res = resid(x, W.r.p);
  DGNP_REQUIRE(std::isfinite(res), DGNP_E_NONFINITE, "non-finite initial residual");
  st.res0 = res;
  st.res_hist[0] = res;
  int code = DGNP_E_NOCONV;
  for (int it = 0; it <= o.max_newton; ++it) {
    if (res <= o.rtol * st.res0 || res <= o.atol) {
      code = DGNP_OK;
      break;
    }
    if (it == o.max_newton) break;
    const auto ts = clk::now();
    // the potential block depends on the concentrations only, so the initial
    // guess's potential hierarchy serves the first Newton step; not with
    // electrodes, whose Butler-Volmer term adds a potential-dependent part
    set_state(c, x, o.prec, s, false, false, (phi_current && !c.has_electrode ? PC_CONC : PC_ALL) | PC_WARM);
    phi_current = false;
    st.t_setup += since(ts);
    vcopy<double>(W.r.p, W.b.p, N, s);
    vscale<double>(-1.0, W.b.p, N, s);
    vfill<double>(W.dx.p, 0.0, N, s);
    // Linear tolerance: the fixed relative tolerance of the paper's Newton-Krylov
    // solver, loosened on the final steps to what still takes the Newton
    // residual below its target (a linear residual of a tenth of the target
    // leaves the nonlinear remainder as the only other contribution).
    const double goal = std::max(o.rtol * st.res0, o.atol);
    const double eta = std::max(o.lin_rtol, std::min(0.5, 0.1 * goal / res));
    const auto tk = clk::now();
    LinResult lr = fgmres(c, W.b.p, W.dx.p, eta * res, o.restart, o.max_lin_it, f32, false, o.pc_kind, true,
                          o.verbose, s);
    precond_check(c);
    st.t_krylov += since(tk);
    st.lin_its_total += lr.its;
    st.refine_its_total += lr.refinements;
    if (it < DGNP_MAX_HIST) st.lin_its[it] = lr.its;
    // backtracking line search
    double lam = 1.0, rt = 0.0;
    bool ok = false;
    for (int cut = 0; cut <= 10; ++cut) {
      vcopy<double>(x, W.xt.p, N, s);
      vaxpy<double>(lam, W.dx.p, W.xt.p, N, s);
      rt = resid(W.xt.p, W.rt.p);
      if (std::isfinite(rt) && rt <= (1.0 - 1e-4 * lam) * res) {
        ok = true;
        break;
      }
      lam *= 0.5;
    }
    if (o.verbose)
      fprintf(stderr, "newton %d: |R| %.3e -> %.3e (lambda %.3g, %d its, lin res %.2e, eta %.2e)\n", it, res, rt,
              lam, lr.its, lr.res / res, eta);
    if (!ok) {
      code = DGNP_E_BREAKDOWN;
      break;
    }
    vcopy<double>(W.xt.p, x, N, s);
    std::swap(W.r.p, W.rt.p);
    res = rt;
    st.newton_its = it + 1;
    if (it + 1 < DGNP_MAX_HIST) st.res_hist[it + 1] = res;
  }
  DGNP_HIP(hipStreamSynchronize(s));
  st.res_final = res;
  st.status = code;
  st.t_total = since(t0);
  return code;
}

// kernel arguments of objective `kind` (0: outflow flux of species 1 through
// x = x_max; 1: reaction rate on the first electrode face)
KArgs objective_args(const dgnp_ctx& c, int kind) {
  KArgs A = c.kargs();
  DGNP_REQUIRE(kind == 0 || kind == 1, DGNP_E_ARG, "objective must be 0 (outflow) or 1 (electrode)");
  A.objective_kind = kind;
  A.objective_tag = 1;
  if (kind == 1) {
    A.objective_tag = -1;
    for (int t = 2 * c.dim - 1; t >= 0; --t)
      if (c.c_bc[t] == DGNP_C_ELECTRODE) A.objective_tag = t;
    DGNP_REQUIRE(A.objective_tag >= 0, DGNP_E_ARG, "objective 1 needs an electrode face");
  }
  return A;
}

// per-element partial sums of the objective kernel: (J, dJ/dPe, dJ/dJ0, dJ/dphi_app)
static std::array<double, 4> objective_sums(dgnp_ctx& c, const double* x, int kind, double* g, hipStream_t s) {
  launch_dg(c.dim, c.p, c.m, false, M_OBJG, objective_args(c, kind), x, nullptr, g, c.d_aux.p, s);
  std::vector<double> part(static_cast<size_t>(4 * c.E));
  DGNP_HIP(hipMemcpyAsync(part.data(), c.d_aux.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  DGNP_HIP(hipStreamSynchronize(s));
  std::array<double, 4> sum = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e = 0; e < c.E; ++e)
    for (int i = 0; i < 4; ++i) sum[size_t(i)] += part[size_t(4 * e + i)];
  return sum;
}

double objective_value(dgnp_ctx& c, const double* x, int kind) {
  hipStream_t s = c.work;
  DGNP_HIP(hipDeviceSynchronize());
  return objective_sums(c, x, kind, nullptr, s)[0];
}

// dJ/dtheta for the exchange currents and applied potentials of the electrode
// faces: the objective's explicit derivatives (objective 1, on its face) minus
// lambda^T dR/dtheta, summed per box face from the boundary-data kernel mode
void electrode_gradient(dgnp_ctx& c, const double* x, int kind, const double* lambda, double* dJ_dj0,
                        double* dJ_dpa) {
  hipStream_t s = c.work;
  DGNP_HIP(hipDeviceSynchronize());
  const KArgs A = objective_args(c, kind);
  const std::array<double, 4> ex = objective_sums(c, x, kind, nullptr, s);
  for (int t = 0; t < 6; ++t) {
    if (dJ_dj0) dJ_dj0[t] = 0.0;
    if (dJ_dpa) dJ_dpa[t] = 0.0;
  }
  if (!c.has_electrode) return;
  if (kind == 1) {
    if (dJ_dj0) dJ_dj0[A.objective_tag] = ex[2];
    if (dJ_dpa) dJ_dpa[A.objective_tag] = ex[3];
  }
  launch_dg(c.dim, c.p, c.m, false, M_DATAT, c.kargs(), x, lambda, nullptr, c.d_aux.p, s);
  std::vector<double> zeta(size_t(2) * c.n_bface * c.nqf);
  DGNP_HIP(hipMemcpyAsync(zeta.data(), c.d_aux.p, zeta.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  DGNP_HIP(hipStreamSynchronize(s));
  for (int t = 0; t < 2 * c.dim; ++t) {
    if (c.c_bc[t] != DGNP_C_ELECTRODE) continue;
    const int64_t f0 = c.btag_off[t], f1 = f0 + c.E / c.n[t / 2];
    double sp = 0.0, sj = 0.0;
    for (int64_t bf = f0; bf < f1; ++bf)
      for (int q = 0; q < c.nqf; ++q) {
        sp += zeta[size_t(bf) * c.nqf + q];
        sj += zeta[(size_t(c.n_bface) + bf) * c.nqf + q];
      }
    if (dJ_dj0) dJ_dj0[t] -= sj;
    if (dJ_dpa) dJ_dpa[t] -= sp;
  }
}

// ---------------------------------------------------------------------------
// Adjoint: J^T lambda = dJ/dx, gradients dJ/dtheta = dJ/dtheta|_x - lambda^T dR/dtheta
// ---------------------------------------------------------------------------
int adjoint_solve(dgnp_ctx& c, const double* x, int kind, double* dJ_dbc, double* dJ_dPe, double* J_out,
                  double* lambda, const dgnp_solve_opts& o, dgnp_solve_stats& st) {
  const auto t0 = clk::now();
  hipStream_t s = c.work;
  const int64_t N = c.N;
  st = dgnp_solve_stats{};
  DGNP_REQUIRE(o.restart >= 1 && o.restart <= MAXV - 8, DGNP_E_ARG, "restart must be 1..120");
  DGNP_REQUIRE(o.prec == DGNP_F64 || o.prec == DGNP_F32, DGNP_E_ARG, "prec must be F64 or F32");
  const auto ts = clk::now();
  set_state(c, x, o.prec, s);
  st.t_setup = since(ts);
  DevBuf<double> g, lam, dr, red;
  g.alloc(size_t(N));
  lam.alloc(size_t(N));
  dr.alloc(size_t(N));
  red.alloc(size_t(reduce_scratch_size()));
  const std::array<double, 4> ex = objective_sums(c, c.d_x.p, kind, g.p, s);
  const double J = ex[0], dJdPe_x = ex[1];
  const double gn = vnorm2(g.p, N, red.p, s);
  vfill<double>(lam.p, 0.0, N, s);
  const auto tk = clk::now();
  LinResult lr = fgmres(c, g.p, lam.p, o.rtol * gn, o.restart, o.max_lin_it, o.prec == DGNP_F32, true, o.pc_kind,
                        true, o.verbose, s);
  precond_check(c);
  st.t_krylov = since(tk);
  st.lin_its_total = lr.its;
  st.refine_its_total = lr.refinements;
  st.res0 = gn;
  st.res_final = lr.res;
  launch_dg(c.dim, c.p, c.m, false, M_DPE, c.kargs(), c.d_x.p, nullptr, dr.p, nullptr, s);
  const double ldr = vdot(lam.p, dr.p, N, red.p, s);
  if (dJ_dPe) *dJ_dPe = dJdPe_x - ldr;
  if (J_out) *J_out = J;
  if (dJ_dbc && c.n_bnode > 0) {
    launch_dg(c.dim, c.p, c.m, false, M_DATAT, c.kargs(), c.d_x.p, lam.p, nullptr, c.d_aux.p, s);
    std::vector<double> zeta(static_cast<size_t>(c.m) * c.n_bface * c.nqf);
    DGNP_HIP(hipMemcpyAsync(zeta.data(), c.d_aux.p, zeta.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DGNP_HIP(hipStreamSynchronize(s));
    const int nn = c.nn, nq = c.nq;
    for (int t = 0; t < 2 * c.dim; ++t) {
      if (c.bnode_off[t] < 0) continue;
      const int64_t nf = c.E / c.n[t / 2];
      for (int64_t lin = 0; lin < nf; ++lin) {
        const int64_t bf = c.btag_off[t] + lin;
        for (int k = 1; k < c.m; ++k)
          for (int jn = 0; jn < c.nfn; ++jn) {
            const int ji = jn % nn, jj = jn / nn;
            double acc = 0.0;
            for (int qf = 0; qf < c.nqf; ++qf) {
              const int qi = qf % nq, qj = qf / nq;
              double psi = c.ref.B[size_t(qi * nn + ji)];
              if (c.dim == 3) psi *= c.ref.B[size_t(qj * nn + jj)];
              acc += psi * zeta[(size_t(k) * c.n_bface + bf) * c.nqf + qf];
            }
            dJ_dbc[size_t(k - 1) * c.n_bnode + c.bnode_off[t] + lin * c.nfn + jn] = -acc;
          }
      }
    }
  }
  if (lambda) vcopy<double>(lam.p, lambda, N, s);
  DGNP_HIP(hipStreamSynchronize(s));
  st.t_total = since(t0);
  st.status = lr.converged ? DGNP_OK : DGNP_E_NOCONV;
  return st.status;
}

}  // namespace dgnp
