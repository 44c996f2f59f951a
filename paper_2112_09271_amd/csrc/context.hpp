// Library context: mesh tables, reference tables, boundary data, state and
// preconditioner storage of one problem on one GPU.
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {
struct Precond;  // preconditioner storage (precond.hip)
void precond_destroy(Precond*);
struct Krylov;   // FGMRES storage (solver.hip)
void krylov_destroy(Krylov*);
}  // namespace dgnp

struct dgnp_ctx {
  int dim = 3, p = 1, m = 2, nn = 2, nq = 3, nb = 8, nqv = 27, nqf = 9, nfn = 4;
  int64_t E = 0, Nf = 0, N = 0, F = 0, n_bface = 0, n_bnode = 0;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  double z[4] = {}, D[4] = {}, a[4] = {}, b[4] = {};
  double delta = 0, c_ip = 10;
  int phi_mg = 1;                 // DGNP_PHIMG_Q1 / _P / _PG (AUTO resolved at setup)
  int conc_pc = 0;                // DGNP_CPC_BILU / _GMG
  int gmg_nu = 2;                 // smoothing steps per side of the concentration V-cycle
  int mms = 0;
  dgnp_velocity vel{};
  int c_bc[6] = {}, phi_bc[6] = {};
  double phi_val[6] = {};
  std::vector<int> nbr;          // [E][2d]
  std::vector<int> face_elems;   // [F][2]
  std::vector<int> face_axis;    // [F]
  int64_t btag_off[6] = {};      // first boundary face of each box face
  int64_t bnode_off[6] = {};     // first data node of each box face (-1: no data)
  std::vector<double> bc_conc;   // [m-1][n_bnode]
  std::vector<double> src_vol;   // caller sources [m][E][nqv] (empty: none, or the manufactured solution's)
  std::vector<double> dir_face;  // caller boundary data [m][n_bface][nqf] (empty: from bc_conc / phi_val)
  dgnp::DevAllocator allocator;  // device workspace allocator (the caller's hook or hipMalloc)
  // Butler-Volmer electrodes (faces tagged DGNP_C_ELECTRODE)
  bool has_electrode = false;
  int bv_ion = 1, bv_prof = 0;
  double bv_aa = 0, bv_ac = 0, bv_j0[6] = {}, bv_phi_app[6] = {};
  dgnp::RefTables ref;
  hipStream_t stream = nullptr;   // the caller's stream at setup
  hipStream_t work = nullptr;     // library stream for the synchronous drivers (graph capture)
  uint64_t state_epoch = 0;       // bumped by every set_state (invalidates captured graphs)

  dgnp::DevBuf<int> d_nbr;
  dgnp::DevBuf<double> d_bcq;    // [m][n_bface][nqf]
  dgnp::DevBuf<double> d_src;    // [m][E][nqv] (manufactured solutions only)
  dgnp::DevBuf<double> d_aux;    // objective partial sums etc.
  double* obj_scratch = nullptr;  // static partial-sum array of the allocation-free objective (this device)

  // linearisation point
  dgnp::DevBuf<double> d_x;
  dgnp::DevBuf<float> d_x32;
  bool has_state = false, has_state32 = false;
  // tabulated linearisation data of the 3-D Jacobian apply (kernels_jac.hip):
  // volume [E][m+2][nq^3] and face [E][6][m+1][nq^2] tables per precision
  bool jac_tab = true;             // use them (DGNP_JAC_GENERAL=1: the general operator kernel)
  dgnp::DevBuf<double> d_jtv, d_jtf;
  dgnp::DevBuf<float> d_jtv32, d_jtf32;

  dgnp::Precond* pc = nullptr;
  dgnp::Krylov* kry = nullptr;

  // optional per-kernel event timing
  bool profiling = false;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, std::pair<double, int64_t>> timers;
  hipEvent_t ev_get() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void ev_resolve() {
    for (auto& p : pending) {
      float ms = 0.0f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& t = timers[p.name];
        t.first += 1e-3 * ms;
        t.second += 1;
      }
      ev_pool.push_back(p.a);
      ev_pool.push_back(p.b);
    }
    pending.clear();
  }

  ~dgnp_ctx() {
    ev_resolve();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    dgnp::krylov_destroy(kry);
    dgnp::precond_destroy(pc);
    if (work) (void)hipStreamDestroy(work);
  }
  dgnp::KArgs kargs() const;
};

namespace dgnp {
// records a pair of events around a region on stream s when profiling is on
struct ScopeTimer {
  dgnp_ctx& c;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ScopeTimer(dgnp_ctx& ctx, const char* nm, hipStream_t st) : c(ctx), name(nm), s(st) {
    if (c.profiling) {
      a = c.ev_get();
      if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
    }
  }
  ~ScopeTimer() {
    if (!a) return;
    hipEvent_t b = c.ev_get();
    if (b && hipEventRecord(b, s) == hipSuccess) c.pending.push_back({name, a, b});
    if (c.pending.size() > 100000) c.ev_resolve();
  }
};
void build_tables(dgnp_ctx& c);                 // mesh, faces, boundary data (tables.cpp)
void mms_exact(const dgnp_ctx& c, const double* x, double* phi, double* c1);
void mms_source(const dgnp_ctx& c, const double* x, double* s_phi, double* s_c1);
}  // namespace dgnp
