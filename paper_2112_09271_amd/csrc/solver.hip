// Host drivers: linearisation state and matrix-free Jacobian applies.
#include "blas.hpp"
#include "solver.hpp"

namespace dgnp {

void set_state(dgnp_ctx& c, const double* x, int prec, hipStream_t s) {
  c.d_x.alloc(size_t(c.N));
  vcopy<double>(x, c.d_x.p, c.N, s);
  c.has_state = true;
  c.has_state32 = false;
  if (prec == DGNP_F32) {
    c.d_x32.alloc(size_t(c.N));
    cvt_d2f(c.d_x.p, c.d_x32.p, c.N, s);
    c.has_state32 = true;
  }
  precond_numeric(c, prec == DGNP_F32, s);
  DGNP_HIP(hipStreamSynchronize(s));
}

void jac_apply(dgnp_ctx& c, const void* v, void* y, bool f32, bool transpose, hipStream_t s) {
  DGNP_REQUIRE(c.has_state, DGNP_E_STATE, "jacobian_apply before set_state");
  DGNP_REQUIRE(!f32 || c.has_state32, DGNP_E_STATE, "float apply needs set_state with DGNP_F32");
  const void* xs = f32 ? static_cast<const void*>(c.d_x32.p) : static_cast<const void*>(c.d_x.p);
  launch_dg(c.dim, c.p, c.m, f32, transpose ? M_JACT : M_JAC, c.kargs(), xs, v, y, nullptr, s);
}

dgnp_solve_opts default_solve_opts() {
  dgnp_solve_opts o{};
  o.rtol = 1e-8;
  o.atol = 0.0;
  o.max_newton = 30;
  o.prec = DGNP_F64;
  o.lin_rtol = 1e-3;
  o.restart = 30;
  o.max_lin_it = 600;
  o.pc_kind = DGNP_PC_P2;
  o.verbose = 0;
  return o;
}

int newton_solve(dgnp_ctx&, double*, const dgnp_solve_opts&, dgnp_solve_stats& st) {
  st.status = DGNP_E_STATE;
  throw Error(DGNP_E_STATE, "solver not available");
}

int adjoint_solve(dgnp_ctx&, const double*, double*, double*, double*, double*, const dgnp_solve_opts&,
                  dgnp_solve_stats& st) {
  st.status = DGNP_E_STATE;
  throw Error(DGNP_E_STATE, "adjoint not available");
}

}  // namespace dgnp
