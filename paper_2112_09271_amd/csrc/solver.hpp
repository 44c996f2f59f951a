// Host drivers: state, operator applies, preconditioner, Newton-FGMRES, adjoint.
#pragma once

#include "context.hpp"

namespace dgnp {

void precond_symbolic(dgnp_ctx& c);                                   // precond.hip
// parts of the numeric preconditioner set-up: the potential block with its
// inverse blocks and multigrid hierarchy, and the concentration BILU(0) factors
// set-up parts; PC_WARM: the potential's power iteration may start from the
// previous set-up's last vector (within one Newton solve)
enum { PC_PHI = 1, PC_CONC = 2, PC_ALL = 3, PC_WARM = 4 };
void precond_numeric(dgnp_ctx& c, bool f32, hipStream_t s, bool assemble_only = false,
                     int parts = PC_ALL);  // precond.hip
void precond_apply(dgnp_ctx& c, const void* r, void* z, bool f32, bool transpose, int pc_kind,
                   hipStream_t s);                                     // precond.hip
void get_block(dgnp_ctx& c, int field, int64_t elem, int slot, double* out);
void precond_invalidate(dgnp_ctx& c);
// true when the concentration sweeps of this apply run as one resident grid per
// direction (line or element dataflow) rather than one launch per level
bool precond_sweeps_resident(const dgnp_ctx& c, bool f32, bool transpose);
// clears a dataflow sweep that hit its wait limit; throws DGNP_E_BREAKDOWN if report (synchronises)
void precond_check(dgnp_ctx& c, bool report = true);
void vcycle_phi(dgnp_ctx& c, const double* b, double* x, hipStream_t s);     // precond.hip
void vcycle_phi(dgnp_ctx& c, const float* b, float* x, hipStream_t s);
void phi_block_apply(dgnp_ctx& c, const double* x, double* y, hipStream_t s); // precond.hip
void phi_block_apply(dgnp_ctx& c, const float* x, float* y, hipStream_t s);
// y = A_phiphi x: assembled blocks or (matfree) the matrix-free operator       // precond.hip
void phi_apply(dgnp_ctx& c, const void* x, void* y, bool f32, bool matfree, hipStream_t s);

void set_state(dgnp_ctx& c, const double* x, int prec, hipStream_t s, bool assemble_only = false,
               bool apply_only = false, int parts = PC_ALL);
// vmask: fields of v that are read (the others count as zero); phi_rows (forward
// apply only): only the potential rows of y = J v are formed and written, as
// y = base - (J v) when base is not null
void jac_apply(dgnp_ctx& c, const void* v, void* y, bool f32, bool transpose, hipStream_t s,
               unsigned vmask = ~0u, bool phi_rows = false, const void* base = nullptr);
dgnp_solve_opts default_solve_opts();
KArgs objective_args(const dgnp_ctx& c, int kind);  // kernel arguments of objective 0 / 1
double objective_value(dgnp_ctx& c, const double* x, int kind);
void electrode_gradient(dgnp_ctx& c, const double* x, int kind, const double* lambda, double* dJ_dj0,
                        double* dJ_dpa);
int newton_solve(dgnp_ctx& c, double* x, const dgnp_solve_opts& o, dgnp_solve_stats& st);
int adjoint_solve(dgnp_ctx& c, const double* x, int kind, double* dJ_dbc, double* dJ_dPe, double* J_out,
                  double* lambda, const dgnp_solve_opts& o, dgnp_solve_stats& st);

}  // namespace dgnp
