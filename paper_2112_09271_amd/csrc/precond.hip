// Block preconditioner storage and applies.
#include "solver.hpp"

namespace dgnp {

struct Precond {};

void precond_destroy(Precond* p) { delete p; }
void precond_symbolic(dgnp_ctx&) {}
void precond_numeric(dgnp_ctx&, bool, hipStream_t) {}
void precond_apply(dgnp_ctx&, const void*, void*, bool, bool, int, hipStream_t) {
  throw Error(DGNP_E_STATE, "preconditioner not available");
}
void get_block(dgnp_ctx&, int, int64_t, int, double*) {
  throw Error(DGNP_E_STATE, "no assembled blocks");
}

}  // namespace dgnp
