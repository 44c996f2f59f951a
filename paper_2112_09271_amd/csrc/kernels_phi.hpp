// Matrix-free potential-potential block (3-D, orders 2 and 3) for p-multigrid.
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {

void upload_ref_tables_phi(const RefTables* tabs, int count);
// kappa tables of the linearisation point (FP64 state xs [m][E][NB]):
// kv [E][(p+2)^3] = kappa w detJ at the volume Gauss points,
// kf [E][6][(p+2)^2] = kappa w_face at the face Gauss points of the own traces
template <typename T>
void launch_phi_kappa(int p, int m, const KArgs& A, const double* xs, T* kv, T* kf, hipStream_t s);
// y = A_phiphi u (u, y: [E][NB])
template <typename T>
void launch_phi_op(int p, const KArgs& A, const T* u, const T* kv, const T* kf, T* y, hipStream_t s);

}  // namespace dgnp
