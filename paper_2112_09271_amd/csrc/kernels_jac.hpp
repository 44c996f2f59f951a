// Jacobian apply with tabulated linearisation data (kernels_jac.hip).
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {
void upload_ref_tables_jac(const RefTables* tabs, int count);
// entries of the volume table [E][m+2][nq^3] followed by the velocity factors
// [n0 + n1][3][nq + 2] (return value) and of the face table [E][6][m+1][nq^2]
// (*nf) of a 3-D problem of order p with m fields on n[0] x n[1] x n[2] elements
size_t jlin_table_sizes(int p, int m, int64_t E, const int* n, size_t* nf);
// tables of the state xs (double [m][E][nb]) in the precision T
template <typename T>
void launch_jlin_tables(int p, int m, const KArgs& A, const double* xs, T* tv, T* tf, hipStream_t s);
// y = J v (coupling = false; input fields masked by A.vin_mask) or the potential
// rows of J v for the concentration part of v (coupling = true; y[0, N_f) =
// A.jbase - (J v) rows when A.jbase is set)
template <typename T>
void launch_jlin(int p, int m, bool coupling, const KArgs& A, const T* v, const T* tv, const T* tf, T* y,
                 hipStream_t s);
}  // namespace dgnp
