// Launchers of the concentration-block multigrid kernels (kernels_gmg.hip).
// Layouts: blocks [field][E][2d+1][nb][nb] (field stride fs), vectors
// [field][E][nb] (field stride E nb), Pi [2^d][nb][nb] (Pi[c][k][i]: coarse
// basis function i at fine node k of child c); nfine = element counts of the
// fine grid per axis (each even).
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {
// Ac = P^T Af P per field for the Ec coarse elements
void launch_gmg_galerkin(int nb, int dim, int nfields, const double* Af, int64_t fsf, const int* nbr,
                         const int* nfine, const double* Pi, double* Ac, int64_t fsc, int64_t Ec, hipStream_t s);
// rc = P^T r (nff, nfc: entries per field on the fine / coarse level)
template <typename T>
void launch_gmg_restrict(int nb, int dim, int nfields, const T* Pi, const int* nfine, const T* r, int64_t nff,
                         T* rc, int64_t nfc, hipStream_t s);
// x += P xc
template <typename T>
void launch_gmg_prolong(int nb, int dim, int nfields, const T* Pi, const int* nfine, const T* xc, int64_t nfc, T* x,
                        int64_t nff, hipStream_t s);
// inverse of every field's dense matrix of the block level (blk, nbr, E):
// M, MT [nfields][n][n] with n = E nb <= 1024 receive the inverse and its
// transpose; *err is set to 1 when a pivot vanishes (not cleared here)
void launch_gmg_dense_inverse(int nb, int dim, int nfields, const double* blk, int64_t fs, const int* nbr,
                               int64_t E, double* M, double* MT, int* err, hipStream_t s);
// r = b - A x, or b - A^T x with transpose; block rows of ld >= nb entries
template <typename T>
void launch_gmg_resid(int nb, int dim, int nfields, bool transpose, const T* blk, int64_t fs, int ld, const int* nbr,
                      int64_t E, const T* x, const T* b, T* r, hipStream_t s);
}  // namespace dgnp
