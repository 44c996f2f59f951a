// Launchers of the block kernels (kernels_block.hip) and CSR kernels (kernels_csr.hip).
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {
void upload_ref_tables_block(const RefTables* tabs, int count);
void upload_gll_nodes(const RefTables* tabs, int count);
// diagonal field blocks of fields f0 .. f0 + nf - 1 (blk holds all m fields)
void launch_assemble(int dim, int p, int m, int f0, int nf, const KArgs& A, const double* xs, double* blk,
                     hipStream_t s);
void launch_block_inverse(int nb, int64_t E, const double* blk, int nslot, double* out, hipStream_t s);
// BILU(0) of nfields field blocks (block stride fstride), one hyperplane level
// per launch: D_i^{-1} and every scaled off-diagonal block of the level's
// elements.  b32 (not null): each finished block also stored in single
// precision there, same layout; over all levels every slot of every element.
void launch_ilu_factor(int nb, int dim, int nfields, int64_t fstride, double* blk, const int* nbr,
                       const int* lev, int64_t first, int64_t count, hipStream_t s, float* b32 = nullptr);
// kind 0: forward, 1: backward (in may alias out), 2: transposed forward,
// 3: transposed backward (aux holds the forward result and is overwritten).
// nfields independent field blocks at block stride bstride / vector stride vstride.
template <typename T>
void launch_ilu_solve(int kind, int nb, int dim, const T* blk, const int* nbr, const int* lev, int64_t first,
                      int64_t count, int nfields, int64_t bstride, int64_t vstride, const T* in, T* out, T* aux,
                      hipStream_t s);
// dataflow sweeps (kind 0 forward, 1 backward) over the level order `order`;
// every entry is published with its sweep count in packed 64-bit words,
// wp[nfields][Nf * W] with W = 1 word per float entry and 2 per double (the
// words of one buffer start at equal counts, zero at first); grid from
// ilu_dataflow_grid (resident on the device at once)
template <typename T>
int ilu_dataflow_grid(int nb, int dim, int64_t E, int nfields);
template <typename T>
void launch_ilu_dataflow(int kind, int nb, int dim, const T* blk, const int* nbr, const int* order, int64_t E,
                         int nfields, int64_t bstride, int64_t vstride, const T* in, T* out, uint64_t* wp, int* err,
                         int spin_limit, int grid, hipStream_t s);
// line sweeps (single precision, packed words as launch_ilu_dataflow):
// lines of `len` elements along axis ax, first elements line_first[0..nline)
// ordered by level, element stride lstride; grid from ilu_lines_grid
int ilu_lines_grid(int nb, int dim, int nline, int nfields);
void launch_ilu_lines(int kind, int nb, int dim, const float* blk, const int* nbr, const int* line_first, int nline,
                      int len, int64_t lstride, int ax, int nfields, int64_t bstride, int64_t vstride,
                      const float* in, float* out, uint64_t* wp, int* err, int spin_limit, int grid, hipStream_t s);
// Row stride of the potential block and of its inverse diagonal blocks as
// launch_bspmv, launch_bdiag and launch_cheb_blk read them: single-precision
// blocks of up to 32 rows have rows padded to a multiple of four floats (zeros
// in the padding); all others are stored unpadded.
inline int pot_ld(int nb, bool f32) { return (f32 && nb <= 32) ? ((nb + 3) & ~3) : nb; }
// y = alpha A x + beta b over the element-block graph (block rows of pot_ld);
// nsys independent systems in one launch, the k-th at blk + k bstride with
// vectors at x, b, y + k vstride
template <typename T>
void launch_bspmv(int nb, int dim, int64_t E, const T* blk, const int* nbr, const T* x, const T* b, T alpha,
                  T beta, T* y, hipStream_t s, int nsys = 1, int64_t bstride = 0, int64_t vstride = 0);
template <typename T>
void launch_bdiag(int nb, int64_t E, const T* dinv, const T* x, T* y, hipStream_t s);
// restriction (d1 not null): also d1 = c1 (dinv .* b), the first Chebyshev
// step of the vertex level from a zero guess
template <typename T>
void launch_q1(bool prolong, int dim, int p, const int* n, const T* a, T* b, T beta, int64_t E, int64_t nvert,
               hipStream_t s, const T* dinv = nullptr, T c1 = T(0), T* d1 = nullptr);
void launch_q1_galerkin(int dim, int p, int64_t E, const double* blk, double* gal, hipStream_t s);
// st[nvert][3^dim]: the Galerkin vertex operator as a dense 3^dim-point stencil per vertex
void launch_vertex_stencil(int dim, const double* gal, const int* nbr, const int* n, int64_t nvert, double* st,
                           hipStream_t s);

// fused Chebyshev step (r = base - A u - sub; d = c1 Dinv r + c2 dprev; x_out = x_in + d),
// null u / sub / dprev / x_in drop their terms, null r_out / d_out skip those stores
template <typename T>
void launch_cheb_blk(int nb, int dim, int64_t E, const T* blk, const int* nbr, const T* dinv, const T* u,
                     const T* base, const T* sub, const T* dprev, const T* x_in, T c1, T c2, T* r_out, T* d_out,
                     T* x_out, hipStream_t s);
// p-multigrid: corner values of the state (m fields, order p -> [m][E][2^d]);
// transfers between order p and p = 1 DG functions element by element:
// prolong: b = P a + beta b; restrict: b = P^T (a - sub) (sub may be null)
void launch_p1_inject(int dim, int p, const double* x, double* x1, int m, int64_t E, hipStream_t s);
template <typename T>
void launch_p1(bool prolong, int dim, int p, const T* a, const T* sub, T* b, T beta, int64_t E, hipStream_t s);
template <typename T>
void launch_cheb_csr(int n, const int* rp, const int* ci, const T* v, const T* dinv, const T* u, const T* base,
                     const T* dprev, const T* x_in, T c1, T c2, T* r_out, T* d_out, T* x_out, hipStream_t s);

// CSR: y = alpha * A x + beta * b (b may be null); nnz (if known) picks one
// 64-lane wave per row for rows of 32 or more entries on average, else 8 lanes
template <typename T>
void launch_csr_spmv(int n, const int* rp, const int* ci, const T* v, const T* x, const T* b, T alpha, T beta,
                     T* y, hipStream_t s, int64_t nnz = 0);
template <typename T>
void launch_vmul(int64_t n, const T* d, const T* x, T* y, hipStream_t s);  // y = d .* x
template <typename T>
void launch_dense_gemv(int n, const T* M, const T* x, T* y, hipStream_t s, int nsys = 1,
                       int64_t xs = 0);  // y = M x for nsys systems (M + k n^2, x and y + k xs)
}  // namespace dgnp
