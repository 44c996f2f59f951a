// Vector kernels (blas.hip): conversions, axpy-type updates, reductions.
#pragma once

#include "dgnp_impl.hpp"

namespace dgnp {
// most vectors one reduction call handles (the Krylov basis of the longest restart)
constexpr int MAXV = 128;
void cvt_d2f(const double* x, float* y, int64_t n, hipStream_t s);
// rows of nb doubles -> rows of ld >= nb floats, zero-padded
void cvt_d2f_rows(const double* x, float* y, int64_t rows, int nb, int ld, hipStream_t s);
void cvt_f2d(const float* x, double* y, int64_t n, hipStream_t s);
template <typename T> void vfill(T* x, T v, int64_t n, hipStream_t s);
template <typename T> void vcopy(const T* x, T* y, int64_t n, hipStream_t s);
template <typename T> void vaxpy(T a, const T* x, T* y, int64_t n, hipStream_t s);        // y += a x
template <typename T> void vaxpby(T a, const T* x, T b, T* y, int64_t n, hipStream_t s);  // y = a x + b y
template <typename T> void vscale(T a, T* x, int64_t n, hipStream_t s);
template <typename T> void vsub(const T* x, const T* y, T* z, int64_t n, hipStream_t s);  // z = x - y
// out[j] = <V_j, w> for j < k, V column-major [k][n] (double accumulation)
void vdots(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* out_dev,
           hipStream_t s);
// the same with the results in out[0..k) and the block partials in scratch
// (k * reduce-blocks entries); the _f variant reads w in single precision and
// also stores it widened to double in w64
void vdots_into(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* out, double* scratch,
                hipStream_t s);
void vscale_dual(double a, const double* x, double* y, float* y32, int64_t n, hipStream_t s);  // y = a x, y32 = (float) y
// w -= sum_j h[j] V_j
// y = sum_j h[j] Z_j (Z of type T) accumulated in double into y (y += when accumulate)
template <typename T>
void vcombine(const T* Z, int64_t ldz, int k, const double* h_dev, double* y, int64_t n, hipStream_t s);
double vnorm2(const double* x, int64_t n, double* scratch_dev, hipStream_t s);  // synchronises
double vnorm2(const float* x, int64_t n, double* scratch_dev, hipStream_t s);   // synchronises
// Delayed classical Gram-Schmidt, step j (see blas.hip): dcgs_reduce forms the
// coefficient block coef[2 MAXV + 8] from V[:, <j], u and w (w null: only
// s, sigma and alpha, for the last column of a cycle; w_f32: w in single
// precision, widened into w64); dcgs_update writes V[:, j], the next u and
// its preconditioner-input copy m, and (zd not null) copies zs to zd in the same
// pass.  partial holds dcgs_partial_size() doubles, zero-filled once before the
// first use (the tail holds a counter that each reduction leaves at zero).  hout (not null: host memory
// mapped for the device, DCGS_COEF doubles) receives the entries of the block
// that the host reads, written by the reduction's last kernel, and then, as a
// 64-bit integer at DCGS_FLAG after a system-scope release, the number seq.
void dcgs_reduce(const double* V, int64_t ldv, int j, const double* u, const void* w, bool w_f32, double* w64,
                 int64_t n, double* partial, double* coef, hipStream_t s, double* hout = nullptr,
                 unsigned long long seq = 0);
template <typename TM>
void dcgs_update(double* V, int64_t ldv, int j, const double* coef, double* u, const double* w, TM* m,
                 const TM* zs, TM* zd, int64_t n, hipStream_t s);
int64_t dcgs_partial_size();
constexpr int DCGS_ALPHA = 2 * MAXV + 1, DCGS_HJJ = 2 * MAXV + 2, DCGS_RHO = 2 * MAXV + 4, DCGS_FLAG = 2 * MAXV + 7,
              DCGS_COEF = 2 * MAXV + 8;
// *out = x . x (accumulated in double) without a host wait; scratch holds the block partials
void vsq_into(const float* x, int64_t n, double* out, double* scratch, hipStream_t s);
// x /= sqrt(*ss_dev), read on the device (no change when *ss_dev <= 0)
template <typename T>
void vscale_rsqrt_inplace(const double* ss_dev, T* x, int64_t n, hipStream_t s);
template <typename T>
void vfill_hash(T* x, int64_t n, hipStream_t s);  // deterministic values in [-0.5, 0.5)
double vdot(const double* x, const double* y, int64_t n, double* scratch_dev, hipStream_t s);
int64_t reduce_scratch_size();
}  // namespace dgnp
