// Scalar CSR kernels for the coarse levels of the algebraic multigrid hierarchy.
#include "kernels_block.hpp"

namespace dgnp {

// one 8-lane group per row
template <typename T>
__global__ void k_csr_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const T* __restrict__ v, const T* __restrict__ x, const T* __restrict__ b, T alpha,
                           T beta, T* __restrict__ y) {
  const int64_t gid = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int row = int(gid >> 3), lane = int(gid & 7);
  T acc = T(0);
  if (row < n)
    for (int k = rp[row] + lane; k < rp[row + 1]; k += 8) acc += v[k] * x[ci[k]];
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 4, 64);
  if (row < n && lane == 0) y[row] = alpha * acc + (b ? beta * b[row] : T(0));
}

// one 64-lane wave per row, for matrices with long rows (the aggregation
// restriction R = P^T: tens of entries per row)
template <typename T>
__global__ void k_csr_spmv_wide(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                const T* __restrict__ v, const T* __restrict__ x, const T* __restrict__ b, T alpha,
                                T beta, T* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  T acc = T(0);
  if (row < n)
    for (int k = rp[row] + lane; k < rp[row + 1]; k += 64) acc += v[k] * x[ci[k]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (row < n && lane == 0) y[row] = alpha * acc + (b ? beta * b[row] : T(0));
}

template <typename T>
void launch_csr_spmv(int n, const int* rp, const int* ci, const T* v, const T* x, const T* b, T alpha, T beta,
                     T* y, hipStream_t s, int64_t nnz) {
  if (n <= 0) return;
  if (nnz >= int64_t(n) * 32) {
    hipLaunchKernelGGL(k_csr_spmv_wide<T>, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, n, rp, ci, v, x, b, alpha,
                       beta, y);
  } else {
    const int64_t thr = int64_t(n) * 8;
    hipLaunchKernelGGL(k_csr_spmv<T>, dim3(unsigned((thr + 255) / 256)), dim3(256), 0, s, n, rp, ci, v, x, b,
                       alpha, beta, y);
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_csr_spmv<double>(int, const int*, const int*, const double*, const double*, const double*,
                                      double, double, double*, hipStream_t, int64_t);
template void launch_csr_spmv<float>(int, const int*, const int*, const float*, const float*, const float*,
                                     float, float, float*, hipStream_t, int64_t);

template <typename T>
__global__ void k_vmul(int64_t n, const T* __restrict__ d, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = d[i] * x[i];
}

template <typename T>
void launch_vmul(int64_t n, const T* d, const T* x, T* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_vmul<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, d, x, y);
  DGNP_HIP(hipGetLastError());
}
template void launch_vmul<double>(int64_t, const double*, const double*, double*, hipStream_t);
template void launch_vmul<float>(int64_t, const float*, const float*, float*, hipStream_t);

// dense row-major n x n matrix-vector product, one 64-lane wave per row;
// blockIdx.y: one of several systems, the k-th at M + k n^2, x + k xs, y + k xs
template <typename T>
__global__ void k_dense_gemv(int n, const T* __restrict__ M, const T* __restrict__ x, T* __restrict__ y,
                             int64_t xs) {
  M += blockIdx.y * int64_t(n) * n;
  x += blockIdx.y * xs;
  y += blockIdx.y * xs;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  T acc = T(0);
  if (row < n)
    for (int c = lane; c < n; c += 64) acc += M[int64_t(row) * n + c] * x[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (row < n && lane == 0) y[row] = acc;
}

template <typename T>
void launch_dense_gemv(int n, const T* M, const T* x, T* y, hipStream_t s, int nsys, int64_t xs) {
  if (n <= 0 || nsys <= 0) return;
  hipLaunchKernelGGL(k_dense_gemv<T>, dim3(unsigned((n + 3) / 4), unsigned(nsys)), dim3(256), 0, s, n, M, x, y, xs);
  DGNP_HIP(hipGetLastError());
}
template void launch_dense_gemv<double>(int, const double*, const double*, double*, hipStream_t, int, int64_t);
template void launch_dense_gemv<float>(int, const float*, const float*, float*, hipStream_t, int, int64_t);

// One Chebyshev smoothing step on a scalar (CSR) level, fused:
//   r = base - A u          (u null: r = base)
//   d = c1 * dinv .* r + c2 * dprev   (dprev null: no second term)
//   x_out = x_in + d        (x_in null: x_out = d)
// with optional stores of r and d.  One 8-lane group per row.  x_out must not
// alias u (other rows read u).
template <typename T>
__global__ void k_cheb_csr(int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v,
                           const T* __restrict__ dinv, const T* u, const T* base, const T* dprev, const T* x_in,
                           T c1, T c2, T* r_out, T* d_out, T* x_out) {
  const int64_t gid = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int row = int(gid >> 3), lane = int(gid & 7);
  T acc = T(0);
  if (row < n && u)
    for (int k = rp[row] + lane; k < rp[row + 1]; k += 8) acc += v[k] * u[ci[k]];
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 4, 64);
  if (row < n && lane == 0) {
    const T r = base[row] - acc;
    T d = c1 * (dinv[row] * r);
    if (dprev) d += c2 * dprev[row];
    if (r_out) r_out[row] = r;
    if (d_out) d_out[row] = d;
    x_out[row] = (x_in ? x_in[row] : T(0)) + d;
  }
}

template <typename T>
void launch_cheb_csr(int n, const int* rp, const int* ci, const T* v, const T* dinv, const T* u, const T* base,
                     const T* dprev, const T* x_in, T c1, T c2, T* r_out, T* d_out, T* x_out, hipStream_t s) {
  if (n <= 0) return;
  const int64_t thr = int64_t(n) * 8;
  hipLaunchKernelGGL(k_cheb_csr<T>, dim3(unsigned((thr + 255) / 256)), dim3(256), 0, s, n, rp, ci, v, dinv, u,
                     base, dprev, x_in, c1, c2, r_out, d_out, x_out);
  DGNP_HIP(hipGetLastError());
}
template void launch_cheb_csr<double>(int, const int*, const int*, const double*, const double*, const double*,
                                      const double*, const double*, const double*, double, double, double*,
                                      double*, double*, hipStream_t);
template void launch_cheb_csr<float>(int, const int*, const int*, const float*, const float*, const float*,
                                     const float*, const float*, const float*, float, float, float*, float*,
                                     float*, hipStream_t);

}  // namespace dgnp
