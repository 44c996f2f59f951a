// Vector kernels for the Krylov and Newton drivers.  Reductions are two-pass
// (fixed block partials, then one block), so results do not depend on timing.
#include "blas.hpp"
#include <cmath>

namespace dgnp {

static constexpr int VB = 256;
static constexpr int RED_BLOCKS = 1024;

static inline unsigned grid_for(int64_t n) {
  // one element per thread up to the grid limit: enough waves in flight to
  // cover memory latency on vectors of a few hundred thousand entries
  int64_t g = (n + VB - 1) / VB;
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return unsigned(g);
}

__global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB)
    y[i] = float(x[i]);
}
// y[r][c] = x[r][c] for c < nb, 0 for nb <= c < ld (rows of nb doubles to rows of ld floats)
__global__ void k_d2f_rows(const double* __restrict__ x, float* __restrict__ y, int64_t rows, int nb, int ld) {
  const int64_t n = rows * ld;
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    const int64_t r = i / ld;
    const int c = int(i - r * ld);
    y[i] = c < nb ? float(x[r * nb + c]) : 0.f;
  }
}
__global__ void k_f2d(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB)
    y[i] = double(x[i]);
}
template <typename T>
__global__ void k_fill(T* __restrict__ x, T v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) x[i] = v;
}
template <typename T>
__global__ void k_copy(const T* __restrict__ x, T* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) y[i] = x[i];
}
// y = a x + b y; y is not read when b == 0 (it may be uninitialised memory)
template <typename T>
__global__ void k_axpby(T a, const T* __restrict__ x, T b, T* __restrict__ y, int64_t n) {
  if (b == T(0)) {
    for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) y[i] = a * x[i];
  } else {
    for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB)
      y[i] = a * x[i] + b * y[i];
  }
}
template <typename T>
__global__ void k_axpy(T a, const T* __restrict__ x, T* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB)
    y[i] += a * x[i];
}
// z = x - y
template <typename T>
__global__ void k_sub(const T* __restrict__ x, const T* __restrict__ y, T* __restrict__ z, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) z[i] = x[i] - y[i];
}
template <typename T>
__global__ void k_scale(T a, T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) x[i] *= a;
}

void cvt_d2f(const double* x, float* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(VB), 0, s, x, y, n);
}
void cvt_d2f_rows(const double* x, float* y, int64_t rows, int nb, int ld, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_d2f_rows, dim3(grid_for(rows * ld)), dim3(VB), 0, s, x, y, rows, nb, ld);
}
void cvt_f2d(const float* x, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n)), dim3(VB), 0, s, x, y, n);
}
template <typename T>
void vfill(T* x, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(VB), 0, s, x, v, n);
}
template <typename T>
void vcopy(const T* x, T* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(n)), dim3(VB), 0, s, x, y, n);
}
template <typename T>
void vaxpy(T a, const T* x, T* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy<T>, dim3(grid_for(n)), dim3(VB), 0, s, a, x, y, n);
}
template <typename T>
void vaxpby(T a, const T* x, T b, T* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n)), dim3(VB), 0, s, a, x, b, y, n);
}
// y = a x and y32 = float(a x)
__global__ void k_scale_dual(double a, const double* __restrict__ x, double* __restrict__ y, float* __restrict__ y32,
                             int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    const double v = a * x[i];
    y[i] = v;
    y32[i] = float(v);
  }
}
void vscale_dual(double a, const double* x, double* y, float* y32, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_dual, dim3(grid_for(n)), dim3(VB), 0, s, a, x, y, y32, n);
}
template <typename T>
void vsub(const T* x, const T* y, T* z, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub<T>, dim3(grid_for(n)), dim3(VB), 0, s, x, y, z, n);
}
template void vsub<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void vsub<float>(const float*, const float*, float*, int64_t, hipStream_t);
template <typename T>
void vscale(T a, T* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale<T>, dim3(grid_for(n)), dim3(VB), 0, s, a, x, n);
}
template void vfill<double>(double*, double, int64_t, hipStream_t);
template void vfill<float>(float*, float, int64_t, hipStream_t);
template void vcopy<double>(const double*, double*, int64_t, hipStream_t);
template void vcopy<float>(const float*, float*, int64_t, hipStream_t);
template void vaxpy<double>(double, const double*, double*, int64_t, hipStream_t);
template void vaxpy<float>(float, const float*, float*, int64_t, hipStream_t);
template void vaxpby<double>(double, const double*, double, double*, int64_t, hipStream_t);
template void vaxpby<float>(float, const float*, float, float*, int64_t, hipStream_t);
template void vscale<double>(double, double*, int64_t, hipStream_t);
template void vscale<float>(float, float*, int64_t, hipStream_t);

// x[i] = pseudo-random value in [-0.5, 0.5) from a counter-based hash of i (splitmix64)
template <typename T>
__global__ void k_hash_fill(T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    uint64_t z = uint64_t(i) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = T(double(z % 1000003ull) / 1000003.0 - 0.5);
  }
}
template <typename T>
void vfill_hash(T* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_hash_fill<T>, dim3(grid_for(n)), dim3(VB), 0, s, x, n);
}
template void vfill_hash<double>(double*, int64_t, hipStream_t);
template void vfill_hash<float>(float*, int64_t, hipStream_t);

// ---- reductions ---------------------------------------------------------------
// sum over the block (returned to every thread): wave sums by lane shuffles,
// then the VB / 64 wave sums through LDS; sh holds at least VB / 64 doubles
__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < VB / 64; ++k) t += sh[k];
  return t;
}

// partial[j][blk] = sum over the block's chunk of V_j * w
__global__ void k_dots_partial(const double* __restrict__ V, int64_t ldv, const double* __restrict__ w,
                               int64_t n, double* __restrict__ partial) {
  __shared__ double sh[VB];
  const int j = blockIdx.y;
  const double* v = V + j * ldv;
  double a0 = 0.0, a1 = 0.0;
  const int64_t st = int64_t(gridDim.x) * VB;
  int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x;
  for (; i + st < n; i += 2 * st) {
    a0 += v[i] * w[i];
    a1 += v[i + st] * w[i + st];
  }
  if (i < n) a0 += v[i] * w[i];
  double s = block_sum(a0 + a1, sh);
  if (threadIdx.x == 0) partial[int64_t(j) * RED_BLOCKS + blockIdx.x] = s;
}

__global__ void k_dots_final(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  __shared__ double sh[VB];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += VB) acc += partial[int64_t(j) * RED_BLOCKS + i];
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = s;
}

int64_t reduce_scratch_size() { return int64_t(MAXV) * RED_BLOCKS + MAXV; }

static unsigned red_grid(int64_t n) {
  int64_t g = (n + VB * 8 - 1) / (VB * 8);
  if (g < 1) g = 1;
  if (g > RED_BLOCKS) g = RED_BLOCKS;
  return unsigned(g);
}

void vdots_into(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* out, double* scratch,
                hipStream_t s) {
  if (k <= 0) return;
  unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_dots_partial, dim3(g, unsigned(k)), dim3(VB), 0, s, V, ldv, w, n, scratch);
  hipLaunchKernelGGL(k_dots_final, dim3(unsigned(k)), dim3(VB), 0, s, scratch, int(g), out);
}


void vdots(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* out_dev,
           hipStream_t s) {
  // out_dev must have room for MAXV results followed by the k * RED_BLOCKS partials
  if (k <= 0) return;
  double* partial = out_dev + MAXV;
  unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_dots_partial, dim3(g, unsigned(k)), dim3(VB), 0, s, V, ldv, w, n, partial);
  hipLaunchKernelGGL(k_dots_final, dim3(unsigned(k)), dim3(VB), 0, s, partial, int(g), out_dev);
}

double vdot(const double* x, const double* y, int64_t n, double* scratch_dev, hipStream_t s) {
  vdots(x, 0, 1, y, n, scratch_dev, s);
  double h = 0.0;
  DGNP_HIP(hipMemcpyAsync(&h, scratch_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  DGNP_HIP(hipStreamSynchronize(s));
  return h;
}

double vnorm2(const double* x, int64_t n, double* scratch_dev, hipStream_t s) {
  double d = vdot(x, x, n, scratch_dev, s);
  return std::isnan(d) ? d : (d > 0.0 ? sqrt(d) : 0.0);  // a NaN entry must not read as a zero norm
}

// partial[blk] = sum over the block's chunk of x^2 (accumulated in double)
__global__ void k_sq_partial(const float* __restrict__ x, int64_t n, double* __restrict__ partial) {
  __shared__ double sh[VB];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    const double v = double(x[i]);
    acc += v * v;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void vsq_into(const float* x, int64_t n, double* out, double* scratch, hipStream_t s) {
  unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_sq_partial, dim3(g), dim3(VB), 0, s, x, n, scratch);
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(VB), 0, s, scratch, int(g), out);
}

// x /= sqrt(*ss) with *ss read on the device (x unchanged when *ss <= 0)
template <typename T>
__global__ void k_scale_rsqrt_inplace(const double* __restrict__ ss, T* __restrict__ x, int64_t n) {
  const double q = *ss;
  if (!(q > 0.0)) return;
  const double a = 1.0 / sqrt(q);
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB)
    x[i] = T(a * double(x[i]));
}
template <typename T>
void vscale_rsqrt_inplace(const double* ss_dev, T* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_rsqrt_inplace<T>, dim3(grid_for(n)), dim3(VB), 0, s, ss_dev, x, n);
}
template void vscale_rsqrt_inplace<double>(const double*, double*, int64_t, hipStream_t);
template void vscale_rsqrt_inplace<float>(const double*, float*, int64_t, hipStream_t);

double vnorm2(const float* x, int64_t n, double* scratch_dev, hipStream_t s) {
  double* partial = scratch_dev + MAXV;
  unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_sq_partial, dim3(g), dim3(VB), 0, s, x, n, partial);
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(VB), 0, s, partial, int(g), scratch_dev);
  double h = 0.0;
  DGNP_HIP(hipMemcpyAsync(&h, scratch_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  DGNP_HIP(hipStreamSynchronize(s));
  return std::isnan(h) ? h : (h > 0.0 ? sqrt(h) : 0.0);
}

// ---- delayed classical Gram-Schmidt (reorthogonalisation one step late) -------
// Step j of the Arnoldi process works on u, the new direction after one
// projection pass (scaled to about unit length), and w = Op z with z = P u.
// One reduction gives s = V_{<j}^T u, sigma = u.u, c = V_{<j}^T w, tau = u.w and
// w.w; then v_j = (u - V s) / alpha with alpha = sqrt(sigma - s.s), and the
// first projection of w against V_{<j} and v_j leaves the next direction.
// Coefficient block (device, contiguous): [s | sigma] at 0, [c | tau] at MAXV,
// then w.w, alpha, h_jj, 1/alpha, rho, 1/rho at 2 MAXV + 0..5.
static constexpr int DC_WW = 2 * MAXV, DC_ALPHA = 2 * MAXV + 1, DC_HJJ = 2 * MAXV + 2, DC_IALPHA = 2 * MAXV + 3,
                     DC_RHO = 2 * MAXV + 4, DC_IRHO = 2 * MAXV + 5, DC_FLAG = DCGS_FLAG;
// block partials: rows 0 .. 2 MAXV of RED_BLOCKS each, then the completion
// counter of the final reduction (zero between reductions)
static constexpr int64_t DC_COUNT = int64_t(2 * MAXV + 1) * RED_BLOCKS;

// partial[r][y][blk], r = 0: L_y . u, r = 1: L_y . w, row 2 MAXV: w . w
// (y = j only); L_y = V_y for y < j, L_j = u.  For single-precision w the
// block row y = j also stores w widened to double in w64 (if not null).
template <typename TW>
__global__ void k_dcgs_dots(const double* __restrict__ V, int64_t ldv, int j, const double* __restrict__ u,
                            const TW* __restrict__ w, double* __restrict__ w64, int64_t n,
                            double* __restrict__ partial) {
  __shared__ double sh[VB];
  const int y = blockIdx.y;
  const bool last = y == j;
  const double* L = last ? u : V + int64_t(y) * ldv;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    const double l = L[i];
    a0 += l * u[i];
    if (w) {
      const double wi = double(w[i]);
      a1 += l * wi;
      if (last) {
        a2 += wi * wi;
        if (w64) w64[i] = wi;
      }
    }
  }
  const double s0 = block_sum(a0, sh);
  __syncthreads();
  if (threadIdx.x == 0) partial[int64_t(y) * RED_BLOCKS + blockIdx.x] = s0;
  if (w) {
    const double s1 = block_sum(a1, sh);
    __syncthreads();
    if (threadIdx.x == 0) partial[int64_t(MAXV + y) * RED_BLOCKS + blockIdx.x] = s1;
    if (last) {
      const double s2 = block_sum(a2, sh);
      if (threadIdx.x == 0) partial[int64_t(2 * MAXV) * RED_BLOCKS + blockIdx.x] = s2;
    }
  }
}

// alpha, h_jj, rho and their reciprocals from the reduced dot products (run
// by one whole block); with hout (host memory mapped for the device), the
// entries the host reads are stored there as well: s_0..s_j, c_0..c_j, w.w and
// the scalars (h_jj = 0, rho = 1 without w)
__device__ void dcgs_scalars_block(double* __restrict__ out, int j, int with_w, double* __restrict__ hout,
                                   double* sh, unsigned long long seq) {
  double ss = 0.0, sc = 0.0, cc = 0.0;
  for (int k = threadIdx.x; k < j; k += VB) {
    const double sk = out[k];
    ss += sk * sk;
    if (with_w) {
      const double ck = out[MAXV + k];
      sc += sk * ck;
      cc += ck * ck;
    }
  }
  ss = block_sum(ss, sh);
  __syncthreads();
  sc = block_sum(sc, sh);
  __syncthreads();
  cc = block_sum(cc, sh);
  if (hout) {
    for (int k = threadIdx.x; k <= j; k += VB) {
      hout[k] = out[k];
      if (with_w) hout[MAXV + k] = out[MAXV + k];
    }
  }
  if (threadIdx.x == 0) {
    const double a2 = out[j] - ss;
    const double alpha = __builtin_isnan(a2) ? a2 : (a2 > 0.0 ? sqrt(a2) : 0.0);  // NaN reaches the host check
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    out[DC_ALPHA] = alpha;
    out[DC_IALPHA] = ia;
    double hjj = 0.0, rho = 1.0;
    if (with_w) {
      hjj = (out[MAXV + j] - sc) * ia;
      const double ww = out[DC_WW];
      const double r2 = ww - cc - hjj * hjj;  // |w - V c - v_j h_jj|^2 by Pythagoras: only a scale
      rho = r2 > 0.0 ? sqrt(r2) : sqrt(ww);
      if (!(rho > 0.0)) rho = 1.0;
      out[DC_HJJ] = hjj;
      out[DC_RHO] = rho;
      out[DC_IRHO] = 1.0 / rho;
    }
    if (hout) {
      hout[DC_WW] = with_w ? out[DC_WW] : 0.0;
      hout[DC_ALPHA] = alpha;
      hout[DC_IALPHA] = ia;
      hout[DC_HJJ] = hjj;
      hout[DC_RHO] = rho;
      hout[DC_IRHO] = 1.0 / rho;
    }
  }
  if (!hout) return;
  // the sequence number goes last: every entry above is visible to the host
  // before it (system-scope release after the block's stores)
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(hout + DC_FLAG), seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// out[row] = sum of the row's block partials for the rows 0..j, MAXV..MAXV+j
// and 2 MAXV (the last two groups only with w), one block per row; the block
// that finishes last (device-wide counter, reset by that block for the next
// reduction) then forms the scalars
__global__ void k_dcgs_final(const double* __restrict__ partial, int nblk, int j, int with_w,
                             double* __restrict__ out, double* __restrict__ hout, unsigned* __restrict__ count,
                             unsigned long long seq) {
  __shared__ double sh[VB];
  __shared__ int s_last;
  const int o = blockIdx.x;
  const int row = o <= j ? o : (o <= 2 * j + 1 ? MAXV + (o - j - 1) : 2 * MAXV);
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += VB) acc += partial[int64_t(row) * RED_BLOCKS + i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    out[row] = t;
    __threadfence();  // the sum is visible device-wide before the count says so
    s_last = atomicAdd(count, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();  // every other block's sum is visible to this block
  if (threadIdx.x == 0) *count = 0u;
  dcgs_scalars_block(out, j, with_w, hout, sh, seq);
}

// v_j = (u - V s) / alpha into V column j; u <- (w - V c - v_j h_jj) / rho and
// its copy m = (TM) u (the next preconditioner input).  V is read once.
template <typename TM>
__global__ void k_dcgs_update(double* __restrict__ V, int64_t ldv, int j, const double* __restrict__ coef,
                              double* __restrict__ u, const double* __restrict__ w, TM* __restrict__ m,
                              const TM* __restrict__ zs, TM* __restrict__ zd, int64_t n) {
  const double ia = coef[DC_IALPHA], hjj = coef[DC_HJJ], irho = coef[DC_IRHO];
  const double* sv = coef;
  const double* cv = coef + MAXV;
  double* vj = V + int64_t(j) * ldv;
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double as0 = 0.0, as1 = 0.0, ac0 = 0.0, ac1 = 0.0;
    int k = 0;
    for (; k + 2 <= j; k += 2) {
      const double x0 = V[int64_t(k) * ldv + i], x1 = V[int64_t(k + 1) * ldv + i];
      as0 += sv[k] * x0;
      ac0 += cv[k] * x0;
      as1 += sv[k + 1] * x1;
      ac1 += cv[k + 1] * x1;
    }
    if (k < j) {
      const double x0 = V[int64_t(k) * ldv + i];
      as0 += sv[k] * x0;
      ac0 += cv[k] * x0;
    }
    const double v = (u[i] - (as0 + as1)) * ia;
    vj[i] = v;
    const double un = (w[i] - (ac0 + ac1) - v * hjj) * irho;
    u[i] = un;
    m[i] = TM(un);
    if (zd) zd[i] = zs[i];
  }
}

void dcgs_reduce(const double* V, int64_t ldv, int j, const double* u, const void* w, bool w_f32, double* w64,
                 int64_t n, double* partial, double* coef, hipStream_t s, double* hout, unsigned long long seq) {
  const unsigned g = red_grid(n);
  const dim3 grid(g, unsigned(j + 1));
  if (!w)
    hipLaunchKernelGGL(k_dcgs_dots<double>, grid, dim3(VB), 0, s, V, ldv, j, u, static_cast<const double*>(nullptr),
                       static_cast<double*>(nullptr), n, partial);
  else if (w_f32)
    hipLaunchKernelGGL(k_dcgs_dots<float>, grid, dim3(VB), 0, s, V, ldv, j, u, static_cast<const float*>(w), w64, n,
                       partial);
  else
    hipLaunchKernelGGL(k_dcgs_dots<double>, grid, dim3(VB), 0, s, V, ldv, j, u, static_cast<const double*>(w),
                       static_cast<double*>(nullptr), n, partial);
  const unsigned nout = w ? unsigned(2 * j + 3) : unsigned(j + 1);
  hipLaunchKernelGGL(k_dcgs_final, dim3(nout), dim3(VB), 0, s, partial, int(g), j, w ? 1 : 0, coef, hout,
                     reinterpret_cast<unsigned*>(partial + DC_COUNT), seq);
}

template <typename TM>
void dcgs_update(double* V, int64_t ldv, int j, const double* coef, double* u, const double* w, TM* m,
                 const TM* zs, TM* zd, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_dcgs_update<TM>, dim3(grid_for(n)), dim3(VB), 0, s, V, ldv, j, coef, u, w, m, zs, zd, n);
}
template void dcgs_update<double>(double*, int64_t, int, const double*, double*, const double*, double*,
                                  const double*, double*, int64_t, hipStream_t);
template void dcgs_update<float>(double*, int64_t, int, const double*, double*, const double*, float*,
                                 const float*, float*, int64_t, hipStream_t);
int64_t dcgs_partial_size() { return DC_COUNT + 8; }

template <typename T>
__global__ void k_combine(const T* __restrict__ Z, int64_t ldz, int k, const double* __restrict__ h,
                          double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(VB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double a0 = y[i], a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      a0 += h[j] * double(Z[j * ldz + i]);
      a1 += h[j + 1] * double(Z[(j + 1) * ldz + i]);
      a2 += h[j + 2] * double(Z[(j + 2) * ldz + i]);
      a3 += h[j + 3] * double(Z[(j + 3) * ldz + i]);
    }
    for (; j < k; ++j) a0 += h[j] * double(Z[j * ldz + i]);
    y[i] = (a0 + a1) + (a2 + a3);
  }
}

template <typename T>
void vcombine(const T* Z, int64_t ldz, int k, const double* h_dev, double* y, int64_t n, hipStream_t s) {
  if (k <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_combine<T>, dim3(grid_for(n)), dim3(VB), 0, s, Z, ldz, k, h_dev, y, n);
}
template void vcombine<double>(const double*, int64_t, int, const double*, double*, int64_t, hipStream_t);
template void vcombine<float>(const float*, int64_t, int, const double*, double*, int64_t, hipStream_t);

}  // namespace dgnp
