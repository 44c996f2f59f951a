// Geometric multigrid on the concentration blocks (Sec. 4.1: an h-multigrid
// preconditioner for A_{c_k c_k} whose smoother is the block ILU(0) and whose
// coarsest grid is solved directly).  The levels are the structured box
// coarsened by 2 along every axis; the coarse space of each level (degree-p
// polynomials on every coarse element) lies inside the next finer one, and the
// prolongation P evaluates a coarse element's polynomial at the nodes of its
// 2^d children: on child c it is the nb x nb matrix Pi_c, the tensor product of
// the 1-D Lagrange interpolants of the coarse nodes at the child's nodes.
// Coarse operators are Galerkin products R A P with R = P^T, which keep the
// 2d+1 block pattern of the element graph.
//
// Kernels: the Galerkin product (double), restriction and prolongation, and
// the level residual b - A x or b - A^T x on the unfactored blocks.  The ILU(0)
// factorisation and sweeps of the coarse levels and the coarsest dense solve
// reuse the kernels of the fine level (kernels_block.hip).
//
// Child numbering: bit a of c is set for the upper half of the parent along
// axis a; the fine element of child c of coarse element (X, Y, Z) is
// (2X + bit0, 2Y + bit1, 2Z + bit2) in the lexicographic order of the fine grid.
#include "kernels_gmg.hpp"

namespace dgnp {

namespace {
constexpr int GT = 256;

struct Dims {
  int x, y, z;  // fine element counts per axis (z = 1 in 2-D)
};

__device__ __forceinline__ int64_t fine_child(const Dims& f, int64_t ec, int c) {
  const int cx = f.x / 2, cy = f.y / 2;
  const int64_t X = ec % cx, Y = (ec / cx) % cy, Z = ec / (int64_t(cx) * cy);
  return (2 * X + (c & 1)) + int64_t(f.x) * ((2 * Y + ((c >> 1) & 1)) + int64_t(f.y) * (2 * Z + ((c >> 2) & 1)));
}

// parent and child index of fine element e
__device__ __forceinline__ int64_t parent_of(const Dims& f, int64_t e, int* child) {
  const int64_t x = e % f.x, y = (e / f.x) % f.y, z = e / (int64_t(f.x) * f.y);
  *child = int(x & 1) | int(y & 1) << 1 | int(z & 1) << 2;
  return (x >> 1) + int64_t(f.x / 2) * ((y >> 1) + int64_t(f.y / 2) * (z >> 1));
}
}  // namespace

// Galerkin product: coarse block (Ec, slot s) = sum of Pi_c^T A_{e,t} Pi_c' over
// the fine blocks (child e = child c of Ec, its slot t) whose column element
// (child c' of Ec, or of Ec's neighbour in slot s) maps to it: for s = 0 the
// 2^d diagonal blocks and the 2^d d couplings between children, for a face
// slot the 2^(d-1) couplings across that face.  One work-group per (coarse
// element, field, coarse slot); the products run one after the other through
// LDS, the next fine block loaded into registers while the current one is
// multiplied, and each thread accumulates fixed entries of the coarse block
// in registers.  The child prolongations sit in LDS when they fit (n_b <= 27).
template <int NB, int DIM>
__global__ void __launch_bounds__(GT) k_gmg_galerkin(const double* __restrict__ Af, int64_t fsf,
                                                     const int* __restrict__ nbr, Dims fd,
                                                     const double* __restrict__ Pi, double* __restrict__ Ac,
                                                     int64_t fsc) {
  constexpr int NS = 2 * DIM + 1, NC = 1 << DIM, BB = NB * NB, PER = (BB + GT - 1) / GT;
  constexpr bool PI_LDS = NB <= 27;
  constexpr int MAXC = NC * (DIM + 1);  // contributions of the diagonal slot
  const int64_t ec = blockIdx.x;
  const int s = blockIdx.z, tid = threadIdx.x;
  Af += blockIdx.y * fsf;
  Ac += blockIdx.y * fsc;
  __shared__ double sA[BB], sT[BB];
  __shared__ double sPi[PI_LDS ? NC * BB : 1];
  if constexpr (PI_LDS)
    for (int i = tid; i < NC * BB; i += GT) sPi[i] = Pi[i];
  const double* PiS = PI_LDS ? sPi : Pi;
  // the contributions (child, fine slot, column child), listed by one thread
  __shared__ int64_t ce[MAXC];
  __shared__ int ct[MAXC], cc[MAXC], ccp[MAXC];
  __shared__ int s_n;
  if (tid == 0) {
    int n = 0;
    for (int c = 0; c < NC; ++c) {
      const int64_t e = fine_child(fd, ec, c);
      for (int t = 0; t < NS; ++t) {
        int cp = c;
        if (t == 0) {
          if (s != 0) continue;
        } else {
          const int a = (t - 1) >> 1, up = (t - 1) & 1;
          // a lower child going up, or an upper child going down, stays inside
          // the coarse element; otherwise the neighbour is in coarse slot t
          const bool inside = ((c >> a) & 1) != up;
          if (inside ? s != 0 : s != t) continue;
          if (nbr[e * 2 * DIM + t - 1] < 0) continue;
          cp = c ^ (1 << a);
        }
        ce[n] = e;
        ct[n] = t;
        cc[n] = c;
        ccp[n] = cp;
        ++n;
      }
    }
    s_n = n;
  }
  __syncthreads();
  const int n = s_n;
  double acc[PER], pre[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    acc[q] = 0.0;
    const int i = tid + q * GT;
    pre[q] = (n > 0 && i < BB) ? Af[(ce[0] * NS + ct[0]) * BB + i] : 0.0;
  }
  for (int k = 0; k < n; ++k) {
    __syncthreads();  // the previous product has finished reading sA / sT
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * GT;
      if (i < BB) sA[i] = pre[q];
    }
    __syncthreads();
    if (k + 1 < n) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = tid + q * GT;
        if (i < BB) pre[q] = Af[(ce[k + 1] * NS + ct[k + 1]) * BB + i];
      }
    }
    const double* Pc = PiS + ccp[k] * BB;  // A_{e,t} Pi_c'
    for (int i = tid; i < BB; i += GT) {
      const int r = i / NB, col = i % NB;
      double v = 0.0;
#pragma unroll 9
      for (int j = 0; j < NB; ++j) v += sA[r * NB + j] * Pc[j * NB + col];
      sT[i] = v;
    }
    __syncthreads();
    const double* Pr = PiS + cc[k] * BB;  // Pi_c^T (A Pi_c')
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * GT;
      if (i < BB) {
        const int r = i / NB, col = i % NB;
        double v = 0.0;
#pragma unroll 9
        for (int j = 0; j < NB; ++j) v += Pr[j * NB + r] * sT[j * NB + col];
        acc[q] += v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = tid + q * GT;
    if (i < BB) Ac[(ec * NS + s) * BB + i] = acc[q];
  }
}

// The same Galerkin product for blocks of 17..32 rows on the FP64 matrix
// cores: both products of a contribution, T = A_{e,t} Pi_c' and then
// Pi_c^T T, are padded to 32 x 32 and split into four 16 x 16 tiles, one per
// wave (v_mfma_f64_16x16x4f64, the k loop in steps of four with entries past
// NB read as zero).  Lane l of wave w holds A operand rows 16 (w >> 1) + l % 16
// and B operand columns 16 (w & 1) + l % 16 at k = 4 s + l / 16; the four
// accumulator entries of a lane are rows 16 (w >> 1) + 4 q + l / 16 of column
// 16 (w & 1) + l % 16.  The fine block of the next contribution is read into
// registers while the current one is multiplied; T passes through LDS; the
// coarse block accumulates in the tiles' registers.
typedef double gv4d __attribute__((ext_vector_type(4)));
template <int NB, int DIM>
__global__ void __launch_bounds__(GT) k_gmg_galerkin_mf(const double* __restrict__ Af, int64_t fsf,
                                                        const int* __restrict__ nbr, Dims fd,
                                                        const double* __restrict__ Pi, double* __restrict__ Ac,
                                                        int64_t fsc) {
  static_assert(NB > 16 && NB <= 32, "32 x 32 padded tiles");
  constexpr int NS = 2 * DIM + 1, NC = 1 << DIM, BB = NB * NB, KS = (NB + 3) / 4;
  constexpr int MAXC = NC * (DIM + 1);
  const int64_t ec = blockIdx.x;
  const int s = blockIdx.z, tid = threadIdx.x;
  Af += blockIdx.y * fsf;
  Ac += blockIdx.y * fsc;
  __shared__ double sPi[NC * BB], sT[BB];
  for (int i = tid; i < NC * BB; i += GT) sPi[i] = Pi[i];
  __shared__ int64_t ce[MAXC];
  __shared__ int ct[MAXC], cc[MAXC], ccp[MAXC];
  __shared__ int s_n;
  if (tid == 0) {
    int n = 0;
    for (int c = 0; c < NC; ++c) {
      const int64_t e = fine_child(fd, ec, c);
      for (int t = 0; t < NS; ++t) {
        int cp = c;
        if (t == 0) {
          if (s != 0) continue;
        } else {
          const int a = (t - 1) >> 1, up = (t - 1) & 1;
          const bool inside = ((c >> a) & 1) != up;
          if (inside ? s != 0 : s != t) continue;
          if (nbr[e * 2 * DIM + t - 1] < 0) continue;
          cp = c ^ (1 << a);
        }
        ce[n] = e;
        ct[n] = t;
        cc[n] = c;
        ccp[n] = cp;
        ++n;
      }
    }
    s_n = n;
  }
  __syncthreads();
  const int n = s_n;
  const int l = tid & 63, w = tid >> 6, lk = l >> 4;
  const int ia = 16 * (w >> 1) + (l & 15), jb = 16 * (w & 1) + (l & 15);
  auto load_a = [&](int k, double (&dst)[KS]) {
    const double* A = Af + (ce[k] * NS + ct[k]) * BB;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = 4 * q + lk;
      dst[q] = (ia < NB && kk < NB) ? A[ia * NB + kk] : 0.0;
    }
  };
  double xa[KS], na[KS];
  if (n > 0) load_a(0, xa);
  gv4d accC = gv4d{0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < n; ++k) {
    if (k + 1 < n) load_a(k + 1, na);
    const double* Pc = sPi + ccp[k] * BB;
    gv4d accT = gv4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = 4 * q + lk;
      const double b = (jb < NB && kk < NB) ? Pc[kk * NB + jb] : 0.0;
      accT = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[q], b, accT, 0, 0, 0);
    }
    __syncthreads();  // the previous contribution has finished reading sT
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = 16 * (w >> 1) + 4 * q + lk, col = jb;
      if (rr < NB && col < NB) sT[rr * NB + col] = accT[q];
    }
    __syncthreads();
    const double* Pr = sPi + cc[k] * BB;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = 4 * q + lk;
      const double a = (ia < NB && kk < NB) ? Pr[kk * NB + ia] : 0.0;
      const double b = (jb < NB && kk < NB) ? sT[kk * NB + jb] : 0.0;
      accC = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, accC, 0, 0, 0);
    }
    if (k + 1 < n) {
#pragma unroll
      for (int q = 0; q < KS; ++q) xa[q] = na[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rr = 16 * (w >> 1) + 4 * q + lk, col = jb;
    if (rr < NB && col < NB) Ac[(ec * NS + s) * BB + rr * NB + col] = accC[q];
  }
}

// rc = P^T r: one thread per (coarse entry, field)
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(GT) k_gmg_restrict(const T* __restrict__ Pi, Dims fd, const T* __restrict__ r,
                                                     int64_t nff, T* __restrict__ rc, int64_t nfc) {
  constexpr int NC = 1 << DIM, BB = NB * NB;
  const int64_t g = blockIdx.x * int64_t(GT) + threadIdx.x;
  if (g >= nfc) return;
  const int i = int(g % NB);
  const int64_t ec = g / NB;
  r += blockIdx.y * nff;
  rc += blockIdx.y * nfc;
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const T* rf = r + fine_child(fd, ec, c) * NB;
    const T* P = Pi + c * BB + i;
#pragma unroll 8
    for (int k = 0; k < NB; ++k) acc += P[k * NB] * rf[k];
  }
  rc[g] = acc;
}

// x += P xc: one thread per (fine entry, field)
template <typename T, int NB>
__global__ void __launch_bounds__(GT) k_gmg_prolong(const T* __restrict__ Pi, Dims fd, const T* __restrict__ xc,
                                                    int64_t nfc, T* __restrict__ x, int64_t nff) {
  const int64_t g = blockIdx.x * int64_t(GT) + threadIdx.x;
  if (g >= nff) return;
  const int k = int(g % NB);
  int c = 0;
  const int64_t ec = parent_of(fd, g / NB, &c);
  xc += blockIdx.y * nfc + ec * NB;
  x += blockIdx.y * nff;
  const T* P = Pi + (c * NB + k) * NB;
  T acc = T(0);
#pragma unroll 8
  for (int i = 0; i < NB; ++i) acc += P[i] * xc[i];
  x[g] += acc;
}

// r = b - A x (TR = false) or b - A^T x (TR = true) on a level's unfactored
// blocks [field][E][slot][NB][ld] (rows of ld >= NB entries): one thread per
// (entry, field)
template <typename T, int NB, int DIM, bool TR>
__global__ void __launch_bounds__(GT) k_gmg_resid(const T* __restrict__ blk, int64_t fs, int ld,
                                                  const int* __restrict__ nbr, int64_t E, const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ r, int64_t nf) {
  constexpr int NS = 2 * DIM + 1;
  const int BB = NB * ld;
  const int64_t g = blockIdx.x * int64_t(GT) + threadIdx.x;
  if (g >= nf) return;
  const int row = int(g % NB);
  const int64_t e = g / NB;
  blk += blockIdx.y * fs;
  x += blockIdx.y * nf;
  b += blockIdx.y * nf;
  r += blockIdx.y * nf;
  T acc = T(0);
  for (int t = 0; t < NS; ++t) {
    const int64_t j = t == 0 ? e : int64_t(nbr[e * 2 * DIM + t - 1]);
    if (j < 0) continue;
    const T* xj = x + j * NB;
    if constexpr (!TR) {
      const T* a = blk + (e * NS + t) * BB + row * ld;
#pragma unroll 8
      for (int col = 0; col < NB; ++col) acc += a[col] * xj[col];
    } else {
      // block of row j that couples j to e: the opposite slot of t
      const int tj = t == 0 ? 0 : (((t - 1) ^ 1) + 1);
      const T* a = blk + (j * NS + tj) * BB + row;
#pragma unroll 8
      for (int col = 0; col < NB; ++col) acc += a[col * ld] * xj[col];
    }
  }
  r[g] = b[g] - acc;
}

// Dense matrix of one field of a block level (the coarsest): M[(i nb + r) n +
// j nb + q] = block (i, slot t) [r][q] with j the slot's neighbour; one thread
// per (block entry, field).  M must be zeroed before.
template <int NB, int DIM>
__global__ void __launch_bounds__(GT) k_gmg_densify(const double* __restrict__ blk, int64_t fs,
                                                    const int* __restrict__ nbr, int64_t E, double* __restrict__ M,
                                                    int n) {
  constexpr int NS = 2 * DIM + 1, BB = NB * NB;
  const int64_t g = blockIdx.x * int64_t(GT) + threadIdx.x;
  if (g >= E * NS * BB) return;
  const int rq = int(g % BB), t = int((g / BB) % NS);
  const int64_t i = g / (BB * NS);
  const int64_t j = t == 0 ? i : int64_t(nbr[i * 2 * DIM + t - 1]);
  if (j < 0) return;
  const int r = rq / NB, q = rq % NB;
  M[blockIdx.y * int64_t(n) * n + (i * NB + r) * n + j * NB + q] = blk[blockIdx.y * fs + g];
}

// In-place inverse of one dense n x n matrix per work-group (row-major) by
// Gauss-Jordan elimination with partial pivoting (ties to the lower row),
// then its transpose into MT.  When a pivot vanishes or is not finite, *err
// is set and both matrices are filled with NaN, so that the solve using them
// reports a non-finite vector.  n <= 1024; up to order 128 the elimination
// runs on a copy in LDS (each step is then bound by barriers, not by global
// memory round trips).
constexpr int DI = 1024;
constexpr int DI_LDS = 128;  // matrices up to this order are eliminated in LDS
template <bool SH>
__global__ void __launch_bounds__(DI) k_dense_inverse(double* __restrict__ Mg, double* __restrict__ MT, int n,
                                                      int* __restrict__ err) {
  Mg += blockIdx.x * int64_t(n) * n;
  MT += blockIdx.x * int64_t(n) * n;
  __shared__ double sM[SH ? DI_LDS * DI_LDS : 1];
  double* M = SH ? sM : Mg;
  if constexpr (SH) {
    for (int64_t idx = threadIdx.x; idx < int64_t(n) * n; idx += DI) sM[idx] = Mg[idx];
    __syncthreads();
  }
  __shared__ int perm[DI];
  __shared__ double colk[DI];
  __shared__ double rv[DI / 64];
  __shared__ int ri[DI / 64];
  __shared__ int s_piv, s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += DI) {
      const double v = fabs(M[int64_t(i) * n + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wave] = best;
      ri[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = rv[0];
      int p = ri[0];
      for (int w = 1; w < DI / 64; ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < p)) {
          b = rv[w];
          p = ri[w];
        }
      s_piv = p;
      s_bad = !(b > 0.0) || !isfinite(b);
      perm[k] = p;
    }
    __syncthreads();
    if (s_bad) {
      // a singular level: NaN everywhere, so the first use reports it
      for (int64_t idx = tid; idx < int64_t(n) * n; idx += DI) Mg[idx] = MT[idx] = __builtin_nan("");
      if (tid == 0) *err = 1;
      return;
    }
    const int p = s_piv;
    if (p != k)
      for (int j = tid; j < n; j += DI) {
        const double t = M[int64_t(k) * n + j];
        M[int64_t(k) * n + j] = M[int64_t(p) * n + j];
        M[int64_t(p) * n + j] = t;
      }
    __syncthreads();
    const double d = 1.0 / M[int64_t(k) * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += DI) M[int64_t(k) * n + j] = (j == k ? 1.0 : M[int64_t(k) * n + j]) * d;
    for (int i = tid; i < n; i += DI) colk[i] = i == k ? 0.0 : M[int64_t(i) * n + k];
    __syncthreads();
    for (int64_t idx = tid; idx < int64_t(n) * n; idx += DI) {
      const int i = int(idx / n), j = int(idx % n);
      const double f = colk[i];
      if (i == k || f == 0.0) continue;
      M[idx] = (j == k ? 0.0 : M[idx]) - f * M[int64_t(k) * n + j];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < n; i += DI) {
        const double t = M[int64_t(i) * n + k];
        M[int64_t(i) * n + k] = M[int64_t(i) * n + p];
        M[int64_t(i) * n + p] = t;
      }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < int64_t(n) * n; idx += DI) {
    MT[(idx % n) * n + idx / n] = M[idx];
    if constexpr (SH) Mg[idx] = M[idx];
  }
}

// ---------------------------------------------------------------------------
#define GMG_NB_SWITCH(nb, dim, CALL)                              \
  do {                                                            \
    if (dim == 3) {                                               \
      switch (nb) {                                               \
        case 8: { constexpr int NB_ = 8, D_ = 3; CALL; } break;   \
        case 27: { constexpr int NB_ = 27, D_ = 3; CALL; } break; \
        case 64: { constexpr int NB_ = 64, D_ = 3; CALL; } break; \
        default: throw Error(DGNP_E_ARG, "unsupported block size"); \
      }                                                           \
    } else {                                                      \
      switch (nb) {                                               \
        case 4: { constexpr int NB_ = 4, D_ = 2; CALL; } break;   \
        case 9: { constexpr int NB_ = 9, D_ = 2; CALL; } break;   \
        case 16: { constexpr int NB_ = 16, D_ = 2; CALL; } break; \
        default: throw Error(DGNP_E_ARG, "unsupported block size"); \
      }                                                           \
    }                                                             \
  } while (0)

static Dims dims_of(int dim, const int* n) { return Dims{n[0], n[1], dim == 3 ? n[2] : 1}; }

// 17..32-row blocks on the matrix cores, the others on the vector ALU
template <int NB, int DIM>
static void galerkin_t(dim3 g, const double* Af, int64_t fsf, const int* nbr, Dims fd, const double* Pi, double* Ac,
                       int64_t fsc, hipStream_t s) {
  if constexpr (NB > 16 && NB <= 32)
    hipLaunchKernelGGL((k_gmg_galerkin_mf<NB, DIM>), g, dim3(GT), 0, s, Af, fsf, nbr, fd, Pi, Ac, fsc);
  else
    hipLaunchKernelGGL((k_gmg_galerkin<NB, DIM>), g, dim3(GT), 0, s, Af, fsf, nbr, fd, Pi, Ac, fsc);
}

void launch_gmg_galerkin(int nb, int dim, int nfields, const double* Af, int64_t fsf, const int* nbr,
                         const int* nfine, const double* Pi, double* Ac, int64_t fsc, int64_t Ec, hipStream_t s) {
  if (Ec == 0 || nfields == 0) return;
  const Dims fd = dims_of(dim, nfine);
  const dim3 g = dim3(unsigned(Ec), unsigned(nfields), unsigned(2 * dim + 1));
  GMG_NB_SWITCH(nb, dim, (galerkin_t<NB_, D_>)(g, Af, fsf, nbr, fd, Pi, Ac, fsc, s));
  DGNP_HIP(hipGetLastError());
}

template <typename T>
void launch_gmg_restrict(int nb, int dim, int nfields, const T* Pi, const int* nfine, const T* r, int64_t nff,
                         T* rc, int64_t nfc, hipStream_t s) {
  if (nfc == 0 || nfields == 0) return;
  const Dims fd = dims_of(dim, nfine);
  const dim3 g = dim3(unsigned((nfc + GT - 1) / GT), unsigned(nfields));
  GMG_NB_SWITCH(nb, dim, hipLaunchKernelGGL((k_gmg_restrict<T, NB_, D_>), g, dim3(GT), 0, s, Pi, fd, r, nff, rc, nfc));
  DGNP_HIP(hipGetLastError());
}

template <typename T>
void launch_gmg_prolong(int nb, int dim, int nfields, const T* Pi, const int* nfine, const T* xc, int64_t nfc, T* x,
                        int64_t nff, hipStream_t s) {
  if (nff == 0 || nfields == 0) return;
  const Dims fd = dims_of(dim, nfine);
  const dim3 g = dim3(unsigned((nff + GT - 1) / GT), unsigned(nfields));
  GMG_NB_SWITCH(nb, dim, (void)D_; hipLaunchKernelGGL((k_gmg_prolong<T, NB_>), g, dim3(GT), 0, s, Pi, fd, xc, nfc, x, nff));
  DGNP_HIP(hipGetLastError());
}

template <typename T>
void launch_gmg_resid(int nb, int dim, int nfields, bool transpose, const T* blk, int64_t fs, int ld, const int* nbr,
                      int64_t E, const T* x, const T* b, T* r, hipStream_t s) {
  const int64_t nf = E * nb;
  if (nf == 0 || nfields == 0) return;
  const dim3 g = dim3(unsigned((nf + GT - 1) / GT), unsigned(nfields));
  if (transpose)
    GMG_NB_SWITCH(nb, dim, hipLaunchKernelGGL((k_gmg_resid<T, NB_, D_, true>), g, dim3(GT), 0, s, blk, fs, ld, nbr, E, x, b, r, nf));
  else
    GMG_NB_SWITCH(nb, dim, hipLaunchKernelGGL((k_gmg_resid<T, NB_, D_, false>), g, dim3(GT), 0, s, blk, fs, ld, nbr, E, x, b, r, nf));
  DGNP_HIP(hipGetLastError());
}

void launch_gmg_dense_inverse(int nb, int dim, int nfields, const double* blk, int64_t fs, const int* nbr,
                               int64_t E, double* M, double* MT, int* err, hipStream_t s) {
  const int n = int(E * nb);
  if (n == 0 || nfields == 0) return;
  DGNP_REQUIRE(n <= DI, DGNP_E_ARG, "dense inverse on the device: at most 1024 unknowns");
  DGNP_HIP(hipMemsetAsync(M, 0, size_t(nfields) * n * n * sizeof(double), s));
  const int NS = 2 * dim + 1;
  const int64_t cnt = E * NS * int64_t(nb) * nb;
  const dim3 g = dim3(unsigned((cnt + GT - 1) / GT), unsigned(nfields));
  GMG_NB_SWITCH(nb, dim, hipLaunchKernelGGL((k_gmg_densify<NB_, D_>), g, dim3(GT), 0, s, blk, fs, nbr, E, M, n));
  DGNP_HIP(hipGetLastError());
  if (n <= DI_LDS)
    hipLaunchKernelGGL(k_dense_inverse<true>, dim3(unsigned(nfields)), dim3(DI), 0, s, M, MT, n, err);
  else
    hipLaunchKernelGGL(k_dense_inverse<false>, dim3(unsigned(nfields)), dim3(DI), 0, s, M, MT, n, err);
  DGNP_HIP(hipGetLastError());
}

template void launch_gmg_restrict<double>(int, int, int, const double*, const int*, const double*, int64_t, double*,
                                          int64_t, hipStream_t);
template void launch_gmg_restrict<float>(int, int, int, const float*, const int*, const float*, int64_t, float*,
                                         int64_t, hipStream_t);
template void launch_gmg_prolong<double>(int, int, int, const double*, const int*, const double*, int64_t, double*,
                                         int64_t, hipStream_t);
template void launch_gmg_prolong<float>(int, int, int, const float*, const int*, const float*, int64_t, float*,
                                        int64_t, hipStream_t);
template void launch_gmg_resid<double>(int, int, int, bool, const double*, int64_t, int, const int*, int64_t,
                                       const double*, const double*, double*, hipStream_t);
template void launch_gmg_resid<float>(int, int, int, bool, const float*, int64_t, int, const int*, int64_t,
                                      const float*, const float*, float*, hipStream_t);

}  // namespace dgnp
