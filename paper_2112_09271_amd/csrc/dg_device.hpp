// Device helpers shared by the DG operator and block-assembly kernels:
// reference tables in constant memory (one copy per translation unit, filled
// by that unit's upload function), LDS table copies, sum-factorised
// interpolation / integration, face traces and face integration, velocity.
#pragma once

#include "dgnp_impl.hpp"
#include "pointwise.hpp"

namespace dgnp {

static __constant__ double c_tab[3][2 * 5 * 4 + 5 + 5 + 2 * 4];  // per p: B, Dq, wq, xq, Dend(-1), Dend(+1)
static __constant__ float c_tabf[3][2 * 5 * 4 + 5 + 5 + 2 * 4];   // float copy

static inline void upload_ref_tables_tu(const RefTables* tabs, int count) {
  double host[3][2 * 5 * 4 + 5 + 5 + 2 * 4] = {};
  for (int i = 0; i < count && i < 3; ++i) {
    const RefTables& t = tabs[i];
    const int nn = t.nn, nq = t.nq;
    double* d = host[t.p - 1];
    for (int q = 0; q < nq; ++q)
      for (int a = 0; a < nn; ++a) {
        d[q * nn + a] = t.B[q * nn + a];
        d[nq * nn + q * nn + a] = t.Dq[q * nn + a];
      }
    for (int q = 0; q < nq; ++q) {
      d[2 * nq * nn + q] = t.wq[q];
      d[2 * nq * nn + nq + q] = t.xq[q];
    }
    for (int a = 0; a < nn; ++a) {
      d[2 * nq * nn + 2 * nq + a] = t.Dend[0][a];
      d[2 * nq * nn + 2 * nq + nn + a] = t.Dend[1][a];
    }
  }
  DGNP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tab), host, sizeof(host)));
  float hostf[3][2 * 5 * 4 + 5 + 5 + 2 * 4];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2 * 5 * 4 + 5 + 5 + 2 * 4; ++j) hostf[i][j] = float(host[i][j]);
  DGNP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tabf), hostf, sizeof(hostf)));
}

#define DG_NT(D, P) (((D) == 3 && (P) == 3) ? 128 : 64)

template <int DIM, int P>
struct Sz {
  static constexpr int NN = P + 1, NQ = P + 2;
  static constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  static constexpr int NQV = DIM == 3 ? NQ * NQ * NQ : NQ * NQ;
  static constexpr int NFN = DIM == 3 ? NN * NN : NN;
  static constexpr int NQF = DIM == 3 ? NQ * NQ : NQ;
  static constexpr int NT = DG_NT(DIM, P);
};

// LDS copy of the 1-D tables
template <int P, typename T>
struct STab {
  static constexpr int NN = P + 1, NQ = P + 2;
  T B[NQ * NN], D[NQ * NN], W[NQ], X[NQ], De[2][NN];
};

template <int P, typename T>
__device__ inline void load_tab(STab<P, T>& t, int tid, int nt) {
  constexpr int NN = P + 1, NQ = P + 2;
  const double* c = c_tab[P - 1];
  for (int i = tid; i < NQ * NN; i += nt) {
    t.B[i] = T(c[i]);
    t.D[i] = T(c[NQ * NN + i]);
  }
  for (int i = tid; i < NQ; i += nt) {
    t.W[i] = T(c[2 * NQ * NN + i]);
    t.X[i] = T(c[2 * NQ * NN + NQ + i]);
  }
  for (int i = tid; i < 2 * NN; i += nt) t.De[i / NN][i % NN] = T(c[2 * NQ * NN + 2 * NQ + i]);
}

// Compile-time-indexed table access: with unrolled loops the offsets are
// constants, so the entries are scalar loads from constant memory (uniform
// across the wave) instead of per-lane LDS loads.
template <typename T, int P>
struct CT {
  static constexpr int NN = P + 1, NQ = P + 2;
  static __device__ __forceinline__ const T* base();
  static __device__ __forceinline__ T B(int q, int a) { return base()[q * NN + a]; }
  static __device__ __forceinline__ T D(int q, int a) { return base()[NQ * NN + q * NN + a]; }
  static __device__ __forceinline__ T De(int s, int a) { return base()[2 * NQ * NN + 2 * NQ + s * NN + a]; }
};
template <>
__device__ __forceinline__ const double* CT<double, 1>::base() { return c_tab[0]; }
template <>
__device__ __forceinline__ const double* CT<double, 2>::base() { return c_tab[1]; }
template <>
__device__ __forceinline__ const double* CT<double, 3>::base() { return c_tab[2]; }
template <>
__device__ __forceinline__ const float* CT<float, 1>::base() { return c_tabf[0]; }
template <>
__device__ __forceinline__ const float* CT<float, 2>::base() { return c_tabf[1]; }
template <>
__device__ __forceinline__ const float* CT<float, 3>::base() { return c_tabf[2]; }

// ---------------------------------------------------------------------------
// Line-per-thread sum factorisation (3-D): each thread contracts one complete
// 1-D line held in registers.  NA arrays (state, input) of MF fields each:
//   u[NA][MF][NB] -> q[NA][MF][DIM+1][NQV] (value, d/dx, d/dy, d/dz).
template <int P, int MF, int NA, int NT, typename T>
__device__ inline void interp_lines(const T* __restrict__ u, T* __restrict__ q, T* t1, T* t2, const T* ih,
                                    int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  constexpr int NB = NN * NN * NN, NQV = NQ * NQ * NQ;
  using C = CT<T, P>;
  // x lines: (arr, f, c, b)
  for (int ln = tid; ln < NA * MF * NN * NN; ln += NT) {
    const T* up = u + ln * NN;
    T x[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) x[a] = up[a];
    T* o = t1 + ln * 2 * NQ;  // [arr][f][c][b][2][NQ]
#pragma unroll
    for (int qx = 0; qx < NQ; ++qx) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int a = 0; a < NN; ++a) {
        s0 += C::B(qx, a) * x[a];
        s1 += C::D(qx, a) * x[a];
      }
      o[qx] = s0;
      o[NQ + qx] = s1;
    }
  }
  __syncthreads();
  // y lines: (arr, f, c, qx)
  for (int ln = tid; ln < NA * MF * NN * NQ; ln += NT) {
    const int qx = ln % NQ, afc = ln / NQ;  // afc = (arr, f, c)
    T v0[NN], v1[NN];
#pragma unroll
    for (int b = 0; b < NN; ++b) {
      v0[b] = t1[((afc * NN + b) * 2 + 0) * NQ + qx];
      v1[b] = t1[((afc * NN + b) * 2 + 1) * NQ + qx];
    }
    T* o = t2 + afc * 3 * NQ * NQ;  // [arr][f][c][3][qy][qx]
#pragma unroll
    for (int qy = 0; qy < NQ; ++qy) {
      T s00 = T(0), s01 = T(0), s10 = T(0);
#pragma unroll
      for (int b = 0; b < NN; ++b) {
        s00 += C::B(qy, b) * v0[b];
        s01 += C::D(qy, b) * v0[b];
        s10 += C::B(qy, b) * v1[b];
      }
      o[(0 * NQ + qy) * NQ + qx] = s00;
      o[(1 * NQ + qy) * NQ + qx] = s01;
      o[(2 * NQ + qy) * NQ + qx] = s10;
    }
  }
  __syncthreads();
  // z lines: (arr, f, qy, qx)
  for (int ln = tid; ln < NA * MF * NQ * NQ; ln += NT) {
    const int qxy = ln % (NQ * NQ), af = ln / (NQ * NQ);
    T w0[NN], w1[NN], w2[NN];
#pragma unroll
    for (int c = 0; c < NN; ++c) {
      const T* tp = t2 + (af * NN + c) * 3 * NQ * NQ + qxy;
      w0[c] = tp[0];
      w1[c] = tp[NQ * NQ];
      w2[c] = tp[2 * NQ * NQ];
    }
    T* o = q + af * 4 * NQV + qxy;  // [arr][f][4][NQV]
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      T v = T(0), gz = T(0), gy = T(0), gx = T(0);
#pragma unroll
      for (int c = 0; c < NN; ++c) {
        v += C::B(qz, c) * w0[c];
        gz += C::D(qz, c) * w0[c];
        gy += C::B(qz, c) * w1[c];
        gx += C::B(qz, c) * w2[c];
      }
      o[qz * NQ * NQ] = v;
      o[NQV + qz * NQ * NQ] = gx * ih[0];
      o[2 * NQV + qz * NQ * NQ] = gy * ih[1];
      o[3 * NQV + qz * NQ * NQ] = gz * ih[2];
    }
  }
  __syncthreads();
}

// Transposed line contractions (3-D): c[MF][4][NQV] -> o[MF][NB] (overwritten)
template <int P, int MF, int NT, typename T>
__device__ inline void integrate_lines(const T* __restrict__ c, T* __restrict__ o, T* t1, T* t2, int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  constexpr int NB = NN * NN * NN, NQV = NQ * NQ * NQ;
  using C = CT<T, P>;
  // z lines: (f, qy, qx)
  for (int ln = tid; ln < MF * NQ * NQ; ln += NT) {
    const int qxy = ln % (NQ * NQ), f = ln / (NQ * NQ);
    const T* cp = c + f * 4 * NQV + qxy;
    T cv[NQ], cx[NQ], cy[NQ], cz[NQ];
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      cv[qz] = cp[qz * NQ * NQ];
      cx[qz] = cp[NQV + qz * NQ * NQ];
      cy[qz] = cp[2 * NQV + qz * NQ * NQ];
      cz[qz] = cp[3 * NQV + qz * NQ * NQ];
    }
    T* op = t2 + f * NN * 3 * NQ * NQ + qxy;  // [f][c][3][qy][qx]
#pragma unroll
    for (int cc = 0; cc < NN; ++cc) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int qz = 0; qz < NQ; ++qz) {
        s0 += C::B(qz, cc) * cv[qz] + C::D(qz, cc) * cz[qz];
        s1 += C::B(qz, cc) * cy[qz];
        s2 += C::B(qz, cc) * cx[qz];
      }
      op[(cc * 3 + 0) * NQ * NQ] = s0;
      op[(cc * 3 + 1) * NQ * NQ] = s1;
      op[(cc * 3 + 2) * NQ * NQ] = s2;
    }
  }
  __syncthreads();
  // y lines: (f, c, qx)
  for (int ln = tid; ln < MF * NN * NQ; ln += NT) {
    const int qx = ln % NQ, fc = ln / NQ;  // fc = (f, c)
    const T* tp = t2 + fc * 3 * NQ * NQ + qx;
    T a0[NQ], a1[NQ], a2[NQ];
#pragma unroll
    for (int qy = 0; qy < NQ; ++qy) {
      a0[qy] = tp[qy * NQ];
      a1[qy] = tp[NQ * NQ + qy * NQ];
      a2[qy] = tp[2 * NQ * NQ + qy * NQ];
    }
    T* op = t1 + fc * NN * 2 * NQ + qx;  // [f][c][b][2][qx]
#pragma unroll
    for (int b = 0; b < NN; ++b) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) {
        s0 += C::B(qy, b) * a0[qy] + C::D(qy, b) * a1[qy];
        s1 += C::B(qy, b) * a2[qy];
      }
      op[(b * 2 + 0) * NQ] = s0;
      op[(b * 2 + 1) * NQ] = s1;
    }
  }
  __syncthreads();
  // x lines: (f, c, b)
  for (int ln = tid; ln < MF * NN * NN; ln += NT) {
    const T* tp = t1 + ln * 2 * NQ;
    T b0[NQ], b1[NQ];
#pragma unroll
    for (int qx = 0; qx < NQ; ++qx) {
      b0[qx] = tp[qx];
      b1[qx] = tp[NQ + qx];
    }
#pragma unroll
    for (int a = 0; a < NN; ++a) {
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) s += C::B(qx, a) * b0[qx] + C::D(qx, a) * b1[qx];
      o[ln * NN + a] = s;
    }
  }
  __syncthreads();
  (void)NB;
}

// ---------------------------------------------------------------------------
// sum-factorised interpolation: u[MF][NB] -> q[MF][DIM+1][NQV] (value, d/dx...)
template <int DIM, int P, int MF, int NT, typename T>
__device__ inline void interp(const T* __restrict__ u, T* __restrict__ q, T* t1, T* t2,
                              const STab<P, T>& tb, const T* ih, int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  if constexpr (DIM == 3) {
    constexpr int NB = NN * NN * NN, NQV = NQ * NQ * NQ;
    for (int i = tid; i < MF * NN * NN * NQ; i += NT) {
      const int qx = i % NQ, r = i / NQ, cb = r % (NN * NN), f = r / (NN * NN);
      const T* up = u + f * NB + cb * NN;
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int a = 0; a < NN; ++a) {
        s0 += tb.B[qx * NN + a] * up[a];
        s1 += tb.D[qx * NN + a] * up[a];
      }
      t1[((f * 2 + 0) * NN * NN + cb) * NQ + qx] = s0;
      t1[((f * 2 + 1) * NN * NN + cb) * NQ + qx] = s1;
    }
    __syncthreads();
    for (int i = tid; i < MF * NN * NQ * NQ; i += NT) {
      const int qx = i % NQ, qy = (i / NQ) % NQ, c = (i / (NQ * NQ)) % NN, f = i / (NQ * NQ * NN);
      T s00 = T(0), s01 = T(0), s10 = T(0);
#pragma unroll
      for (int b = 0; b < NN; ++b) {
        const T t0v = t1[((f * 2 + 0) * NN * NN + c * NN + b) * NQ + qx];
        const T t1v = t1[((f * 2 + 1) * NN * NN + c * NN + b) * NQ + qx];
        s00 += tb.B[qy * NN + b] * t0v;
        s01 += tb.D[qy * NN + b] * t0v;
        s10 += tb.B[qy * NN + b] * t1v;
      }
      const int o = (c * NQ + qy) * NQ + qx;
      t2[(f * 3 + 0) * NN * NQ * NQ + o] = s00;
      t2[(f * 3 + 1) * NN * NQ * NQ + o] = s01;
      t2[(f * 3 + 2) * NN * NQ * NQ + o] = s10;
    }
    __syncthreads();
    for (int i = tid; i < MF * NQV; i += NT) {
      const int qxy = i % (NQ * NQ), qz = (i / (NQ * NQ)) % NQ, f = i / NQV;
      T v = T(0), gz = T(0), gy = T(0), gx = T(0);
#pragma unroll
      for (int c = 0; c < NN; ++c) {
        const T a0 = t2[(f * 3 + 0) * NN * NQ * NQ + c * NQ * NQ + qxy];
        v += tb.B[qz * NN + c] * a0;
        gz += tb.D[qz * NN + c] * a0;
        gy += tb.B[qz * NN + c] * t2[(f * 3 + 1) * NN * NQ * NQ + c * NQ * NQ + qxy];
        gx += tb.B[qz * NN + c] * t2[(f * 3 + 2) * NN * NQ * NQ + c * NQ * NQ + qxy];
      }
      const int qi = qz * NQ * NQ + qxy;
      q[(f * 4 + 0) * NQV + qi] = v;
      q[(f * 4 + 1) * NQV + qi] = gx * ih[0];
      q[(f * 4 + 2) * NQV + qi] = gy * ih[1];
      q[(f * 4 + 3) * NQV + qi] = gz * ih[2];
    }
    __syncthreads();
  } else {
    constexpr int NB = NN * NN, NQV = NQ * NQ;
    for (int i = tid; i < MF * NN * NQ; i += NT) {
      const int qx = i % NQ, b = (i / NQ) % NN, f = i / (NQ * NN);
      const T* up = u + f * NB + b * NN;
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int a = 0; a < NN; ++a) {
        s0 += tb.B[qx * NN + a] * up[a];
        s1 += tb.D[qx * NN + a] * up[a];
      }
      t1[((f * 2 + 0) * NN + b) * NQ + qx] = s0;
      t1[((f * 2 + 1) * NN + b) * NQ + qx] = s1;
    }
    __syncthreads();
    for (int i = tid; i < MF * NQV; i += NT) {
      const int qx = i % NQ, qy = (i / NQ) % NQ, f = i / NQV;
      T v = T(0), gy = T(0), gx = T(0);
#pragma unroll
      for (int b = 0; b < NN; ++b) {
        const T t0v = t1[((f * 2 + 0) * NN + b) * NQ + qx];
        v += tb.B[qy * NN + b] * t0v;
        gy += tb.D[qy * NN + b] * t0v;
        gx += tb.B[qy * NN + b] * t1[((f * 2 + 1) * NN + b) * NQ + qx];
      }
      const int qi = qy * NQ + qx;
      q[(f * 3 + 0) * NQV + qi] = v;
      q[(f * 3 + 1) * NQV + qi] = gx * ih[0];
      q[(f * 3 + 2) * NQV + qi] = gy * ih[1];
    }
    __syncthreads();
  }
}

// transposed contraction: coefficients c[MF][DIM+1][NQV] (weights and chain-rule
// factors already applied) -> o[MF][NB] (overwritten)
template <int DIM, int P, int MF, int NT, typename T>
__device__ inline void integrate(const T* __restrict__ c, T* __restrict__ o, T* t1, T* t2,
                                 const STab<P, T>& tb, int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  if constexpr (DIM == 3) {
    constexpr int NB = NN * NN * NN, NQV = NQ * NQ * NQ;
    for (int i = tid; i < MF * NN * NQ * NQ; i += NT) {
      const int qxy = i % (NQ * NQ), cc = (i / (NQ * NQ)) % NN, f = i / (NQ * NQ * NN);
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int qz = 0; qz < NQ; ++qz) {
        const int qi = qz * NQ * NQ + qxy;
        s0 += tb.B[qz * NN + cc] * c[(f * 4 + 0) * NQV + qi] + tb.D[qz * NN + cc] * c[(f * 4 + 3) * NQV + qi];
        s1 += tb.B[qz * NN + cc] * c[(f * 4 + 2) * NQV + qi];
        s2 += tb.B[qz * NN + cc] * c[(f * 4 + 1) * NQV + qi];
      }
      const int o2 = cc * NQ * NQ + qxy;
      t2[(f * 3 + 0) * NN * NQ * NQ + o2] = s0;
      t2[(f * 3 + 1) * NN * NQ * NQ + o2] = s1;
      t2[(f * 3 + 2) * NN * NQ * NQ + o2] = s2;
    }
    __syncthreads();
    for (int i = tid; i < MF * NN * NN * NQ; i += NT) {
      const int qx = i % NQ, b = (i / NQ) % NN, cc = (i / (NQ * NN)) % NN, f = i / (NQ * NN * NN);
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) {
        const int o2 = (cc * NQ + qy) * NQ + qx;
        s0 += tb.B[qy * NN + b] * t2[(f * 3 + 0) * NN * NQ * NQ + o2] +
              tb.D[qy * NN + b] * t2[(f * 3 + 1) * NN * NQ * NQ + o2];
        s1 += tb.B[qy * NN + b] * t2[(f * 3 + 2) * NN * NQ * NQ + o2];
      }
      t1[((f * 2 + 0) * NN * NN + cc * NN + b) * NQ + qx] = s0;
      t1[((f * 2 + 1) * NN * NN + cc * NN + b) * NQ + qx] = s1;
    }
    __syncthreads();
    for (int i = tid; i < MF * NB; i += NT) {
      const int a = i % NN, cb = (i / NN) % (NN * NN), f = i / NB;
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx)
        s += tb.B[qx * NN + a] * t1[((f * 2 + 0) * NN * NN + cb) * NQ + qx] +
             tb.D[qx * NN + a] * t1[((f * 2 + 1) * NN * NN + cb) * NQ + qx];
      o[i] = s;
    }
    __syncthreads();
  } else {
    constexpr int NB = NN * NN, NQV = NQ * NQ;
    for (int i = tid; i < MF * NN * NQ; i += NT) {
      const int qx = i % NQ, b = (i / NQ) % NN, f = i / (NQ * NN);
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) {
        const int qi = qy * NQ + qx;
        s0 += tb.B[qy * NN + b] * c[(f * 3 + 0) * NQV + qi] + tb.D[qy * NN + b] * c[(f * 3 + 2) * NQV + qi];
        s1 += tb.B[qy * NN + b] * c[(f * 3 + 1) * NQV + qi];
      }
      t1[((f * 2 + 0) * NN + b) * NQ + qx] = s0;
      t1[((f * 2 + 1) * NN + b) * NQ + qx] = s1;
    }
    __syncthreads();
    for (int i = tid; i < MF * NB; i += NT) {
      const int a = i % NN, b = (i / NN) % NN, f = i / NB;
      T s = T(0);
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx)
        s += tb.B[qx * NN + a] * t1[((f * 2 + 0) * NN + b) * NQ + qx] +
             tb.D[qx * NN + a] * t1[((f * 2 + 1) * NN + b) * NQ + qx];
      o[i] = s;
    }
    __syncthreads();
  }
}

// node index of (normal coordinate l, tangential i, j) for a face of axis ax
template <int DIM, int NN>
__device__ inline int face_node(int ax, int l, int i, int j) {
  if constexpr (DIM == 3) {
    const int s1 = ax == 0 ? NN : 1;
    const int s2 = ax == 2 ? NN : NN * NN;
    const int sa = ax == 0 ? 1 : (ax == 1 ? NN : NN * NN);
    return l * sa + i * s1 + j * s2;
  } else {
    const int s1 = ax == 0 ? NN : 1;
    const int sa = ax == 0 ? 1 : NN;
    return l * sa + i * s1;
  }
}

// traces at the face Gauss points: out[MF][2][NQF] = (value, d/dx_ax)
template <int DIM, int P, int MF, int NT, typename T>
__device__ inline void trace(const T* __restrict__ u, int ax, int side, T* __restrict__ out, T* tn,
                             T* tm, const STab<P, T>& tb, T ihax, int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NFN = DIM == 3 ? NN * NN : NN;
  const int lend = side < 0 ? 0 : P;
  const T* De = tb.De[side < 0 ? 0 : 1];
  for (int idx = tid; idx < MF * NFN; idx += NT) {
    const int f = idx / NFN, ij = idx % NFN;
    const int i = ij % NN, j = ij / NN;
    const T* uf = u + f * NB;
    T dn = T(0);
#pragma unroll
    for (int l = 0; l < NN; ++l) dn += De[l] * uf[face_node<DIM, NN>(ax, l, i, j)];
    tn[(f * 2 + 0) * NFN + ij] = uf[face_node<DIM, NN>(ax, lend, i, j)];
    tn[(f * 2 + 1) * NFN + ij] = dn * ihax;
  }
  __syncthreads();
  if constexpr (DIM == 3) {
    for (int idx = tid; idx < MF * 2 * NN * NQ; idx += NT) {
      const int qi = idx % NQ, j = (idx / NQ) % NN, fc = idx / (NQ * NN);
      T s = T(0);
#pragma unroll
      for (int i = 0; i < NN; ++i) s += tb.B[qi * NN + i] * tn[fc * NFN + j * NN + i];
      tm[(fc * NN + j) * NQ + qi] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < MF * 2 * NQ * NQ; idx += NT) {
      const int qi = idx % NQ, qj = (idx / NQ) % NQ, fc = idx / (NQ * NQ);
      T s = T(0);
#pragma unroll
      for (int j = 0; j < NN; ++j) s += tb.B[qj * NN + j] * tm[(fc * NN + j) * NQ + qi];
      out[fc * NQ * NQ + qj * NQ + qi] = s;
    }
    __syncthreads();
  } else {
    for (int idx = tid; idx < MF * 2 * NQ; idx += NT) {
      const int qi = idx % NQ, fc = idx / NQ;
      T s = T(0);
#pragma unroll
      for (int i = 0; i < NN; ++i) s += tb.B[qi * NN + i] * tn[fc * NFN + i];
      out[fc * NQ + qi] = s;
    }
    __syncthreads();
  }
}

// o[MF][NB] += integral of cf[MF][2][NQF] against (value, dscale * d/dx_ax)
template <int DIM, int P, int MF, int NT, typename T>
__device__ inline void face_integrate(const T* __restrict__ cf, T* __restrict__ o, int ax, int side,
                                      T* tn, T* tm, const STab<P, T>& tb, T dscale, int tid) {
  constexpr int NN = P + 1, NQ = P + 2;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NFN = DIM == 3 ? NN * NN : NN;
  const int lend = side < 0 ? 0 : P;
  const T* De = tb.De[side < 0 ? 0 : 1];
  if constexpr (DIM == 3) {
    for (int idx = tid; idx < MF * 2 * NN * NQ; idx += NT) {
      const int qi = idx % NQ, j = (idx / NQ) % NN, fc = idx / (NQ * NN);
      T s = T(0);
#pragma unroll
      for (int qj = 0; qj < NQ; ++qj) s += tb.B[qj * NN + j] * cf[fc * NQ * NQ + qj * NQ + qi];
      tm[(fc * NN + j) * NQ + qi] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < MF * 2 * NFN; idx += NT) {
      const int i = idx % NN, j = (idx / NN) % NN, fc = idx / NFN;
      T s = T(0);
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) s += tb.B[qi * NN + i] * tm[(fc * NN + j) * NQ + qi];
      tn[fc * NFN + j * NN + i] = s;
    }
    __syncthreads();
  } else {
    for (int idx = tid; idx < MF * 2 * NFN; idx += NT) {
      const int i = idx % NN, fc = idx / NFN;
      T s = T(0);
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) s += tb.B[qi * NN + i] * cf[fc * NQ + qi];
      tn[fc * NFN + i] = s;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < MF * NB; idx += NT) {
    const int f = idx / NB, node = idx % NB;
    int cx = node % NN, cy = (node / NN) % NN, cz = node / (NN * NN);
    int l, i, j;
    if constexpr (DIM == 3) {
      l = ax == 0 ? cx : (ax == 1 ? cy : cz);
      i = ax == 0 ? cy : cx;
      j = ax == 2 ? cy : cz;
    } else {
      l = ax == 0 ? cx : cy;
      i = ax == 0 ? cy : cx;
      j = 0;
    }
    const int ij = j * NN + i;
    T add = dscale * De[l] * tn[(f * 2 + 1) * NFN + ij];
    if (l == lend) add += tn[(f * 2 + 0) * NFN + ij];
    o[idx] += add;
  }
  __syncthreads();
}

// physical constants of the pointwise fluxes in the arithmetic T
template <typename T, int MF>
__device__ inline Phys<T, MF> make_phys(const KArgs& A) {
  Phys<T, MF> ph;
  for (int k = 0; k < MF - 1; ++k) {
    ph.zD[k] = T(A.z[k] * A.D[k]);
    ph.D[k] = T(A.D[k]);
    ph.a[k] = T(A.a[k]);
    ph.b[k] = T(A.b[k]);
    ph.bv_dc[k] = T(A.bv_dc[k]);
  }
  ph.delta = T(A.delta);
  ph.bv_r = A.bv_r;
  ph.bv_z = T(A.bv_z);
  ph.bv_aa = T(A.bv_aa);
  ph.bv_ac = T(A.bv_ac);
  return ph;
}

// shape of the exchange current across the box in z (the parabola of Sec. 5.2
// with mean 1, or 1)
__device__ inline double j0_profile(const KArgs& A, double z) {
  if (A.bv_prof == 0) return 1.0;
  const double t = (z - A.bv_zc) / A.bv_zhalf;
  return 0.6 * (2.0 - t * t);
}

__device__ inline void velocity_hat(const KArgs& A, const double* x, int dim, double* uh) {
  uh[0] = uh[1] = uh[2] = 0.0;
  if (A.vel_kind == DGNP_VEL_VORTEX) {
    double sx, cx, sy, cy;
    sincospi(x[0], &sx, &cx);
    sincospi(x[1], &sy, &cy);
    uh[0] = sx * cy;
    uh[1] = -cx * sy;
  } else if (A.vel_kind == DGNP_VEL_POISEUILLE_X) {
    const double yy = x[1] - A.vel_ylo;
    uh[0] = 6.0 * yy * (A.vel_H - yy) / (A.vel_H * A.vel_H);
  } else {
    for (int i = 0; i < dim; ++i) uh[i] = A.vel_param[i];
  }
}

}  // namespace dgnp
