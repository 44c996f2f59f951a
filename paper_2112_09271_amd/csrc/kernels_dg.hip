// Matrix-free DG operator kernels for gfx950: residual (Eqs. NPDG / chargeDG),
// Jacobian apply, its exact transpose, d/dPe, objective gradient and
// lambda^T dR/d(boundary data).
//
// One work-group per element.  The element's nodal values are staged in LDS,
// values and gradients at the (p+2)^d Gauss points come from sum-factorised
// 1-D contractions (x, then y, then z), the pointwise fluxes of pointwise.hpp
// turn them into test coefficients, and the transposed contractions integrate
// them back.  The 2d faces of the element are then processed element-centric:
// traces (value and normal derivative) of the own and the neighbour element at
// the face Gauss points, the numerical flux, and integration into the own
// element only.  Each face flux is therefore evaluated by both of its
// elements, but every output entry has exactly one writer: no atomics, and
// results are bitwise reproducible.
#include "dgnp_impl.hpp"
#include "pointwise.hpp"

namespace dgnp {

__constant__ double c_tab[3][2 * 5 * 4 + 5 + 5 + 2 * 4];  // per p: B, Dq, wq, xq, Dend(-1), Dend(+1)

void upload_ref_tables(const RefTables* tabs, int count) {
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

template <int DIM, int P, int MF, typename T, int MODE>
__global__ void __launch_bounds__(DG_NT(DIM, P))
    k_dg(KArgs A, const T* __restrict__ xs, const T* __restrict__ vin, T* __restrict__ out,
         double* __restrict__ aux) {
  using S = Sz<DIM, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NFN = S::NFN, NQF = S::NQF,
                NT = S::NT;
  constexpr int NBT = MF * NB;
  constexpr int QV = MF * (DIM + 1) * NQV;
  constexpr int S1 = DIM == 3 ? MF * 2 * NN * NN * NQ : MF * 2 * NN * NQ;
  constexpr int S2 = DIM == 3 ? MF * 3 * NN * NQ * NQ : 0;
  constexpr int VOLR = 2 * QV + S1 + S2;
  constexpr int TRQ = MF * 2 * NQF;
  constexpr int TRN = MF * 2 * NFN;
  constexpr int TRM = DIM == 3 ? MF * 2 * NN * NQ : 0;
  constexpr int FACER = 2 * NBT + 5 * TRQ + TRN + TRM;
  constexpr int REG = VOLR > FACER ? VOLR : FACER;
  constexpr bool HAS_V = (MODE == M_JAC || MODE == M_JACT || MODE == M_DATAT);
  __shared__ T pool[3 * NBT + REG];
  __shared__ STab<P, T> tb;

  T* s_x = pool;
  T* s_v = pool + NBT;
  T* s_o = pool + 2 * NBT;
  T* R = pool + 3 * NBT;
  const int tid = threadIdx.x;
  load_tab<P, T>(tb, tid, NT);

  Phys<T, MF> ph;
  for (int k = 0; k < MF - 1; ++k) {
    ph.zD[k] = T(A.z[k] * A.D[k]);
    ph.D[k] = T(A.D[k]);
    ph.a[k] = T(A.a[k]);
    ph.b[k] = T(A.b[k]);
  }
  ph.delta = T(A.delta);

  const int64_t e = blockIdx.x;
  const int64_t Nf = A.E * NB;
  int eid[3];
  eid[0] = int(e % A.n[0]);
  eid[1] = int((e / A.n[0]) % A.n[1]);
  eid[2] = DIM == 3 ? int(e / (int64_t(A.n[0]) * A.n[1])) : 0;
  T ih[3];
  for (int i = 0; i < 3; ++i) ih[i] = T(2.0 / A.h[i]);

  for (int i = tid; i < NBT; i += NT) {
    const int f = i / NB, l = i % NB;
    s_x[i] = xs[f * Nf + e * NB + l];
    if constexpr (HAS_V) s_v[i] = vin[f * Nf + e * NB + l];
  }
  __syncthreads();

  // ------------------------------------------------------------------ volume
  if constexpr (MODE == M_RES || MODE == M_JAC || MODE == M_JACT || MODE == M_DPE) {
    T* q_x = R;
    T* q_v = R + QV;
    T* t1 = R + 2 * QV;
    T* t2 = t1 + S1;
    interp<DIM, P, MF, NT, T>(s_x, q_x, t1, t2, tb, ih, tid);
    if constexpr (HAS_V) interp<DIM, P, MF, NT, T>(s_v, q_v, t1, t2, tb, ih, tid);
    for (int qi = tid; qi < NQV; qi += NT) {
      int qc[3];
      qc[0] = qi % NQ;
      qc[1] = (qi / NQ) % NQ;
      qc[2] = qi / (NQ * NQ);
      double xp[3];
      T w = T(A.detJ);
      for (int d = 0; d < DIM; ++d) {
        xp[d] = A.lo[d] + (eid[d] + 0.5 * (double(tb.X[qc[d]]) + 1.0)) * A.h[d];
        w *= tb.W[qc[d]];
      }
      double uhd[3];
      velocity_hat(A, xp, DIM, uhd);
      T u[DIM], uh[DIM];
      for (int d = 0; d < DIM; ++d) {
        uh[d] = T(uhd[d]);
        u[d] = T(A.Pe * uhd[d]);
      }
      T val[MF], grad[MF][DIM];
      for (int f = 0; f < MF; ++f) {
        val[f] = q_x[(f * (DIM + 1)) * NQV + qi];
        for (int d = 0; d < DIM; ++d) grad[f][d] = q_x[(f * (DIM + 1) + 1 + d) * NQV + qi];
      }
      T cv[MF], cg[MF][DIM];
      if constexpr (MODE == M_RES) {
        T src[MF];
        for (int f = 0; f < MF; ++f) src[f] = A.src ? T(A.src[(f * A.E + e) * NQV + qi]) : T(0);
        vol_res<T, MF, DIM>(ph, val, grad, u, src, cv, cg);
      } else if constexpr (MODE == M_JAC) {
        T dv[MF], dg[MF][DIM];
        for (int f = 0; f < MF; ++f) {
          dv[f] = q_v[(f * (DIM + 1)) * NQV + qi];
          for (int d = 0; d < DIM; ++d) dg[f][d] = q_v[(f * (DIM + 1) + 1 + d) * NQV + qi];
          cv[f] = T(0);
        }
        vol_jac<T, MF, DIM>(ph, val, grad, u, dv, dg, cg);
      } else if constexpr (MODE == M_JACT) {
        T gw[MF][DIM];
        for (int f = 0; f < MF; ++f)
          for (int d = 0; d < DIM; ++d) gw[f][d] = q_v[(f * (DIM + 1) + 1 + d) * NQV + qi];
        vol_jacT<T, MF, DIM>(ph, val, grad, u, gw, cv, cg);
      } else {
        for (int f = 0; f < MF; ++f) cv[f] = T(0);
        vol_dpe<T, MF, DIM>(ph, val, uh, cg);
      }
      for (int f = 0; f < MF; ++f) {
        q_v[(f * (DIM + 1)) * NQV + qi] = cv[f] * w;
        for (int d = 0; d < DIM; ++d) q_v[(f * (DIM + 1) + 1 + d) * NQV + qi] = cg[f][d] * w * ih[d];
      }
    }
    __syncthreads();
    integrate<DIM, P, MF, NT, T>(q_v, s_o, t1, t2, tb, tid);
  } else {
    for (int i = tid; i < NBT; i += NT) s_o[i] = T(0);
    __syncthreads();
  }

  // ------------------------------------------------------------------- faces
  double obj_j = 0.0, obj_dpe = 0.0;
  for (int slot = 0; slot < 2 * DIM; ++slot) {
    const int ax = slot >> 1;
    const int side = (slot & 1) ? 1 : -1;
    const int nb = A.nbr[e * 2 * DIM + slot];
    const bool interior = nb >= 0;
    const int cbc = interior ? 0 : A.c_bc[slot];
    const bool phid = interior ? false : (A.phi_bc[slot] == DGNP_PHI_DIRICHLET);
    if constexpr (MODE == M_OBJG) {
      if (interior || slot != A.objective_tag) continue;
    } else if constexpr (MODE == M_DATAT) {
      if (interior || (cbc != BC_DIRICHLET && cbc != BC_INFLOW)) continue;
    } else if constexpr (MODE == M_DPE) {
      if (!interior && cbc == BC_WALL) continue;
    } else {
      if (!interior && cbc == BC_WALL && !phid) continue;
    }
    T* n_x = R;
    T* n_v = R + NBT;
    T* tox = R + 2 * NBT;
    T* tov = tox + TRQ;
    T* tnx = tov + TRQ;
    T* tnv = tnx + TRQ;
    T* cf = tnv + TRQ;
    T* tn = cf + TRQ;
    T* tm = tn + TRN;
    trace<DIM, P, MF, NT, T>(s_x, ax, side, tox, tn, tm, tb, ih[ax], tid);
    if constexpr (HAS_V) trace<DIM, P, MF, NT, T>(s_v, ax, side, tov, tn, tm, tb, ih[ax], tid);
    const bool need_nb = interior && (MODE == M_RES || MODE == M_JAC || MODE == M_JACT || MODE == M_DPE);
    if (need_nb) {
      for (int i = tid; i < NBT; i += NT) {
        const int f = i / NB, l = i % NB;
        n_x[i] = xs[f * Nf + int64_t(nb) * NB + l];
        if constexpr (HAS_V) n_v[i] = vin[f * Nf + int64_t(nb) * NB + l];
      }
      __syncthreads();
      trace<DIM, P, MF, NT, T>(n_x, ax, -side, tnx, tn, tm, tb, ih[ax], tid);
      if constexpr (HAS_V) trace<DIM, P, MF, NT, T>(n_v, ax, -side, tnv, tn, tm, tb, ih[ax], tid);
    }
    // boundary-face index for the data arrays
    int64_t bf = 0;
    if (!interior) {
      int64_t lin;
      if constexpr (DIM == 3)
        lin = ax == 0 ? eid[1] + int64_t(A.n[1]) * eid[2]
                      : (ax == 1 ? eid[0] + int64_t(A.n[0]) * eid[2] : eid[0] + int64_t(A.n[0]) * eid[1]);
      else
        lin = ax == 0 ? eid[1] : eid[0];
      bf = A.btag_off[slot] + lin;
    }
    const int t1ax = DIM == 3 ? (ax == 0 ? 1 : 0) : 1 - ax;
    const int t2ax = DIM == 3 ? (ax == 2 ? 1 : 2) : 0;
    const int own = side > 0 ? 0 : 1;  // own element is the minus side when the face is at +1
    for (int qf = tid; qf < NQF; qf += NT) {
      const int qi = qf % NQ, qj = qf / NQ;
      double xp[3];
      xp[ax] = A.lo[ax] + (eid[ax] + (side > 0 ? 1.0 : 0.0)) * A.h[ax];
      xp[t1ax] = A.lo[t1ax] + (eid[t1ax] + 0.5 * (double(tb.X[qi]) + 1.0)) * A.h[t1ax];
      T w = T(0.5 * A.h[t1ax]) * tb.W[qi];
      if constexpr (DIM == 3) {
        xp[t2ax] = A.lo[t2ax] + (eid[t2ax] + 0.5 * (double(tb.X[qj]) + 1.0)) * A.h[t2ax];
        w *= T(0.5 * A.h[t2ax]) * tb.W[qj];
      }
      double uhd[3];
      velocity_hat(A, xp, DIM, uhd);
      T Fo[MF], Go[MF];
      if (interior) {
        const T un = T(A.Pe * uhd[ax]);
        T v[2][MF], g[2][MF];
        for (int f = 0; f < MF; ++f) {
          v[own][f] = tox[(f * 2 + 0) * NQF + qf];
          g[own][f] = tox[(f * 2 + 1) * NQF + qf];
          v[1 - own][f] = tnx[(f * 2 + 0) * NQF + qf];
          g[1 - own][f] = tnx[(f * 2 + 1) * NQF + qf];
        }
        if constexpr (MODE == M_RES) {
          face_res<T, MF>(ph, v, g, un, own, Fo, Go);
        } else if constexpr (MODE == M_JAC || MODE == M_JACT) {
          T tv[2][MF], tg[2][MF];
          for (int f = 0; f < MF; ++f) {
            tv[own][f] = tov[(f * 2 + 0) * NQF + qf];
            tg[own][f] = tov[(f * 2 + 1) * NQF + qf];
            tv[1 - own][f] = tnv[(f * 2 + 0) * NQF + qf];
            tg[1 - own][f] = tnv[(f * 2 + 1) * NQF + qf];
          }
          if constexpr (MODE == M_JAC)
            face_jac<T, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
          else
            face_jacT<T, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
        } else if constexpr (MODE == M_DPE) {
          face_dpe<T, MF>(ph, v, g, un, T(uhd[ax]), own, Fo, Go);
        }
        for (int f = 0; f < MF; ++f) {
          cf[(f * 2 + 0) * NQF + qf] = Fo[f] * w;
          cf[(f * 2 + 1) * NQF + qf] = Go[f] * w;
        }
      } else {
        const T sd = T(side);
        const T un = T(side * A.Pe * uhd[ax]);
        const T uhn = T(side * uhd[ax]);
        T v[MF], g[MF], gd[MF];
        for (int f = 0; f < MF; ++f) {
          v[f] = tox[(f * 2 + 0) * NQF + qf];
          g[f] = sd * tox[(f * 2 + 1) * NQF + qf];
          gd[f] = T(A.bcq[(f * A.n_bface + bf) * NQF + qf]);
        }
        if constexpr (MODE == M_RES) {
          bnd_res<T, MF>(ph, v, g, un, cbc, phid, gd, Fo, Go);
        } else if constexpr (MODE == M_JAC || MODE == M_JACT) {
          T tv[MF], tg[MF];
          for (int f = 0; f < MF; ++f) {
            tv[f] = tov[(f * 2 + 0) * NQF + qf];
            tg[f] = sd * tov[(f * 2 + 1) * NQF + qf];
          }
          if constexpr (MODE == M_JAC)
            bnd_jac<T, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
          else
            bnd_jacT<T, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
        } else if constexpr (MODE == M_DPE) {
          bnd_dpe<T, MF>(ph, v, g, un, uhn, cbc, gd, Fo, Go);
        } else if constexpr (MODE == M_OBJG) {
          // J = int (q_1 . n) c_1: dJ/dc_1 = Q, dJ/d(dphi/dn) = -z_1 D_1 c_1
          const T Q = un - ph.zD[0] * g[0];
          for (int f = 0; f < MF; ++f) Fo[f] = Go[f] = T(0);
          Fo[1] = Q;
          Go[0] = -ph.zD[0] * v[1];
          obj_j += double(Q * v[1] * w);
          obj_dpe += double(uhn * v[1] * w);
        } else if constexpr (MODE == M_DATAT) {
          T wv[MF], wg[MF], od[MF];
          for (int f = 0; f < MF; ++f) {
            wv[f] = tov[(f * 2 + 0) * NQF + qf];
            wg[f] = sd * tov[(f * 2 + 1) * NQF + qf];
          }
          bnd_dataT<T, MF>(ph, g, wv, wg, un, cbc, od);
          for (int f = 1; f < MF; ++f) aux[(f * A.n_bface + bf) * NQF + qf] = double(od[f] * w);
          for (int f = 0; f < MF; ++f) Fo[f] = Go[f] = T(0);
        }
        for (int f = 0; f < MF; ++f) {
          cf[(f * 2 + 0) * NQF + qf] = Fo[f] * w;
          cf[(f * 2 + 1) * NQF + qf] = Go[f] * w * sd;
        }
      }
    }
    __syncthreads();
    if constexpr (MODE != M_DATAT)
      face_integrate<DIM, P, MF, NT, T>(cf, s_o, ax, side, tn, tm, tb, ih[ax], tid);
  }
  if constexpr (MODE == M_OBJG) {
    __shared__ double rj[NT], rp[NT];
    rj[tid] = obj_j;
    rp[tid] = obj_dpe;
    __syncthreads();
    if (tid == 0) {
      double sj = 0.0, sp = 0.0;
      for (int i = 0; i < NT; ++i) {
        sj += rj[i];
        sp += rp[i];
      }
      aux[2 * e + 0] = sj;
      aux[2 * e + 1] = sp;
    }
  }
  if constexpr (MODE != M_DATAT) {
    for (int i = tid; i < NBT; i += NT) {
      const int f = i / NB, l = i % NB;
      out[f * Nf + e * NB + l] = s_o[i];
    }
  }
}

template <int DIM, int P, int MF, typename T, int MODE>
static void launch_t(const KArgs& A, const void* xs, const void* vin, void* out, double* aux,
                     hipStream_t s) {
  using S = Sz<DIM, P>;
  hipLaunchKernelGGL((k_dg<DIM, P, MF, T, MODE>), dim3(unsigned(A.E)), dim3(S::NT), 0, s, A,
                     static_cast<const T*>(xs), static_cast<const T*>(vin), static_cast<T*>(out), aux);
  DGNP_HIP(hipGetLastError());
}

template <int DIM, int P, int MF>
static void launch_mode(bool f32, int mode, const KArgs& A, const void* xs, const void* vin, void* out,
                        double* aux, hipStream_t s) {
  if (f32) {
    if (mode == M_JAC) return launch_t<DIM, P, MF, float, M_JAC>(A, xs, vin, out, aux, s);
    if (mode == M_JACT) return launch_t<DIM, P, MF, float, M_JACT>(A, xs, vin, out, aux, s);
    throw Error(DGNP_E_ARG, "float arithmetic is offered for the Jacobian applies only");
  }
  switch (mode) {
    case M_RES: return launch_t<DIM, P, MF, double, M_RES>(A, xs, vin, out, aux, s);
    case M_JAC: return launch_t<DIM, P, MF, double, M_JAC>(A, xs, vin, out, aux, s);
    case M_JACT: return launch_t<DIM, P, MF, double, M_JACT>(A, xs, vin, out, aux, s);
    case M_DPE: return launch_t<DIM, P, MF, double, M_DPE>(A, xs, vin, out, aux, s);
    case M_OBJG: return launch_t<DIM, P, MF, double, M_OBJG>(A, xs, vin, out, aux, s);
    case M_DATAT: return launch_t<DIM, P, MF, double, M_DATAT>(A, xs, vin, out, aux, s);
  }
  throw Error(DGNP_E_ARG, "unknown operator mode");
}

template <int DIM, int P>
static void launch_m(int m, bool f32, int mode, const KArgs& A, const void* xs, const void* vin,
                     void* out, double* aux, hipStream_t s) {
  if (m == 2) return launch_mode<DIM, P, 2>(f32, mode, A, xs, vin, out, aux, s);
  if (m == 3) return launch_mode<DIM, P, 3>(f32, mode, A, xs, vin, out, aux, s);
  throw Error(DGNP_E_ARG, "number of ions must be 2 or 3");
}

void launch_dg(int dim, int p, int m, bool f32, int mode, const KArgs& A, const void* xs,
               const void* vin, void* out, double* aux, hipStream_t s) {
  if (A.E == 0) return;
  if (dim == 3) {
    if (p == 1) return launch_m<3, 1>(m, f32, mode, A, xs, vin, out, aux, s);
    if (p == 2) return launch_m<3, 2>(m, f32, mode, A, xs, vin, out, aux, s);
    if (p == 3) return launch_m<3, 3>(m, f32, mode, A, xs, vin, out, aux, s);
  } else if (dim == 2) {
    if (p == 1) return launch_m<2, 1>(m, f32, mode, A, xs, vin, out, aux, s);
    if (p == 2) return launch_m<2, 2>(m, f32, mode, A, xs, vin, out, aux, s);
    if (p == 3) return launch_m<2, 3>(m, f32, mode, A, xs, vin, out, aux, s);
  }
  throw Error(DGNP_E_ARG, "unsupported dimension / order");
}

}  // namespace dgnp
