// Matrix-free potential-potential block for p-multigrid smoothing (3-D).
//
// The derivative of the charge equation (Eq. chargeDG) with respect to the
// potential is the SIPG diffusion operator with the coefficient
// kappa(c) = sum_k b_k c_k of the linearisation point (plus a Robin term on
// Butler-Volmer electrode faces, the only place where the equation is
// nonlinear in the potential):
//   (A u, v) = sum_K int_K kappa grad u . grad v
//            + sum_F int_F ( -{kappa du/dn}[v] - [u]{kappa dv/dn} + {kappa} delta [u][v] )
//            + sum_{F potential-Dirichlet} int_F ( -kappa du/dn v - u kappa dv/dn + kappa delta u v ).
// kappa is tabulated once per linearisation point at the volume Gauss points
// (times weight and Jacobian) and at the face Gauss points of each element's
// own traces (times the face weight), so one apply reads only the input, the
// tables and the output instead of all fields of state and input.
//
// One work-group per element, as the general operator kernel: sum-factorised
// volume term, then the 6 faces element-centric (own and neighbour traces at
// the face Gauss points, flux, integration into the own element only).
#include <cstdlib>

#include "dg_device.hpp"
#include "kernels_phi.hpp"

namespace dgnp {

void upload_ref_tables_phi(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

#define PHI_NT(P) ((P) == 3 ? 256 : 128)

// kv[e][q] = kappa w_q detJ at the volume Gauss points; kf[e][fc][qf] = kappa
// w_f at the Gauss points of face fc from the element's own traces (on an
// electrode face: the Robin coefficient -z_r dg/dphi w_f of the Butler-Volmer
// term instead)
template <int P, int MF, typename T>
__global__ void __launch_bounds__(PHI_NT(P)) k_phi_kappa(KArgs A, const double* __restrict__ xs, T* __restrict__ kv,
                                                         T* __restrict__ kf) {
  using S = Sz<3, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NQF = S::NQF;
  constexpr int NT = PHI_NT(P);
  using C = CT<double, P>;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t Nf = A.E * NB;
  const double* wq = C::base() + 2 * NQ * NN;  // Gauss weights
  for (int qi = tid; qi < NQV; qi += NT) {
    const int qx = qi % NQ, qy = (qi / NQ) % NQ, qz = qi / (NQ * NQ);
    double kap = 0.0;
    for (int k = 1; k < MF; ++k) {
      const double* x = xs + k * Nf + e * NB;
      double s = 0.0;
      for (int c = 0; c < NN; ++c)
        for (int b = 0; b < NN; ++b)
          for (int a = 0; a < NN; ++a)
            s += C::B(qx, a) * C::B(qy, b) * C::B(qz, c) * x[(c * NN + b) * NN + a];
      kap += A.b[k - 1] * s;
    }
    kv[e * NQV + qi] = T(kap * A.detJ * wq[qx] * wq[qy] * wq[qz]);
  }
  for (int idx = tid; idx < 6 * NQF; idx += NT) {
    const int qf = idx % NQF, fc = idx / NQF;
    const int ax = fc >> 1, l = (fc & 1) ? P : 0;
    const int qi = qf % NQ, qj = qf / NQ;
    const int t1ax = ax == 0 ? 1 : 0, t2ax = ax == 2 ? 1 : 2;
    double val[MF];
    for (int f = 0; f < MF; ++f) {
      const double* x = xs + f * Nf + e * NB;
      double s = 0.0;
      for (int j = 0; j < NN; ++j)
        for (int i = 0; i < NN; ++i) s += C::B(qi, i) * C::B(qj, j) * x[face_node<3, NN>(ax, l, i, j)];
      val[f] = s;
    }
    double kap = 0.0;
    for (int k = 1; k < MF; ++k) kap += A.b[k - 1] * val[k];
    const double w = 0.25 * A.h[t1ax] * A.h[t2ax] * wq[qi] * wq[qj];
    double coef = kap * w;
    if (A.nbr[e * 6 + fc] < 0 && A.c_bc[fc] == BC_ELECTRODE) {
      // electrode face: the Butler-Volmer term -z_r g v of the charge equation,
      // linearised in the potential, is a Robin term with coefficient -z_r dg/dphi
      const int ex = int(e % A.n[0]), ey = int((e / A.n[0]) % A.n[1]), ez = int(e / (int64_t(A.n[0]) * A.n[1]));
      const int64_t lin = ax == 0 ? ey + int64_t(A.n[1]) * ez : (ax == 1 ? ex + int64_t(A.n[0]) * ez : ex + int64_t(A.n[0]) * ey);
      const int64_t bf = A.btag_off[fc] + lin;
      double gd[MF];
      for (int f = 0; f < MF; ++f) gd[f] = A.bcq[(f * A.n_bface + bf) * NQF + qf];
      const Phys<double, MF> ph = make_phys<double, MF>(A);
      coef = -ph.bv_z * bv_rate(ph, val, gd).dphi * w;
    }
    kf[(e * 6 + fc) * NQF + qf] = T(coef);
  }
}

// y = A_phiphi u
template <int P, typename T, int NT>
__global__ void __launch_bounds__(NT) k_phi_op(KArgs A, const T* __restrict__ u, const T* __restrict__ kv,
                                               const T* __restrict__ kf, T* __restrict__ y, int64_t eper) {
  using S = Sz<3, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NFN = S::NFN, NQF = S::NQF;
  static_assert(NT >= NQ * NN && NT >= 2 * NN && NT >= 6, "the table loads take one lane per entry");
  constexpr int VOLR = 4 * NQV + NN * NN * 2 * NQ + NN * 3 * NQ * NQ;
  constexpr int NROW = 6 * 2 * 2;  // face, side (own, neighbour), value / d/dx_ax
  constexpr int FACR = NROW * NFN + NROW * NQF;
  constexpr int REG = VOLR > FACR ? VOLR : FACR;
  static_assert(6 * 2 * NQF <= NROW * NFN, "face coefficients must fit in the node-trace area");
  static_assert(6 * 2 * NFN <= NROW * NQF, "transposes must fit in the face-point area");
  __shared__ T s_u[NB];
  __shared__ T s_o[NB];
  __shared__ T R[REG];
  __shared__ int s_nb[6];
  __shared__ T s_de[2][NN];
  __shared__ T s_B[NQ * NN];  // B(q, a) for the lane-indexed contractions of the face traces
  const int64_t bid = blockIdx.x;
  const int64_t e = (bid % 8) * eper + bid / 8;  // one slab of elements per XCD, as the operator kernel
  if (e >= A.E) return;
  const int tid = threadIdx.x;
  using C = CT<T, P>;
  T ih[3];
  for (int i = 0; i < 3; ++i) ih[i] = T(2.0 / A.h[i]);
  const T delta = T(A.delta);
  for (int i = tid; i < NB; i += NT) s_u[i] = u[e * NB + i];
  if (tid < 6) s_nb[tid] = A.nbr[e * 6 + tid];
  if (tid < 2 * NN) s_de[tid / NN][tid % NN] = C::De(tid / NN, tid % NN);
  if (tid < NQ * NN) s_B[tid] = C::B(tid / NN, tid % NN);
  __syncthreads();

  // volume: kappa grad u . grad v
  {
    T* q = R;
    T* t1 = R + 4 * NQV;
    T* t2 = t1 + NN * NN * 2 * NQ;
    interp_lines<P, 1, 1, NT, T>(s_u, q, t1, t2, ih, tid);
    for (int qi = tid; qi < NQV; qi += NT) {
      const T kw = kv[e * NQV + qi];
      q[qi] = T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) q[(1 + d) * NQV + qi] *= kw * ih[d];
    }
    __syncthreads();
    integrate_lines<P, 1, NT, T>(q, s_o, t1, t2, tid);
  }

  // faces: fn [NROW][NFN] node traces, fq [NROW][NQF] face-point traces;
  // cf [6][2][NQF] over fn, tnt [6][2][NFN] over fq
  T* fn = R;
  T* fq = R + NROW * NFN;
  T* cf = fn;
  T* tnt = fq;
  for (int idx = tid; idx < 12 * NFN; idx += NT) {
    const int ij = idx % NFN, pr = idx / NFN;  // pr = face * 2 + side
    const int sd = pr & 1, fc = pr >> 1;
    const int ax = fc >> 1;
    const int side = (fc & 1) ? 1 : -1;
    const int sside = sd == 0 ? side : -side;
    const int i = ij % NN, j = ij / NN;
    const T* src = nullptr;
    if (sd == 0)
      src = s_u;
    else if (s_nb[fc] >= 0)
      src = u + int64_t(s_nb[fc]) * NB;
    T val = T(0), dn = T(0);
    if (src) {
      T x[NN];
#pragma unroll
      for (int l = 0; l < NN; ++l) x[l] = src[face_node<3, NN>(ax, l, i, j)];
      val = sside < 0 ? x[0] : x[P];
#pragma unroll
      for (int l = 0; l < NN; ++l) dn += (sside < 0 ? C::De(0, l) : C::De(1, l)) * x[l];
      dn *= ih[ax];
    }
    fn[(2 * pr + 0) * NFN + ij] = val;
    fn[(2 * pr + 1) * NFN + ij] = dn;
  }
  __syncthreads();
  // node traces to face points, one lane per (row, qi): first along i with
  // the lane's B(qi, .), then along j with compile-time B(qj, .)
  for (int idx = tid; idx < NROW * NQ; idx += NT) {
    const int row = idx / NQ, qi = idx % NQ;
    T b[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) b[i] = s_B[qi * NN + i];
    T yv[NN];
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      T t = T(0);
#pragma unroll
      for (int i = 0; i < NN; ++i) t += b[i] * fn[row * NFN + j * NN + i];
      yv[j] = t;
    }
#pragma unroll
    for (int qj = 0; qj < NQ; ++qj) {
      T t = T(0);
#pragma unroll
      for (int j = 0; j < NN; ++j) t += C::B(qj, j) * yv[j];
      fq[row * NQF + qj * NQ + qi] = t;
    }
  }
  __syncthreads();
  // fluxes: coefficients of v and dv/dx_ax of the own element (kappa tables
  // carry the face weight); side = +1 on a +x_ax face, where the own element is
  // the minus element of the interior face
  for (int idx = tid; idx < 6 * NQF; idx += NT) {
    const int qf = idx % NQF, fc = idx / NQF;
    const int ax = fc >> 1;
    const T side = (fc & 1) ? T(1) : T(-1);
    const int nb = s_nb[fc];
    const T uo = fq[((fc * 2 + 0) * 2 + 0) * NQF + qf];
    const T dno = fq[((fc * 2 + 0) * 2 + 1) * NQF + qf];
    const T ko = kf[(e * 6 + fc) * NQF + qf];
    T F = T(0), G = T(0);
    if (nb >= 0) {
      const T un = fq[((fc * 2 + 1) * 2 + 0) * NQF + qf];
      const T dnn = fq[((fc * 2 + 1) * 2 + 1) * NQF + qf];
      const T kn = kf[(int64_t(nb) * 6 + (fc ^ 1)) * NQF + qf];
      const T jmp = uo - un;
      F = -T(0.5) * side * (ko * dno + kn * dnn) + T(0.5) * (ko + kn) * delta * jmp;
      G = -T(0.5) * side * ko * jmp;
    } else if (A.phi_bc[fc] == DGNP_PHI_DIRICHLET) {
      F = -side * ko * dno + ko * delta * uo;
      G = -side * ko * uo;
    } else if (A.c_bc[fc] == BC_ELECTRODE) {
      F = ko * uo;  // Robin coefficient of the electrode term (weight included)
    }
    cf[(fc * 2 + 0) * NQF + qf] = F;
    cf[(fc * 2 + 1) * NQF + qf] = G * ih[ax];
  }
  __syncthreads();
  // face-point coefficients back to node traces, one lane per (row, j): first
  // along qj with the lane's B(., j), then along qi with compile-time B(., i)
  for (int idx = tid; idx < 12 * NN; idx += NT) {
    const int rc = idx / NN, j = idx % NN;
    T b[NQ];
#pragma unroll
    for (int qj = 0; qj < NQ; ++qj) b[qj] = s_B[qj * NN + j];
    T yv[NQ];
#pragma unroll
    for (int qi = 0; qi < NQ; ++qi) {
      T t = T(0);
#pragma unroll
      for (int qj = 0; qj < NQ; ++qj) t += b[qj] * cf[rc * NQF + qj * NQ + qi];
      yv[qi] = t;
    }
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      T t = T(0);
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) t += C::B(qi, i) * yv[qi];
      tnt[rc * NFN + j * NN + i] = t;
    }
  }
  __syncthreads();
  for (int node = tid; node < NB; node += NT) {
    const int cx = node % NN, cy = (node / NN) % NN, cz = node / (NN * NN);
    T acc = s_o[node];
#pragma unroll
    for (int fc = 0; fc < 6; ++fc) {
      const int ax = fc >> 1;
      const int sdi = fc & 1;
      const int l = ax == 0 ? cx : (ax == 1 ? cy : cz);
      const int i = ax == 0 ? cy : cx;
      const int j = ax == 2 ? cy : cz;
      const int ij = j * NN + i;
      acc += s_de[sdi][l] * tnt[(fc * 2 + 1) * NFN + ij];
      if (l == (sdi ? P : 0)) acc += tnt[(fc * 2 + 0) * NFN + ij];
    }
    y[e * NB + node] = acc;
  }
}

template <typename T>
void launch_phi_kappa(int p, int m, const KArgs& A, const double* xs, T* kv, T* kf, hipStream_t s) {
  if (A.E == 0) return;
  const dim3 g(unsigned(A.E));
  if (p == 2 && m == 3) hipLaunchKernelGGL((k_phi_kappa<2, 3, T>), g, dim3(PHI_NT(2)), 0, s, A, xs, kv, kf);
  else if (p == 2 && m == 2) hipLaunchKernelGGL((k_phi_kappa<2, 2, T>), g, dim3(PHI_NT(2)), 0, s, A, xs, kv, kf);
  else if (p == 3 && m == 3) hipLaunchKernelGGL((k_phi_kappa<3, 3, T>), g, dim3(PHI_NT(3)), 0, s, A, xs, kv, kf);
  else if (p == 3 && m == 2) hipLaunchKernelGGL((k_phi_kappa<3, 2, T>), g, dim3(PHI_NT(3)), 0, s, A, xs, kv, kf);
  else throw Error(DGNP_E_ARG, "potential operator tables: orders 2 and 3, 2 or 3 ions");
  DGNP_HIP(hipGetLastError());
}

// threads per element: one wave (64), or 128 / 256 by DGNP_PHI_NT (A/B
// measurement).  Most phases have fewer items than 256 lanes (16 to 192 at
// p = 3), so one wave per element keeps the lanes busy and lets more elements
// share a CU: on the 12.6M-DOF channel, p = 3, 106 / 135 / 193 us per apply in
// single precision and 216 / 223 / 310 us in double with 64 / 128 / 256 threads.
template <int P, typename T>
static void phi_op_t(const KArgs& A, const T* u, const T* kv, const T* kf, T* y, hipStream_t s) {
  const int64_t eper = (A.E + 7) / 8;
  const dim3 g(unsigned(8 * eper));
  const char* env = getenv("DGNP_PHI_NT");
  const int nt = env ? atoi(env) : 64;
  if (nt == 64) hipLaunchKernelGGL((k_phi_op<P, T, 64>), g, dim3(64), 0, s, A, u, kv, kf, y, eper);
  else if (nt == 128) hipLaunchKernelGGL((k_phi_op<P, T, 128>), g, dim3(128), 0, s, A, u, kv, kf, y, eper);
  else hipLaunchKernelGGL((k_phi_op<P, T, 256>), g, dim3(256), 0, s, A, u, kv, kf, y, eper);
  DGNP_HIP(hipGetLastError());
}

template <typename T>
void launch_phi_op(int p, const KArgs& A, const T* u, const T* kv, const T* kf, T* y, hipStream_t s) {
  if (A.E == 0) return;
  if (p == 2) phi_op_t<2, T>(A, u, kv, kf, y, s);
  else if (p == 3) phi_op_t<3, T>(A, u, kv, kf, y, s);
  else throw Error(DGNP_E_ARG, "potential operator: orders 2 and 3");
}

template void launch_phi_kappa<double>(int, int, const KArgs&, const double*, double*, double*, hipStream_t);
template void launch_phi_kappa<float>(int, int, const KArgs&, const double*, float*, float*, hipStream_t);
template void launch_phi_op<double>(int, const KArgs&, const double*, const double*, const double*, double*,
                                    hipStream_t);
template void launch_phi_op<float>(int, const KArgs&, const float*, const float*, const float*, float*, hipStream_t);

}  // namespace dgnp
