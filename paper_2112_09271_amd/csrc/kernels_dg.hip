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
#include "dg_device.hpp"

namespace dgnp {

void upload_ref_tables(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

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
