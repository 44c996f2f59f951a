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
#include <mutex>

#include "dg_device.hpp"

namespace dgnp {

void upload_ref_tables(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

#define OP_NT(D, P) ((D) == 3 ? ((P) == 3 ? 256 : 128) : 64)

// One work-group per element.  Phases (each a parallel loop followed by a
// barrier):
//   volume   sum-factorised interpolation of the state (and input vector) to the
//            Gauss points, pointwise flux, transposed contraction -> s_o;
//   faces    all 2d faces together: F1 traces (value and d/dx_ax) at the face
//            nodes of own and neighbour element (neighbours read from global
//            memory), F2/F3 tangential interpolation to the face Gauss points,
//            F4 numerical flux -> own-side coefficients, F5 tangential
//            transposes, F6 accumulation into the own element's nodes.
// Block b works on element (b mod 8) * ceil(E/8) + b / 8: work-groups are
// dispatched round-robin over the 8 XCDs, so each XCD sweeps one contiguous
// slab of elements and the neighbour reads of the face terms stay in its L2.
template <int DIM, int P, int MF, typename T, int MODE>
__global__ void __launch_bounds__(OP_NT(DIM, P))
    k_dg(KArgs A, const T* __restrict__ xs, const T* __restrict__ vin, T* __restrict__ out,
         double* __restrict__ aux, int64_t eper) {
  using S = Sz<DIM, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NFN = S::NFN, NQF = S::NQF;
  constexpr int NT = OP_NT(DIM, P);
  constexpr bool JACF = (MODE == M_JAC || MODE == M_JACP);  // forward Jacobian (all rows / potential rows)
  constexpr bool HAS_V = (JACF || MODE == M_JACT || MODE == M_DATAT);
  constexpr bool VOLUME = (MODE == M_RES || JACF || MODE == M_JACT || MODE == M_DPE);
  constexpr int OUTF = MODE == M_JACP ? 1 : MF;  // output fields formed (M_JACP: the potential's)
  constexpr bool NEED_NB = VOLUME;  // objective and data modes use the own trace only
  constexpr int NARR = HAS_V ? 2 : 1;
  constexpr int NC = DIM + 1;
  constexpr int NFACE = 2 * DIM;
  constexpr int NBT = MF * NB;
  constexpr int QV = MF * NC * NQV;
  constexpr int S1 = DIM == 3 ? MF * 2 * NN * NN * NQ : MF * 2 * NN * NQ;
  constexpr int S2 = DIM == 3 ? MF * 3 * NN * NQ * NQ : 0;
  constexpr int VOLR = 2 * QV + NARR * (S1 + S2);
  constexpr int NROW = NFACE * 2 * NARR * MF * 2;  // trace rows: face, side, array, field, value/dn
  constexpr int NCF = NFACE * MF * 2 * NQF;
  constexpr int FACR = NROW * NQF + (NROW * NFN > NCF ? NROW * NFN : NCF);
  constexpr int REG = VOLR > FACR ? VOLR : FACR;
  __shared__ T s_xv[NARR * NBT];  // state, then input vector (contiguous for the line contractions)
  __shared__ T s_o[NBT];
  __shared__ T R[REG];
  __shared__ STab<P, T> tb;
  __shared__ int s_nb[NFACE];
  T* s_x = s_xv;
  T* s_v = s_xv + (NARR - 1) * NBT;

  const int64_t bid = blockIdx.x;
  const int64_t e = (bid % 8) * eper + bid / 8;
  if (e >= A.E) return;
  const int tid = threadIdx.x;
  load_tab<P, T>(tb, tid, NT);
  const Phys<T, MF> ph = make_phys<T, MF>(A);
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
    if constexpr (HAS_V) s_v[i] = ((A.vin_mask >> f) & 1u) ? vin[f * Nf + e * NB + l] : T(0);
  }
  if (tid < NFACE) s_nb[tid] = A.nbr[e * NFACE + tid];
  __syncthreads();

  // ---------------------------------------------------------------- volume
  if constexpr (VOLUME) {
    T* q_x = R;
    T* q_v = R + QV;
    T* t1 = R + 2 * QV;
    T* t2 = t1 + NARR * S1;
    if constexpr (DIM == 3) {
      interp_lines<P, MF, NARR, NT, T>(s_xv, q_x, t1, t2, ih, tid);
    } else {
      interp<DIM, P, MF, NT, T>(s_x, q_x, t1, t2, tb, ih, tid);
      if constexpr (HAS_V) interp<DIM, P, MF, NT, T>(s_v, q_v, t1, t2, tb, ih, tid);
    }
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
        val[f] = q_x[(f * NC) * NQV + qi];
        for (int d = 0; d < DIM; ++d) grad[f][d] = q_x[(f * NC + 1 + d) * NQV + qi];
      }
      T cv[MF], cg[MF][DIM];
      if constexpr (MODE == M_RES) {
        T src[MF];
        for (int f = 0; f < MF; ++f) src[f] = A.src ? T(A.src[(f * A.E + e) * NQV + qi]) : T(0);
        vol_res<T, MF, DIM>(ph, val, grad, u, src, cv, cg);
      } else if constexpr (JACF) {
        T dv[MF], dg[MF][DIM];
        for (int f = 0; f < MF; ++f) {
          dv[f] = q_v[(f * NC) * NQV + qi];
          for (int d = 0; d < DIM; ++d) dg[f][d] = q_v[(f * NC + 1 + d) * NQV + qi];
          cv[f] = T(0);
        }
        vol_jac<T, MF, DIM>(ph, val, grad, u, dv, dg, cg);
      } else if constexpr (MODE == M_JACT) {
        T gw[MF][DIM];
        for (int f = 0; f < MF; ++f)
          for (int d = 0; d < DIM; ++d) gw[f][d] = q_v[(f * NC + 1 + d) * NQV + qi];
        vol_jacT<T, MF, DIM>(ph, val, grad, u, gw, cv, cg);
      } else {
        for (int f = 0; f < MF; ++f) cv[f] = T(0);
        vol_dpe<T, MF, DIM>(ph, val, uh, cg);
      }
      for (int f = 0; f < OUTF; ++f) {
        q_v[(f * NC) * NQV + qi] = cv[f] * w;
        for (int d = 0; d < DIM; ++d) q_v[(f * NC + 1 + d) * NQV + qi] = cg[f][d] * w * ih[d];
      }
    }
    __syncthreads();
    if constexpr (DIM == 3)
      integrate_lines<P, OUTF, NT, T>(q_v, s_o, t1, t2, tid);
    else
      integrate<DIM, P, OUTF, NT, T>(q_v, s_o, t1, t2, tb, tid);
  } else {
    for (int i = tid; i < NBT; i += NT) s_o[i] = T(0);
    __syncthreads();
  }

  // ----------------------------------------------------------------- faces
  // face region: [fq: NROW * NQF][fn: max(NROW * NFN, NCF)].  F1 writes the
  // node traces fn, F2/F3 interpolate them to fq, F4 reads fq and writes the
  // coefficients cf over fn, F5 writes the transposes tnt over fq.
  T* fq = R;
  T* fn = R + NROW * NQF;
  T* cf = fn;
  T* tnt = R;
  static_assert(NFACE * MF * 2 * NFN <= NROW * NQF, "transposes must fit in the face-point area");
  // F1: face-node traces (value and d/dx_ax together) of own and neighbour
  // element; pair row pr = (face, side, array, field) -> rows 2 pr (value),
  // 2 pr + 1 (normal derivative).  The state's concentration derivatives are
  // used by the residual only.
  {
    using C = CT<T, P>;
    for (int idx = tid; idx < (NROW / 2) * NFN; idx += NT) {
      const int ij = idx % NFN;
      int pr = idx / NFN;
      const int f = pr % MF;
      const int ar = (pr / MF) % NARR;
      const int sd = (pr / (MF * NARR)) % 2;
      const int fc = pr / (MF * NARR * 2);
      const int ax = fc >> 1;
      const int side = (fc & 1) ? 1 : -1;
      const int sside = sd == 0 ? side : -side;
      const int i = ij % NN, j = ij / NN;
      const T* u = nullptr;
      if (sd == 0)
        u = (ar == 0 ? s_x : s_v) + f * NB;
      else if (NEED_NB && s_nb[fc] >= 0 && (ar == 0 || ((A.vin_mask >> f) & 1u)))
        u = (ar == 0 ? xs : vin) + f * Nf + int64_t(s_nb[fc]) * NB;
      const bool need_dn = MODE == M_RES || ar == 1 || f == 0;
      T val = T(0), dn = T(0);
      if (u) {
        T x[NN];
#pragma unroll
        for (int l = 0; l < NN; ++l) x[l] = u[face_node<DIM, NN>(ax, l, i, j)];
        val = sside < 0 ? x[0] : x[P];
        if (need_dn) {
#pragma unroll
          for (int l = 0; l < NN; ++l) dn += (sside < 0 ? C::De(0, l) : C::De(1, l)) * x[l];
          dn *= ih[ax];
        }
      }
      fn[(2 * pr + 0) * NFN + ij] = val;
      fn[(2 * pr + 1) * NFN + ij] = dn;
    }
  }
  __syncthreads();
  // F2/F3: both tangential interpolations of one trace row in registers
  {
    using C = CT<T, P>;
    for (int row = tid; row < NROW; row += NT) {
      T x[NFN];
#pragma unroll
      for (int k = 0; k < NFN; ++k) x[k] = fn[row * NFN + k];
      if constexpr (DIM == 3) {
        T y[NN][NQ];  // interpolated along the first tangential direction
#pragma unroll
        for (int j = 0; j < NN; ++j)
#pragma unroll
          for (int qi = 0; qi < NQ; ++qi) {
            T s = T(0);
#pragma unroll
            for (int i = 0; i < NN; ++i) s += C::B(qi, i) * x[j * NN + i];
            y[j][qi] = s;
          }
#pragma unroll
        for (int qj = 0; qj < NQ; ++qj)
#pragma unroll
          for (int qi = 0; qi < NQ; ++qi) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < NN; ++j) s += C::B(qj, j) * y[j][qi];
            fq[row * NQF + qj * NQ + qi] = s;
          }
      } else {
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < NN; ++i) s += C::B(qi, i) * x[i];
          fq[row * NQF + qi] = s;
        }
      }
    }
  }
  __syncthreads();
  // F4: numerical fluxes at every face point of every face
  double obj_j = 0.0, obj_dpe = 0.0, obj_j0 = 0.0, obj_pa = 0.0;
  auto trow = [&](int fc, int sd, int ar, int f, int c2) { return ((((fc * 2 + sd) * NARR + ar) * MF + f) * 2 + c2); };
  for (int idx = tid; idx < NFACE * NQF; idx += NT) {
    const int qf = idx % NQF, fc = idx / NQF;
    const int ax = fc >> 1;
    const int side = (fc & 1) ? 1 : -1;
    const int nb = s_nb[fc];
    const bool interior = nb >= 0;
    const int cbc = interior ? 0 : A.c_bc[fc];
    const bool phid = interior ? false : (A.phi_bc[fc] == DGNP_PHI_DIRICHLET);
    T Fo[MF], Go[MF];
    for (int f = 0; f < MF; ++f) Fo[f] = Go[f] = T(0);
    bool active;
    if constexpr (MODE == M_OBJG)
      active = !interior && fc == A.objective_tag;
    else if constexpr (MODE == M_DATAT)
      active = !interior && (cbc == BC_DIRICHLET || cbc == BC_INFLOW || cbc == BC_ELECTRODE);
    else if constexpr (MODE == M_DPE)
      active = interior || cbc != BC_WALL;
    else
      active = interior || cbc != BC_WALL || phid;
    T w = T(0);
    if (active) {
      const int qi = qf % NQ, qj = qf / NQ;
      const int t1ax = DIM == 3 ? (ax == 0 ? 1 : 0) : 1 - ax;
      const int t2ax = DIM == 3 ? (ax == 2 ? 1 : 2) : 0;
      double xp[3];
      xp[ax] = A.lo[ax] + (eid[ax] + (side > 0 ? 1.0 : 0.0)) * A.h[ax];
      xp[t1ax] = A.lo[t1ax] + (eid[t1ax] + 0.5 * (double(tb.X[qi]) + 1.0)) * A.h[t1ax];
      w = T(0.5 * A.h[t1ax]) * tb.W[qi];
      if constexpr (DIM == 3) {
        xp[t2ax] = A.lo[t2ax] + (eid[t2ax] + 0.5 * (double(tb.X[qj]) + 1.0)) * A.h[t2ax];
        w *= T(0.5 * A.h[t2ax]) * tb.W[qj];
      }
      double uhd[3];
      velocity_hat(A, xp, DIM, uhd);
      if (interior) {
        const int own = side > 0 ? 0 : 1;  // the own element is the minus side of a +1 face
        const T un = T(A.Pe * uhd[ax]);
        T v[2][MF], g[2][MF];
        for (int f = 0; f < MF; ++f) {
          v[own][f] = fq[trow(fc, 0, 0, f, 0) * NQF + qf];
          g[own][f] = fq[trow(fc, 0, 0, f, 1) * NQF + qf];
          v[1 - own][f] = fq[trow(fc, 1, 0, f, 0) * NQF + qf];
          g[1 - own][f] = fq[trow(fc, 1, 0, f, 1) * NQF + qf];
        }
        if constexpr (MODE == M_RES) {
          face_res<T, MF>(ph, v, g, un, own, Fo, Go);
        } else if constexpr (JACF || MODE == M_JACT) {
          T tv[2][MF], tg[2][MF];
          for (int f = 0; f < MF; ++f) {
            tv[own][f] = fq[trow(fc, 0, NARR - 1, f, 0) * NQF + qf];
            tg[own][f] = fq[trow(fc, 0, NARR - 1, f, 1) * NQF + qf];
            tv[1 - own][f] = fq[trow(fc, 1, NARR - 1, f, 0) * NQF + qf];
            tg[1 - own][f] = fq[trow(fc, 1, NARR - 1, f, 1) * NQF + qf];
          }
          if constexpr (JACF)
            face_jac<T, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
          else
            face_jacT<T, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
        } else if constexpr (MODE == M_DPE) {
          face_dpe<T, MF>(ph, v, g, un, T(uhd[ax]), own, Fo, Go);
        }
      } else {
        int64_t lin;
        if constexpr (DIM == 3)
          lin = ax == 0 ? eid[1] + int64_t(A.n[1]) * eid[2]
                        : (ax == 1 ? eid[0] + int64_t(A.n[0]) * eid[2] : eid[0] + int64_t(A.n[0]) * eid[1]);
        else
          lin = ax == 0 ? eid[1] : eid[0];
        const int64_t bf = A.btag_off[fc] + lin;
        const T sd = T(side);
        const T un = T(side * A.Pe * uhd[ax]);
        const T uhn = T(side * uhd[ax]);
        T v[MF], g[MF], gd[MF];
        for (int f = 0; f < MF; ++f) {
          v[f] = fq[trow(fc, 0, 0, f, 0) * NQF + qf];
          g[f] = sd * fq[trow(fc, 0, 0, f, 1) * NQF + qf];
          gd[f] = T(A.bcq[(f * A.n_bface + bf) * NQF + qf]);
        }
        if constexpr (MODE == M_RES) {
          bnd_res<T, MF>(ph, v, g, un, cbc, phid, gd, Fo, Go);
        } else if constexpr (JACF || MODE == M_JACT) {
          T tv[MF], tg[MF];
          for (int f = 0; f < MF; ++f) {
            tv[f] = fq[trow(fc, 0, NARR - 1, f, 0) * NQF + qf];
            tg[f] = sd * fq[trow(fc, 0, NARR - 1, f, 1) * NQF + qf];
          }
          if constexpr (JACF)
            bnd_jac<T, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
          else
            bnd_jacT<T, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
        } else if constexpr (MODE == M_DPE) {
          bnd_dpe<T, MF>(ph, v, g, un, uhn, cbc, gd, Fo, Go);
        } else if constexpr (MODE == M_OBJG) {
          if (A.objective_kind == 1) {
            // J = int g (the reacting ion's rate on an electrode face)
            const BvRate<T> r = bv_rate(ph, v, gd);
            Fo[0] = r.dphi;
            for (int k = 1; k < MF; ++k) Fo[k] = r.dc * ph.bv_dc[k - 1];
            obj_j += double(r.g * w);
            obj_j0 += double(r.dj0 * w) * (DIM == 3 ? j0_profile(A, xp[2]) : 1.0);
            obj_pa += double(r.dpa * w);
          } else {
            // J = int (q_1 . n) c_1: dJ/dc_1 = Q, dJ/d(dphi/dn) = -z_1 D_1 c_1
            const T Q = un - ph.zD[0] * g[0];
            Fo[1] = Q;
            Go[0] = -ph.zD[0] * v[1];
            obj_j += double(Q * v[1] * w);
            obj_dpe += double(uhn * v[1] * w);
          }
        } else if constexpr (MODE == M_DATAT) {
          T wv[MF], wg[MF], od[MF];
          for (int f = 0; f < MF; ++f) {
            wv[f] = fq[trow(fc, 0, NARR - 1, f, 0) * NQF + qf];
            wg[f] = sd * fq[trow(fc, 0, NARR - 1, f, 1) * NQF + qf];
          }
          bnd_dataT<T, MF>(ph, v, g, wv, wg, un, cbc, gd, od);
          if (cbc == BC_ELECTRODE) {  // applied potential, exchange-current amplitude
            aux[(0 * A.n_bface + bf) * NQF + qf] = double(od[0] * w);
            aux[(1 * A.n_bface + bf) * NQF + qf] = double(od[1] * w) * (DIM == 3 ? j0_profile(A, xp[2]) : 1.0);
          } else {
            for (int f = 1; f < MF; ++f) aux[(f * A.n_bface + bf) * NQF + qf] = double(od[f] * w);
          }
        }
        for (int f = 0; f < MF; ++f) Go[f] *= sd;  // outward normal derivative -> d/dx_ax
      }
    }
    // cf layout [face][field][value / dn][qf]
    for (int f = 0; f < OUTF; ++f) {
      cf[((fc * MF + f) * 2 + 0) * NQF + qf] = Fo[f] * w;
      cf[((fc * MF + f) * 2 + 1) * NQF + qf] = Go[f] * w * ih[ax];
    }
  }
  __syncthreads();
  if constexpr (MODE == M_OBJG) {
    __shared__ double rj[4][NT];
    rj[0][tid] = obj_j;
    rj[1][tid] = obj_dpe;
    rj[2][tid] = obj_j0;
    rj[3][tid] = obj_pa;
    __syncthreads();
    if (tid < 4) {
      double sj = 0.0;
      for (int i = 0; i < NT; ++i) sj += rj[tid][i];
      aux[4 * e + tid] = sj;
    }
    if (out == nullptr) return;  // the value alone (no gradient)
  }
  if constexpr (MODE == M_DATAT) return;
  // F5: both tangential transposes of one coefficient row in registers
  {
    using C = CT<T, P>;
    for (int ro = tid; ro < NFACE * OUTF * 2; ro += NT) {
      const int rc = ((ro / (2 * OUTF)) * MF + (ro / 2) % OUTF) * 2 + (ro & 1);  // row of cf / tnt
      T x[NQF];
#pragma unroll
      for (int k = 0; k < NQF; ++k) x[k] = cf[rc * NQF + k];
      if constexpr (DIM == 3) {
        T y[NN][NQ];  // transposed along the second tangential direction
#pragma unroll
        for (int j = 0; j < NN; ++j)
#pragma unroll
          for (int qi = 0; qi < NQ; ++qi) {
            T s = T(0);
#pragma unroll
            for (int qj = 0; qj < NQ; ++qj) s += C::B(qj, j) * x[qj * NQ + qi];
            y[j][qi] = s;
          }
#pragma unroll
        for (int j = 0; j < NN; ++j)
#pragma unroll
          for (int i = 0; i < NN; ++i) {
            T s = T(0);
#pragma unroll
            for (int qi = 0; qi < NQ; ++qi) s += C::B(qi, i) * y[j][qi];
            tnt[rc * NFN + j * NN + i] = s;
          }
      } else {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          T s = T(0);
#pragma unroll
          for (int qi = 0; qi < NQ; ++qi) s += C::B(qi, i) * x[qi];
          tnt[rc * NFN + i] = s;
        }
      }
    }
  }
  __syncthreads();
  // F6: every node gathers its value / normal-derivative contributions of all faces
  for (int idx = tid; idx < OUTF * NB; idx += NT) {
    const int f = idx / NB, node = idx % NB;
    const int cx = node % NN, cy = (node / NN) % NN, cz = node / (NN * NN);
    T acc = s_o[idx];
#pragma unroll
    for (int fc = 0; fc < NFACE; ++fc) {
      const int ax = fc >> 1;
      const int sdi = fc & 1;
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
      const int rc = fc * MF + f;
      const int ij = j * NN + i;
      acc += tb.De[sdi][l] * tnt[(rc * 2 + 1) * NFN + ij];
      if (l == (sdi ? P : 0)) acc += tnt[(rc * 2 + 0) * NFN + ij];
    }
    if constexpr (MODE == M_JACP) {
      const T* jb = static_cast<const T*>(A.jbase);
      out[f * Nf + e * NB + node] = jb ? jb[f * Nf + e * NB + node] - acc : acc;
    } else {
      out[f * Nf + e * NB + node] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Allocation-free objective value: the per-element partial sums of the
// objective kernel go to a static device array instead of library or caller
// workspace; one work-group then adds them in a fixed order.  The array is
// shared by every call on one GPU (calls that overlap on a GPU race) and
// needs no clearing: the objective kernel writes the two partials of every
// element before the sum reads them.
static constexpr int64_t OBJ_SCRATCH_ELEMS = int64_t(1) << 18;
static __device__ __align__(256) double scratch[4 * OBJ_SCRATCH_ELEMS];

static std::mutex g_scratch_mu;
static double* g_scratch_dev[64] = {};  // the array's address on each device

double* objective_scratch_init() {
  int dev = 0;
  DGNP_HIP(hipGetDevice(&dev));
  DGNP_REQUIRE(dev >= 0 && dev < 64, DGNP_E_ARG, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    DGNP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}

int64_t objective_scratch_max_elements() { return OBJ_SCRATCH_ELEMS; }

__global__ void __launch_bounds__(256) k_obj_sum(const double* __restrict__ part, int64_t E, double* __restrict__ J) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < E; e += 256) acc += part[4 * e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = sh[0];
}

void objective_noalloc(int dim, int p, int m, const KArgs& A, const double* x, double* scratch_dev, double* J_dev,
                       hipStream_t s) {
  // A selects the objective (objective_kind, objective_tag)
  DGNP_REQUIRE(A.E <= OBJ_SCRATCH_ELEMS, DGNP_E_ARG,
               "allocation-free objective: at most 262144 elements (2^18) per problem");
  DGNP_REQUIRE(scratch_dev, DGNP_E_STATE, "allocation-free objective: scratch not set up on this device");
  launch_dg(dim, p, m, false, M_OBJG, A, x, nullptr, nullptr, scratch_dev, s);
  hipLaunchKernelGGL(k_obj_sum, dim3(1), dim3(256), 0, s, scratch_dev, A.E, J_dev);
  DGNP_HIP(hipGetLastError());
}

template <int DIM, int P, int MF, typename T, int MODE>
static void launch_t(const KArgs& A, const void* xs, const void* vin, void* out, double* aux,
                     hipStream_t s) {
  const int64_t eper = (A.E + 7) / 8;
  hipLaunchKernelGGL((k_dg<DIM, P, MF, T, MODE>), dim3(unsigned(8 * eper)), dim3(OP_NT(DIM, P)), 0, s, A,
                     static_cast<const T*>(xs), static_cast<const T*>(vin), static_cast<T*>(out), aux, eper);
  DGNP_HIP(hipGetLastError());
}

template <int DIM, int P, int MF>
static void launch_mode(bool f32, int mode, const KArgs& A, const void* xs, const void* vin, void* out,
                        double* aux, hipStream_t s) {
  if (f32) {
    if (mode == M_JAC) return launch_t<DIM, P, MF, float, M_JAC>(A, xs, vin, out, aux, s);
    if (mode == M_JACP) return launch_t<DIM, P, MF, float, M_JACP>(A, xs, vin, out, aux, s);
    if (mode == M_JACT) return launch_t<DIM, P, MF, float, M_JACT>(A, xs, vin, out, aux, s);
    throw Error(DGNP_E_ARG, "float arithmetic is offered for the Jacobian applies only");
  }
  switch (mode) {
    case M_RES: return launch_t<DIM, P, MF, double, M_RES>(A, xs, vin, out, aux, s);
    case M_JAC: return launch_t<DIM, P, MF, double, M_JAC>(A, xs, vin, out, aux, s);
    case M_JACP: return launch_t<DIM, P, MF, double, M_JACP>(A, xs, vin, out, aux, s);
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
