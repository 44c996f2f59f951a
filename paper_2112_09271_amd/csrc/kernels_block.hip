// Block kernels of the preconditioner (gfx950):
//  * assembly of the diagonal field blocks A_ff of the Jacobian (Sec. 4,
//    Eq. blockmatrix) on the element graph: one n_b x n_b block per element
//    (volume + own-side face terms) and one per neighbour slot;
//  * in-LDS Gauss-Jordan inversion of element blocks;
//  * element-block ILU(0) (BILU(0)) factorisation over hyperplane levels
//    ix + iy + iz = const of the lexicographic element order, and the
//    level-scheduled forward / backward solves and their transposes;
//  * block sparse matrix-vector products and block-diagonal applies;
//  * the trilinear (Q1) vertex <-> DG node transfers and the Galerkin
//    product of the potential block onto the Q1 vertex space.
#include <algorithm>
#include <type_traits>

#include "dg_device.hpp"
#include "kernels_block.hpp"

namespace dgnp {

void upload_ref_tables_block(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

static constexpr int BT = 256;  // threads per block kernel

// ===========================================================================
// Assembly.  One work-group per (element, field).  blk[f][e][s][i][j]: s = 0
// diagonal block, s = 1 + slot coupling to the neighbour across `slot`; row i
// = test function, column j = trial function.
//
// The pointwise Jacobian of the field's own flux is tabulated at every
// quadrature point for each pair (alpha, beta) of test derivative alpha
// (d/dx_1..d/dx_d) and trial component beta (value, d/dx_1..d/dx_d), and the
// element matrix
//   A_ij = sum_q sum_{alpha,beta} T_alpha(q, i) M_q[alpha][beta] T_beta(q, j)
// is formed by sum factorisation over the tensor-product structure: a pair
// (alpha, beta) factorises along direction d into E_a(q_d, i_d) E_b(q_d, j_d)
// with E = interpolation (B) or derivative (D) rows, so the quadrature sum is
// contracted one direction at a time, pairs whose remaining factors agree
// being summed before the next contraction.  Pairs whose coefficient vanishes
// at every point of the element are skipped.  Face terms (value and normal
// derivative of test and trial on both sides) factorise the same way over the
// two tangential directions.  2-D problems run the same code with a third
// direction of one node and one point.
// ===========================================================================
// a0, a1 or a2 by a run-time index d (selects, not an indexed array)
template <typename T>
__device__ __forceinline__ T sel3(T a0, T a1, T a2, int d) {
  return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

template <int DIM>
struct AsmPairs {
  static constexpr int NC = DIM + 1;
  static constexpr int NCB = DIM * NC;  // alpha = 1..DIM, beta = 0..DIM
  // factor type of pair c along direction d: 2 * (test derivative) + (trial derivative)
  static constexpr int ty(int c, int d) { return d >= DIM ? 0 : 2 * (c / NC == d) + (c % NC == 1 + d); }
  static constexpr int key(int c) { return ty(c, 1) + 4 * ty(c, 2); }
  static constexpr int nkeys() {
    int n = 0;
    for (int k = 0; k < 16; ++k) {
      bool hit = false;
      for (int c = 0; c < NCB; ++c) hit = hit || key(c) == k;
      n += hit ? 1 : 0;
    }
    return n;
  }
};

template <int DIM, int P, int MF>
__global__ void __launch_bounds__(BT, P >= 2 ? 3 : 1)
    k_assemble(KArgs A, const double* __restrict__ xs, double* __restrict__ blk, int f0) {
  using S = Sz<DIM, P>;
  using PR = AsmPairs<DIM>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NQF = S::NQF, NFN = S::NFN;
  constexpr int N3 = DIM == 3 ? NN : 1, Q3 = DIM == 3 ? NQ : 1;  // third direction (padded in 2-D)
  constexpr int NC = DIM + 1;
  constexpr int NCB = PR::NCB;
  constexpr int NKMAX = PR::nkeys();
  constexpr int NBT = MF * NB;
  constexpr int NN2 = NN * NN;
  constexpr int QV = MF * NC * NQV;
  constexpr int S1 = DIM == 3 ? MF * 2 * NN * NN * NQ : MF * 2 * NN * NQ;
  constexpr int S2 = DIM == 3 ? MF * 3 * NN * NQ * NQ : 0;
  constexpr int Y1K = NN2 * NQ * Q3;   // per key: [q3][q2][i1 j1]
  constexpr int Y2G = NN2 * NN2 * Q3;  // per third-direction type: [q3][i2 j2][i1 j1]
  constexpr int VOL1 = NKMAX * Y1K;
  // LDS of the volume part, by lifetime: M (pointwise coefficients) from the
  // pointwise step to direction 1; the interpolation temporaries before it
  // (above M); Y1 from direction 1 to the last direction-2 pass (over the
  // temporaries); Y2 over M.  At order 3 Y2 holds one third-direction type at
  // a time (the LDS then admits three work-groups per CU), below it every type
  // at once (fewer barriers; LDS is not the limit there)
  constexpr bool Y2ONE = P >= 3;
  constexpr int Y2SZ = Y2ONE ? Y2G : 4 * Y2G;
  constexpr int MSZ = NCB * NQV;
  constexpr int OY1 = MSZ > Y2SZ ? MSZ : Y2SZ;
  // loop unrolling of the face slots: at order 3 one slot at a time and two
  // block entries per step, which keeps the registers within three
  // work-groups per CU
  constexpr int UNR_SLOT = Y2ONE ? 1 : 2 * DIM;
  constexpr int UNR_ENT = Y2ONE ? 2 : (NB * NB + BT - 1) / BT;
  constexpr int VOLA = MSZ + QV + S1 + S2, VOLB = OY1 + VOL1;
  constexpr int VOLR = VOLA > VOLB ? VOLA : VOLB;
  constexpr int NFACE = 2 * DIM;
  constexpr int NROWF = NFACE * 2 * MF * 2;  // face trace rows: face, side (own / neighbour), field, value / dn
  constexpr int ZSZ = 8 * NN2 * Q3;
  constexpr int CSZ = 8 * NN2 * N3 * N3;
  constexpr int TRS = NROWF * (NFN + NQF);
  constexpr int FACR = NFACE * NQF * 8 + (TRS > ZSZ + CSZ ? TRS : ZSZ + CSZ);
  constexpr int REG = VOLR > FACR ? VOLR : FACR;
  constexpr int ENT = (NB * NB + BT - 1) / BT;
  constexpr int NSLOT = 2 * DIM + 1;
  __shared__ double s_x[NBT];
  __shared__ double R[REG];
  __shared__ double G[4 * NQ * NN2];  // G[t][q][i][j] = E_{t>>1}(q, i) E_{t&1}(q, j)
  __shared__ STab<P, double> tb;
  __shared__ int s_nz[NCB];
  __shared__ int s_keys[16], s_t3[4], s_nk, s_n3;

  const int tid = threadIdx.x;
  const int64_t e = blockIdx.x;
  const int f = f0 + int(blockIdx.y);
  load_tab<P, double>(tb, tid, BT);
  const Phys<double, MF> ph = make_phys<double, MF>(A);
  const int64_t Nf = A.E * NB;
  int eid[3];
  eid[0] = int(e % A.n[0]);
  eid[1] = int((e / A.n[0]) % A.n[1]);
  eid[2] = DIM == 3 ? int(e / (int64_t(A.n[0]) * A.n[1])) : 0;
  double ih[3];
  for (int i = 0; i < 3; ++i) ih[i] = 2.0 / A.h[i];
  for (int i = tid; i < NBT; i += BT) s_x[i] = xs[(i / NB) * Nf + e * NB + (i % NB)];
  if (tid < NCB) s_nz[tid] = 0;
  __syncthreads();
  for (int idx = tid; idx < 4 * NQ * NN2; idx += BT) {
    const int j = idx % NN, i = (idx / NN) % NN, q = (idx / NN2) % NQ, t = idx / (NQ * NN2);
    G[idx] = ((t >> 1) ? tb.D[q * NN + i] : tb.B[q * NN + i]) * ((t & 1) ? tb.D[q * NN + j] : tb.B[q * NN + j]);
  }

  double acc[ENT];
  for (int k = 0; k < ENT; ++k) acc[k] = 0.0;
  // ---- volume
  {
    double* M = R;  // M[c][q]
    double* q_x = R + MSZ;
    double* t1 = q_x + QV;
    double* t2 = t1 + S1;
    double* Y1 = R + OY1;
    double* Y2 = R;
    interp<DIM, P, MF, BT, double>(s_x, q_x, t1, t2, tb, ih, tid);
    for (int qi = tid; qi < NQV; qi += BT) {
      const int qc[3] = {qi % NQ, (qi / NQ) % NQ, qi / (NQ * NQ)};
      double xp[3], w = A.detJ;
      for (int d = 0; d < DIM; ++d) {
        xp[d] = A.lo[d] + (eid[d] + 0.5 * (tb.X[qc[d]] + 1.0)) * A.h[d];
        w *= tb.W[qc[d]];
      }
      double uh[3];
      velocity_hat(A, xp, DIM, uh);
      double u[DIM];
      for (int d = 0; d < DIM; ++d) u[d] = A.Pe * uh[d];
      double val[MF], grad[MF][DIM];
      for (int g = 0; g < MF; ++g) {
        val[g] = q_x[(g * NC) * NQV + qi];
        for (int d = 0; d < DIM; ++d) grad[g][d] = q_x[(g * NC + 1 + d) * NQV + qi];
      }
      // unit trial directions, written with compile-time indices only (the
      // field f is a run-time value) so that the arrays stay in registers
      for (int beta = 0; beta < NC; ++beta) {
        double dv[MF], dg[MF][DIM], cg[MF][DIM];
#pragma unroll
        for (int g = 0; g < MF; ++g) {
          dv[g] = (beta == 0 && g == f) ? 1.0 : 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) dg[g][d] = (beta == 1 + d && g == f) ? 1.0 : 0.0;
        }
        vol_jac<double, MF, DIM>(ph, val, grad, u, dv, dg, cg);
        const double sb = beta == 0 ? 1.0 : ih[beta - 1];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          double cf = 0.0;
#pragma unroll
          for (int g = 0; g < MF; ++g) cf = g == f ? cg[g][d] : cf;
          const double m = cf * w * sb * ih[d];
          M[(d * NC + beta) * NQV + qi] = m;
          if (m != 0.0) s_nz[d * NC + beta] = 1;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      int nk = 0, n3 = 0;
      for (int k = 0; k < 16; ++k) {
        bool hit = false;
        for (int c = 0; c < NCB; ++c) hit = hit || (s_nz[c] && PR::key(c) == k);
        if (hit) s_keys[nk++] = k;
      }
      for (int t = 0; t < 4; ++t) {
        bool hit = false;
        for (int kk = 0; kk < nk; ++kk) hit = hit || (s_keys[kk] >> 2) == t;
        if (hit) s_t3[n3++] = t;
      }
      s_nk = nk;
      s_n3 = n3;
    }
    __syncthreads();
    const int nk = s_nk, n3 = s_n3;
    // direction 1: Y1[key][q3][q2][i1 j1] = sum_{pairs of key} sum_q1 G_t1(q1, i1, j1) M_c(q1, q2, q3)
    for (int o = tid; o < nk * Y1K; o += BT) {
      const int kk = o / Y1K, r = o % Y1K;
      const int ij = r % NN2, q2 = (r / NN2) % NQ, q3 = r / (NN2 * NQ);
      const int key = s_keys[kk];
      double s = 0.0;
      for (int c = 0; c < NCB; ++c) {
        if (!s_nz[c] || PR::key(c) != key) continue;
        const double* g = G + PR::ty(c, 0) * NQ * NN2 + ij;
        const double* m = M + c * NQV + NQ * (q2 + NQ * q3);
#pragma unroll
        for (int q1 = 0; q1 < NQ; ++q1) s += g[q1 * NN2] * m[q1];
      }
      Y1[o] = s;
    }
    __syncthreads();
    // direction 2: Y2[t3][q3][i2 j2][i1 j1] = sum_{keys with t3} sum_q2 G_t2(q2, i2, j2) Y1[key][q3][q2][i1 j1]
    if constexpr (Y2ONE) {
      for (int gg = 0; gg < n3; ++gg) {
        const int t3 = s_t3[gg];
        for (int o = tid; o < Y2G; o += BT) {
          const int ij1 = o % NN2, ij2 = (o / NN2) % NN2, q3 = o / (NN2 * NN2);
          double s = 0.0;
          for (int kk = 0; kk < nk; ++kk) {
            const int key = s_keys[kk];
            if ((key >> 2) != t3) continue;
            const double* g = G + (key & 3) * NQ * NN2 + ij2;
            const double* y = Y1 + kk * Y1K + q3 * NQ * NN2 + ij1;
  #pragma unroll
            for (int q2 = 0; q2 < NQ; ++q2) s += g[q2 * NN2] * y[q2 * NN2];
          }
          Y2[o] = s;
        }
        __syncthreads();
        for (int k = 0; k < ENT; ++k) {
          const int idx = tid + k * BT;
          if (idx >= NB * NB) break;
          const int i = idx / NB, j = idx % NB;
          const int i1 = i % NN, i2 = (i / NN) % NN, i3 = i / NN2;
          const int j1 = j % NN, j2 = (j / NN) % NN, j3 = j / NN2;
          const double* y = Y2 + (i2 * NN + j2) * NN2 + i1 * NN + j1;
          double s = acc[k];
          for (int q3 = 0; q3 < Q3; ++q3) {
            const double g = DIM == 3 ? G[((t3 * NQ + q3) * NN + i3) * NN + j3] : 1.0;
            s += g * y[q3 * NN2 * NN2];
          }
          acc[k] = s;
        }
        __syncthreads();
      }
    } else {
      // every type at once: Y2[t3][q3][i2 j2][i1 j1], then A_ij = sum_t3 sum_q3 G_t3(q3, i3, j3) Y2[t3]..
      for (int o = tid; o < n3 * Y2G; o += BT) {
        const int gg = o / Y2G, r = o % Y2G;
        const int ij1 = r % NN2, ij2 = (r / NN2) % NN2, q3 = r / (NN2 * NN2);
        const int t3 = s_t3[gg];
        double s = 0.0;
        for (int kk = 0; kk < nk; ++kk) {
          const int key = s_keys[kk];
          if ((key >> 2) != t3) continue;
          const double* g = G + (key & 3) * NQ * NN2 + ij2;
          const double* y = Y1 + kk * Y1K + q3 * NQ * NN2 + ij1;
#pragma unroll
          for (int q2 = 0; q2 < NQ; ++q2) s += g[q2 * NN2] * y[q2 * NN2];
        }
        Y2[o] = s;
      }
      __syncthreads();
      for (int k = 0; k < ENT; ++k) {
        const int idx = tid + k * BT;
        if (idx >= NB * NB) break;
        const int i = idx / NB, j = idx % NB;
        const int i1 = i % NN, i2 = (i / NN) % NN, i3 = i / NN2;
        const int j1 = j % NN, j2 = (j / NN) % NN, j3 = j / NN2;
        const double* y = Y2 + (i2 * NN + j2) * NN2 + i1 * NN + j1;
        double s = 0.0;
        for (int gg = 0; gg < n3; ++gg) {
          const int t3 = s_t3[gg];
          for (int q3 = 0; q3 < Q3; ++q3) {
            const double g = DIM == 3 ? G[((t3 * NQ + q3) * NN + i3) * NN + j3] : 1.0;
            s += g * y[gg * Y2G + q3 * NN2 * NN2];
          }
        }
        acc[k] = s;
      }
      __syncthreads();
    }
  }

  // ---- faces
  // FA: node traces (value, d/dx_ax) of the state on both sides of every face
  //     (rows: face, side, field, value / dn; the neighbour read from global memory);
  // FB: both tangential interpolations of every row to the face points;
  // FC: the pointwise face Jacobian for every (face, point, trial direction),
  //     Mf[face][qf][test value / dn][trial: own v, own g, nb v, nb g];
  // then, face by face, the tangential contractions and the expansion below.
  double* MfA = R;                               // [NFACE][NQF][8]
  double* fnod = MfA + NFACE * NQF * 8;          // [NROWF][NFN]
  double* fq = fnod + NROWF * NFN;               // [NROWF][NQF]
  double* Z = fnod;                              // [8][q2][i1 j1]
  double* Cf = Z + ZSZ;                          // [8][i2 j2][i1 j1]
  double* out = blk + ((int64_t(f) * A.E + e) * NSLOT) * NB * NB;
  {
    for (int idx = tid; idx < (NROWF / 2) * NFN; idx += BT) {
      const int ij = idx % NFN, pr = idx / NFN;
      const int c = pr % MF, sd = (pr / MF) % 2, fc = pr / (2 * MF);
      const int ax = fc >> 1;
      const int side = (fc & 1) ? 1 : -1;
      const int sside = sd == 0 ? side : -side;
      const int nbe = A.nbr[e * 2 * DIM + fc];
      const double* u = nullptr;
      if (sd == 0)
        u = s_x + c * NB;
      else if (nbe >= 0)
        u = xs + c * Nf + int64_t(nbe) * NB;
      const int i = ij % NN, j = ij / NN;
      double val = 0.0, dn = 0.0;
      if (u) {
        const double* De = tb.De[sside < 0 ? 0 : 1];
        for (int l = 0; l < NN; ++l) {
          const double x = u[face_node<DIM, NN>(ax, l, i, j)];
          dn += De[l] * x;
          if (l == (sside < 0 ? 0 : P)) val = x;
        }
        dn *= sel3(ih[0], ih[1], ih[2], ax);
      }
      fnod[(2 * pr + 0) * NFN + ij] = val;
      fnod[(2 * pr + 1) * NFN + ij] = dn;
    }
    __syncthreads();
    for (int row = tid; row < NROWF; row += BT) {
      const double* x = fnod + row * NFN;
      if constexpr (DIM == 3) {
        double y[NN][NQ];
        for (int j = 0; j < NN; ++j)
          for (int qi = 0; qi < NQ; ++qi) {
            double t = 0.0;
            for (int i = 0; i < NN; ++i) t += tb.B[qi * NN + i] * x[j * NN + i];
            y[j][qi] = t;
          }
        for (int qj = 0; qj < NQ; ++qj)
          for (int qi = 0; qi < NQ; ++qi) {
            double t = 0.0;
            for (int j = 0; j < NN; ++j) t += tb.B[qj * NN + j] * y[j][qi];
            fq[row * NQF + qj * NQ + qi] = t;
          }
      } else {
        for (int qi = 0; qi < NQ; ++qi) {
          double t = 0.0;
          for (int i = 0; i < NN; ++i) t += tb.B[qi * NN + i] * x[i];
          fq[row * NQF + qi] = t;
        }
      }
    }
    __syncthreads();
    auto trow = [&](int fc, int sd, int c, int c2) { return ((fc * 2 + sd) * MF + c) * 2 + c2; };
    for (int idx = tid; idx < NFACE * NQF * 4; idx += BT) {
      const int beta = idx % 4, qf = (idx / 4) % NQF, fc = idx / (4 * NQF);
      const int ax = fc >> 1, side = (fc & 1) ? 1 : -1;
      const int nbe = A.nbr[e * 2 * DIM + fc];
      const bool interior = nbe >= 0;
      const int cbc = interior ? 0 : A.c_bc[fc];
      const bool phid = interior ? false : (A.phi_bc[fc] == DGNP_PHI_DIRICHLET);
      double* M = MfA + (fc * NQF + qf) * 8;
      if (!interior && (beta >= 2 || (cbc == BC_WALL && !phid))) {
        M[0 * 4 + beta] = 0.0;
        M[1 * 4 + beta] = 0.0;
        continue;
      }
      const int t1ax = DIM == 3 ? (ax == 0 ? 1 : 0) : 1 - ax;
      const int t2ax = DIM == 3 ? (ax == 2 ? 1 : 2) : 0;
      const int qi = qf % NQ, qj = qf / NQ;
      // the face point: the face's coordinate along ax, Gauss points along
      // the tangential axes (every array index fixed at compile time: arrays
      // indexed by a run-time axis would live in scratch memory)
      double xp[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double ed = d < DIM ? double(eid[d]) : 0.0;
        const double xd = d == ax ? (side > 0 ? 1.0 : 0.0) : 0.5 * (tb.X[d == t1ax ? qi : qj] + 1.0);
        xp[d] = d < DIM ? A.lo[d] + (ed + xd) * A.h[d] : 0.0;
      }
      const double ihx = sel3(ih[0], ih[1], ih[2], ax);
      double w = 0.5 * sel3(A.h[0], A.h[1], A.h[2], t1ax) * tb.W[qi];
      if constexpr (DIM == 3) w *= 0.5 * sel3(A.h[0], A.h[1], A.h[2], t2ax) * tb.W[qj];
      double uh[3];
      velocity_hat(A, xp, DIM, uh);
      const double uax = sel3(uh[0], uh[1], uh[2], ax);
      double fo = 0.0, go = 0.0;
      if (interior) {
        const double un = A.Pe * uax;
        const int own = side > 0 ? 0 : 1;
        double v[2][MF], g[2][MF], tv[2][MF], tg[2][MF];
        const int sdb = beta < 2 ? own : 1 - own;
#pragma unroll
        for (int c = 0; c < MF; ++c) {
          // own side first when it is the minus side (selects: see above)
          const double vo = fq[trow(fc, 0, c, 0) * NQF + qf], go_ = fq[trow(fc, 0, c, 1) * NQF + qf];
          const double vn = fq[trow(fc, 1, c, 0) * NQF + qf], gn = fq[trow(fc, 1, c, 1) * NQF + qf];
          v[0][c] = own == 0 ? vo : vn;
          v[1][c] = own == 0 ? vn : vo;
          g[0][c] = own == 0 ? go_ : gn;
          g[1][c] = own == 0 ? gn : go_;
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            tv[s2][c] = (s2 == sdb && c == f && beta % 2 == 0) ? 1.0 : 0.0;
            tg[s2][c] = (s2 == sdb && c == f && beta % 2 == 1) ? 1.0 : 0.0;
          }
        }
        double Fo[MF], Go[MF];
        face_jac<double, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
#pragma unroll
        for (int c = 0; c < MF; ++c) {
          fo = c == f ? Fo[c] : fo;
          go = c == f ? Go[c] : go;
        }
        const double sb = (beta % 2 == 0) ? 1.0 : ihx;
        M[0 * 4 + beta] = fo * w * sb;
        M[1 * 4 + beta] = go * w * sb * ihx;
      } else {
        int64_t lin;
        if constexpr (DIM == 3)
          lin = ax == 0 ? eid[1] + int64_t(A.n[1]) * eid[2]
                        : (ax == 1 ? eid[0] + int64_t(A.n[0]) * eid[2] : eid[0] + int64_t(A.n[0]) * eid[1]);
        else
          lin = ax == 0 ? eid[1] : eid[0];
        const int64_t bf = A.btag_off[fc] + lin;
        const double un = side * A.Pe * uax;
        double v[MF], g[MF], gd[MF], tv[MF], tg[MF];
#pragma unroll
        for (int c = 0; c < MF; ++c) {
          v[c] = fq[trow(fc, 0, c, 0) * NQF + qf];
          g[c] = side * fq[trow(fc, 0, c, 1) * NQF + qf];
          gd[c] = A.bcq[(c * A.n_bface + bf) * NQF + qf];
          tv[c] = (c == f && beta == 0) ? 1.0 : 0.0;
          tg[c] = (c == f && beta == 1) ? 1.0 : 0.0;
        }
        double Fo[MF], Go[MF];
        bnd_jac<double, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
#pragma unroll
        for (int c = 0; c < MF; ++c) {
          fo = c == f ? Fo[c] : fo;
          go = c == f ? Go[c] : go;
        }
        const double sb = beta == 0 ? 1.0 : side * ihx;
        M[0 * 4 + beta] = fo * w * sb;
        M[1 * 4 + beta] = go * w * sb * side * ihx;
      }
    }
    __syncthreads();
  }
#pragma unroll UNR_SLOT
  for (int slot = 0; slot < 2 * DIM; ++slot) {
    const int ax = slot >> 1, side = (slot & 1) ? 1 : -1;
    const int nb = A.nbr[e * 2 * DIM + slot];
    const bool interior = nb >= 0;
    const int cbc = interior ? 0 : A.c_bc[slot];
    const bool phid = interior ? false : (A.phi_bc[slot] == DGNP_PHI_DIRICHLET);
    double* ob = out + int64_t(1 + slot) * NB * NB;
    if (!interior && cbc == BC_WALL && !phid) {
      for (int idx = tid; idx < NB * NB; idx += BT) ob[idx] = 0.0;
      continue;
    }
    const int t1ax = DIM == 3 ? (ax == 0 ? 1 : 0) : 1 - ax;
    const int t2ax = DIM == 3 ? (ax == 2 ? 1 : 2) : 0;
    const double* Mf = MfA + slot * NQF * 8;
    __syncthreads();
    // first tangential direction: Z[ab][qj][i1 j1] = sum_qi B(qi, i1) B(qi, j1) Mf[qi, qj][ab]
#pragma unroll 1
    for (int o = tid; o < 8 * Q3 * NN2; o += BT) {
      const int ij = o % NN2, qj = (o / NN2) % Q3, ab = o / (Q3 * NN2);
      if ((ab & 3) >= 2 && !interior) continue;
      double s = 0.0;
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) s += G[qi * NN2 + ij] * Mf[(qj * NQ + qi) * 8 + ab];
      Z[o] = s;
    }
    __syncthreads();
    // second tangential direction: Cf[ab][i2 j2][i1 j1] = sum_qj B(qj, i2) B(qj, j2) Z[ab][qj][i1 j1]
#pragma unroll 1
    for (int o = tid; o < 8 * N3 * N3 * NN2; o += BT) {
      const int ij1 = o % NN2, ij2 = (o / NN2) % (N3 * N3), ab = o / (N3 * N3 * NN2);
      if ((ab & 3) >= 2 && !interior) continue;
      double s = 0.0;
      if constexpr (DIM == 3) {
#pragma unroll
        for (int qj = 0; qj < NQ; ++qj) s += G[qj * NN2 + ij2] * Z[(ab * Q3 + qj) * NN2 + ij1];
      } else {
        s = Z[ab * NN2 + ij1];
      }
      Cf[o] = s;
    }
    __syncthreads();
    // expansion over the normal direction: value (l == endpoint) and normal-derivative rows
    const int lend_own = side < 0 ? 0 : P;
    const int lend_nb = side < 0 ? P : 0;
    const double* De_own = tb.De[side < 0 ? 0 : 1];
    const double* De_nb = tb.De[side < 0 ? 1 : 0];
#pragma unroll UNR_ENT
    for (int k = 0; k < ENT; ++k) {
      const int idx = tid + k * BT;
      if (idx >= NB * NB) break;
      const int i = idx / NB, j = idx % NB;
      // node coordinates picked by run-time axes with selects (an array
      // indexed at run time would live in scratch memory)
      const int i0 = i % NN, i1 = (i / NN) % NN, i2 = DIM == 3 ? i / NN2 : 0;
      const int j0 = j % NN, j1 = (j / NN) % NN, j2 = DIM == 3 ? j / NN2 : 0;
      auto pick = [](int a0, int a1, int a2, int d) { return d == 0 ? a0 : (d == 1 ? a1 : a2); };
      const int li = pick(i0, i1, i2, ax), lj = pick(j0, j1, j2, ax);
      const int tix = pick(i0, i1, i2, t1ax) * NN + pick(j0, j1, j2, t1ax);
      const int t2x = DIM == 3 ? pick(i0, i1, i2, t2ax) * N3 + pick(j0, j1, j2, t2ax) : 0;
      const double* c = Cf + t2x * NN2 + tix;
      constexpr int CS = N3 * N3 * NN2;  // stride between pairs ab
      const double pi0 = li == lend_own ? 1.0 : 0.0, pi1 = De_own[li];
      const double pj0 = lj == lend_own ? 1.0 : 0.0, pj1 = De_own[lj];
      acc[k] += pi0 * (pj0 * c[0 * CS] + pj1 * c[1 * CS]) + pi1 * (pj0 * c[4 * CS] + pj1 * c[5 * CS]);
      double so = 0.0;
      if (interior) {
        const double nj0 = lj == lend_nb ? 1.0 : 0.0, nj1 = De_nb[lj];
        so = pi0 * (nj0 * c[2 * CS] + nj1 * c[3 * CS]) + pi1 * (nj0 * c[6 * CS] + nj1 * c[7 * CS]);
      }
      ob[idx] = so;
    }
    __syncthreads();
  }
  for (int k = 0; k < ENT; ++k) {
    const int idx = tid + k * BT;
    if (idx < NB * NB) out[idx] = acc[k];
  }
}

template <int DIM, int P>
static void assemble_t(int m, int f0, int nf, const KArgs& A, const double* xs, double* blk, hipStream_t s) {
  const dim3 grid = dim3(unsigned(A.E), unsigned(nf));
  if (m == 2)
    hipLaunchKernelGGL((k_assemble<DIM, P, 2>), grid, dim3(BT), 0, s, A, xs, blk, f0);
  else
    hipLaunchKernelGGL((k_assemble<DIM, P, 3>), grid, dim3(BT), 0, s, A, xs, blk, f0);
  DGNP_HIP(hipGetLastError());
}

void launch_assemble(int dim, int p, int m, int f0, int nf, const KArgs& A, const double* xs, double* blk,
                     hipStream_t s) {
  DGNP_REQUIRE(m == 2 || m == 3, DGNP_E_ARG, "number of ions must be 2 or 3");
  DGNP_REQUIRE(f0 >= 0 && nf >= 0 && f0 + nf <= m, DGNP_E_ARG, "field range out of bounds");
  if (nf == 0 || A.E == 0) return;
  if (dim == 3) {
    if (p == 1) return assemble_t<3, 1>(m, f0, nf, A, xs, blk, s);
    if (p == 2) return assemble_t<3, 2>(m, f0, nf, A, xs, blk, s);
    if (p == 3) return assemble_t<3, 3>(m, f0, nf, A, xs, blk, s);
  } else {
    if (p == 1) return assemble_t<2, 1>(m, f0, nf, A, xs, blk, s);
    if (p == 2) return assemble_t<2, 2>(m, f0, nf, A, xs, blk, s);
    if (p == 3) return assemble_t<2, 3>(m, f0, nf, A, xs, blk, s);
  }
  throw Error(DGNP_E_ARG, "unsupported dimension / order");
}

// ===========================================================================
// Gauss-Jordan inversion (sweep form) with partial pivoting of an NB x NB
// matrix (NB <= 64) held in LDS with leading dimension LD.  The matrix lives in
// registers during the elimination: lane r of every wave holds row r, and wave
// w holds the columns 16 j + 4 w + t (t = 0..3), i.e. panels of four
// consecutive columns dealt round the four waves.  Rows are never
// interchanged; step k pivots column k on the unused row p of largest
// magnitude (ties: smallest row), so that on exit
//   A^{-1}[i][j] = a[rsrc[i]][csrc[j]],  rsrc[k] = p_k,  csrc[p_k] = k.
// Step k with pivot p and inv = 1 / x[p][k]: every row r != p takes
// x[r][c] -= g_r x[p][c] for c != k with g_r = x[r][k] inv, and x[r][k] = -g_r;
// row p takes x[p][c] *= inv and x[p][k] = inv.
// Per panel of four steps the owning wave alone runs the four pivot searches
// and applies each step to its own panel columns (everything the next search
// needs), then publishes the pivots, their inverses and the multipliers g_r;
// after one barrier every wave applies the four steps to its other columns,
// taking the pivot row's entries from lane p of its own registers.  Each entry
// sees the same operations in the same order as in a step-by-step sweep; the
// published data are double-buffered, so one barrier per panel suffices.
// ===========================================================================
// v (a double) of lane `lane` (wave-uniform) of the calling wave
__device__ inline double readlane_d(double v, int lane) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), lane));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// maximum of v over the 64 lanes of the wave (all lanes active), wave-uniform:
// lane exchanges inside each row of 16 lanes (quad permutations, then row
// rotations by 4 and 8), then the four row maxima through scalar registers
__device__ inline int wave_max_i32(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xF, 0xF, false));  // row_ror 4
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false));  // row_ror 8
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// exchange buffers of gj_invert: per parity, the multipliers [64 rows][4 steps]
// and the four inverse pivots (doubles), and the four pivot rows (ints)
constexpr int GJ_SHD = 2 * (4 * 64 + 4);
constexpr int GJ_SHI = 2 * 4;

template <int NB, int LD>
__device__ void gj_invert(double* a, double* sh, int* shi, int* rsrc, int* csrc, int tid) {
  static_assert(NB <= 64 && BT == 256, "one row per lane, four waves");
  constexpr int NC = 4 * ((NB + 15) / 16);  // registers per lane: column groups of 16, four per wave
  const int r = tid & 63, w = tid >> 6;
  const bool rowok = r < NB;
  double x[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c = 16 * (j >> 2) + 4 * w + (j & 3);
    x[j] = (rowok && c < NB) ? a[r * LD + c] : 0.0;
  }
  bool used = !rowok;
#pragma unroll
  for (int kp = 0; kp < NB; kp += 4) {
    const int pn = kp >> 2, wk = pn & 3, jk = 4 * (pn >> 2);  // panel, owner wave, owner's first register
    const int tt = NB - kp < 4 ? NB - kp : 4;
    double* gb = sh + (pn & 1) * (4 * 64 + 4);
    int* pb = shi + 4 * (pn & 1);
    if (w == wk) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= tt) break;
        const double xk = x[jk + t];
        // pivot: largest |x| among unused rows, compared on the upper word of its
        // bit pattern (sign, exponent, 20 mantissa bits: non-negative doubles
        // order like these integers), ties to the smallest row; the reduction is
        // on 32-bit keys and a ballot picks the row
        const int key = used ? -1 : int(uint32_t(uint64_t(__double_as_longlong(fabs(xk))) >> 32));
        const int mk = wave_max_i32(key);
        const uint64_t hit = __ballot(key == mk);
        const int p = __ffsll(static_cast<unsigned long long>(hit)) - 1;
        const double inv = 1.0 / readlane_d(xk, p);
        const double g = (r == p || !rowok) ? 0.0 : xk * inv;
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          if (t2 == t || t2 >= tt) continue;
          const double pr = readlane_d(x[jk + t2], p);
          x[jk + t2] = r == p ? x[jk + t2] * inv : fma(-g, pr, x[jk + t2]);
        }
        x[jk + t] = r == p ? inv : -g;
        gb[r * 4 + t] = g;
        if (r == p) {
          used = true;
          pb[t] = p;
          gb[256 + t] = inv;
          rsrc[kp + t] = p;
          csrc[p] = kp + t;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= tt) break;
      const int p = __builtin_amdgcn_readfirstlane(pb[t]);
      const double inv = gb[256 + t];
      const double g = gb[r * 4 + t];
      if (r == p) used = true;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int c = 16 * (j >> 2) + 4 * w + (j & 3);
        if (c >= NB || (w == wk && j >= jk && j < jk + 4)) continue;  // past the end, or the owner's panel
        const double pr = readlane_d(x[j], p);
        x[j] = r == p ? x[j] * inv : fma(-g, pr, x[j]);
      }
    }
  }
  if (rowok) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = 16 * (j >> 2) + 4 * w + (j & 3);
      if (c < NB) a[r * LD + c] = x[j];
    }
  }
  __syncthreads();
}

// out[e] = inverse of the diagonal block of element e (blk slot 0)
template <int NB>
__global__ void __launch_bounds__(BT) k_block_inverse(const double* __restrict__ blk, int nslot,
                                                      double* __restrict__ out) {
  constexpr int LD = NB + 1;
  __shared__ double a[NB * LD];
  __shared__ double sh[GJ_SHD];
  __shared__ int shi[GJ_SHI], rsrc[NB], csrc[NB];
  const int64_t e = blockIdx.x;
  const double* src = blk + e * nslot * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += BT) a[(idx / NB) * LD + idx % NB] = src[idx];
  __syncthreads();
  gj_invert<NB, LD>(a, sh, shi, rsrc, csrc, threadIdx.x);
  for (int idx = threadIdx.x; idx < NB * NB; idx += BT)
    out[e * NB * NB + idx] = a[rsrc[idx / NB] * LD + csrc[idx % NB]];
}

// ===========================================================================
// BILU(0) factorisation of the concentration field blocks (blockIdx.y picks
// the field, at block stride fstride), one hyperplane level per launch.  For
// the 2d+1-point block stencil in lexicographic order ILU(0) changes only the
// diagonal blocks: D_i = A_ii - sum_{j lower} A_ij D_j^{-1} A_ji.  Stored in
// place: slot 0 <- D_i^{-1}; slot 1+s <- D_i^{-1} A_{i,nbr(s)} for every
// neighbour (lower ones = Lhat, upper ones = Uhat), so that
//   M = D (I + Lhat)(I + Uhat).
// The level kernel forms D_i, inverts it and scales all six off-diagonal
// blocks of element i: the upper ones are read by the next levels, the lower
// ones only by element i's own Schur product, which has already run.
//
// Products of two NB x NB blocks run on a 16 x 16 thread grid: thread (ty, tx)
// owns rows ty + 16 i and columns tx + 16 j, and the operands stream through
// LDS in panels of KP columns / rows.
// ===========================================================================
template <int NB>
struct BlkGemm {
  static constexpr int RT = (NB + 15) / 16;  // rows (and columns) per thread
  static constexpr int KP = NB < 16 ? NB : 16;
  static constexpr int PLD = KP + 1;         // padded row length of the left panel
};

// acc += Lft * Rgt over all k, both operands NB x NB row-major in global memory.
// Panels are fetched into registers two ahead of their use (the panel loop is
// unrolled, so the two register buffers are addressed at compile time).
template <int NB>
__device__ inline void gemm_gg(double (&acc)[BlkGemm<NB>::RT][BlkGemm<NB>::RT], const double* __restrict__ L,
                               const double* __restrict__ Rm, double* pa, double* pb, int tid) {
  using G = BlkGemm<NB>;
  constexpr int PE = (NB * G::KP + BT - 1) / BT;  // panel elements per thread
  constexpr int NP = (NB + G::KP - 1) / G::KP;    // panels
  const int ty = tid >> 4, tx = tid & 15;
  double ra[2][PE], rb[2][PE];
  auto fetch = [&](int p, double (&xa)[PE], double (&xb)[PE]) {
    const int k0 = p * G::KP;
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int idx = tid + q * BT;
      const int r = idx / G::KP, kk = idx % G::KP;
      xa[q] = (idx < NB * G::KP && k0 + kk < NB) ? L[r * NB + k0 + kk] : 0.0;
      const int kr = idx / NB, cc = idx % NB;
      xb[q] = (idx < NB * G::KP && k0 + kr < NB) ? Rm[(k0 + kr) * NB + cc] : 0.0;
    }
  };
  fetch(0, ra[0], rb[0]);
  if (NP > 1) fetch(1, ra[1], rb[1]);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int k0 = p * G::KP;
    const int kn = (NB - k0) < G::KP ? (NB - k0) : G::KP;
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int idx = tid + q * BT;
      if (idx < NB * G::KP) {
        pa[(idx / G::KP) * G::PLD + idx % G::KP] = ra[p & 1][q];
        pb[idx] = rb[p & 1][q];
      }
    }
    __syncthreads();
    if (p + 2 < NP) fetch(p + 2, ra[p & 1], rb[p & 1]);
#pragma unroll 4
    for (int kk = 0; kk < kn; ++kk) {
      double av[G::RT], bv[G::RT];
#pragma unroll
      for (int i = 0; i < G::RT; ++i) {
        const int r = ty + 16 * i;
        av[i] = r < NB ? pa[r * G::PLD + kk] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < G::RT; ++j) {
        const int c = tx + 16 * j;
        bv[j] = c < NB ? pb[kk * NB + c] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < G::RT; ++i)
#pragma unroll
        for (int j = 0; j < G::RT; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
}

// B <- Dinv * B in place (B in global memory); Dinv[i][k] = a[rsrc[i]][csrc[k]]
// with the LDS array a of leading dimension LD
template <int NB, int LD>
__device__ inline void scale_block(double* __restrict__ B, const double* a, const int* rsrc, const int* csrc,
                                   double* pb, int tid, float* __restrict__ B32) {
  using G = BlkGemm<NB>;
  constexpr int PE = (NB * G::KP + BT - 1) / BT;
  constexpr int NP = (NB + G::KP - 1) / G::KP;
  const int ty = tid >> 4, tx = tid & 15;
  double acc[G::RT][G::RT];
#pragma unroll
  for (int i = 0; i < G::RT; ++i)
#pragma unroll
    for (int j = 0; j < G::RT; ++j) acc[i][j] = 0.0;
  int arow[G::RT];
#pragma unroll
  for (int i = 0; i < G::RT; ++i) {
    const int r = ty + 16 * i;
    arow[i] = r < NB ? rsrc[r] * LD : 0;
  }
  double rb[2][PE];
  auto fetch = [&](int p, double (&xb)[PE]) {
    const int k0 = p * G::KP;
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int idx = tid + q * BT;
      const int kr = idx / NB, cc = idx % NB;
      xb[q] = (idx < NB * G::KP && k0 + kr < NB) ? B[(k0 + kr) * NB + cc] : 0.0;
    }
  };
  fetch(0, rb[0]);
  if (NP > 1) fetch(1, rb[1]);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int k0 = p * G::KP;
    const int kn = (NB - k0) < G::KP ? (NB - k0) : G::KP;
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int idx = tid + q * BT;
      if (idx < NB * G::KP) pb[idx] = rb[p & 1][q];
    }
    __syncthreads();
    if (p + 2 < NP) fetch(p + 2, rb[p & 1]);
#pragma unroll 4
    for (int kk = 0; kk < kn; ++kk) {
      const int kc = csrc[k0 + kk];
      double av[G::RT], bv[G::RT];
#pragma unroll
      for (int i = 0; i < G::RT; ++i) {
        const int r = ty + 16 * i;
        av[i] = r < NB ? a[arow[i] + kc] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < G::RT; ++j) {
        const int c = tx + 16 * j;
        bv[j] = c < NB ? pb[kk * NB + c] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < G::RT; ++i)
#pragma unroll
        for (int j = 0; j < G::RT; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < G::RT; ++i)
#pragma unroll
    for (int j = 0; j < G::RT; ++j) {
      const int r = ty + 16 * i, c = tx + 16 * j;
      if (r < NB && c < NB) {
        B[r * NB + c] = acc[i][j];
        if (B32) B32[r * NB + c] = float(acc[i][j]);
      }
    }
}

// ---- 64-row blocks on the FP64 matrix cores ----------------------------------
// v_mfma_f64_16x16x4f64 (D = A B + C, A 16 x 4, B 4 x 16): A[i][k] sits in lane
// i + 16 k, B[k][j] in lane j + 16 k, and D[i][j] in lane j + 16 (i % 4) as
// element i / 4 of the four-double accumulator.  Wave w of the work-group owns
// the 16-row strip 16 w .. 16 w + 15 of a 64 x 64 product, as four 16 x 16
// tiles; the operands are read from global memory (L2) straight into
// registers, one 16-wide k panel ahead, so no LDS staging or barrier is needed.
typedef double v4d __attribute__((ext_vector_type(4)));

// acc += L R over the wave's strip; L, R 64 x 64 row-major
__device__ inline void gemm_mfma64(v4d (&acc)[4], const double* __restrict__ L, const double* __restrict__ R,
                                   int tid) {
  const int l = tid & 63, w = tid >> 6, li = l & 15, lk = l >> 4;
  const double* lp = L + (16 * w + li) * 64 + lk;  // A[i][k0 + 4 s + lk]
  const double* rp = R + lk * 64 + li;             // B[k0 + 4 s + lk][16 t + li]
  double ca[4], cb[4][4], na[4], nb[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ca[s] = lp[4 * s];
#pragma unroll
    for (int t = 0; t < 4; ++t) cb[s][t] = rp[(4 * s) * 64 + 16 * t];
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p + 1 < 4) {
      const int k0 = 16 * (p + 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        na[s] = lp[k0 + 4 * s];
#pragma unroll
        for (int t = 0; t < 4; ++t) nb[s][t] = rp[(k0 + 4 * s) * 64 + 16 * t];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[s], cb[s][t], acc[t], 0, 0, 0);
    if (p + 1 < 4) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ca[s] = na[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) cb[s][t] = nb[s][t];
      }
    }
  }
}

// B <- Dinv B in place (B 64 x 64 row-major in global memory), Dinv[i][k] =
// a[rsrc[i] LD + csrc[k]] in LDS.  Every wave reads all of B, so the strips are
// written only after the work-group's barrier.
template <int LD>
__device__ inline void scale_mfma64(double* __restrict__ B, const double* a, const int* rsrc, const int* csrc,
                                    int tid, float* __restrict__ B32) {
  const int l = tid & 63, w = tid >> 6, li = l & 15, lk = l >> 4;
  const int arow = rsrc[16 * w + li] * LD;
  const double* rp = B + lk * 64 + li;
  v4d acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  double cb[4][4], nb[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) cb[s][t] = rp[(4 * s) * 64 + 16 * t];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p + 1 < 4) {
      const int k0 = 16 * (p + 1);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) nb[s][t] = rp[(k0 + 4 * s) * 64 + 16 * t];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double av = a[arow + csrc[16 * p + 4 * s + lk]];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cb[s][t], acc[t], 0, 0, 0);
    }
    if (p + 1 < 4) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) cb[s][t] = nb[s][t];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = (16 * w + 4 * q + lk) * 64 + 16 * t + li;
      B[o] = acc[t][q];
      if (B32) B32[o] = float(acc[t][q]);
    }
}

// ---- 17..32-row blocks on the FP64 matrix cores (padded to 32 x 32) ----------
// Wave w owns the 16 x 16 tile (w >> 1, w & 1) of the padded product; its k
// loop runs over KS = ceil(NB / 4) steps of four, entries past NB read as 0.
template <int NB>
struct Mf32 {
  static constexpr bool on = NB > 16 && NB <= 32;
  static constexpr int KS = (NB + 3) / 4;
};

// per-lane operand lists of one padded product: A[i][4 s + lk] and B[4 s + lk][j]
template <int NB>
__device__ inline void mf32_load_a(double (&xa)[Mf32<NB>::KS], const double* __restrict__ L, int tid) {
  const int l = tid & 63, w = tid >> 6, i = 16 * (w >> 1) + (l & 15), lk = l >> 4;
#pragma unroll
  for (int s = 0; s < Mf32<NB>::KS; ++s) {
    const int k = 4 * s + lk;
    xa[s] = (L && i < NB && k < NB) ? L[i * NB + k] : 0.0;
  }
}
template <int NB>
__device__ inline void mf32_load_b(double (&xb)[Mf32<NB>::KS], const double* __restrict__ R, int tid) {
  const int l = tid & 63, w = tid >> 6, j = 16 * (w & 1) + (l & 15), lk = l >> 4;
#pragma unroll
  for (int s = 0; s < Mf32<NB>::KS; ++s) {
    const int k = 4 * s + lk;
    xb[s] = (R && j < NB && k < NB) ? R[k * NB + j] : 0.0;
  }
}
template <int NB>
__device__ inline void mf32_mma(v4d& acc, const double (&xa)[Mf32<NB>::KS], const double (&xb)[Mf32<NB>::KS]) {
#pragma unroll
  for (int s = 0; s < Mf32<NB>::KS; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], xb[s], acc, 0, 0, 0);
}
// Dinv[i][k] = a[rsrc[i] LD + csrc[k]] (LDS) as the A operand
template <int NB, int LD>
__device__ inline void mf32_load_dinv(double (&xa)[Mf32<NB>::KS], const double* a, const int* rsrc,
                                      const int* csrc, int tid) {
  const int l = tid & 63, w = tid >> 6, i = 16 * (w >> 1) + (l & 15), lk = l >> 4;
  const int arow = i < NB ? rsrc[i] * LD : 0;
#pragma unroll
  for (int s = 0; s < Mf32<NB>::KS; ++s) {
    const int k = 4 * s + lk;
    xa[s] = (i < NB && k < NB) ? a[arow + csrc[k]] : 0.0;
  }
}
// rows and columns of the lane's four accumulator entries
template <int NB>
__device__ inline void mf32_out(int tid, int q, int& rr, int& cc) {
  const int l = tid & 63, w = tid >> 6;
  rr = 16 * (w >> 1) + 4 * q + (l >> 4);
  cc = 16 * (w & 1) + (l & 15);
}

// single-precision copy of a block that is all zeros (no neighbour there)
template <int NB>
__device__ inline void zero_block32(float* f, int tid) {
  if (f)
    for (int idx = tid; idx < NB * NB; idx += BT) f[idx] = 0.0f;
}

// b32 (not null): every block the kernel finalises is also stored in single
// precision there (same layout and field stride as blk)
template <int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_factor(double* __restrict__ blk, int64_t fstride,
                                                   const int* __restrict__ nbr, const int* __restrict__ lev_elems,
                                                   int64_t first, float* __restrict__ b32) {
  using G = BlkGemm<NB>;
  constexpr int LD = NB + 1;
  constexpr int NSLOT = 2 * DIM + 1;
  __shared__ double a[NB * LD];
  __shared__ double sh[GJ_SHD];
  __shared__ int shi[GJ_SHI], rsrc[NB], csrc[NB];
  const int tid = threadIdx.x;
  blk += blockIdx.y * fstride;
  const int64_t i = lev_elems[first + blockIdx.x];
  double* bi = blk + i * NSLOT * NB * NB;
  float* fi = b32 ? b32 + blockIdx.y * fstride + i * NSLOT * NB * NB : nullptr;
  if constexpr (NB == 64) {
    // Schur complement on the matrix cores, then a = A_ii - sum
    v4d acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < 2 * DIM; s += 2) {
      const int j = nbr[i * 2 * DIM + s];
      if (j < 0) continue;
      gemm_mfma64(acc, bi + int64_t(1 + s) * NB * NB, blk + (int64_t(j) * NSLOT + 1 + (s + 1)) * NB * NB, tid);
    }
    {
      const int l = tid & 63, w = tid >> 6, li = l & 15, lk = l >> 4;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = 16 * w + 4 * q + lk, cc = 16 * t + li;
          a[rr * LD + cc] = bi[rr * NB + cc] - acc[t][q];
        }
    }
    __syncthreads();
    gj_invert<NB, LD>(a, sh, shi, rsrc, csrc, tid);
    for (int idx = tid; idx < NB * NB; idx += BT) {
      const double dv = a[rsrc[idx / NB] * LD + csrc[idx % NB]];
      bi[idx] = dv;
      if (fi) fi[idx] = float(dv);
    }
    // every off-diagonal block: the upper ones (read by later levels) and the
    // lower ones (read only by this element's Schur product above)
    for (int s = 0; s < 2 * DIM; ++s) {
      float* f32s = fi ? fi + int64_t(1 + s) * NB * NB : nullptr;
      if (nbr[i * 2 * DIM + s] < 0) {
        zero_block32<NB>(f32s, tid);
        continue;
      }
      scale_mfma64<LD>(bi + int64_t(1 + s) * NB * NB, a, rsrc, csrc, tid, f32s);
    }
  } else if constexpr (Mf32<NB>::on) {
    constexpr int KS = Mf32<NB>::KS;
    // every operand of the three Schur products and of the six block scalings
    // (upper and lower) is requested up front; the scalings' blocks wait in
    // registers through the inversion
    double la[DIM][KS], rb[DIM][KS], ub[DIM][KS], lb[DIM][KS];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int j = nbr[i * 2 * DIM + 2 * d];
      mf32_load_a<NB>(la[d], j >= 0 ? bi + int64_t(1 + 2 * d) * NB * NB : nullptr, tid);
      mf32_load_b<NB>(rb[d], j >= 0 ? blk + (int64_t(j) * NSLOT + 2 + 2 * d) * NB * NB : nullptr, tid);
      mf32_load_b<NB>(lb[d], j >= 0 ? bi + int64_t(1 + 2 * d) * NB * NB : nullptr, tid);
      const bool up = nbr[i * 2 * DIM + 2 * d + 1] >= 0;
      mf32_load_b<NB>(ub[d], up ? bi + int64_t(2 + 2 * d) * NB * NB : nullptr, tid);
    }
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) mf32_mma<NB>(acc, la[d], rb[d]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int rr, cc;
      mf32_out<NB>(tid, q, rr, cc);
      if (rr < NB && cc < NB) a[rr * LD + cc] = bi[rr * NB + cc] - acc[q];
    }
    __syncthreads();
    gj_invert<NB, LD>(a, sh, shi, rsrc, csrc, tid);
    for (int idx = tid; idx < NB * NB; idx += BT) {
      const double dv = a[rsrc[idx / NB] * LD + csrc[idx % NB]];
      bi[idx] = dv;
      if (fi) fi[idx] = float(dv);
    }
    double da[KS];
    mf32_load_dinv<NB, LD>(da, a, rsrc, csrc, tid);
    v4d ua[2 * DIM];  // slot 1 + s: s even lower, s odd upper
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      ua[2 * d] = v4d{0.0, 0.0, 0.0, 0.0};
      ua[2 * d + 1] = v4d{0.0, 0.0, 0.0, 0.0};
      mf32_mma<NB>(ua[2 * d], da, lb[d]);
      mf32_mma<NB>(ua[2 * d + 1], da, ub[d]);
    }
    __syncthreads();  // all reads of the blocks are done before any is overwritten
#pragma unroll
    for (int s = 0; s < 2 * DIM; ++s) {
      float* B32 = fi ? fi + int64_t(1 + s) * NB * NB : nullptr;
      if (nbr[i * 2 * DIM + s] < 0) {
        zero_block32<NB>(B32, tid);
        continue;
      }
      double* B = bi + int64_t(1 + s) * NB * NB;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int rr, cc;
        mf32_out<NB>(tid, q, rr, cc);
        if (rr < NB && cc < NB) {
          B[rr * NB + cc] = ua[s][q];
          if (B32) B32[rr * NB + cc] = float(ua[s][q]);
        }
      }
    }
  } else {
    __shared__ double pa[NB * G::PLD];
    __shared__ double pb[G::KP * NB];
    const int ty = tid >> 4, tx = tid & 15;
    for (int idx = tid; idx < NB * NB; idx += BT) a[(idx / NB) * LD + idx % NB] = bi[idx];
    // Schur complement of the lower neighbours (slots 0, 2, 4 = -x, -y, -z):
    // A_ij times the scaled block of j toward i (D_j^{-1} A_ji)
    double acc[G::RT][G::RT];
#pragma unroll
    for (int r = 0; r < G::RT; ++r)
#pragma unroll
      for (int c = 0; c < G::RT; ++c) acc[r][c] = 0.0;
    for (int s = 0; s < 2 * DIM; s += 2) {
      const int j = nbr[i * 2 * DIM + s];
      if (j < 0) continue;
      gemm_gg<NB>(acc, bi + int64_t(1 + s) * NB * NB, blk + (int64_t(j) * NSLOT + 1 + (s + 1)) * NB * NB, pa, pb,
                  tid);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < G::RT; ++r)
#pragma unroll
      for (int c = 0; c < G::RT; ++c) {
        const int rr = ty + 16 * r, cc = tx + 16 * c;
        if (rr < NB && cc < NB) a[rr * LD + cc] -= acc[r][c];
      }
    __syncthreads();
    gj_invert<NB, LD>(a, sh, shi, rsrc, csrc, tid);
    for (int idx = tid; idx < NB * NB; idx += BT) {
      const double dv = a[rsrc[idx / NB] * LD + csrc[idx % NB]];
      bi[idx] = dv;
      if (fi) fi[idx] = float(dv);
    }
    // every off-diagonal block (slots 1 + s: s even lower, s odd upper)
    for (int s = 0; s < 2 * DIM; ++s) {
      float* f32s = fi ? fi + int64_t(1 + s) * NB * NB : nullptr;
      if (nbr[i * 2 * DIM + s] < 0) {
        zero_block32<NB>(f32s, tid);
        continue;
      }
      scale_block<NB, LD>(bi + int64_t(1 + s) * NB * NB, a, rsrc, csrc, pb, tid, f32s);
    }
  }
}

// ===========================================================================
// Level-scheduled solves.  Four threads per block row, each handling a
// contiguous quarter of the row; partial sums combined with lane shuffles.
// ===========================================================================
// Single-precision blocks whose rows split into four 16-byte aligned parts
// (NB a multiple of 16): a lane reads its part of a row with 16-byte loads.
template <typename T, int NB>
struct VecRows {
  static constexpr bool on = std::is_same<T, float>::value && NB % 16 == 0;
};

template <typename T, int NB>
__device__ inline T row_dot4(const T* __restrict__ M, const T* x, int r, int part) {
  constexpr int QL = (NB + 3) / 4;
  T acc = T(0);
  const int c0 = part * QL;
  if constexpr (VecRows<T, NB>::on) {
    // QL a multiple of 4 floats: each lane's part of the row is 16-byte aligned
    const float4* mp = reinterpret_cast<const float4*>(M + r * NB + c0);
#pragma unroll
    for (int k = 0; k < QL / 4; ++k) {
      const float4 v = mp[k];
      acc += v.x * x[c0 + 4 * k] + v.y * x[c0 + 4 * k + 1] + v.z * x[c0 + 4 * k + 2] + v.w * x[c0 + 4 * k + 3];
    }
  } else {
#pragma unroll
    for (int c = 0; c < QL; ++c)
      if (c0 + c < NB) acc += M[r * NB + c0 + c] * x[c0 + c];
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  return acc;
}

template <typename T, int NB>
__device__ inline T col_dot4(const T* __restrict__ M, const T* x, int c, int part) {
  constexpr int QL = (NB + 3) / 4;
  T acc = T(0);
  const int r0 = part * QL;
#pragma unroll
  for (int r = 0; r < QL; ++r)
    if (r0 + r < NB) acc += M[(r0 + r) * NB + c] * x[r0 + r];
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  return acc;
}

// forward: w_i = D_i^{-1} r_i - sum_{s lower} Lhat_{i,s} w_nbr
// blockIdx.y selects one of several independent field blocks: block storage
// advances by bstride, vectors by vstride.
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_fwd(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                const int* __restrict__ lev_elems, int64_t first,
                                                const T* __restrict__ r, T* __restrict__ w, int64_t bstride,
                                                int64_t vstride) {
  constexpr int NSLOT = 2 * DIM + 1;
  blk += blockIdx.y * bstride;
  r += blockIdx.y * vstride;
  w += blockIdx.y * vstride;
  __shared__ T xs[DIM + 1][NB];
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  const int64_t i = lev_elems[first + blockIdx.x];
  int nb[DIM];
  for (int d = 0; d < DIM; ++d) nb[d] = nbr[i * 2 * DIM + 2 * d];
  for (int idx = tid; idx < NB; idx += BT) {
    xs[0][idx] = r[i * NB + idx];
    for (int d = 0; d < DIM; ++d) xs[1 + d][idx] = nb[d] >= 0 ? w[int64_t(nb[d]) * NB + idx] : T(0);
  }
  __syncthreads();
  const T* bi = blk + i * NSLOT * NB * NB;
  if (row < NB) {
    T acc = row_dot4<T, NB>(bi, xs[0], row, part);
    for (int d = 0; d < DIM; ++d)
      if (nb[d] >= 0) acc -= row_dot4<T, NB>(bi + int64_t(1 + 2 * d) * NB * NB, xs[1 + d], row, part);
    if (part == 0) w[i * NB + row] = acc;
  }
}

// backward: z_i = w_i - sum_{s upper} Uhat_{i,s} z_nbr   (z may alias w)
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_bwd(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                const int* __restrict__ lev_elems, int64_t first,
                                                const T* w, T* z, int64_t bstride, int64_t vstride) {
  constexpr int NSLOT = 2 * DIM + 1;
  blk += blockIdx.y * bstride;
  w += blockIdx.y * vstride;
  z += blockIdx.y * vstride;
  __shared__ T xs[DIM][NB];
  __shared__ T wi[NB];
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  const int64_t i = lev_elems[first + blockIdx.x];
  int nb[DIM];
  for (int d = 0; d < DIM; ++d) nb[d] = nbr[i * 2 * DIM + 2 * d + 1];
  for (int idx = tid; idx < NB; idx += BT) {
    wi[idx] = w[i * NB + idx];
    for (int d = 0; d < DIM; ++d) xs[d][idx] = nb[d] >= 0 ? z[int64_t(nb[d]) * NB + idx] : T(0);
  }
  __syncthreads();
  const T* bi = blk + i * NSLOT * NB * NB;
  if (row < NB) {
    T acc = T(0);
    for (int d = 0; d < DIM; ++d)
      if (nb[d] >= 0) acc += row_dot4<T, NB>(bi + int64_t(2 + 2 * d) * NB * NB, xs[d], row, part);
    if (part == 0) z[i * NB + row] = wi[row] - acc;
  }
}

// transposed forward: a_i = r_i - sum_{j lower} Uhat_{j->i}^T a_j
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_fwdT(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                 const int* __restrict__ lev_elems, int64_t first,
                                                 const T* __restrict__ r, T* __restrict__ aw, int64_t bstride,
                                                 int64_t vstride) {
  constexpr int NSLOT = 2 * DIM + 1;
  blk += blockIdx.y * bstride;
  r += blockIdx.y * vstride;
  aw += blockIdx.y * vstride;
  __shared__ T xs[DIM][NB];
  const int tid = threadIdx.x, col = tid >> 2, part = tid & 3;
  const int64_t i = lev_elems[first + blockIdx.x];
  int nb[DIM];
  for (int d = 0; d < DIM; ++d) nb[d] = nbr[i * 2 * DIM + 2 * d];
  for (int idx = tid; idx < NB; idx += BT)
    for (int d = 0; d < DIM; ++d) xs[d][idx] = nb[d] >= 0 ? aw[int64_t(nb[d]) * NB + idx] : T(0);
  __syncthreads();
  if (col < NB) {
    T acc = T(0);
    for (int d = 0; d < DIM; ++d)
      if (nb[d] >= 0) {
        const T* U = blk + (int64_t(nb[d]) * NSLOT + 2 + 2 * d) * NB * NB;  // nb's +d slot
        acc += col_dot4<T, NB>(U, xs[d], col, part);
      }
    if (part == 0) aw[i * NB + col] = r[i * NB + col] - acc;
  }
}

// transposed backward: b_i = a_i - sum_{j upper} Lhat_{j->i}^T b_j, z_i = D_i^{-T} b_i
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_bwdT(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                 const int* __restrict__ lev_elems, int64_t first,
                                                 T* __restrict__ bw, T* __restrict__ z, int64_t bstride,
                                                 int64_t vstride) {
  constexpr int NSLOT = 2 * DIM + 1;
  blk += blockIdx.y * bstride;
  bw += blockIdx.y * vstride;
  z += blockIdx.y * vstride;
  __shared__ T xs[DIM][NB];
  __shared__ T bi_s[NB];
  const int tid = threadIdx.x, col = tid >> 2, part = tid & 3;
  const int64_t i = lev_elems[first + blockIdx.x];
  int nb[DIM];
  for (int d = 0; d < DIM; ++d) nb[d] = nbr[i * 2 * DIM + 2 * d + 1];
  for (int idx = tid; idx < NB; idx += BT)
    for (int d = 0; d < DIM; ++d) xs[d][idx] = nb[d] >= 0 ? bw[int64_t(nb[d]) * NB + idx] : T(0);
  __syncthreads();
  if (col < NB) {
    T acc = T(0);
    for (int d = 0; d < DIM; ++d)
      if (nb[d] >= 0) {
        const T* Lm = blk + (int64_t(nb[d]) * NSLOT + 1 + 2 * d) * NB * NB;  // nb's -d slot
        acc += col_dot4<T, NB>(Lm, xs[d], col, part);
      }
    if (part == 0) {
      const T b = bw[i * NB + col] - acc;
      bw[i * NB + col] = b;
      bi_s[col] = b;
    }
  }
  __syncthreads();
  if (col < NB) {
    const T v = col_dot4<T, NB>(blk + i * NSLOT * NB * NB, bi_s, col, part);
    if (part == 0) z[i * NB + col] = v;
  }
}

// ===========================================================================
// Block sparse products.  y_i = alpha * sum_s A_{i,s} x_{nbr(s)} + beta * b_i
// ===========================================================================
// Potential-block kernels (block sparse product, block-diagonal apply, fused
// Chebyshev step) read the potential block and its inverse diagonal blocks.
// In single precision, blocks of up to 32 rows are stored with every row
// padded to LD = a multiple of four floats (zeros in the padding), so that a
// lane reads four consecutive entries of a row with one 16-byte load and a
// work-group's loads cover whole cache lines; eight lanes share a row (lanes
// with part >= LD / 4 hold zeros).  Double precision and larger blocks keep
// unpadded rows (LD = NB) and four lanes per row.
template <typename T, int NB>
struct PotRows {
  static constexpr bool VEC = std::is_same<T, float>::value && NB <= 32;
  static constexpr int LD = VEC ? ((NB + 3) & ~3) : NB;
  static constexpr int QV = LD / 4;
  // single-precision rows take 8 lanes each; blocks of up to 8 (16) rows
  // share a work-group four (two) at a time, 64 (128) lanes per element
  static constexpr int EPB = VEC ? (NB <= 8 ? 4 : (NB <= 16 ? 2 : 1)) : 1;
};

__device__ inline float dot4(const float4& a, const float4& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}
__device__ inline float sum8(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}
__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_bspmv(const T* __restrict__ blk, const int* __restrict__ nbr,
                                              const T* __restrict__ x, const T* __restrict__ b, T alpha,
                                              T beta, T* __restrict__ y, int64_t bstride, int64_t vstride,
                                              int64_t E) {
  constexpr int NSLOT = 2 * DIM + 1;
  using PR = PotRows<T, NB>;
  const int tid = threadIdx.x;
  // blockIdx.y: one of several independent systems at block / vector strides
  blk += blockIdx.y * bstride;
  x += blockIdx.y * vstride;
  if (b) b += blockIdx.y * vstride;
  y += blockIdx.y * vstride;
  if constexpr (PR::VEC) {
    constexpr int LD = PR::LD, QV = PR::QV, EPB = PR::EPB, TPE = BT / EPB;
    __shared__ __align__(16) float xv[EPB][NSLOT][LD];
    const int el = tid / TPE, lt = tid % TPE;  // element of the group, lane within it
    const int64_t i = int64_t(blockIdx.x) * EPB + el;
    const bool live = i < E;
    const int row = lt >> 3, part = lt & 7;
    const bool on = live && row < NB && part < QV;
    const float* bi = blk + i * NSLOT * NB * LD + row * LD + 4 * part;
    float4 mr[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) mr[s] = on ? ld4(bi + s * NB * LD) : make_float4(0.f, 0.f, 0.f, 0.f);
    int nb[NSLOT];
    nb[0] = live ? int(i) : -1;
    for (int s = 0; s < 2 * DIM; ++s) nb[1 + s] = live ? nbr[i * 2 * DIM + s] : -1;
    for (int idx = lt; idx < NSLOT * LD; idx += TPE) {
      const int sl = idx / LD, c = idx - sl * LD;
      xv[el][sl][c] = (c < NB && nb[sl] >= 0) ? x[int64_t(nb[sl]) * NB + c] : 0.f;
    }
    __syncthreads();
    float acc = 0.f;
    if (on) {
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
        if (nb[s] >= 0) acc += dot4(mr[s], ld4(&xv[el][s][4 * part]));
    }
    acc = sum8(acc);
    if (live && row < NB && part == 0) y[i * NB + row] = alpha * acc + (b ? beta * b[i * NB + row] : 0.f);
  } else {
    const int64_t i = blockIdx.x;
    __shared__ T xs[NSLOT][NB];
    const int row = tid >> 2, part = tid & 3;
    int nb[NSLOT];
    nb[0] = int(i);
    for (int s = 0; s < 2 * DIM; ++s) nb[1 + s] = nbr[i * 2 * DIM + s];
    for (int idx = tid; idx < NB; idx += BT)
      for (int s = 0; s < NSLOT; ++s) xs[s][idx] = nb[s] >= 0 ? x[int64_t(nb[s]) * NB + idx] : T(0);
    __syncthreads();
    const T* bi = blk + i * NSLOT * NB * NB;
    if (row < NB) {
      T acc = T(0);
      for (int s = 0; s < NSLOT; ++s)
        if (nb[s] >= 0) acc += row_dot4<T, NB>(bi + int64_t(s) * NB * NB, xs[s], row, part);
      if (part == 0) y[i * NB + row] = alpha * acc + (b ? beta * b[i * NB + row] : T(0));
    }
  }
}

// y_i = Dinv_i x_i
template <typename T, int NB>
__global__ void __launch_bounds__(BT) k_bdiag(const T* __restrict__ dinv, const T* __restrict__ x,
                                              T* __restrict__ y) {
  using PR = PotRows<T, NB>;
  const int tid = threadIdx.x;
  const int64_t i = blockIdx.x;
  if constexpr (PR::VEC) {
    constexpr int LD = PR::LD, QV = PR::QV;
    __shared__ __align__(16) float xv[LD];
    const int row = tid >> 3, part = tid & 7;
    const bool on = row < NB && part < QV;
    const float4 dr = on ? ld4(dinv + (i * NB + row) * LD + 4 * part) : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int idx = tid; idx < LD; idx += BT) xv[idx] = idx < NB ? x[i * NB + idx] : 0.f;
    __syncthreads();
    const float v = sum8(on ? dot4(dr, ld4(&xv[4 * part])) : 0.f);
    if (row < NB && part == 0) y[i * NB + row] = v;
  } else {
    __shared__ T xs[NB];
    const int row = tid >> 2, part = tid & 3;
    for (int idx = tid; idx < NB; idx += BT) xs[idx] = x[i * NB + idx];
    __syncthreads();
    if (row < NB) {
      const T v = row_dot4<T, NB>(dinv + i * NB * NB, xs, row, part);
      if (part == 0) y[i * NB + row] = v;
    }
  }
}

// ===========================================================================
// Q1 vertex space.  Vertex (vx, vy, vz) of the (n+1)^d grid; element e owns
// vertices (ix + ox, iy + oy, iz + oz), o in {0,1}^d, with trilinear shape
// N_o(xi) = prod_d (o_d ? (1 + xi_d) : (1 - xi_d)) / 2 at the GLL nodes.
// ===========================================================================
__constant__ double c_gll[3][4];

void upload_gll_nodes(const RefTables* tabs, int count) {
  double h[3][4] = {};
  for (int i = 0; i < count; ++i)
    for (int a = 0; a < tabs[i].nn; ++a) h[tabs[i].p - 1][a] = tabs[i].xn[a];
  DGNP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gll), h, sizeof(h)));
}

template <int DIM, int P>
__device__ inline double q1_shape(int node, int o) {
  constexpr int NN = P + 1;
  int ic[3] = {node % NN, (node / NN) % NN, node / (NN * NN)};
  double t = 1.0;
  for (int d = 0; d < DIM; ++d) {
    const double xi = c_gll[P - 1][ic[d]];
    t *= ((o >> d) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);
  }
  return t;
}

__device__ inline int64_t vert_id(const int* n, int dim, const int* eid, int o) {
  int64_t v = 0, st = 1;
  for (int d = 0; d < dim; ++d) {
    v += (eid[d] + ((o >> d) & 1)) * st;
    st *= (n[d] + 1);
  }
  return v;
}

// x_dg[e][node] = beta * x_dg + sum_o N_o(node) xv[vertex(e, o)]
template <typename T, int DIM, int P>
__global__ void k_q1_prolong(int3 n3, const T* __restrict__ xv, T* __restrict__ xdg, T beta, int64_t E) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  const int64_t gid = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (gid >= E * NB) return;
  const int64_t e = gid / NB;
  const int node = int(gid % NB);
  int n[3] = {n3.x, n3.y, n3.z};
  int eid[3] = {int(e % n[0]), int((e / n[0]) % n[1]), DIM == 3 ? int(e / (int64_t(n[0]) * n[1])) : 0};
  double acc = 0.0;
  for (int o = 0; o < (1 << DIM); ++o) acc += q1_shape<DIM, P>(node, o) * double(xv[vert_id(n, DIM, eid, o)]);
  xdg[gid] = T(acc) + (beta != T(0) ? beta * xdg[gid] : T(0));
}

// rv[v] = sum over elements e containing v of sum_node N_{o(e,v)}(node) r[e][node]
// 2^DIM lanes per vertex: lane o takes the element of which v is corner o and
// contracts its nodal values with the corner's trilinear shape one direction
// at a time; the lanes' sums are combined by shuffles (a fixed order).
template <typename T, int DIM, int P>
__global__ void k_q1_restrict(int3 n3, const T* __restrict__ r, T* __restrict__ rv, int64_t nvert,
                              const T* __restrict__ dinv, T c1, T* __restrict__ d1) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t v = t / NV;
  const int o = int(t % NV);
  if (v >= nvert) return;  // whole groups of NV lanes leave together
  const int n[3] = {n3.x, n3.y, n3.z};
  const int vc[3] = {int(v % (n[0] + 1)), int((v / (n[0] + 1)) % (n[1] + 1)),
                     DIM == 3 ? int(v / (int64_t(n[0] + 1) * (n[1] + 1))) : 0};
  int eid[3] = {0, 0, 0};
  bool ok = true;
  for (int d = 0; d < DIM; ++d) {
    eid[d] = vc[d] - ((o >> d) & 1);
    if (eid[d] < 0 || eid[d] >= n[d]) ok = false;
  }
  double acc = 0.0;
  if (ok) {
    const int64_t e = eid[0] + int64_t(n[0]) * (eid[1] + int64_t(n[1]) * eid[2]);
    double phi[3][NN];
    for (int d = 0; d < 3; ++d)
      for (int i = 0; i < NN; ++i) {
        const double xi = c_gll[P - 1][i];
        phi[d][i] = ((o >> d) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);
      }
    const T* re = r + e * NB;
    constexpr int NK = DIM == 3 ? NN : 1;
    for (int k = 0; k < NK; ++k) {
      double sj = 0.0;
      for (int j = 0; j < NN; ++j) {
        double si = 0.0;
#pragma unroll
        for (int i = 0; i < NN; ++i) si += phi[0][i] * double(re[(k * NN + j) * NN + i]);
        sj += phi[1][j] * si;
      }
      acc += (DIM == 3 ? phi[2][k] : 1.0) * sj;
    }
  }
#pragma unroll
  for (int m = 1; m < NV; m <<= 1) acc += __shfl_xor(acc, m, 64);
  if (o == 0) {
    const T rvv = T(acc);
    rv[v] = rvv;
    // first Chebyshev step of the vertex level from a zero guess, as the CSR
    // smoother computes it: d_1 = c1 (D^{-1} r)
    if (d1) d1[v] = c1 * (dinv[v] * rvv);
  }
}

// ---------------------------------------------------------------------------
// p-multigrid transfers between the order-p DG space and the p = 1 DG space on
// the same mesh: element by element, the p = 1 function (values at the 2^d
// corners) is interpolated at the order-p GLL nodes (prolongation), and the
// restriction is its transpose.
// ---------------------------------------------------------------------------
// x1[f][e][o] = x[f][e][corner node o]  (m fields; the GLL nodes include the corners)
template <int DIM, int P>
__global__ void k_p1_inject(const double* __restrict__ x, double* __restrict__ x1, int m, int64_t E) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= int64_t(m) * E * NV) return;
  const int o = int(t % NV);
  const int64_t fe = t / NV;  // f * E + e
  int node = 0, st = 1;
  for (int d = 0; d < DIM; ++d) {
    node += ((o >> d) & 1) * P * st;
    st *= NN;
  }
  x1[t] = x[fe * NB + node];
}

// xp[e][node] = sum_o N_o(node) x1[e][o] + beta xp[e][node]   (one thread per node)
template <typename T, int DIM, int P>
__global__ void k_p1_prolong(const T* __restrict__ x1, T* __restrict__ xp, T beta, int64_t E) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  const int64_t gid = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (gid >= E * NB) return;
  const int64_t e = gid / NB;
  const int node = int(gid % NB);
  double acc = 0.0;
#pragma unroll
  for (int o = 0; o < NV; ++o) acc += q1_shape<DIM, P>(node, o) * double(x1[e * NV + o]);
  xp[gid] = T(acc) + (beta != T(0) ? beta * xp[gid] : T(0));
}

// r1[e][o] = sum_node N_o(node) (rp[e][node] - sub[e][node])   (sub may be null);
// one thread per (element, corner), contracted one direction at a time
template <typename T, int DIM, int P>
__global__ void k_p1_restrict(const T* __restrict__ rp, const T* __restrict__ sub, T* __restrict__ r1, int64_t E) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= E * NV) return;
  const int64_t e = t / NV;
  const int o = int(t % NV);
  double phi[3][NN];
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < NN; ++i) {
      const double xi = c_gll[P - 1][i];
      phi[d][i] = ((o >> d) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);
    }
  const T* re = rp + e * NB;
  const T* se = sub ? sub + e * NB : nullptr;
  constexpr int NK = DIM == 3 ? NN : 1;
  double acc = 0.0;
  for (int k = 0; k < NK; ++k) {
    double sj = 0.0;
    for (int j = 0; j < NN; ++j) {
      double si = 0.0;
#pragma unroll
      for (int i = 0; i < NN; ++i) {
        const int node = (k * NN + j) * NN + i;
        si += phi[0][i] * (double(re[node]) - (se ? double(se[node]) : 0.0));
      }
      sj += phi[1][j] * si;
    }
    acc += (DIM == 3 ? phi[2][k] : 1.0) * sj;
  }
  r1[t] = T(acc);
}

// gal[e][s][u][v] = sum_ij N_u(i) A_{e,s}[i][j] N_v(j)   (s = 0 diag, 1 + slot).
// The rows are contracted first: lane t of the G = BT / NB row groups owns
// column j = t mod NB and the rows g, g + G, ... of its group g = t / NB, so
// every load instruction of a wave reads consecutive entries of the block
// (address t + NB G r); the groups' partial sums W_g[u][j] are added in group
// order, then gal = W N.
template <int DIM, int P>
__global__ void __launch_bounds__(BT) k_q1_galerkin(const double* __restrict__ blk, double* __restrict__ gal) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  constexpr int NSLOT = 2 * DIM + 1;
  constexpr int G = BT / NB;  // row groups
  static_assert(G >= 1, "one row group at least");
  __shared__ double sN[NB <= 8 ? 1 : NB * NV];
  __shared__ double Wg[NB <= 8 ? 1 : G * NV * NB];
  __shared__ double W[NV * NB];
  const int64_t e = blockIdx.x;
  const int s = blockIdx.y;
  const int t = threadIdx.x;
  const double* A = blk + (e * NSLOT + s) * NB * NB;
  if constexpr (NB <= 8) {
    // blocks of at most 8 rows: T = A N straight from the block, then N^T T
    // (the row groups would be mostly empty)
    for (int idx = t; idx < NB * NV; idx += BT) {
      const int i = idx / NV, v = idx % NV;
      double acc = 0.0;
      for (int j = 0; j < NB; ++j) acc += A[i * NB + j] * q1_shape<DIM, P>(j, v);
      W[idx] = acc;
    }
    __syncthreads();
    for (int idx = t; idx < NV * NV; idx += BT) {
      const int u = idx / NV, v = idx % NV;
      double acc = 0.0;
      for (int i = 0; i < NB; ++i) acc += q1_shape<DIM, P>(i, u) * W[i * NV + v];
      gal[(e * NSLOT + s) * NV * NV + idx] = acc;
    }
    return;
  }
  for (int idx = t; idx < NB * NV; idx += BT) sN[idx] = q1_shape<DIM, P>(idx / NV, idx % NV);
  __syncthreads();
  if (t < G * NB) {
    const int j = t % NB, g = t / NB;
    double w[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) w[u] = 0.0;
    for (int i = g; i < NB; i += G) {
      const double a = A[i * NB + j];
#pragma unroll
      for (int u = 0; u < NV; ++u) w[u] += sN[i * NV + u] * a;
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) Wg[(g * NV + u) * NB + j] = w[u];
  }
  __syncthreads();
  for (int idx = t; idx < NV * NB; idx += BT) {
    double w = 0.0;
    for (int g = 0; g < G; ++g) w += Wg[g * NV * NB + idx];
    W[idx] = w;
  }
  __syncthreads();
  for (int idx = t; idx < NV * NV; idx += BT) {
    const int u = idx / NV, v = idx % NV;
    double acc = 0.0;
    for (int j = 0; j < NB; ++j) acc += W[u * NB + j] * sN[j * NV + v];
    gal[(e * NSLOT + s) * NV * NV + idx] = acc;
  }
}

// ===========================================================================
// Dataflow (sync-free) forward / backward BILU(0) sweeps.  One launch per
// sweep instead of one per hyperplane level: the grid is small enough to be
// resident on the device at once, work-group b takes the elements b, b + G,
// b + 2G, ... of the level order (reversed for the backward sweep), and an
// element waits only for the neighbours it reads.  Every exchanged vector
// entry travels together with its sweep count in 64-bit words (count high,
// 32 value bits low: one word per single-precision entry, two per double, the
// low half of the double first), written and read with device-scope relaxed
// atomics.  A consumer polls each word it needs until the word carries the
// sweep's count; since a word is written and read whole, the value bits it
// holds are the ones published with that count, and no ordering between
// different words (no counter, no fence, no wait for store completion) is
// needed.  An element that has completed s sweeps expects count s + 1, so no
// reset is needed between sweeps (and a captured graph can replay them).  The
// plain result is also written to `out` for the kernels that follow.  The
// residency of the whole grid makes the schedule deadlock-free (the least
// unfinished element always has its inputs); a wait that exceeds its spin
// limit sets *err and ends the work-group, so the sweep cannot hang.  Once
// *err is set, every other wait of the sweep ends at its next look at the flag
// and every later sweep returns at entry; a work-group that ends early writes
// NaN into the rows of the element it was about to compute (it is their only
// writer), so the failure reaches the Krylov coefficients as a non-finite
// value and the host reports it at once.
// ===========================================================================
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a wait gives up after spin_limit polls, or earlier when another work-group
// has already given up (the flag is looked at every 64 polls)
__device__ __forceinline__ bool df_give_up(int spins, int spin_limit, const int* err) {
  return spins > spin_limit || ((spins & 63) == 0 && ld_dev(err) != 0);
}

// the rows of element i of an ended sweep: NaN (one writer per element)
template <typename T, int NB>
__device__ __forceinline__ void df_poison(T* out, int64_t i, int tid) {
  for (int idx = tid; idx < NB; idx += BT) st_dev(out + i * NB + idx, T(__builtin_nan("")));
}

// true (in every thread) when an earlier wait of this or another sweep gave up
__device__ __forceinline__ bool df_failed(const int* err, int* s_abort, int tid) {
  if (tid == 0) *s_abort = ld_dev(err) != 0;
  __syncthreads();
  return *s_abort != 0;
}

// packed words per vector entry
template <typename T>
struct DfWords;
template <>
struct DfWords<float> {
  static constexpr int W = 1;
  __device__ static unsigned half(float v, int) { return __float_as_uint(v); }
  __device__ static float join(const unsigned* h) { return __uint_as_float(h[0]); }
};
template <>
struct DfWords<double> {
  static constexpr int W = 2;
  __device__ static unsigned half(double v, int k) {
    const uint64_t b = uint64_t(__double_as_longlong(v));
    return unsigned(k == 0 ? b : b >> 32);
  }
  __device__ static double join(const unsigned* h) {
    return __longlong_as_double((long long)((uint64_t(h[1]) << 32) | uint64_t(h[0])));
  }
};

// publish entry `e` (word index e * W) with sweep count `target`
template <typename T>
__device__ __forceinline__ void df_publish(uint64_t* wp, int64_t e, unsigned target, T v) {
  constexpr int W = DfWords<T>::W;
#pragma unroll
  for (int k = 0; k < W; ++k) st_dev(wp + e * W + k, (uint64_t(target) << 32) | uint64_t(DfWords<T>::half(v, k)));
}

// the sweep count published with entry e (its first word)
template <typename T>
__device__ __forceinline__ unsigned df_count(const uint64_t* wp, int64_t e) {
  return unsigned(ld_dev(wp + e * DfWords<T>::W) >> 32);
}

// poll entry e until every word of it carries `target`; false when the wait
// gave up (then *err is set)
template <typename T, int SLEEP>
__device__ __forceinline__ bool df_fetch(const uint64_t* wp, int64_t e, unsigned target, int spin_limit, int* err,
                                         T* v) {
  constexpr int W = DfWords<T>::W;
  unsigned h[W];
  int spins = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const uint64_t* src = wp + e * W + k;
    uint64_t word = ld_dev(src);
    while (unsigned(word >> 32) != target) {
      if (df_give_up(++spins, spin_limit, err)) {
        st_dev(err, 1);
        return false;
      }
      __builtin_amdgcn_s_sleep(SLEEP);
      word = ld_dev(src);
    }
    h[k] = unsigned(word);
  }
  *v = DfWords<T>::join(h);
  return true;
}

// kind 0 (forward): w_i = D_i^{-1} r_i - sum_{s lower} Lhat_{i,s} w_nbr
// kind 1 (backward): z_i = w_i - sum_{s upper} Uhat_{i,s} z_nbr   (z may alias w)
template <typename T, int NB, int DIM, int KIND>
__global__ void __launch_bounds__(BT) k_ilu_dfp(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                const int* __restrict__ order, int64_t E, const T* in, T* out,
                                                int64_t bstride, int64_t vstride, uint64_t* wp, int* err,
                                                int spin_limit) {
  constexpr int NSLOT = 2 * DIM + 1;
  constexpr int QL = (NB + 3) / 4;
  blk += blockIdx.y * bstride;
  in += blockIdx.y * vstride;
  out += blockIdx.y * vstride;
  wp += blockIdx.y * vstride * DfWords<T>::W;
  __shared__ T xs[DIM + 1][NB];
  __shared__ int s_nb[DIM];
  __shared__ int s_abort;
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  if (df_failed(err, &s_abort, tid)) {
    if (int64_t(blockIdx.x) < E) df_poison<T, NB>(out, order[KIND == 0 ? blockIdx.x : E - 1 - blockIdx.x], tid);
    return;
  }
  for (int64_t t = blockIdx.x; t < E; t += gridDim.x) {
    const int64_t i = order[KIND == 0 ? t : E - 1 - t];
    if (tid < DIM) s_nb[tid] = nbr[i * 2 * DIM + 2 * tid + KIND];
    // the element's own block rows do not depend on the neighbours: fetch them first
    const T* bi = blk + i * NSLOT * NB * NB;
    T m[DIM + 1][QL];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
      const int slot = KIND == 0 ? (b == 0 ? 0 : 1 + 2 * (b - 1)) : (b == 0 ? 0 : 2 + 2 * (b - 1));
#pragma unroll
      for (int c = 0; c < QL; ++c) {
        const int cc = part * QL + c;
        m[b][c] = (row < NB && cc < NB && (KIND == 0 || b > 0)) ? bi[int64_t(slot) * NB * NB + row * NB + cc]
                                                                  : T(0);
      }
    }
    for (int idx = tid; idx < NB; idx += BT) xs[0][idx] = in[i * NB + idx];
    const unsigned target = df_count<T>(wp, i * NB) + 1u;
    __syncthreads();
    for (int idx = tid; idx < DIM * NB; idx += BT) {
      const int d = idx / NB, l = idx % NB;
      const int j = s_nb[d];
      T v = T(0);
      if (j >= 0 && !df_fetch<T, 1>(wp, int64_t(j) * NB + l, target, spin_limit, err, &v)) s_abort = 1;
      xs[1 + d][l] = v;
    }
    __syncthreads();
    if (s_abort) {
      df_poison<T, NB>(out, i, tid);
      return;
    }
    if (row < NB) {
      T acc = T(0);
      if constexpr (KIND == 0) {
#pragma unroll
        for (int c = 0; c < QL; ++c) acc += m[0][c] * xs[0][part * QL + c < NB ? part * QL + c : 0];
      }
#pragma unroll
      for (int b = 1; b <= DIM; ++b) {
        T sb = T(0);
#pragma unroll
        for (int c = 0; c < QL; ++c) sb += m[b][c] * xs[b][part * QL + c < NB ? part * QL + c : 0];
        acc -= sb;
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (KIND == 1) acc = xs[0][row] + acc;
      if (part == 0) {
        df_publish<T>(wp, i * NB + row, target, acc);
        out[i * NB + row] = acc;
      }
    }
    __syncthreads();
  }
}

// Line variant of the single-precision dataflow sweeps: a work-group walks a
// line of elements along axis ax in the sweep's direction, so the neighbour
// along the line is the element it has just computed (kept in LDS) and only
// the neighbours across lines are polled.  Lines are ordered by the level of
// their first element, work-group b takes lines b, b + G, ... (reversed for
// the backward sweep), which keeps the schedule deadlock-free on a resident
// grid as for the element variant.  The block rows of the next element are
// fetched while the current element waits for its neighbours and computes.
// line_first: first element of each line (lowest coordinate along ax); the
// line's elements are line_first + p * lstride, p = 0 .. len - 1.
template <int NB, int DIM, int KIND>
__global__ void __launch_bounds__(BT) k_ilu_dfl(const float* __restrict__ blk, const int* __restrict__ nbr,
                                                const int* __restrict__ line_first, int nline, int len,
                                                int64_t lstride, int ax, const float* in, float* out,
                                                int64_t bstride, int64_t vstride, uint64_t* wp, int* err,
                                                int spin_limit) {
  constexpr int NSLOT = 2 * DIM + 1;
  constexpr int QL = (NB + 3) / 4;
  blk += blockIdx.y * bstride;
  in += blockIdx.y * vstride;
  out += blockIdx.y * vstride;
  wp += blockIdx.y * vstride;
  __shared__ float xs[DIM + 1][NB];  // [0]: own input; [1 + d]: neighbour across direction d
  __shared__ int s_abort;
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  if (df_failed(err, &s_abort, tid)) {
    if (int(blockIdx.x) < nline) {
      const int64_t first = line_first[KIND == 0 ? blockIdx.x : nline - 1 - blockIdx.x];
      df_poison<float, NB>(out, KIND == 0 ? first : first + int64_t(len - 1) * lstride, tid);
    }
    return;
  }
  // rows of the element's own blocks that the sweep reads: D^{-1} and the
  // lower blocks (forward) or the upper blocks (backward)
  auto fetch = [&](int64_t e, float (&m)[DIM + 1][QL]) {
    const float* be = blk + e * NSLOT * NB * NB;
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
      const int slot = KIND == 0 ? (b == 0 ? 0 : 1 + 2 * (b - 1)) : (b == 0 ? 0 : 2 + 2 * (b - 1));
      if constexpr (VecRows<float, NB>::on) {
        const float4* mp = reinterpret_cast<const float4*>(be + int64_t(slot) * NB * NB + row * NB + part * QL);
#pragma unroll
        for (int k = 0; k < QL / 4; ++k) {
          const float4 v = (row < NB && (KIND == 0 || b > 0)) ? mp[k] : make_float4(0.f, 0.f, 0.f, 0.f);
          m[b][4 * k] = v.x;
          m[b][4 * k + 1] = v.y;
          m[b][4 * k + 2] = v.z;
          m[b][4 * k + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int c = 0; c < QL; ++c) {
          const int cc = part * QL + c;
          m[b][c] = (row < NB && cc < NB && (KIND == 0 || b > 0)) ? be[int64_t(slot) * NB * NB + row * NB + cc]
                                                                    : 0.0f;
        }
      }
    }
  };
  for (int c = blockIdx.x; c < nline; c += gridDim.x) {
    const int64_t first = line_first[KIND == 0 ? c : nline - 1 - c];
    const int64_t step = KIND == 0 ? lstride : -lstride;
    const int64_t start = KIND == 0 ? first : first + int64_t(len - 1) * lstride;
    // blocks of up to 32 rows: the next element's rows are fetched while the
    // current one waits; 64-row blocks are fetched in place, which keeps the
    // registers for more resident lines
    constexpr bool PF = NB <= 32;
    float m[DIM + 1][QL], mn[PF ? DIM + 1 : 1][PF ? QL : 1];
    if constexpr (PF) fetch(start, m);
    for (int q = 0; q < len; ++q) {
      const int64_t i = start + q * step;
      if constexpr (PF) {
        if (q + 1 < len) fetch(i + step, mn);
      } else {
        fetch(i, m);
      }
      for (int idx = tid; idx < NB; idx += BT) xs[0][idx] = in[i * NB + idx];
      const unsigned target = unsigned(ld_dev(wp + i * NB) >> 32) + 1u;
      for (int idx = tid; idx < DIM * NB; idx += BT) {
        const int d = idx / NB, l = idx % NB;
        if (d == ax) {
          if (q == 0) xs[1 + d][l] = 0.0f;  // the line starts at the domain boundary
          continue;                          // otherwise: the previous element's result
        }
        const int j = nbr[i * 2 * DIM + 2 * d + KIND];
        float v = 0.0f;
        if (j >= 0) {
          const uint64_t* src = wp + int64_t(j) * NB + l;
          uint64_t word = ld_dev(src);
          int spins = 0;
          while (unsigned(word >> 32) != target) {
            if (df_give_up(++spins, spin_limit, err)) {
              st_dev(err, 1);
              s_abort = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            word = ld_dev(src);
          }
          v = __uint_as_float(unsigned(word));
        }
        xs[1 + d][l] = v;
      }
      __syncthreads();
      if (s_abort) {
        df_poison<float, NB>(out, i, tid);
        return;
      }
      float acc = 0.0f;
      if (row < NB) {
        if constexpr (KIND == 0) {
#pragma unroll
          for (int cq = 0; cq < QL; ++cq) acc += m[0][cq] * xs[0][part * QL + cq < NB ? part * QL + cq : 0];
        }
#pragma unroll
        for (int b = 1; b <= DIM; ++b) {
          float sb = 0.0f;
#pragma unroll
          for (int cq = 0; cq < QL; ++cq) sb += m[b][cq] * xs[b][part * QL + cq < NB ? part * QL + cq : 0];
          acc -= sb;
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (KIND == 1) acc = xs[0][row] + acc;
      }
      __syncthreads();  // every read of xs is done before the next element's inputs land there
      if (row < NB && part == 0) {
        st_dev(wp + i * NB + row, (uint64_t(target) << 32) | uint64_t(__float_as_uint(acc)));
        out[i * NB + row] = acc;
        xs[1 + ax][row] = acc;
      }
      if constexpr (PF) {
#pragma unroll
        for (int b = 0; b <= DIM; ++b)
#pragma unroll
          for (int cq = 0; cq < QL; ++cq) m[b][cq] = mn[b][cq];
      }
    }
    __syncthreads();  // the last result of the line is in xs before the next line clears it
  }
}

// ===========================================================================
// host launchers
// ===========================================================================
template <int NB>
static void inv_t(int64_t E, const double* blk, int nslot, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_block_inverse<NB>, dim3(unsigned(E)), dim3(BT), 0, s, blk, nslot, out);
}

void launch_block_inverse(int nb, int64_t E, const double* blk, int nslot, double* out, hipStream_t s) {
  if (E == 0) return;
  switch (nb) {
    case 4: inv_t<4>(E, blk, nslot, out, s); break;
    case 9: inv_t<9>(E, blk, nslot, out, s); break;
    case 16: inv_t<16>(E, blk, nslot, out, s); break;
    case 8: inv_t<8>(E, blk, nslot, out, s); break;
    case 27: inv_t<27>(E, blk, nslot, out, s); break;
    case 64: inv_t<64>(E, blk, nslot, out, s); break;
    default: throw Error(DGNP_E_ARG, "unsupported block size");
  }
  DGNP_HIP(hipGetLastError());
}

template <int NB, int DIM>
static void fac_t(int nfields, int64_t fstride, double* blk, const int* nbr, const int* lev, int64_t first,
                  int64_t count, float* b32, hipStream_t s) {
  hipLaunchKernelGGL((k_ilu_factor<NB, DIM>), dim3(unsigned(count), unsigned(nfields)), dim3(BT), 0, s, blk,
                     fstride, nbr, lev, first, b32);
}

static void fac_dispatch(int nb, int dim, int nfields, int64_t fstride, double* blk, const int* nbr,
                         const int* lev, int64_t first, int64_t count, float* b32, hipStream_t s) {
  if (dim == 3) {
    switch (nb) {
      case 8: fac_t<8, 3>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      case 27: fac_t<27, 3>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      case 64: fac_t<64, 3>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: fac_t<4, 2>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      case 9: fac_t<9, 2>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      case 16: fac_t<16, 2>(nfields, fstride, blk, nbr, lev, first, count, b32, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}

void launch_ilu_factor(int nb, int dim, int nfields, int64_t fstride, double* blk, const int* nbr,
                       const int* lev, int64_t first, int64_t count, hipStream_t s, float* b32) {
  if (count == 0 || nfields == 0) return;
  fac_dispatch(nb, dim, nfields, fstride, blk, nbr, lev, first, count, b32, s);
}


template <typename T, int NB, int DIM>
static void solve_t(int kind, const T* blk, const int* nbr, const int* lev, int64_t first, int64_t count,
                    int nfields, int64_t bstride, int64_t vstride, const T* in, T* out, T* aux, hipStream_t s) {
  const dim3 g = dim3(unsigned(count), unsigned(nfields)), b = dim3(BT);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL((k_ilu_fwd<T, NB, DIM>), g, b, 0, s, blk, nbr, lev, first, in, out, bstride, vstride);
      break;
    case 1:
      hipLaunchKernelGGL((k_ilu_bwd<T, NB, DIM>), g, b, 0, s, blk, nbr, lev, first, in, out, bstride, vstride);
      break;
    case 2:
      hipLaunchKernelGGL((k_ilu_fwdT<T, NB, DIM>), g, b, 0, s, blk, nbr, lev, first, in, out, bstride, vstride);
      break;
    case 3:
      hipLaunchKernelGGL((k_ilu_bwdT<T, NB, DIM>), g, b, 0, s, blk, nbr, lev, first, aux, out, bstride, vstride);
      break;
  }
}

template <typename T>
void launch_ilu_solve(int kind, int nb, int dim, const T* blk, const int* nbr, const int* lev, int64_t first,
                      int64_t count, int nfields, int64_t bstride, int64_t vstride, const T* in, T* out, T* aux,
                      hipStream_t s) {
  if (count == 0 || nfields == 0) return;
  if (dim == 3) {
    switch (nb) {
      case 8: solve_t<T, 8, 3>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      case 27: solve_t<T, 27, 3>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      case 64: solve_t<T, 64, 3>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: solve_t<T, 4, 2>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      case 9: solve_t<T, 9, 2>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      case 16: solve_t<T, 16, 2>(kind, blk, nbr, lev, first, count, nfields, bstride, vstride, in, out, aux, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_ilu_solve<double>(int, int, int, const double*, const int*, const int*, int64_t, int64_t, int,
                                       int64_t, int64_t, const double*, double*, double*, hipStream_t);
template void launch_ilu_solve<float>(int, int, int, const float*, const int*, const int*, int64_t, int64_t, int,
                                      int64_t, int64_t, const float*, float*, float*, hipStream_t);

template <typename T, int NB, int DIM>
static void bsp_t(int64_t E, const T* blk, const int* nbr, const T* x, const T* b, T alpha, T beta, T* y,
                  int nsys, int64_t bstride, int64_t vstride, hipStream_t s) {
  constexpr int EPB = PotRows<T, NB>::EPB;
  hipLaunchKernelGGL((k_bspmv<T, NB, DIM>), dim3(unsigned((E + EPB - 1) / EPB), unsigned(nsys)), dim3(BT), 0, s,
                     blk, nbr, x, b, alpha, beta, y, bstride, vstride, E);
}

template <typename T>
void launch_bspmv(int nb, int dim, int64_t E, const T* blk, const int* nbr, const T* x, const T* b, T alpha,
                  T beta, T* y, hipStream_t s, int nsys, int64_t bstride, int64_t vstride) {
  if (E == 0 || nsys == 0) return;
#define BSP_ARGS E, blk, nbr, x, b, alpha, beta, y, nsys, bstride, vstride, s
  if (dim == 3) {
    switch (nb) {
      case 8: bsp_t<T, 8, 3>(BSP_ARGS); break;
      case 27: bsp_t<T, 27, 3>(BSP_ARGS); break;
      case 64: bsp_t<T, 64, 3>(BSP_ARGS); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: bsp_t<T, 4, 2>(BSP_ARGS); break;
      case 9: bsp_t<T, 9, 2>(BSP_ARGS); break;
      case 16: bsp_t<T, 16, 2>(BSP_ARGS); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
#undef BSP_ARGS
  DGNP_HIP(hipGetLastError());
}
template void launch_bspmv<double>(int, int, int64_t, const double*, const int*, const double*, const double*,
                                   double, double, double*, hipStream_t, int, int64_t, int64_t);
template void launch_bspmv<float>(int, int, int64_t, const float*, const int*, const float*, const float*,
                                  float, float, float*, hipStream_t, int, int64_t, int64_t);

template <typename T>
void launch_bdiag(int nb, int64_t E, const T* dinv, const T* x, T* y, hipStream_t s) {
  if (E == 0) return;
  const dim3 g = dim3(unsigned(E)), b = dim3(BT);
  switch (nb) {
    case 4: hipLaunchKernelGGL((k_bdiag<T, 4>), g, b, 0, s, dinv, x, y); break;
    case 8: hipLaunchKernelGGL((k_bdiag<T, 8>), g, b, 0, s, dinv, x, y); break;
    case 9: hipLaunchKernelGGL((k_bdiag<T, 9>), g, b, 0, s, dinv, x, y); break;
    case 16: hipLaunchKernelGGL((k_bdiag<T, 16>), g, b, 0, s, dinv, x, y); break;
    case 27: hipLaunchKernelGGL((k_bdiag<T, 27>), g, b, 0, s, dinv, x, y); break;
    case 64: hipLaunchKernelGGL((k_bdiag<T, 64>), g, b, 0, s, dinv, x, y); break;
    default: throw Error(DGNP_E_ARG, "unsupported block size");
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_bdiag<double>(int, int64_t, const double*, const double*, double*, hipStream_t);
template void launch_bdiag<float>(int, int64_t, const float*, const float*, float*, hipStream_t);

template <typename T, int DIM, int P>
static void q1_t(bool prolong, const int* n, const T* a, T* b, T beta, int64_t E, int64_t nvert, const T* dinv,
                 T c1, T* d1, hipStream_t s) {
  int3 n3 = make_int3(n[0], n[1], n[2]);
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  if (prolong) {
    const int64_t tot = E * NB;
    hipLaunchKernelGGL((k_q1_prolong<T, DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, n3, a, b,
                       beta, E);
  } else {
    const int64_t tot = nvert << DIM;  // 2^DIM lanes per vertex
    hipLaunchKernelGGL((k_q1_restrict<T, DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, n3, a, b,
                       nvert, dinv, c1, d1);
  }
}

template <typename T>
void launch_q1(bool prolong, int dim, int p, const int* n, const T* a, T* b, T beta, int64_t E, int64_t nvert,
               hipStream_t s, const T* dinv, T c1, T* d1) {
  if (!prolong && d1 && !dinv) throw Error(DGNP_E_ARG, "vertex restriction: first smoothing step without D^-1");
  if (dim == 3) {
    if (p == 1) q1_t<T, 3, 1>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
    else if (p == 2) q1_t<T, 3, 2>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
    else q1_t<T, 3, 3>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
  } else {
    if (p == 1) q1_t<T, 2, 1>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
    else if (p == 2) q1_t<T, 2, 2>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
    else q1_t<T, 2, 3>(prolong, n, a, b, beta, E, nvert, dinv, c1, d1, s);
  }
  DGNP_HIP(hipGetLastError());
}
template <int DIM, int P>
static void p1_inject_t(const double* x, double* x1, int m, int64_t E, hipStream_t s) {
  const int64_t tot = int64_t(m) * E * (1 << DIM);
  hipLaunchKernelGGL((k_p1_inject<DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, x, x1, m, E);
}
void launch_p1_inject(int dim, int p, const double* x, double* x1, int m, int64_t E, hipStream_t s) {
  if (E == 0) return;
  if (dim == 3) {
    if (p == 2) p1_inject_t<3, 2>(x, x1, m, E, s);
    else if (p == 3) p1_inject_t<3, 3>(x, x1, m, E, s);
    else throw Error(DGNP_E_ARG, "p-multigrid needs order 2 or 3");
  } else {
    if (p == 2) p1_inject_t<2, 2>(x, x1, m, E, s);
    else if (p == 3) p1_inject_t<2, 3>(x, x1, m, E, s);
    else throw Error(DGNP_E_ARG, "p-multigrid needs order 2 or 3");
  }
  DGNP_HIP(hipGetLastError());
}

template <typename T, int DIM, int P>
static void p1_t(bool prolong, const T* a, const T* sub, T* b, T beta, int64_t E, hipStream_t s) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  if (prolong) {
    const int64_t tot = E * NB;
    hipLaunchKernelGGL((k_p1_prolong<T, DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, a, b, beta, E);
  } else {
    const int64_t tot = E << DIM;
    hipLaunchKernelGGL((k_p1_restrict<T, DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, a, sub, b, E);
  }
}

template <typename T>
void launch_p1(bool prolong, int dim, int p, const T* a, const T* sub, T* b, T beta, int64_t E, hipStream_t s) {
  if (E == 0) return;
  if (dim == 3) {
    if (p == 2) p1_t<T, 3, 2>(prolong, a, sub, b, beta, E, s);
    else if (p == 3) p1_t<T, 3, 3>(prolong, a, sub, b, beta, E, s);
    else throw Error(DGNP_E_ARG, "p-multigrid needs order 2 or 3");
  } else {
    if (p == 2) p1_t<T, 2, 2>(prolong, a, sub, b, beta, E, s);
    else if (p == 3) p1_t<T, 2, 3>(prolong, a, sub, b, beta, E, s);
    else throw Error(DGNP_E_ARG, "p-multigrid needs order 2 or 3");
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_p1<double>(bool, int, int, const double*, const double*, double*, double, int64_t, hipStream_t);
template void launch_p1<float>(bool, int, int, const float*, const float*, float*, float, int64_t, hipStream_t);

template void launch_q1<double>(bool, int, int, const int*, const double*, double*, double, int64_t, int64_t,
                                hipStream_t, const double*, double, double*);
template void launch_q1<float>(bool, int, int, const int*, const float*, float*, float, int64_t, int64_t,
                               hipStream_t, const float*, float, float*);

void launch_q1_galerkin(int dim, int p, int64_t E, const double* blk, double* gal, hipStream_t s) {
  dim3 g(unsigned(E), unsigned(2 * dim + 1));
  if (dim == 3) {
    if (p == 1) hipLaunchKernelGGL((k_q1_galerkin<3, 1>), g, dim3(BT), 0, s, blk, gal);
    else if (p == 2) hipLaunchKernelGGL((k_q1_galerkin<3, 2>), g, dim3(BT), 0, s, blk, gal);
    else hipLaunchKernelGGL((k_q1_galerkin<3, 3>), g, dim3(BT), 0, s, blk, gal);
  } else {
    if (p == 1) hipLaunchKernelGGL((k_q1_galerkin<2, 1>), g, dim3(BT), 0, s, blk, gal);
    else if (p == 2) hipLaunchKernelGGL((k_q1_galerkin<2, 2>), g, dim3(BT), 0, s, blk, gal);
    else hipLaunchKernelGGL((k_q1_galerkin<2, 3>), g, dim3(BT), 0, s, blk, gal);
  }
  DGNP_HIP(hipGetLastError());
}

// Vertex stencil of the Galerkin operator: st[r][o] = sum of gal[e][s][u][v]
// over every element e that has vertex r (local index u) and every slot s whose
// target element (e itself or its neighbour across face s - 1) has the vertex
// r + offset(o) (local index v); o runs over the 3^d offsets in {-1, 0, 1}^d.
// Elements are visited in increasing index and slots in increasing order,
// which fixes the summation order.  Vertex pairs two layers apart (far sides
// of two face neighbours) couple only through exact zeros and are not stored.
template <int DIM>
__global__ void k_vertex_stencil(const double* __restrict__ gal, const int* __restrict__ nbr, int3 n,
                                 int64_t nvert, double* __restrict__ st) {
  constexpr int NV = 1 << DIM;
  constexpr int NS = DIM == 3 ? 27 : 9;
  constexpr int NSLOT = 2 * DIM + 1;
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= nvert * NS) return;
  const int64_t r = t / NS;
  const int o = int(t % NS);
  const int nv[3] = {n.x + 1, n.y + 1, DIM == 3 ? n.z + 1 : 1};
  const int ne[3] = {n.x, n.y, DIM == 3 ? n.z : 1};
  const int rc[3] = {int(r % nv[0]), int((r / nv[0]) % nv[1]), DIM == 3 ? int(r / (int64_t(nv[0]) * nv[1])) : 0};
  const int oc[3] = {o % 3 - 1, (o / 3) % 3 - 1, DIM == 3 ? o / 9 - 1 : 0};
  int cc[3];
  for (int a = 0; a < 3; ++a) cc[a] = rc[a] + oc[a];
  double acc = 0.0;
  // elements around r in increasing index: the offset bits run from (1,1,1) down
  for (int b = NV - 1; b >= 0; --b) {
    int ec[3] = {0, 0, 0};
    bool ok = true;
    int u = 0;
    for (int a = 0; a < DIM; ++a) {
      const int bit = (b >> a) & 1;  // descending b: last axis most significant
      ec[a] = rc[a] - bit;
      if (ec[a] < 0 || ec[a] >= ne[a]) ok = false;
      u |= bit << a;
    }
    if (!ok) continue;
    const int64_t e = ec[0] + int64_t(ne[0]) * (ec[1] + int64_t(ne[1]) * ec[2]);
    for (int sl = 0; sl < NSLOT; ++sl) {
      int tc[3] = {ec[0], ec[1], ec[2]};
      if (sl > 0) {
        if (nbr[e * 2 * DIM + (sl - 1)] < 0) continue;
        const int ax = (sl - 1) >> 1;
        tc[ax] += ((sl - 1) & 1) ? 1 : -1;
      }
      int v = 0;
      bool in = true;
      for (int a = 0; a < DIM; ++a) {
        const int l = cc[a] - tc[a];
        if (l < 0 || l > 1) in = false;
        v |= (l & 1) << a;
      }
      if (!in) continue;
      acc += gal[((e * NSLOT + sl) * NV + u) * NV + v];
    }
  }
  st[t] = acc;
}

void launch_vertex_stencil(int dim, const double* gal, const int* nbr, const int* n, int64_t nvert, double* st,
                           hipStream_t s) {
  const int ns = dim == 3 ? 27 : 9;
  const int64_t total = nvert * ns;
  if (total == 0) return;
  const int3 nn = make_int3(n[0], n[1], dim == 3 ? n[2] : 1);
  const unsigned g = unsigned((total + BT - 1) / BT);
  if (dim == 3)
    hipLaunchKernelGGL(k_vertex_stencil<3>, dim3(g), dim3(BT), 0, s, gal, nbr, nn, nvert, st);
  else
    hipLaunchKernelGGL(k_vertex_stencil<2>, dim3(g), dim3(BT), 0, s, gal, nbr, nn, nvert, st);
  DGNP_HIP(hipGetLastError());
}

template <typename T, int NB, int DIM>
static void dfp_t(int kind, const T* blk, const int* nbr, const int* order, int64_t E, int nfields, int64_t bstride,
                  int64_t vstride, const T* in, T* out, uint64_t* wp, int* err, int spin_limit, int grid,
                  hipStream_t s) {
  const dim3 g = dim3(unsigned(grid), unsigned(nfields)), b = dim3(BT);
  if (kind == 0)
    hipLaunchKernelGGL((k_ilu_dfp<T, NB, DIM, 0>), g, b, 0, s, blk, nbr, order, E, in, out, bstride, vstride, wp,
                       err, spin_limit);
  else
    hipLaunchKernelGGL((k_ilu_dfp<T, NB, DIM, 1>), g, b, 0, s, blk, nbr, order, E, in, out, bstride, vstride, wp,
                       err, spin_limit);
}

template <typename T, int NB, int DIM>
static int df_resident(int nfields) {
  int dev = 0, ncu = 0;
  DGNP_HIP(hipGetDevice(&dev));
  DGNP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int occ[2] = {0, 0};
  DGNP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], (k_ilu_dfp<T, NB, DIM, 0>), BT, 0));
  DGNP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], (k_ilu_dfp<T, NB, DIM, 1>), BT, 0));
  return (ncu * std::min(occ[0], occ[1])) / (2 * nfields);  // half the resident capacity per field
}

template <typename T>
int ilu_dataflow_grid(int nb, int dim, int64_t E, int nfields) {
  int r = 0;
  if (dim == 3) {
    switch (nb) {
      case 8: r = df_resident<T, 8, 3>(nfields); break;
      case 27: r = df_resident<T, 27, 3>(nfields); break;
      case 64: r = df_resident<T, 64, 3>(nfields); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: r = df_resident<T, 4, 2>(nfields); break;
      case 9: r = df_resident<T, 9, 2>(nfields); break;
      case 16: r = df_resident<T, 16, 2>(nfields); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  if (r < 1) throw Error(DGNP_E_HIP, "no resident work-groups for the dataflow sweep");
  return int(std::min<int64_t>(E, r));
}
template int ilu_dataflow_grid<double>(int, int, int64_t, int);
template int ilu_dataflow_grid<float>(int, int, int64_t, int);

template <typename T>
void launch_ilu_dataflow(int kind, int nb, int dim, const T* blk, const int* nbr, const int* order, int64_t E,
                         int nfields, int64_t bstride, int64_t vstride, const T* in, T* out, uint64_t* wp, int* err,
                         int spin_limit, int grid, hipStream_t s) {
  if (E == 0 || nfields == 0) return;
  if (dim == 3) {
    switch (nb) {
      case 8: dfp_t<T, 8, 3>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 27: dfp_t<T, 27, 3>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 64: dfp_t<T, 64, 3>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: dfp_t<T, 4, 2>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 9: dfp_t<T, 9, 2>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 16: dfp_t<T, 16, 2>(kind, blk, nbr, order, E, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}

template <int NB, int DIM>
static void dfl_t(int kind, const float* blk, const int* nbr, const int* line_first, int nline, int len,
                  int64_t lstride, int ax, int nfields, int64_t bstride, int64_t vstride, const float* in,
                  float* out, uint64_t* wp, int* err, int spin_limit, int grid, hipStream_t s) {
  const dim3 g = dim3(unsigned(grid), unsigned(nfields)), b = dim3(BT);
  if (kind == 0)
    hipLaunchKernelGGL((k_ilu_dfl<NB, DIM, 0>), g, b, 0, s, blk, nbr, line_first, nline, len, lstride, ax, in, out,
                       bstride, vstride, wp, err, spin_limit);
  else
    hipLaunchKernelGGL((k_ilu_dfl<NB, DIM, 1>), g, b, 0, s, blk, nbr, line_first, nline, len, lstride, ax, in, out,
                       bstride, vstride, wp, err, spin_limit);
}

template <int NB, int DIM>
static int dfl_resident(int nfields) {
  int dev = 0, ncu = 0;
  DGNP_HIP(hipGetDevice(&dev));
  DGNP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  int occ[2] = {0, 0};
  DGNP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], (k_ilu_dfl<NB, DIM, 0>), BT, 0));
  DGNP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], (k_ilu_dfl<NB, DIM, 1>), BT, 0));
  // the whole resident capacity: a line sweep runs alone on its stream, and a
  // line is one work-group's sequential work, so every resident work-group
  // shortens the sweep
  return (ncu * std::min(occ[0], occ[1])) / nfields;
}

int ilu_lines_grid(int nb, int dim, int nline, int nfields) {
  int r = 0;
  if (dim == 3) {
    switch (nb) {
      case 8: r = dfl_resident<8, 3>(nfields); break;
      case 27: r = dfl_resident<27, 3>(nfields); break;
      case 64: r = dfl_resident<64, 3>(nfields); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: r = dfl_resident<4, 2>(nfields); break;
      case 9: r = dfl_resident<9, 2>(nfields); break;
      case 16: r = dfl_resident<16, 2>(nfields); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  if (r < 1) throw Error(DGNP_E_HIP, "no resident work-groups for the line sweep");
  return std::min(nline, r);
}

void launch_ilu_lines(int kind, int nb, int dim, const float* blk, const int* nbr, const int* line_first, int nline,
                      int len, int64_t lstride, int ax, int nfields, int64_t bstride, int64_t vstride,
                      const float* in, float* out, uint64_t* wp, int* err, int spin_limit, int grid, hipStream_t s) {
  if (nline == 0 || nfields == 0) return;
  if (ax < 0 || ax >= dim || grid < 1) throw Error(DGNP_E_ARG, "bad line sweep arguments");
  if (dim == 3) {
    switch (nb) {
      case 8: dfl_t<8, 3>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 27: dfl_t<27, 3>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 64: dfl_t<64, 3>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: dfl_t<4, 2>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 9: dfl_t<9, 2>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      case 16: dfl_t<16, 2>(kind, blk, nbr, line_first, nline, len, lstride, ax, nfields, bstride, vstride, in, out, wp, err, spin_limit, grid, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}

template void launch_ilu_dataflow<double>(int, int, int, const double*, const int*, const int*, int64_t, int, int64_t,
                                          int64_t, const double*, double*, uint64_t*, int*, int, int, hipStream_t);
template void launch_ilu_dataflow<float>(int, int, int, const float*, const int*, const int*, int64_t, int, int64_t,
                                         int64_t, const float*, float*, uint64_t*, int*, int, int, hipStream_t);

// One Chebyshev smoothing step on the element-block level, fused:
//   r = base - A u - sub    (u null: no product; sub null: no subtrahend)
//   d = c1 * Dinv r + c2 * dprev   (dprev null: no second term)
//   x_out = x_in + d        (x_in null: x_out = d)
// with optional stores of r and d.  One work-group per element; x_out must not
// alias u (the neighbours read u).  Row layout and lane mapping as for
// k_bspmv (padded single-precision rows for blocks of up to 32 rows).
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_cheb_blk(const T* __restrict__ blk, const int* __restrict__ nbr,
                                                 const T* __restrict__ dinv, const T* u, const T* base,
                                                 const T* sub, const T* dprev, const T* x_in, T c1, T c2,
                                                 T* r_out, T* d_out, T* x_out, int64_t E) {
  constexpr int NSLOT = 2 * DIM + 1;
  using PR = PotRows<T, NB>;
  const int tid = threadIdx.x;
  if constexpr (PR::VEC) {
    constexpr int LD = PR::LD, QV = PR::QV, EPB = PR::EPB, TPE = BT / EPB;
    __shared__ __align__(16) float xv_[EPB][NSLOT][LD];
    __shared__ __align__(16) float rv_[EPB][LD];
    const int el = tid / TPE, lt = tid % TPE;  // element of the group, lane within it
    float(*xv)[LD] = xv_[el];
    float* rv = rv_[el];
    const int64_t i = int64_t(blockIdx.x) * EPB + el;
    const bool live = i < E;
    const int row = lt >> 3, part = lt & 7;
    const bool on = live && row < NB && part < QV;
    // the block rows and the inverse diagonal row go out first: they do not
    // depend on the neighbour table
    const float* bi = blk + i * NSLOT * NB * LD + row * LD + 4 * part;
    float4 mr[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      mr[s] = (u && on) ? ld4(bi + s * NB * LD) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 dr = on ? ld4(dinv + (i * NB + row) * LD + 4 * part) : make_float4(0.f, 0.f, 0.f, 0.f);
    int nb[NSLOT];
    nb[0] = live ? int(i) : -1;
    for (int s = 0; s < 2 * DIM; ++s) nb[1 + s] = live ? nbr[i * 2 * DIM + s] : -1;
    if (u) {
      for (int idx = lt; idx < NSLOT * LD; idx += TPE) {
        const int sl = idx / LD, c = idx - sl * LD;
        xv[sl][c] = (c < NB && nb[sl] >= 0) ? u[int64_t(nb[sl]) * NB + c] : 0.f;
      }
      __syncthreads();
    }
    float acc = 0.f;
    if (u && on) {
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
        if (nb[s] >= 0) acc += dot4(mr[s], ld4(&xv[s][4 * part]));
    }
    acc = sum8(acc);
    if (live && row < NB && part == 0) {
      const float r = base[i * NB + row] - acc - (sub ? sub[i * NB + row] : 0.f);
      rv[row] = r;
      if (r_out) r_out[i * NB + row] = r;
    }
    if (lt < LD - NB) rv[NB + lt] = 0.f;
    __syncthreads();
    const float z = sum8(on ? dot4(dr, ld4(&rv[4 * part])) : 0.f);
    if (live && row < NB && part == 0) {
      const int64_t k = i * NB + row;
      float d = c1 * z;
      if (dprev) d += c2 * dprev[k];
      if (d_out) d_out[k] = d;
      x_out[k] = (x_in ? x_in[k] : 0.f) + d;
    }
  } else {
    const int64_t i = blockIdx.x;
    __shared__ T xs[NSLOT][NB];
    __shared__ T rs[NB];
    const int row = tid >> 2, part = tid & 3;
    int nb[NSLOT];
    nb[0] = int(i);
    for (int s = 0; s < 2 * DIM; ++s) nb[1 + s] = nbr[i * 2 * DIM + s];
    if (u) {
      for (int idx = tid; idx < NB; idx += BT)
        for (int s = 0; s < NSLOT; ++s) xs[s][idx] = nb[s] >= 0 ? u[int64_t(nb[s]) * NB + idx] : T(0);
    }
    const T* bi = blk + i * NSLOT * NB * NB;
    constexpr int QL = (NB + 3) / 4;
    // small blocks: every row part of all blocks is fetched before any product
    // (loads in flight together); large blocks stream block by block
    constexpr bool PRE = NSLOT * QL * int(sizeof(T)) <= 256;
    if constexpr (PRE) {
      T m[NSLOT][QL];
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
#pragma unroll
        for (int c = 0; c < QL; ++c) {
          const int cc = part * QL + c;
          m[s][c] = (u && row < NB && cc < NB && nb[s] >= 0) ? bi[int64_t(s) * NB * NB + row * NB + cc] : T(0);
        }
      if (u) __syncthreads();
      if (row < NB) {
        T acc = T(0);
        if (u) {  // without u the LDS operand is not loaded (and the products vanish)
#pragma unroll
          for (int s = 0; s < NSLOT; ++s)
#pragma unroll
            for (int c = 0; c < QL; ++c) acc += m[s][c] * xs[s][part * QL + c < NB ? part * QL + c : 0];
          acc += __shfl_xor(acc, 1, 64);
          acc += __shfl_xor(acc, 2, 64);
        }
        if (part == 0) {
          const T r = base[i * NB + row] - acc - (sub ? sub[i * NB + row] : T(0));
          rs[row] = r;
          if (r_out) r_out[i * NB + row] = r;
        }
      }
    } else {
      if (u) __syncthreads();
      if (row < NB) {
        T acc = T(0);
        if (u)
          for (int s = 0; s < NSLOT; ++s)
            if (nb[s] >= 0) acc += row_dot4<T, NB>(bi + int64_t(s) * NB * NB, xs[s], row, part);
        if (part == 0) {
          const T r = base[i * NB + row] - acc - (sub ? sub[i * NB + row] : T(0));
          rs[row] = r;
          if (r_out) r_out[i * NB + row] = r;
        }
      }
    }
    __syncthreads();
    if (row < NB) {
      const T z = row_dot4<T, NB>(dinv + i * NB * NB, rs, row, part);
      if (part == 0) {
        const int64_t k = i * NB + row;
        T d = c1 * z;
        if (dprev) d += c2 * dprev[k];
        if (d_out) d_out[k] = d;
        x_out[k] = (x_in ? x_in[k] : T(0)) + d;
      }
    }
  }
}

template <typename T, int NB, int DIM>
static void cheb_blk_t(int64_t E, const T* blk, const int* nbr, const T* dinv, const T* u, const T* base,
                       const T* sub, const T* dprev, const T* x_in, T c1, T c2, T* r_out, T* d_out, T* x_out,
                       hipStream_t s) {
  constexpr int EPB = PotRows<T, NB>::EPB;
  hipLaunchKernelGGL((k_cheb_blk<T, NB, DIM>), dim3(unsigned((E + EPB - 1) / EPB)), dim3(BT), 0, s, blk, nbr, dinv,
                     u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, E);
}

template <typename T>
void launch_cheb_blk(int nb, int dim, int64_t E, const T* blk, const int* nbr, const T* dinv, const T* u,
                     const T* base, const T* sub, const T* dprev, const T* x_in, T c1, T c2, T* r_out, T* d_out,
                     T* x_out, hipStream_t s) {
  if (E == 0) return;
  if (dim == 3) {
    switch (nb) {
      case 8: cheb_blk_t<T, 8, 3>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      case 27: cheb_blk_t<T, 27, 3>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      case 64: cheb_blk_t<T, 64, 3>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: cheb_blk_t<T, 4, 2>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      case 9: cheb_blk_t<T, 9, 2>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      case 16: cheb_blk_t<T, 16, 2>(E, blk, nbr, dinv, u, base, sub, dprev, x_in, c1, c2, r_out, d_out, x_out, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_cheb_blk<double>(int, int, int64_t, const double*, const int*, const double*, const double*,
                                      const double*, const double*, const double*, const double*, double, double, double*,
                                      double*, double*, hipStream_t);
template void launch_cheb_blk<float>(int, int, int64_t, const float*, const int*, const float*, const float*,
                                     const float*, const float*, const float*, const float*, float, float, float*, float*,
                                     float*, hipStream_t);

}  // namespace dgnp
