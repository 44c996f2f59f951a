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
#include "dg_device.hpp"
#include "kernels_block.hpp"

namespace dgnp {

void upload_ref_tables_block(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

static constexpr int BT = 256;  // threads per block kernel

// ===========================================================================
// Assembly.  One work-group per (element, field).  blk[f][e][s][i][j]: s = 0
// diagonal block, s = 1 + slot coupling to the neighbour across `slot`; row i
// = test function, column j = trial function.
// ===========================================================================
template <int DIM, int P, int MF>
__global__ void __launch_bounds__(BT)
    k_assemble(KArgs A, const double* __restrict__ xs, double* __restrict__ blk, int nfields) {
  using S = Sz<DIM, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NQF = S::NQF, NFN = S::NFN;
  constexpr int NC = DIM + 1;                       // value + gradient components
  constexpr int NBT = MF * NB;
  constexpr int QV = MF * NC * NQV;
  constexpr int S1 = DIM == 3 ? MF * 2 * NN * NN * NQ : MF * 2 * NN * NQ;
  constexpr int S2 = DIM == 3 ? MF * 3 * NN * NQ * NQ : 0;
  constexpr int QCH = NQ * NQ > 16 ? 16 : NQ * NQ;  // quadrature points per Y chunk
  constexpr int YCH = QCH * NC * NB;
  constexpr int TRQ = MF * 2 * NQF;
  constexpr int TRN = MF * 2 * NFN;
  constexpr int TRM = DIM == 3 ? MF * 2 * NN * NQ : 0;
  constexpr int VOLR = (QV + S1 + S2) > YCH ? (QV + S1 + S2) : YCH;
  constexpr int FACR = NBT + 2 * TRQ + TRN + TRM + NQF * 8;
  constexpr int REG = VOLR > FACR ? VOLR : FACR;
  constexpr int ENT = (NB * NB + BT - 1) / BT;
  constexpr int NSLOT = 2 * DIM + 1;
  __shared__ double s_x[NBT];
  __shared__ double Mq[NQV * NC * NC];
  __shared__ double R[REG];
  __shared__ STab<P, double> tb;

  const int tid = threadIdx.x;
  const int64_t e = blockIdx.x;
  const int f = blockIdx.y;
  load_tab<P, double>(tb, tid, BT);
  Phys<double, MF> ph;
  for (int k = 0; k < MF - 1; ++k) {
    ph.zD[k] = A.z[k] * A.D[k];
    ph.D[k] = A.D[k];
    ph.a[k] = A.a[k];
    ph.b[k] = A.b[k];
  }
  ph.delta = A.delta;
  const int64_t Nf = A.E * NB;
  int eid[3];
  eid[0] = int(e % A.n[0]);
  eid[1] = int((e / A.n[0]) % A.n[1]);
  eid[2] = DIM == 3 ? int(e / (int64_t(A.n[0]) * A.n[1])) : 0;
  double ih[3];
  for (int i = 0; i < 3; ++i) ih[i] = 2.0 / A.h[i];
  for (int i = tid; i < NBT; i += BT) s_x[i] = xs[(i / NB) * Nf + e * NB + (i % NB)];
  __syncthreads();

  // ---- volume: pointwise Jacobian restricted to field f -> Mq[q][alpha][beta]
  {
    double* q_x = R;
    double* t1 = R + QV;
    double* t2 = t1 + S1;
    interp<DIM, P, MF, BT, double>(s_x, q_x, t1, t2, tb, ih, tid);
    for (int qi = tid; qi < NQV; qi += BT) {
      int qc[3] = {qi % NQ, (qi / NQ) % NQ, qi / (NQ * NQ)};
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
      for (int beta = 0; beta < NC; ++beta) {
        double dv[MF], dg[MF][DIM], cg[MF][DIM];
        for (int g = 0; g < MF; ++g) {
          dv[g] = 0.0;
          for (int d = 0; d < DIM; ++d) dg[g][d] = 0.0;
        }
        if (beta == 0) dv[f] = 1.0; else dg[f][beta - 1] = 1.0;
        vol_jac<double, MF, DIM>(ph, val, grad, u, dv, dg, cg);
        const double sb = beta == 0 ? 1.0 : ih[beta - 1];
        Mq[(qi * NC + 0) * NC + beta] = 0.0;
        for (int d = 0; d < DIM; ++d) Mq[(qi * NC + 1 + d) * NC + beta] = cg[f][d] * w * sb * ih[d];
      }
    }
    __syncthreads();
  }
  // reference tabulation T_alpha(q, i) of basis i at volume point q
  auto tab = [&](int alpha, int q, int i) -> double {
    int qc[3] = {q % NQ, (q / NQ) % NQ, q / (NQ * NQ)};
    int ic[3] = {i % NN, (i / NN) % NN, i / (NN * NN)};
    double t = 1.0;
    for (int d = 0; d < DIM; ++d) {
      const double* M = (alpha == 1 + d) ? tb.D : tb.B;
      t *= M[qc[d] * NN + ic[d]];
    }
    return t;
  };
  double acc[ENT];
  for (int k = 0; k < ENT; ++k) acc[k] = 0.0;
  // Y[qq][beta][i] = sum_alpha T_alpha(q, i) M[q][alpha][beta], in chunks of QCH points
  for (int q0 = 0; q0 < NQV; q0 += QCH) {
    const int nq = (NQV - q0) < QCH ? (NQV - q0) : QCH;
    double* Y = R;
    for (int idx = tid; idx < nq * NC * NB; idx += BT) {
      const int i = idx % NB, beta = (idx / NB) % NC, qq = idx / (NB * NC);
      const int q = q0 + qq;
      double s = 0.0;
      for (int alpha = 1; alpha < NC; ++alpha) s += tab(alpha, q, i) * Mq[(q * NC + alpha) * NC + beta];
      Y[(qq * NC + beta) * NB + i] = s;
    }
    __syncthreads();
    for (int k = 0; k < ENT; ++k) {
      const int idx = tid + k * BT;
      if (idx >= NB * NB) break;
      const int i = idx / NB, j = idx % NB;
      double s = acc[k];
      for (int qq = 0; qq < nq; ++qq)
        for (int beta = 0; beta < NC; ++beta) s += Y[(qq * NC + beta) * NB + i] * tab(beta, q0 + qq, j);
      acc[k] = s;
    }
    __syncthreads();
  }

  // ---- faces
  double* n_x = R;
  double* tox = R + NBT;
  double* tnx = tox + TRQ;
  double* tn = tnx + TRQ;
  double* tm = tn + TRN;
  double* Mf = tm + TRM;  // [qf][2 test][4 trial: own v, own g, nb v, nb g]
  double* out = blk + ((int64_t(f) * A.E + e) * NSLOT) * NB * NB;
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
    trace<DIM, P, MF, BT, double>(s_x, ax, side, tox, tn, tm, tb, ih[ax], tid);
    if (interior) {
      for (int i = tid; i < NBT; i += BT) n_x[i] = xs[(i / NB) * Nf + int64_t(nb) * NB + (i % NB)];
      __syncthreads();
      trace<DIM, P, MF, BT, double>(n_x, ax, -side, tnx, tn, tm, tb, ih[ax], tid);
    }
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
    const int own = side > 0 ? 0 : 1;
    for (int qf = tid; qf < NQF; qf += BT) {
      const int qi = qf % NQ, qj = qf / NQ;
      double xp[3];
      xp[ax] = A.lo[ax] + (eid[ax] + (side > 0 ? 1.0 : 0.0)) * A.h[ax];
      xp[t1ax] = A.lo[t1ax] + (eid[t1ax] + 0.5 * (tb.X[qi] + 1.0)) * A.h[t1ax];
      double w = 0.5 * A.h[t1ax] * tb.W[qi];
      if constexpr (DIM == 3) {
        xp[t2ax] = A.lo[t2ax] + (eid[t2ax] + 0.5 * (tb.X[qj] + 1.0)) * A.h[t2ax];
        w *= 0.5 * A.h[t2ax] * tb.W[qj];
      }
      double uh[3];
      velocity_hat(A, xp, DIM, uh);
      if (interior) {
        const double un = A.Pe * uh[ax];
        double v[2][MF], g[2][MF];
        for (int c = 0; c < MF; ++c) {
          v[own][c] = tox[(c * 2 + 0) * NQF + qf];
          g[own][c] = tox[(c * 2 + 1) * NQF + qf];
          v[1 - own][c] = tnx[(c * 2 + 0) * NQF + qf];
          g[1 - own][c] = tnx[(c * 2 + 1) * NQF + qf];
        }
        for (int beta = 0; beta < 4; ++beta) {
          double tv[2][MF] = {}, tg[2][MF] = {};
          const int sd = beta < 2 ? own : 1 - own;
          if (beta % 2 == 0) tv[sd][f] = 1.0; else tg[sd][f] = 1.0;
          double Fo[MF], Go[MF];
          face_jac<double, MF>(ph, v, g, tv, tg, un, own, Fo, Go);
          const double sb = (beta % 2 == 0) ? 1.0 : ih[ax];
          Mf[(qf * 2 + 0) * 4 + beta] = Fo[f] * w * sb;
          Mf[(qf * 2 + 1) * 4 + beta] = Go[f] * w * sb * ih[ax];
        }
      } else {
        const double un = side * A.Pe * uh[ax];
        double v[MF], g[MF], gd[MF];
        for (int c = 0; c < MF; ++c) {
          v[c] = tox[(c * 2 + 0) * NQF + qf];
          g[c] = side * tox[(c * 2 + 1) * NQF + qf];
          gd[c] = A.bcq[(c * A.n_bface + bf) * NQF + qf];
        }
        for (int beta = 0; beta < 2; ++beta) {
          double tv[MF] = {}, tg[MF] = {};
          if (beta == 0) tv[f] = 1.0; else tg[f] = 1.0;
          double Fo[MF], Go[MF];
          bnd_jac<double, MF>(ph, v, g, tv, tg, un, cbc, phid, gd, Fo, Go);
          const double sb = beta == 0 ? 1.0 : side * ih[ax];
          Mf[(qf * 2 + 0) * 4 + beta] = Fo[f] * w * sb;
          Mf[(qf * 2 + 1) * 4 + beta] = Go[f] * w * sb * side * ih[ax];
          Mf[(qf * 2 + 0) * 4 + 2 + beta] = 0.0;
          Mf[(qf * 2 + 1) * 4 + 2 + beta] = 0.0;
        }
      }
    }
    __syncthreads();
    // face tabulation of basis i on side `sd` of this face: value or d/dxi_ax
    const int lend_own = side < 0 ? 0 : P;
    const int lend_nb = side < 0 ? P : 0;
    auto ftab = [&](int kind, int sdir, int lend, int qf, int i) -> double {
      const int qi = qf % NQ, qj = qf / NQ;
      int ic[3] = {i % NN, (i / NN) % NN, i / (NN * NN)};
      const int l = ic[ax];
      const int it1 = ic[t1ax];
      double t = tb.B[qi * NN + it1];
      if constexpr (DIM == 3) t *= tb.B[qj * NN + ic[t2ax]];
      if (kind == 0) return l == lend ? t : 0.0;
      return t * tb.De[sdir < 0 ? 0 : 1][l];
    };
    for (int k = 0; k < ENT; ++k) {
      const int idx = tid + k * BT;
      if (idx >= NB * NB) break;
      const int i = idx / NB, j = idx % NB;
      double sd = 0.0, so = 0.0;
      for (int qf = 0; qf < NQF; ++qf) {
        const double ti0 = ftab(0, side, lend_own, qf, i), ti1 = ftab(1, side, lend_own, qf, i);
        const double tj0 = ftab(0, side, lend_own, qf, j), tj1 = ftab(1, side, lend_own, qf, j);
        const double* M = Mf + qf * 8;
        sd += ti0 * (M[0] * tj0 + M[1] * tj1) + ti1 * (M[4] * tj0 + M[5] * tj1);
        if (interior) {
          const double nj0 = ftab(0, -side, lend_nb, qf, j), nj1 = ftab(1, -side, lend_nb, qf, j);
          so += ti0 * (M[2] * nj0 + M[3] * nj1) + ti1 * (M[6] * nj0 + M[7] * nj1);
        }
      }
      acc[k] += sd;
      ob[idx] = so;
    }
    __syncthreads();
  }
  for (int k = 0; k < ENT; ++k) {
    const int idx = tid + k * BT;
    if (idx < NB * NB) out[idx] = acc[k];
  }
  (void)nfields;
}

template <int DIM, int P>
static void assemble_t(int m, const KArgs& A, const double* xs, double* blk, hipStream_t s) {
  dim3 grid(unsigned(A.E), unsigned(m));
  if (m == 2)
    hipLaunchKernelGGL((k_assemble<DIM, P, 2>), grid, dim3(BT), 0, s, A, xs, blk, m);
  else
    hipLaunchKernelGGL((k_assemble<DIM, P, 3>), grid, dim3(BT), 0, s, A, xs, blk, m);
  DGNP_HIP(hipGetLastError());
}

void launch_assemble(int dim, int p, int m, const KArgs& A, const double* xs, double* blk, hipStream_t s) {
  DGNP_REQUIRE(m == 2 || m == 3, DGNP_E_ARG, "number of ions must be 2 or 3");
  if (dim == 3) {
    if (p == 1) return assemble_t<3, 1>(m, A, xs, blk, s);
    if (p == 2) return assemble_t<3, 2>(m, A, xs, blk, s);
    if (p == 3) return assemble_t<3, 3>(m, A, xs, blk, s);
  } else {
    if (p == 1) return assemble_t<2, 1>(m, A, xs, blk, s);
    if (p == 2) return assemble_t<2, 2>(m, A, xs, blk, s);
    if (p == 3) return assemble_t<2, 3>(m, A, xs, blk, s);
  }
  throw Error(DGNP_E_ARG, "unsupported dimension / order");
}

// ===========================================================================
// Gauss-Jordan inversion with partial (row) pivoting of an NB x NB matrix held
// in LDS with leading dimension LD.  The row interchanges are undone as
// column interchanges at the end, so a holds A^{-1} on exit.
// ===========================================================================
template <int NB, int LD>
__device__ void gj_invert(double* a, int* piv, double* colk, int tid) {
  const int lane = tid & 63;
  for (int k = 0; k < NB; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int r = k + lane; r < NB; r += 64) {
        const double v = fabs(a[r * LD + k]);
        if (v > best) {
          best = v;
          bi = r;
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
      if (lane == 0) piv[k] = bi;
    }
    __syncthreads();
    const int p = piv[k];
    if (p != k)
      for (int c = tid; c < NB; c += BT) {
        const double t = a[k * LD + c];
        a[k * LD + c] = a[p * LD + c];
        a[p * LD + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / a[k * LD + k];
    for (int r = tid; r < NB; r += BT) colk[r] = a[r * LD + k];
    __syncthreads();
    for (int c = tid; c < NB; c += BT) a[k * LD + c] = (c == k) ? inv : a[k * LD + c] * inv;
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += BT) {
      const int r = idx / NB, c = idx % NB;
      if (r == k) continue;
      const double fr = colk[r];
      if (c == k)
        a[r * LD + c] = -fr * inv;
      else
        a[r * LD + c] -= fr * a[k * LD + c];
    }
    __syncthreads();
  }
  for (int k = NB - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int r = tid; r < NB; r += BT) {
        const double t = a[r * LD + k];
        a[r * LD + k] = a[r * LD + p];
        a[r * LD + p] = t;
      }
    __syncthreads();
  }
}

// out[e] = inverse of the diagonal block of element e (blk slot 0)
template <int NB>
__global__ void __launch_bounds__(BT) k_block_inverse(const double* __restrict__ blk, int nslot,
                                                      double* __restrict__ out) {
  constexpr int LD = NB + 1;
  __shared__ double a[NB * LD];
  __shared__ double colk[NB];
  __shared__ int piv[NB];
  const int64_t e = blockIdx.x;
  const double* src = blk + e * nslot * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += BT) a[(idx / NB) * LD + idx % NB] = src[idx];
  __syncthreads();
  gj_invert<NB, LD>(a, piv, colk, threadIdx.x);
  for (int idx = threadIdx.x; idx < NB * NB; idx += BT) out[e * NB * NB + idx] = a[(idx / NB) * LD + idx % NB];
}

// ===========================================================================
// BILU(0) factorisation of one field block, one hyperplane level per launch.
// For the 2d+1-point block stencil in lexicographic order, ILU(0) changes only
// the diagonal blocks: D_i = A_ii - sum_{j lower} A_ij D_j^{-1} A_ji.  Stored in
// place: slot 0 <- D_i^{-1}; slot 1+s <- D_i^{-1} A_{i,nbr(s)} for every
// neighbour (lower ones = Lhat, upper ones = Uhat), so that
//   M = D (I + Lhat)(I + Uhat).
// ===========================================================================
template <int NB, int DIM>
__global__ void __launch_bounds__(BT) k_ilu_factor(double* __restrict__ blk, const int* __restrict__ nbr,
                                                   const int* __restrict__ lev_elems, int64_t first) {
  constexpr int LD = NB + 1;
  constexpr int NSLOT = 2 * DIM + 1;
  constexpr int PW = 16;  // column panel width
  __shared__ double a[NB * LD];
  __shared__ double pan[NB * PW];
  __shared__ double colk[NB];
  __shared__ int piv[NB];
  const int tid = threadIdx.x;
  const int64_t i = lev_elems[first + blockIdx.x];
  double* bi = blk + i * NSLOT * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += BT) a[(idx / NB) * LD + idx % NB] = bi[idx];
  __syncthreads();
  // Schur updates from the lower neighbours (slots 0, 2, 4 = -x, -y, -z)
  for (int s = 0; s < 2 * DIM; s += 2) {
    const int j = nbr[i * 2 * DIM + s];
    if (j < 0) continue;
    const double* Aij = bi + int64_t(1 + s) * NB * NB;
    const double* Uji = blk + (int64_t(j) * NSLOT + 1 + (s + 1)) * NB * NB;  // j's slot toward i
    for (int idx = tid; idx < NB * NB; idx += BT) {
      const int r = idx / NB, c = idx % NB;
      double acc = 0.0;
      for (int k = 0; k < NB; ++k) acc += Aij[r * NB + k] * Uji[k * NB + c];
      a[r * LD + c] -= acc;
    }
    __syncthreads();
  }
  gj_invert<NB, LD>(a, piv, colk, tid);
  for (int idx = tid; idx < NB * NB; idx += BT) bi[idx] = a[(idx / NB) * LD + idx % NB];
  // scale every neighbour block by D_i^{-1}
  for (int s = 0; s < 2 * DIM; ++s) {
    if (nbr[i * 2 * DIM + s] < 0) continue;
    double* B = bi + int64_t(1 + s) * NB * NB;
    for (int c0 = 0; c0 < NB; c0 += PW) {
      const int w = (NB - c0) < PW ? (NB - c0) : PW;
      __syncthreads();
      for (int idx = tid; idx < NB * w; idx += BT) pan[(idx / w) * PW + idx % w] = B[(idx / w) * NB + c0 + idx % w];
      __syncthreads();
      for (int idx = tid; idx < NB * w; idx += BT) {
        const int r = idx / w, c = idx % w;
        double acc = 0.0;
        for (int k = 0; k < NB; ++k) acc += a[r * LD + k] * pan[k * PW + c];
        B[r * NB + c0 + c] = acc;
      }
    }
  }
}

// ===========================================================================
// Level-scheduled solves.  Four threads per block row, each handling a
// contiguous quarter of the row; partial sums combined with lane shuffles.
// ===========================================================================
template <typename T, int NB>
__device__ inline T row_dot4(const T* __restrict__ M, const T* x, int r, int part) {
  constexpr int QL = (NB + 3) / 4;
  T acc = T(0);
  const int c0 = part * QL;
#pragma unroll
  for (int c = 0; c < QL; ++c)
    if (c0 + c < NB) acc += M[r * NB + c0 + c] * x[c0 + c];
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
template <typename T, int NB, int DIM>
__global__ void __launch_bounds__(BT) k_bspmv(const T* __restrict__ blk, const int* __restrict__ nbr,
                                              const T* __restrict__ x, const T* __restrict__ b, T alpha,
                                              T beta, T* __restrict__ y) {
  constexpr int NSLOT = 2 * DIM + 1;
  __shared__ T xs[NSLOT][NB];
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  const int64_t i = blockIdx.x;
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

// y_i = Dinv_i x_i
template <typename T, int NB>
__global__ void __launch_bounds__(BT) k_bdiag(const T* __restrict__ dinv, const T* __restrict__ x,
                                              T* __restrict__ y) {
  __shared__ T xs[NB];
  const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
  const int64_t i = blockIdx.x;
  for (int idx = tid; idx < NB; idx += BT) xs[idx] = x[i * NB + idx];
  __syncthreads();
  if (row < NB) {
    const T v = row_dot4<T, NB>(dinv + i * NB * NB, xs, row, part);
    if (part == 0) y[i * NB + row] = v;
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
template <typename T, int DIM, int P>
__global__ void k_q1_restrict(int3 n3, const T* __restrict__ r, T* __restrict__ rv, int64_t nvert) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= nvert) return;
  int n[3] = {n3.x, n3.y, n3.z};
  int vc[3] = {int(v % (n[0] + 1)), int((v / (n[0] + 1)) % (n[1] + 1)),
               DIM == 3 ? int(v / (int64_t(n[0] + 1) * (n[1] + 1))) : 0};
  double acc = 0.0;
  for (int o = 0; o < (1 << DIM); ++o) {
    int eid[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < DIM; ++d) {
      eid[d] = vc[d] - ((o >> d) & 1);
      if (eid[d] < 0 || eid[d] >= n[d]) ok = false;
    }
    if (!ok) continue;
    const int64_t e = eid[0] + int64_t(n[0]) * (eid[1] + int64_t(n[1]) * eid[2]);
    for (int node = 0; node < NB; ++node) acc += q1_shape<DIM, P>(node, o) * double(r[e * NB + node]);
  }
  rv[v] = T(acc);
}

// gal[e][s][u][v] = sum_ij N_u(i) A_{e,s}[i][j] N_v(j)   (s = 0 diag, 1 + slot)
template <int DIM, int P>
__global__ void __launch_bounds__(BT) k_q1_galerkin(const double* __restrict__ blk, double* __restrict__ gal) {
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  constexpr int NV = 1 << DIM;
  constexpr int NSLOT = 2 * DIM + 1;
  __shared__ double T[NB * NV];
  const int64_t e = blockIdx.x;
  const int s = blockIdx.y;
  const double* A = blk + (e * NSLOT + s) * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NV; idx += BT) {
    const int i = idx / NV, v = idx % NV;
    double acc = 0.0;
    for (int j = 0; j < NB; ++j) acc += A[i * NB + j] * q1_shape<DIM, P>(j, v);
    T[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NV * NV; idx += BT) {
    const int u = idx / NV, v = idx % NV;
    double acc = 0.0;
    for (int i = 0; i < NB; ++i) acc += q1_shape<DIM, P>(i, u) * T[i * NV + v];
    gal[(e * NSLOT + s) * NV * NV + idx] = acc;
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
static void fac_t(double* blk, const int* nbr, const int* lev, int64_t first, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL((k_ilu_factor<NB, DIM>), dim3(unsigned(count)), dim3(BT), 0, s, blk, nbr, lev, first);
}

void launch_ilu_factor(int nb, int dim, double* blk, const int* nbr, const int* lev, int64_t first,
                       int64_t count, hipStream_t s) {
  if (count == 0) return;
  if (dim == 3) {
    switch (nb) {
      case 8: fac_t<8, 3>(blk, nbr, lev, first, count, s); break;
      case 27: fac_t<27, 3>(blk, nbr, lev, first, count, s); break;
      case 64: fac_t<64, 3>(blk, nbr, lev, first, count, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: fac_t<4, 2>(blk, nbr, lev, first, count, s); break;
      case 9: fac_t<9, 2>(blk, nbr, lev, first, count, s); break;
      case 16: fac_t<16, 2>(blk, nbr, lev, first, count, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
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
                  hipStream_t s) {
  hipLaunchKernelGGL((k_bspmv<T, NB, DIM>), dim3(unsigned(E)), dim3(BT), 0, s, blk, nbr, x, b, alpha, beta, y);
}

template <typename T>
void launch_bspmv(int nb, int dim, int64_t E, const T* blk, const int* nbr, const T* x, const T* b, T alpha,
                  T beta, T* y, hipStream_t s) {
  if (E == 0) return;
  if (dim == 3) {
    switch (nb) {
      case 8: bsp_t<T, 8, 3>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      case 27: bsp_t<T, 27, 3>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      case 64: bsp_t<T, 64, 3>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  } else {
    switch (nb) {
      case 4: bsp_t<T, 4, 2>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      case 9: bsp_t<T, 9, 2>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      case 16: bsp_t<T, 16, 2>(E, blk, nbr, x, b, alpha, beta, y, s); break;
      default: throw Error(DGNP_E_ARG, "unsupported block size");
    }
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_bspmv<double>(int, int, int64_t, const double*, const int*, const double*, const double*,
                                   double, double, double*, hipStream_t);
template void launch_bspmv<float>(int, int, int64_t, const float*, const int*, const float*, const float*,
                                  float, float, float*, hipStream_t);

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
static void q1_t(bool prolong, const int* n, const T* a, T* b, T beta, int64_t E, int64_t nvert, hipStream_t s) {
  int3 n3 = make_int3(n[0], n[1], n[2]);
  constexpr int NN = P + 1;
  constexpr int NB = DIM == 3 ? NN * NN * NN : NN * NN;
  if (prolong) {
    const int64_t tot = E * NB;
    hipLaunchKernelGGL((k_q1_prolong<T, DIM, P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, n3, a, b,
                       beta, E);
  } else {
    hipLaunchKernelGGL((k_q1_restrict<T, DIM, P>), dim3(unsigned((nvert + 255) / 256)), dim3(256), 0, s, n3, a,
                       b, nvert);
  }
}

template <typename T>
void launch_q1(bool prolong, int dim, int p, const int* n, const T* a, T* b, T beta, int64_t E, int64_t nvert,
               hipStream_t s) {
  if (dim == 3) {
    if (p == 1) q1_t<T, 3, 1>(prolong, n, a, b, beta, E, nvert, s);
    else if (p == 2) q1_t<T, 3, 2>(prolong, n, a, b, beta, E, nvert, s);
    else q1_t<T, 3, 3>(prolong, n, a, b, beta, E, nvert, s);
  } else {
    if (p == 1) q1_t<T, 2, 1>(prolong, n, a, b, beta, E, nvert, s);
    else if (p == 2) q1_t<T, 2, 2>(prolong, n, a, b, beta, E, nvert, s);
    else q1_t<T, 2, 3>(prolong, n, a, b, beta, E, nvert, s);
  }
  DGNP_HIP(hipGetLastError());
}
template void launch_q1<double>(bool, int, int, const int*, const double*, double*, double, int64_t, int64_t,
                                hipStream_t);
template void launch_q1<float>(bool, int, int, const int*, const float*, float*, float, int64_t, int64_t,
                               hipStream_t);

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

}  // namespace dgnp
