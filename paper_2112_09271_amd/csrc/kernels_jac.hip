// Jacobian apply with tabulated linearisation data (3-D): y = J(x) v, the exact
// derivative of the residual of Eqs. NPDG / chargeDG (Sec. 3.3) at a fixed
// state x (Sec. 4, Eq. blockmatrix), and its potential rows applied to the
// concentration part of v alone (the coupling A_phi,c z_c of the
// block-triangular preconditioner, Eq. P2).
//
// J(x) v is linear in v; x enters only through point values that stay fixed
// for a whole Newton step.  They are tabulated once per linearisation point:
//   volume, at every Gauss point of every element: c_1 .. c_{m-1} and grad phi
//     (the linearised fluxes need kappa(c), q_k = u - z_k D_k grad phi and c_k);
//   faces, at the Gauss points of each of the element's 6 faces, from the
//     element's own trace: phi, d phi / dx_axis, c_1 .. c_{m-1} (the neighbour's
//     side of an interior face is the neighbour's own record of that face).
// An apply then interpolates only v.  The velocity factors are separable in
// every velocity kind (u_d = Pe alpha_d(x) beta_d(y)): one small table per
// element column and row, built with the state tables, gives them at the 1-D
// point sets, and the apply does no double-precision or transcendental work.
//
// A work-group holds EPB elements (consecutive in the lexicographic order, so
// x-neighbours of the face terms inside the group are read from LDS); every
// phase loops over all (element, item) pairs of the group.  Phases: sum-factorised
// interpolation of v (x, y, z lines), pointwise linearised volume flux,
// transposed contractions (z, y, x), then the 6 faces element-centric: node
// traces of own and neighbour element, tangential interpolation to the face
// Gauss points, linearised numerical flux, tangential transposes, accumulation
// into the own element.  The face flux is taken from the own side's point of
// view (face_jac_own: no side index chosen at run time, which would otherwise
// become chains of selects).  Every output entry has one writer: no atomics,
// and results are bitwise reproducible.
#include <cstdlib>

#include "dg_device.hpp"
#include "kernels_jac.hpp"

namespace dgnp {

void upload_ref_tables_jac(const RefTables* tabs, int count) { upload_ref_tables_tu(tabs, count); }

// Launch shape: elements per work-group and threads.  In single precision the
// kernel is bound by the vector-instruction issue rate (index, address and
// select work beside the contractions), in double precision by latency at
// its occupancy; the number of resident work-groups matters more than busy
// lanes.  Measured on the 12.6M-DOF channel (p = 3), one element per group is
// fastest (FP32: 128 threads, against 733 us with four elements and 256; FP64:
// 256 threads, against 1590 us with two elements and 128); on the 16^3 cube
// (p = 2) one element and 64 threads (FP32) and two elements and 256 threads
// (FP64).  FP64 asks for five waves per SIMD (a register limit of 96), which
// beats the occupancy of four that its unrestricted register count gives
// (796 against 888 us).  The neighbours' inputs of the face traces are read
// directly from global memory: staging them in LDS first cost more (427 against
// 395 us in FP32).
// The coupling block (potential rows only) has a third of the full apply's
// output work and is fastest with fewer threads per element at p = 3 (FP32:
// 64 threads, 257 against 270 us; FP64: 128 threads, 427 against 482 us).
template <int P, typename T, bool CPL = false>
struct Shape {
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int epb = P == 3 ? 1 : (P == 2 ? (F64 ? 2 : 1) : (F64 ? 2 : 4));
  static constexpr int nt = P == 3 ? (CPL ? (F64 ? 128 : 64) : (F64 ? 256 : 128))
                                   : (P == 2 ? (F64 ? 256 : 64) : 256);
};

// ---------------------------------------------------------------------------
// state tables, computed in double from the double state
// tv[e][comp][q]: comp 0 .. m-2 = c_1 .. c_{m-1}, m-1 .. m+1 = d phi/dx, dy, dz
// tf[e][fc][comp][qf]: comp 0 = phi, 1 = d phi/dx_ax, 2 .. m = c_1 .. c_{m-1}
template <int P, int MF, typename T>
__global__ void __launch_bounds__(128) k_jlin_tab(KArgs A, const double* __restrict__ xs, T* __restrict__ tv,
                                                  T* __restrict__ tf) {
  using S = Sz<3, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NQF = S::NQF;
  constexpr int NV = MF + 2, NF = MF + 1;
  using C = CT<double, P>;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t Nf = A.E * NB;
  __shared__ double sx[MF][NB];
  for (int i = tid; i < MF * NB; i += 128) sx[i / NB][i % NB] = xs[(i / NB) * Nf + e * NB + i % NB];
  __syncthreads();
  double ih[3];
  for (int d = 0; d < 3; ++d) ih[d] = 2.0 / A.h[d];
  for (int qi = tid; qi < NQV; qi += 128) {
    const int qx = qi % NQ, qy = (qi / NQ) % NQ, qz = qi / (NQ * NQ);
    double val[MF], gp[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < MF; ++f) val[f] = 0.0;
    for (int c = 0; c < NN; ++c)
      for (int b = 0; b < NN; ++b)
        for (int a = 0; a < NN; ++a) {
          const int l = (c * NN + b) * NN + a;
          const double bbb = C::B(qx, a) * C::B(qy, b) * C::B(qz, c);
          for (int f = 1; f < MF; ++f) val[f] += bbb * sx[f][l];
          gp[0] += C::D(qx, a) * C::B(qy, b) * C::B(qz, c) * sx[0][l];
          gp[1] += C::B(qx, a) * C::D(qy, b) * C::B(qz, c) * sx[0][l];
          gp[2] += C::B(qx, a) * C::B(qy, b) * C::D(qz, c) * sx[0][l];
        }
    for (int k = 1; k < MF; ++k) tv[(e * NV + k - 1) * NQV + qi] = T(val[k]);
    for (int d = 0; d < 3; ++d) tv[(e * NV + MF - 1 + d) * NQV + qi] = T(gp[d] * ih[d]);
  }
  for (int idx = tid; idx < 6 * NQF; idx += 128) {
    const int qf = idx % NQF, fc = idx / NQF;
    const int ax = fc >> 1, sdi = fc & 1, lend = sdi ? P : 0;
    const int qi = qf % NQ, qj = qf / NQ;
    double val[MF], dn = 0.0;
    for (int f = 0; f < MF; ++f) val[f] = 0.0;
    for (int j = 0; j < NN; ++j)
      for (int i = 0; i < NN; ++i) {
        const double bb = C::B(qi, i) * C::B(qj, j);
        for (int f = 0; f < MF; ++f) val[f] += bb * sx[f][face_node<3, NN>(ax, lend, i, j)];
        double d = 0.0;
        for (int l = 0; l < NN; ++l) d += C::De(sdi, l) * sx[0][face_node<3, NN>(ax, l, i, j)];
        dn += bb * d;
      }
    T* o = tf + (e * 6 + fc) * NF * NQF + qf;
    o[0] = T(val[0]);
    o[NQF] = T(dn * ih[ax]);
    for (int k = 1; k < MF; ++k) o[(1 + k) * NQF] = T(val[k]);
  }
}

// velocity factors at the 1-D point sets (the NQ Gauss points, then the lower
// and upper end of the element): every velocity kind is separable,
// u_d = Pe alpha_d(x) beta_d(y), so one row per element column (alpha) and one
// per element row (beta) serve every element:
//   va[(ex * 3 + d) * (NQ + 2) + q] = alpha_d,  vb[(ey * 3 + d) * (NQ + 2) + q] = beta_d
template <int P, typename T>
__global__ void __launch_bounds__(128) k_jlin_vel(KArgs A, T* __restrict__ va, T* __restrict__ vb) {
  constexpr int NN = P + 1, NQ = P + 2, W = NQ + 2;
  const double* cd = CT<double, P>::base();
  const int n0 = A.n[0], n1 = A.n[1];
  const int t = blockIdx.x * 128 + threadIdx.x;
  if (t >= (n0 + n1) * 3 * W) return;
  const bool isx = t < n0 * 3 * W;
  const int r = isx ? t : t - n0 * 3 * W;
  const int q = r % W, d = (r / W) % 3, col = r / (3 * W);
  // point q < NQ: Gauss point; NQ, NQ + 1: lower / upper end of the element
  const double tx = q < NQ ? 0.5 * (cd[2 * NQ * NN + NQ + q] + 1.0) : double(q - NQ);
  const double x = A.lo[0] + (col + tx) * A.h[0];
  const double y = A.lo[1] + (col + tx) * A.h[1];
  double al = 0.0, be = 0.0;
  if (A.vel_kind == DGNP_VEL_VORTEX) {
    double sx, cx, sy, cy;
    sincospi(x, &sx, &cx);
    sincospi(y, &sy, &cy);
    al = d == 0 ? sx : (d == 1 ? -cx : 0.0);
    be = d == 0 ? cy : (d == 1 ? sy : 0.0);
  } else if (A.vel_kind == DGNP_VEL_POISEUILLE_X) {
    const double yy = y - A.vel_ylo;
    al = d == 0 ? 1.0 : 0.0;
    be = d == 0 ? 6.0 * yy * (A.vel_H - yy) / (A.vel_H * A.vel_H) : 0.0;
  } else {
    al = A.vel_param[d];
    be = 1.0;
  }
  if (isx)
    va[r] = T(al);
  else
    vb[r] = T(be);
}

// ---------------------------------------------------------------------------
// the apply.  CPL = false: all rows of J v (input fields masked by vin_mask);
// CPL = true: potential rows of J v for an input whose potential part is zero,
// written as jbase - (J v) when jbase is set (the concentrations of v are read,
// its potential is not).
template <int P, int MF, typename T, bool CPL, int EPB, int NT>
__global__ void __launch_bounds__(NT, (sizeof(T) == 8 ? 5 : 1)) k_jlin(KArgs A, const T* __restrict__ vin, const T* __restrict__ tv,
                                                const T* __restrict__ tf, T* __restrict__ out, int64_t gper) {
  using S = Sz<3, P>;
  constexpr int NN = S::NN, NQ = S::NQ, NB = S::NB, NQV = S::NQV, NFN = S::NFN, NQF = S::NQF;
  constexpr int MI = CPL ? MF - 1 : MF;  // input fields held
  constexpr int FI0 = CPL ? 1 : 0;       // field of the first one
  constexpr int MO = CPL ? 1 : MF;       // output fields formed (from field 0 on)
  constexpr int NV = MF + 2, NFT = MF + 1;
  constexpr int QV = MI * 4 * NQV;
  constexpr int S1 = MI * 2 * NN * NN * NQ;
  constexpr int S2 = MI * 3 * NN * NQ * NQ;
  constexpr int VOLR = QV + S1 + S2;
  constexpr int NROW = 6 * 2 * MI * 2;  // face, side (own, neighbour), field, value / d/dx_ax
  constexpr int NCF = 6 * MO * 2 * NQF;
  constexpr int FACR = NROW * NQF + (NROW * NFN > NCF ? NROW * NFN : NCF);
  constexpr int REG = VOLR > FACR ? VOLR : FACR;
  static_assert(6 * MO * 2 * NFN <= NROW * NQF, "transposes must fit in the face-point area");
  __shared__ T s_v[EPB][MI * NB];
  __shared__ T s_o[EPB][MO * NB];
  __shared__ T R[EPB][REG];
  __shared__ int s_nb[EPB][6];
  __shared__ T s_al[EPB][3][NQ + 2], s_be[EPB][3][NQ + 2];  // velocity factors at x / y points

  const int64_t bid = blockIdx.x;
  const int64_t e0 = ((bid % 8) * gper + bid / 8) * EPB;  // one contiguous slab of groups per XCD
  if (e0 >= A.E) return;
  const int tid = threadIdx.x;
  const int64_t E = A.E, Nf = E * NB;
  using C = CT<T, P>;
  const Phys<T, MF> ph = make_phys<T, MF>(A);
  T ih[3], hh[3];
  for (int i = 0; i < 3; ++i) ih[i] = T(2.0 / A.h[i]);
  // face Jacobian per axis: a quarter of the product of the two tangential widths
  hh[0] = T(0.25 * A.h[1] * A.h[2]);
  hh[1] = T(0.25 * A.h[0] * A.h[2]);
  hh[2] = T(0.25 * A.h[0] * A.h[1]);
  const T peT = T(A.Pe), detT = T(A.detJ);
  // element coordinates (the element count fits in 32 bits; checked at launch)
  auto ecoord = [&](int64_t e, int d) -> int {
    const int ei = int(e);
    return d == 0 ? ei % A.n[0] : (d == 1 ? (ei / A.n[0]) % A.n[1] : ei / (A.n[0] * A.n[1]));
  };

  // ---- load v, neighbours, velocity factors
  for (int g = tid; g < EPB * MI * NB; g += NT) {
    const int el = g / (MI * NB), r = g % (MI * NB);
    const int fi = r / NB, l = r % NB, f = FI0 + fi;
    const int64_t e = e0 + el;
    s_v[el][r] = (e < E && ((A.vin_mask >> f) & 1u)) ? vin[f * Nf + e * NB + l] : T(0);
  }
  for (int g = tid; g < EPB * 6; g += NT) {
    const int el = g / 6;
    const int64_t e = e0 + el;
    s_nb[el][g % 6] = e < E ? A.nbr[e * 6 + g % 6] : -1;
  }
  {
    const T* va = tv + E * NV * NQV;
    const T* vb = va + int64_t(A.n[0]) * 3 * (NQ + 2);
    for (int g = tid; g < EPB * 3 * (NQ + 2); g += NT) {
      const int el = g / (3 * (NQ + 2)), r = g % (3 * (NQ + 2));
      const int64_t e = e0 + el < E ? e0 + el : E - 1;
      s_al[el][r / (NQ + 2)][r % (NQ + 2)] = va[ecoord(e, 0) * 3 * (NQ + 2) + r];
      s_be[el][r / (NQ + 2)][r % (NQ + 2)] = vb[ecoord(e, 1) * 3 * (NQ + 2) + r];
    }
  }
  __syncthreads();

  // ---- volume: interpolation of v (x lines, y lines, z lines)
  // layout per element: q [MI][4][NQV] | t1 [MI][NN][NN][2][NQ] | t2 [MI][NN][3][NQ][NQ]
  for (int g = tid; g < EPB * MI * NN * NN; g += NT) {
    const int el = g / (MI * NN * NN), ln = g % (MI * NN * NN);
    const T* up = &s_v[el][ln * NN];
    T x[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) x[a] = up[a];
    T* o = &R[el][QV + ln * 2 * NQ];
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
  for (int g = tid; g < EPB * MI * NN * NQ; g += NT) {
    const int el = g / (MI * NN * NQ), ln = g % (MI * NN * NQ);
    const int qx = ln % NQ, fc = ln / NQ;  // fc = (field, c)
    const T* t1 = &R[el][QV];
    T v0[NN], v1[NN];
#pragma unroll
    for (int b = 0; b < NN; ++b) {
      v0[b] = t1[((fc * NN + b) * 2 + 0) * NQ + qx];
      v1[b] = t1[((fc * NN + b) * 2 + 1) * NQ + qx];
    }
    T* o = &R[el][QV + S1 + fc * 3 * NQ * NQ];
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
  for (int g = tid; g < EPB * MI * NQ * NQ; g += NT) {
    const int el = g / (MI * NQ * NQ), ln = g % (MI * NQ * NQ);
    const int qxy = ln % (NQ * NQ), fi = ln / (NQ * NQ);
    T w0[NN], w1[NN], w2[NN];
#pragma unroll
    for (int c = 0; c < NN; ++c) {
      const T* tp = &R[el][QV + S1 + (fi * NN + c) * 3 * NQ * NQ + qxy];
      w0[c] = tp[0];
      w1[c] = tp[NQ * NQ];
      w2[c] = tp[2 * NQ * NQ];
    }
    T* o = &R[el][fi * 4 * NQV + qxy];
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

  // ---- pointwise linearised volume flux (gradient coefficients only: the
  // linearised volume terms have no value coefficient)
  for (int g = tid; g < EPB * NQV; g += NT) {
    const int el = g / NQV, qi = g % NQV;
    const int64_t e = e0 + el;
    if (e >= E) continue;
    const int qx = qi % NQ, qy = (qi / NQ) % NQ, qz = qi / (NQ * NQ);
    T val[MF], grad[MF][3], dv[MF], dg[MF][3], vg[MF][3], u[3];
    for (int f = 0; f < MF; ++f) {
      val[f] = dv[f] = T(0);
      for (int d = 0; d < 3; ++d) grad[f][d] = dg[f][d] = T(0);
    }
    const T* ts = tv + e * NV * NQV + qi;
    for (int k = 1; k < MF; ++k) val[k] = ts[(k - 1) * NQV];
    for (int d = 0; d < 3; ++d) grad[0][d] = ts[(MF - 1 + d) * NQV];
    for (int d = 0; d < 3; ++d) u[d] = peT * s_al[el][d][qx] * s_be[el][d][qy];
    const T* q = &R[el][0];
    for (int fi = 0; fi < MI; ++fi) {
      dv[FI0 + fi] = q[(fi * 4) * NQV + qi];
      for (int d = 0; d < 3; ++d) dg[FI0 + fi][d] = q[(fi * 4 + 1 + d) * NQV + qi];
    }
    vol_jac<T, MF, 3>(ph, val, grad, u, dv, dg, vg);
    const T w = detT * C::base()[2 * NQ * NN + qx] * C::base()[2 * NQ * NN + qy] * C::base()[2 * NQ * NN + qz];
    T* o = &R[el][0];
    for (int fo = 0; fo < MO; ++fo)
      for (int d = 0; d < 3; ++d) o[(fo * 4 + 1 + d) * NQV + qi] = vg[fo][d] * w * ih[d];
  }
  __syncthreads();

  // ---- transposed contractions (z, y, x lines) into s_o; t1/t2 reused
  for (int g = tid; g < EPB * MO * NQ * NQ; g += NT) {
    const int el = g / (MO * NQ * NQ), ln = g % (MO * NQ * NQ);
    const int qxy = ln % (NQ * NQ), fo = ln / (NQ * NQ);
    const T* cp = &R[el][fo * 4 * NQV + qxy];
    T cx[NQ], cy[NQ], cz[NQ];
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      cx[qz] = cp[NQV + qz * NQ * NQ];
      cy[qz] = cp[2 * NQV + qz * NQ * NQ];
      cz[qz] = cp[3 * NQV + qz * NQ * NQ];
    }
    T* op = &R[el][QV + S1 + fo * NN * 3 * NQ * NQ + qxy];  // [fo][c][3][qy][qx]
#pragma unroll
    for (int cc = 0; cc < NN; ++cc) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int qz = 0; qz < NQ; ++qz) {
        s0 += C::D(qz, cc) * cz[qz];
        s1 += C::B(qz, cc) * cy[qz];
        s2 += C::B(qz, cc) * cx[qz];
      }
      op[(cc * 3 + 0) * NQ * NQ] = s0;
      op[(cc * 3 + 1) * NQ * NQ] = s1;
      op[(cc * 3 + 2) * NQ * NQ] = s2;
    }
  }
  __syncthreads();
  for (int g = tid; g < EPB * MO * NN * NQ; g += NT) {
    const int el = g / (MO * NN * NQ), ln = g % (MO * NN * NQ);
    const int qx = ln % NQ, fcc = ln / NQ;  // (fo, c)
    const T* tp = &R[el][QV + S1 + fcc * 3 * NQ * NQ + qx];
    T a0[NQ], a1[NQ], a2[NQ];
#pragma unroll
    for (int qy = 0; qy < NQ; ++qy) {
      a0[qy] = tp[qy * NQ];
      a1[qy] = tp[NQ * NQ + qy * NQ];
      a2[qy] = tp[2 * NQ * NQ + qy * NQ];
    }
    T* op = &R[el][QV + fcc * NN * 2 * NQ + qx];  // [fo][c][b][2][qx]
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
  for (int g = tid; g < EPB * MO * NN * NN; g += NT) {
    const int el = g / (MO * NN * NN), ln = g % (MO * NN * NN);
    const T* tp = &R[el][QV + ln * 2 * NQ];
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
      s_o[el][ln * NN + a] = s;
    }
  }
  __syncthreads();

  // ---- faces.  Per element: fq [NROW][NQF] face-point traces, fn [..][NFN]
  // node traces; cf [6][MO][2][NQF] coefficients over fn, tnt [6][MO][2][NFN]
  // transposes over fq.  Trace row of (face, side, field, value / d/dx_ax):
  auto trow = [](int fc, int sd, int fi, int c2) { return ((fc * 2 + sd) * MI + fi) * 2 + c2; };
  // F1: node traces of own (side 0) and neighbour (side 1) element
  for (int g = tid; g < EPB * (NROW / 2) * NFN; g += NT) {
    const int el = g / ((NROW / 2) * NFN), r = g % ((NROW / 2) * NFN);
    const int ij = r % NFN, pr = r / NFN;  // pr = (fc, sd, fi)
    const int fi = pr % MI, sd = (pr / MI) & 1, fc = pr / (2 * MI);
    const int ax = fc >> 1;
    const int side = (fc & 1) ? 1 : -1;
    const int sside = sd == 0 ? side : -side;
    const int i = ij % NN, j = ij / NN;
    const int f = FI0 + fi, nb = s_nb[el][fc];
    const bool has = sd == 0 || (nb >= 0 && ((A.vin_mask >> f) & 1u));
    const T* u = sd == 0 ? &s_v[el][fi * NB] : vin + f * Nf + int64_t(nb >= 0 ? nb : 0) * NB;
    T x[NN];
#pragma unroll
    for (int l = 0; l < NN; ++l) x[l] = has ? u[face_node<3, NN>(ax, l, i, j)] : T(0);
    const T val = sside < 0 ? x[0] : x[P];
    T dn = T(0);
#pragma unroll
    for (int l = 0; l < NN; ++l) dn += (sside < 0 ? C::De(0, l) : C::De(1, l)) * x[l];
    dn *= ih[ax];
    T* fn = &R[el][NROW * NQF];
    fn[(2 * pr + 0) * NFN + ij] = val;
    fn[(2 * pr + 1) * NFN + ij] = dn;
  }
  __syncthreads();
  // F2/F3: node traces to face points, one lane per (row, qi): along i with the
  // lane's B(qi, .), then along j with compile-time B(qj, .)
  for (int g = tid; g < EPB * NROW * NQ; g += NT) {
    const int el = g / (NROW * NQ), r = g % (NROW * NQ);
    const int row = r / NQ, qi = r % NQ;
    const T* fn = &R[el][NROW * NQF + row * NFN];
    T yv[NN];
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      T t = T(0);
#pragma unroll
      for (int i = 0; i < NN; ++i) t += C::B(qi, i) * fn[j * NN + i];
      yv[j] = t;
    }
    T* fq = &R[el][row * NQF];
#pragma unroll
    for (int qj = 0; qj < NQ; ++qj) {
      T t = T(0);
#pragma unroll
      for (int j = 0; j < NN; ++j) t += C::B(qj, j) * yv[j];
      fq[qj * NQ + qi] = t;
    }
  }
  __syncthreads();
  // F4: linearised numerical fluxes -> coefficients of the own element's
  // value and d/dx_ax traces (face weights included)
  for (int g = tid; g < EPB * 6 * NQF; g += NT) {
    const int el = g / (6 * NQF), r = g % (6 * NQF);
    const int qf = r % NQF, fc = r / NQF;
    const int64_t e = e0 + el;
    const int ax = fc >> 1;
    const int side = (fc & 1) ? 1 : -1;
    const int nb = s_nb[el][fc];
    const bool interior = nb >= 0;
    const int cbc = interior ? 0 : A.c_bc[fc];
    const bool phid = interior ? false : (A.phi_bc[fc] == DGNP_PHI_DIRICHLET);
    T Fo[MF], Go[MF];
    for (int f = 0; f < MF; ++f) Fo[f] = Go[f] = T(0);
    T w = T(0);
    const T* fq = &R[el][0];
    if (e < E && (interior || cbc != BC_WALL || phid)) {
      const int qi = qf % NQ, qj = qf / NQ;
      const T* wq = C::base() + 2 * NQ * NN;
      w = hh[ax] * wq[qi] * wq[qj];
      // u . e_ax at the face point: x index (end point of x faces, else the
      // first tangential point), y index (end point of y faces, else the
      // first tangential point of x faces / the second of z faces)
      const int ix = ax == 0 ? NQ + (side > 0) : qi;
      const int iy = ax == 1 ? NQ + (side > 0) : (ax == 0 ? qi : qj);
      const T uax = peT * s_al[el][ax][ix] * s_be[el][ax][iy];
      const T* so = tf + ((e * 6 + fc) * NFT) * NQF + qf;
      const T* sn = tf + ((interior ? int64_t(nb) * 6 + (fc ^ 1) : 0) * NFT) * NQF + qf;
      // the own outward normal is side * e_ax: normal derivatives and the
      // normal velocity are the d/dx_ax ones times sg
      const T sg = T(side);
      T vo[MF], tvo[MF], tgo[MF];
      for (int f = 0; f < MF; ++f) vo[f] = tvo[f] = tgo[f] = T(0);
      vo[0] = so[0];
      for (int k = 1; k < MF; ++k) vo[k] = so[(1 + k) * NQF];
      for (int fi = 0; fi < MI; ++fi) {
        tvo[FI0 + fi] = fq[trow(fc, 0, fi, 0) * NQF + qf];
        tgo[FI0 + fi] = sg * fq[trow(fc, 0, fi, 1) * NQF + qf];
      }
      if (interior) {
        T vn[MF], tvn[MF], tgn[MF], Gn[MF];
        for (int f = 0; f < MF; ++f) vn[f] = tvn[f] = tgn[f] = T(0);
        vn[0] = sn[0];
        for (int k = 1; k < MF; ++k) vn[k] = sn[(1 + k) * NQF];
        for (int fi = 0; fi < MI; ++fi) {
          tvn[FI0 + fi] = fq[trow(fc, 1, fi, 0) * NQF + qf];
          tgn[FI0 + fi] = sg * fq[trow(fc, 1, fi, 1) * NQF + qf];
        }
        face_jac_own<T, MF>(ph, vo, vn, sg * so[NQF], sg * sn[NQF], tvo, tvn, tgo, tgn, sg * uax, Fo, Gn);
        for (int f = 0; f < MF; ++f) Go[f] = sg * Gn[f];  // outward normal derivative -> d/dx_ax
      } else {
        const int ex = ecoord(e, 0), ey = ecoord(e, 1), ez = ecoord(e, 2);
        const int64_t lin =
            ax == 0 ? ey + int64_t(A.n[1]) * ez : (ax == 1 ? ex + int64_t(A.n[0]) * ez : ex + int64_t(A.n[0]) * ey);
        const int64_t bf = A.btag_off[fc] + lin;
        T gd[MF], gno[MF];
        for (int f = 0; f < MF; ++f) gno[f] = T(0);
        gno[0] = sg * so[NQF];
        for (int f = 0; f < MF; ++f) gd[f] = T(A.bcq[(f * A.n_bface + bf) * NQF + qf]);
        bnd_jac<T, MF>(ph, vo, gno, tvo, tgo, sg * uax, cbc, phid, gd, Fo, Go);
        for (int f = 0; f < MF; ++f) Go[f] *= sg;  // outward normal derivative -> d/dx_ax
      }
    }
    T* cf = &R[el][NROW * NQF];
    for (int fo = 0; fo < MO; ++fo) {
      cf[((fc * MO + fo) * 2 + 0) * NQF + qf] = Fo[fo] * w;
      cf[((fc * MO + fo) * 2 + 1) * NQF + qf] = Go[fo] * w * ih[ax];
    }
  }
  __syncthreads();
  // F5: face-point coefficients back to node traces, one lane per (row, j):
  // along qj with the lane's B(., j), then along qi with compile-time B(., i)
  for (int g = tid; g < EPB * 6 * MO * 2 * NN; g += NT) {
    const int el = g / (6 * MO * 2 * NN), r = g % (6 * MO * 2 * NN);
    const int rc = r / NN, j = r % NN;
    const T* cf = &R[el][NROW * NQF + rc * NQF];
    T yv[NQ];
#pragma unroll
    for (int qi = 0; qi < NQ; ++qi) {
      T t = T(0);
#pragma unroll
      for (int qj = 0; qj < NQ; ++qj) t += C::B(qj, j) * cf[qj * NQ + qi];
      yv[qi] = t;
    }
    T* tnt = &R[el][rc * NFN];
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      T t = T(0);
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) t += C::B(qi, i) * yv[qi];
      tnt[j * NN + i] = t;
    }
  }
  __syncthreads();
  // F6: every node gathers its value / normal-derivative contributions
  const T* jb = static_cast<const T*>(A.jbase);
  for (int g = tid; g < EPB * MO * NB; g += NT) {
    const int el = g / (MO * NB), r = g % (MO * NB);
    const int64_t e = e0 + el;
    if (e >= E) continue;
    const int fo = r / NB, node = r % NB;
    const int cx = node % NN, cy = (node / NN) % NN, cz = node / (NN * NN);
    T acc = s_o[el][r];
    const T* tnt = &R[el][0];
#pragma unroll
    for (int fc = 0; fc < 6; ++fc) {
      const int ax = fc >> 1;
      const int sdi = fc & 1;
      const int l = ax == 0 ? cx : (ax == 1 ? cy : cz);
      const int i = ax == 0 ? cy : cx;
      const int j = ax == 2 ? cy : cz;
      const int rc = fc * MO + fo;
      const int ij = j * NN + i;
      acc += C::De(sdi, l) * tnt[(rc * 2 + 1) * NFN + ij];
      if (l == (sdi ? P : 0)) acc += tnt[(rc * 2 + 0) * NFN + ij];
    }
    const int64_t o = fo * Nf + e * NB + node;
    if constexpr (CPL)
      out[o] = jb ? jb[o] - acc : acc;
    else
      out[o] = acc;
  }
}

// ---------------------------------------------------------------------------
template <int P, int MF, typename T>
static void tab_t(const KArgs& A, const double* xs, T* tv, T* tf, hipStream_t s) {
  constexpr int NQ = P + 2;
  hipLaunchKernelGGL((k_jlin_tab<P, MF, T>), dim3(unsigned(A.E)), dim3(128), 0, s, A, xs, tv, tf);
  DGNP_HIP(hipGetLastError());
  T* va = tv + A.E * (MF + 2) * NQ * NQ * NQ;
  T* vb = va + int64_t(A.n[0]) * 3 * (NQ + 2);
  const int nv = (A.n[0] + A.n[1]) * 3 * (NQ + 2);
  hipLaunchKernelGGL((k_jlin_vel<P, T>), dim3(unsigned((nv + 127) / 128)), dim3(128), 0, s, A, va, vb);
  DGNP_HIP(hipGetLastError());
}

template <typename T>
void launch_jlin_tables(int p, int m, const KArgs& A, const double* xs, T* tv, T* tf, hipStream_t s) {
  if (A.E == 0) return;
  if (m == 2) {
    if (p == 1) return tab_t<1, 2, T>(A, xs, tv, tf, s);
    if (p == 2) return tab_t<2, 2, T>(A, xs, tv, tf, s);
    if (p == 3) return tab_t<3, 2, T>(A, xs, tv, tf, s);
  } else if (m == 3) {
    if (p == 1) return tab_t<1, 3, T>(A, xs, tv, tf, s);
    if (p == 2) return tab_t<2, 3, T>(A, xs, tv, tf, s);
    if (p == 3) return tab_t<3, 3, T>(A, xs, tv, tf, s);
  }
  throw Error(DGNP_E_ARG, "tabulated Jacobian: orders 1..3, 2 or 3 ions");
}

template <int P, int MF, typename T, bool CPL, int EPB, int NT>
static void jl_v(const KArgs& A, const T* v, const T* tv, const T* tf, T* y, hipStream_t s) {
  const int64_t groups = (A.E + EPB - 1) / EPB;
  const int64_t gper = (groups + 7) / 8;
  hipLaunchKernelGGL((k_jlin<P, MF, T, CPL, EPB, NT>), dim3(unsigned(8 * gper)), dim3(NT), 0, s, A, v, tv, tf, y,
                     gper);
  DGNP_HIP(hipGetLastError());
}

// launch shape (elements per work-group x threads): the default, or for order 3
// a variant chosen by the value of DGNP_JAC_VARIANT (A/B measurement)
static int jl_variant() {
  const char* e = getenv("DGNP_JAC_VARIANT");
  return e ? atoi(e) : 0;
}

template <int P, int MF, typename T, bool CPL>
static void jl_t(const KArgs& A, const T* v, const T* tv, const T* tf, T* y, hipStream_t s) {
  if constexpr (P >= 2) {
    switch (jl_variant()) {  // elements per work-group * 1000 + threads
      case 1064: return jl_v<P, MF, T, CPL, 1, 64>(A, v, tv, tf, y, s);
      case 1128: return jl_v<P, MF, T, CPL, 1, 128>(A, v, tv, tf, y, s);
      case 1256: return jl_v<P, MF, T, CPL, 1, 256>(A, v, tv, tf, y, s);
      case 2128: return jl_v<P, MF, T, CPL, 2, 128>(A, v, tv, tf, y, s);
      case 2256: return jl_v<P, MF, T, CPL, 2, 256>(A, v, tv, tf, y, s);
      default: break;
    }
  }
  jl_v<P, MF, T, CPL, Shape<P, T, CPL>::epb, Shape<P, T, CPL>::nt>(A, v, tv, tf, y, s);
}

template <typename T>
void launch_jlin(int p, int m, bool coupling, const KArgs& A, const T* v, const T* tv, const T* tf, T* y,
                 hipStream_t s) {
  if (A.E == 0) return;
  DGNP_REQUIRE(A.E < (int64_t(1) << 31), DGNP_E_ARG, "tabulated Jacobian: element count beyond 32 bits");
#define JL_CASE(PP, MM)                                                \
  if (p == PP && m == MM) {                                            \
    if (coupling) return jl_t<PP, MM, T, true>(A, v, tv, tf, y, s);    \
    return jl_t<PP, MM, T, false>(A, v, tv, tf, y, s);                 \
  }
  JL_CASE(1, 2)
  JL_CASE(2, 2)
  JL_CASE(3, 2)
  JL_CASE(1, 3)
  JL_CASE(2, 3)
  JL_CASE(3, 3)
#undef JL_CASE
  throw Error(DGNP_E_ARG, "tabulated Jacobian: orders 1..3, 2 or 3 ions");
}

size_t jlin_table_sizes(int p, int m, int64_t E, const int* n, size_t* nf) {
  const size_t nq = size_t(p) + 2;
  if (nf) *nf = size_t(E) * 6 * (m + 1) * nq * nq;
  return size_t(E) * (m + 2) * nq * nq * nq + size_t(n[0] + n[1]) * 3 * (nq + 2);
}

template void launch_jlin_tables<double>(int, int, const KArgs&, const double*, double*, double*, hipStream_t);
template void launch_jlin_tables<float>(int, int, const KArgs&, const double*, float*, float*, hipStream_t);
template void launch_jlin<double>(int, int, bool, const KArgs&, const double*, const double*, const double*, double*,
                                  hipStream_t);
template void launch_jlin<float>(int, int, bool, const KArgs&, const float*, const float*, const float*, float*,
                                 hipStream_t);

}  // namespace dgnp
