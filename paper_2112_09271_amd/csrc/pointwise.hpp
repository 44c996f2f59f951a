// Pointwise fluxes of the DG scheme for the charge-conservation Nernst-Planck
// model (arXiv 2112.09271, Sec. 3.2-3.3, Eqs. NPDG and chargeDG, nondimensional
// form of Sec. 2.3).  Every function works on one quadrature point and is
// callable on host and device.  Field f = 0 is the potential phi, f = k >= 1 the
// concentration c_k; species constants are indexed k - 1.
//
//   a_k = z_k (D_k - D_m),  b_k = z_k (z_k D_k - z_m D_m),  kappa = sum_k b_k c_k,
//   q_k = u - z_k D_k grad phi.
//
// Volume: the test function enters through "vv * v + vg . grad v".
// Faces: through "Fv * v + G * dv/dn" per side.  On interior faces the normal
// n points from the lower ("minus", side 0) element to the upper ("plus",
// side 1) one, [w] = w_minus - w_plus, {w} = average; the upwind flux is
// {c q}.n + |{q}.n| [c] / 2 and the potential carries SIPG with penalty
// {kappa} delta [phi].  On boundary faces n is the outward normal.
// d|s| = sign(s) ds with sign(0) = 0.
//
// Each linearised flux exists in a forward form (trial -> test coefficients)
// and an exact transpose (test traces -> trial coefficients), so that the
// matrix-free operator and its adjoint come from the same formulas.
#pragma once

#include <hip/hip_runtime.h>

namespace dgnp {

enum { BC_WALL = 0, BC_DIRICHLET = 1, BC_INFLOW = 2, BC_OUTFLOW = 3, BC_ELECTRODE = 4 };

template <typename T, int MF>
struct Phys {
  T zD[MF];     // z_k D_k, index k-1
  T D[MF];
  T a[MF];
  T b[MF];
  T delta;      // interior penalty C_IP p^2 / h
  // Butler-Volmer electrode faces: the reacting ion r (1..m; m is the
  // eliminated one), its valence, the exponents alpha_a n and alpha_c n, and
  // the derivatives of c_r with respect to c_1..c_{m-1} (a unit vector, or
  // -z_k / z_m by electroneutrality when r = m), index k-1
  int bv_r;
  T bv_z, bv_aa, bv_ac;
  T bv_dc[MF];
};

template <typename T>
__host__ __device__ inline T sgn(T s) { return s > T(0) ? T(1) : (s < T(0) ? T(-1) : T(0)); }
template <typename T>
__host__ __device__ inline T pos(T s) { return s > T(0) ? s : T(0); }
template <typename T>
__host__ __device__ inline T neg(T s) { return s < T(0) ? s : T(0); }
template <typename T>
__host__ __device__ inline T fabs_(T s) { return s < T(0) ? -s : s; }

// ----------------------------------------------------------------------------
// Volume terms.  val[f], grad[f][i] of the state; outputs vv[f], vg[f][i].
template <typename T, int MF, int DIM>
__host__ __device__ inline void vol_res(const Phys<T, MF>& ph, const T* val, const T (*grad)[DIM],
                                        const T* u, const T* src, T* vv, T (*vg)[DIM]) {
  T kap = T(0);
  for (int k = 1; k < MF; ++k) kap += ph.b[k - 1] * val[k];
  vv[0] = -src[0];
  for (int i = 0; i < DIM; ++i) {
    T cur = kap * grad[0][i];
    for (int k = 1; k < MF; ++k) cur += ph.a[k - 1] * grad[k][i];
    vg[0][i] = cur;
  }
  for (int k = 1; k < MF; ++k) {
    vv[k] = -src[k];
    for (int i = 0; i < DIM; ++i) {
      T q = u[i] - ph.zD[k - 1] * grad[0][i];
      vg[k][i] = ph.D[k - 1] * grad[k][i] - val[k] * q;
    }
  }
}

// forward linearisation: trial (dval, dgrad) -> test (vg); no value coefficient
template <typename T, int MF, int DIM>
__host__ __device__ inline void vol_jac(const Phys<T, MF>& ph, const T* val, const T (*grad)[DIM],
                                        const T* u, const T* dval, const T (*dgrad)[DIM],
                                        T (*vg)[DIM]) {
  T kap = T(0), dkap = T(0);
  for (int k = 1; k < MF; ++k) {
    kap += ph.b[k - 1] * val[k];
    dkap += ph.b[k - 1] * dval[k];
  }
  for (int i = 0; i < DIM; ++i) {
    T cur = dkap * grad[0][i] + kap * dgrad[0][i];
    for (int k = 1; k < MF; ++k) cur += ph.a[k - 1] * dgrad[k][i];
    vg[0][i] = cur;
  }
  for (int k = 1; k < MF; ++k) {
    for (int i = 0; i < DIM; ++i) {
      T q = u[i] - ph.zD[k - 1] * grad[0][i];
      T dq = -ph.zD[k - 1] * dgrad[0][i];
      vg[k][i] = ph.D[k - 1] * dgrad[k][i] - dval[k] * q - val[k] * dq;
    }
  }
}

// transpose: test gradients gw[f][i] -> trial coefficients (tv[f] value, tg[f][i] gradient)
template <typename T, int MF, int DIM>
__host__ __device__ inline void vol_jacT(const Phys<T, MF>& ph, const T* val, const T (*grad)[DIM],
                                         const T* u, const T (*gw)[DIM], T* tv, T (*tg)[DIM]) {
  T kap = T(0);
  for (int k = 1; k < MF; ++k) kap += ph.b[k - 1] * val[k];
  T gphi_gw0 = T(0);
  for (int i = 0; i < DIM; ++i) gphi_gw0 += grad[0][i] * gw[0][i];
  tv[0] = T(0);
  for (int i = 0; i < DIM; ++i) tg[0][i] = kap * gw[0][i];
  for (int k = 1; k < MF; ++k) {
    T qdot = T(0);
    for (int i = 0; i < DIM; ++i) {
      T q = u[i] - ph.zD[k - 1] * grad[0][i];
      qdot += q * gw[k][i];
      tg[k][i] = ph.D[k - 1] * gw[k][i] + ph.a[k - 1] * gw[0][i];
      tg[0][i] += val[k] * ph.zD[k - 1] * gw[k][i];
    }
    tv[k] = -qdot + ph.b[k - 1] * gphi_gw0;
  }
}

// derivative with respect to the velocity scale (u = Pe * uh)
template <typename T, int MF, int DIM>
__host__ __device__ inline void vol_dpe(const Phys<T, MF>& ph, const T* val, const T* uh, T (*vg)[DIM]) {
  for (int i = 0; i < DIM; ++i) vg[0][i] = T(0);
  for (int k = 1; k < MF; ++k)
    for (int i = 0; i < DIM; ++i) vg[k][i] = -val[k] * uh[i];
}

// ----------------------------------------------------------------------------
// Interior faces.  Traces v[s][f], g[s][f] (value, d/dn) on side s = 0 (minus),
// 1 (plus); un = u.n.  Outputs: coefficients of v and dv/dn on the side `o`.
template <typename T, int MF>
__host__ __device__ inline void face_res(const Phys<T, MF>& ph, const T (*v)[MF], const T (*g)[MF],
                                         T un, int o, T* Fo, T* Go) {
  T kap[2] = {T(0), T(0)};
  for (int k = 1; k < MF; ++k) {
    kap[0] += ph.b[k - 1] * v[0][k];
    kap[1] += ph.b[k - 1] * v[1][k];
  }
  const T sign_o = o == 0 ? T(1) : T(-1);
  T jphi = v[0][0] - v[1][0];
  T cur0 = kap[0] * g[0][0], cur1 = kap[1] * g[1][0], ajc = T(0);
  for (int k = 1; k < MF; ++k) {
    cur0 += ph.a[k - 1] * g[0][k];
    cur1 += ph.a[k - 1] * g[1][k];
    ajc += ph.a[k - 1] * (v[0][k] - v[1][k]);
  }
  T F0 = -T(0.5) * (cur0 + cur1) + T(0.5) * (kap[0] + kap[1]) * ph.delta * jphi;
  Fo[0] = sign_o * F0;
  Go[0] = -T(0.5) * ajc - T(0.5) * kap[o] * jphi;
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Qm = un - zD * g[0][0], Qp = un - zD * g[1][0];
    T Qb = un - zD * T(0.5) * (g[0][0] + g[1][0]);
    T jc = v[0][k] - v[1][k];
    T F = -T(0.5) * D * (g[0][k] + g[1][k]) + D * ph.delta * jc +
          T(0.5) * (v[0][k] * Qm + v[1][k] * Qp) + T(0.5) * fabs_(Qb) * jc;
    Fo[k] = sign_o * F;
    Go[k] = -T(0.5) * D * jc;
  }
}

// forward linearisation; (tv, tg) trial traces on both sides
template <typename T, int MF>
__host__ __device__ inline void face_jac(const Phys<T, MF>& ph, const T (*v)[MF], const T (*g)[MF],
                                         const T (*tv)[MF], const T (*tg)[MF], T un, int o, T* Fo,
                                         T* Go) {
  T kap[2] = {T(0), T(0)}, dkap[2] = {T(0), T(0)};
  for (int k = 1; k < MF; ++k)
    for (int s = 0; s < 2; ++s) {
      kap[s] += ph.b[k - 1] * v[s][k];
      dkap[s] += ph.b[k - 1] * tv[s][k];
    }
  const T sign_o = o == 0 ? T(1) : T(-1);
  T jphi = v[0][0] - v[1][0], djphi = tv[0][0] - tv[1][0];
  T dcur0 = dkap[0] * g[0][0] + kap[0] * tg[0][0];
  T dcur1 = dkap[1] * g[1][0] + kap[1] * tg[1][0];
  T dajc = T(0);
  for (int k = 1; k < MF; ++k) {
    dcur0 += ph.a[k - 1] * tg[0][k];
    dcur1 += ph.a[k - 1] * tg[1][k];
    dajc += ph.a[k - 1] * (tv[0][k] - tv[1][k]);
  }
  T F0 = -T(0.5) * (dcur0 + dcur1) + T(0.5) * (dkap[0] + dkap[1]) * ph.delta * jphi +
         T(0.5) * (kap[0] + kap[1]) * ph.delta * djphi;
  Fo[0] = sign_o * F0;
  Go[0] = -T(0.5) * dajc - T(0.5) * dkap[o] * jphi - T(0.5) * kap[o] * djphi;
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Qm = un - zD * g[0][0], Qp = un - zD * g[1][0];
    T Qb = un - zD * T(0.5) * (g[0][0] + g[1][0]);
    T dQm = -zD * tg[0][0], dQp = -zD * tg[1][0];
    T jc = v[0][k] - v[1][k], djc = tv[0][k] - tv[1][k];
    T F = -T(0.5) * D * (tg[0][k] + tg[1][k]) + D * ph.delta * djc +
          T(0.5) * (tv[0][k] * Qm + v[0][k] * dQm + tv[1][k] * Qp + v[1][k] * dQp) +
          T(0.5) * sgn(Qb) * T(0.5) * (dQm + dQp) * jc + T(0.5) * fabs_(Qb) * djc;
    Fo[k] = sign_o * F;
    Go[k] = -T(0.5) * D * djc;
  }
}

// The same forward linearisation written from one side's point of view: the
// own side (o) and the neighbour side (n), every derivative and the velocity
// taken along the own element's outward normal.  For the own side as the
// minus side this is face_jac with o = 0; for the plus side every normal
// quantity changes sign, and the jumps [w] and the factor sign_o of face_jac
// change sign with it, so that both cases give the same expressions.  Outputs:
// Fo, the coefficient of the own test value (as face_jac), and Gn, that of its
// outward normal derivative (face_jac's Go is sign_o Gn).  No side index is
// taken at run time.
//   vo, vn: state values; gpo, gpn: state d phi/dn; tvo, tvn: trial values;
//   tgo, tgn: trial d/dn (every field); un: u . n.
template <typename T, int MF>
__host__ __device__ inline void face_jac_own(const Phys<T, MF>& ph, const T* vo, const T* vn, T gpo, T gpn,
                                             const T* tvo, const T* tvn, const T* tgo, const T* tgn, T un, T* Fo,
                                             T* Gn) {
  T kapo = T(0), kapn = T(0), dkapo = T(0), dkapn = T(0), sa = T(0), da = T(0);
  for (int k = 1; k < MF; ++k) {
    kapo += ph.b[k - 1] * vo[k];
    kapn += ph.b[k - 1] * vn[k];
    dkapo += ph.b[k - 1] * tvo[k];
    dkapn += ph.b[k - 1] * tvn[k];
    sa += ph.a[k - 1] * (tgo[k] + tgn[k]);
    da += ph.a[k - 1] * (tvo[k] - tvn[k]);
  }
  const T jphi = vo[0] - vn[0], djphi = tvo[0] - tvn[0];
  const T dcur = dkapo * gpo + kapo * tgo[0] + dkapn * gpn + kapn * tgn[0] + sa;
  Fo[0] = -T(0.5) * dcur + T(0.5) * (dkapo + dkapn) * ph.delta * jphi + T(0.5) * (kapo + kapn) * ph.delta * djphi;
  Gn[0] = -T(0.5) * da - T(0.5) * dkapo * jphi - T(0.5) * kapo * djphi;
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    const T Qo = un - zD * gpo, Qn = un - zD * gpn;
    const T Qb = un - zD * T(0.5) * (gpo + gpn);
    const T dQo = -zD * tgo[0], dQn = -zD * tgn[0];
    const T jc = vo[k] - vn[k], djc = tvo[k] - tvn[k];
    Fo[k] = -T(0.5) * D * (tgo[k] + tgn[k]) + D * ph.delta * djc +
            T(0.5) * (tvo[k] * Qo + vo[k] * dQo + tvn[k] * Qn + vn[k] * dQn) +
            T(0.25) * sgn(Qb) * (dQo + dQn) * jc + T(0.5) * fabs_(Qb) * djc;
    Gn[k] = -T(0.5) * D * djc;
  }
}

// transpose: test traces (wv, wg) on both sides -> coefficients of the trial
// value and d/dn on side o
template <typename T, int MF>
__host__ __device__ inline void face_jacT(const Phys<T, MF>& ph, const T (*v)[MF], const T (*g)[MF],
                                          const T (*wv)[MF], const T (*wg)[MF], T un, int o, T* To,
                                          T* Tgo) {
  T kap[2] = {T(0), T(0)};
  for (int k = 1; k < MF; ++k)
    for (int s = 0; s < 2; ++s) kap[s] += ph.b[k - 1] * v[s][k];
  const T so = o == 0 ? T(1) : T(-1);  // d[.]/d(own value)
  T jphi = v[0][0] - v[1][0];
  T W0 = wv[0][0] - wv[1][0];
  T SG0 = wg[0][0] + wg[1][0];
  // potential trial on side o
  To[0] = so * (W0 * T(0.5) * (kap[0] + kap[1]) * ph.delta) -
          so * T(0.5) * (kap[0] * wg[0][0] + kap[1] * wg[1][0]);
  Tgo[0] = -T(0.5) * kap[o] * W0;
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1], ak = ph.a[k - 1], bk = ph.b[k - 1];
    T Qo = un - zD * g[o][0];
    T Qb = un - zD * T(0.5) * (g[0][0] + g[1][0]);
    T jc = v[0][k] - v[1][k];
    T Wk = wv[0][k] - wv[1][k];
    T SGk = wg[0][k] + wg[1][k];
    // concentration value on side o
    T c = Wk * (so * D * ph.delta + T(0.5) * Qo + so * T(0.5) * fabs_(Qb)) - so * T(0.5) * D * SGk;
    c += W0 * bk * (-T(0.5) * g[o][0] + T(0.5) * ph.delta * jphi);
    c += -so * T(0.5) * ak * SG0 - T(0.5) * bk * jphi * wg[o][0];
    To[k] = c;
    Tgo[k] = -T(0.5) * D * Wk - T(0.5) * ak * W0;
    // potential normal derivative through q_k on side o
    Tgo[0] += Wk * (-zD) * (T(0.5) * v[o][k] + T(0.25) * sgn(Qb) * jc);
  }
}

template <typename T, int MF>
__host__ __device__ inline void face_dpe(const Phys<T, MF>& ph, const T (*v)[MF], const T (*g)[MF],
                                         T un, T uhn, int o, T* Fo, T* Go) {
  const T sign_o = o == 0 ? T(1) : T(-1);
  Fo[0] = T(0);
  Go[0] = T(0);
  for (int k = 1; k < MF; ++k) {
    const T zD = ph.zD[k - 1];
    T Qb = un - zD * T(0.5) * (g[0][0] + g[1][0]);
    T jc = v[0][k] - v[1][k];
    T F = T(0.5) * (v[0][k] + v[1][k]) * uhn + T(0.5) * sgn(Qb) * uhn * jc;
    Fo[k] = sign_o * F;
    Go[k] = T(0);
  }
}

// ----------------------------------------------------------------------------
// Butler-Volmer rate of the reacting ion at an electrode point (Sec. 2.1 Eq. bv
// in the nondimensional form of Sec. 2.3, gamma = 1, reductant of constant
// concentration as in Sec. 5.2):
//   g = J0 [exp(alpha_a n eta) - c_r exp(-alpha_c n eta)],  eta = phi_app - phi,
// with the point data gd[0] = phi_app and gd[1] = J0 (exchange current times
// its profile).  It enters the reacting ion's equation as -g v (Eq. NPDG,
// Eq. electrode) and the charge equation as -z_r g v (Eq. chargeDG).
template <typename T>
struct BvRate {
  T g, dphi, dc, dj0, dpa;  // g and its derivatives: phi, c_r, J0, phi_app
};

template <typename T, int MF>
__host__ __device__ inline T bv_conc(const Phys<T, MF>& ph, const T* v) {
  T c = T(0);
  for (int k = 1; k < MF; ++k) c += ph.bv_dc[k - 1] * v[k];
  return c;
}

template <typename T, int MF>
__host__ __device__ inline BvRate<T> bv_rate(const Phys<T, MF>& ph, const T* v, const T* gd) {
  const T eta = gd[0] - v[0];
  const T ea = exp(ph.bv_aa * eta), ec = exp(-ph.bv_ac * eta);
  const T c = bv_conc(ph, v);
  BvRate<T> r;
  r.g = gd[1] * (ea - c * ec);
  r.dphi = gd[1] * (-ph.bv_aa * ea - c * ph.bv_ac * ec);
  r.dc = -gd[1] * ec;
  r.dj0 = ea - c * ec;
  r.dpa = -r.dphi;
  return r;
}

// value coefficients of the electrode terms for a rate (or its linearisation) s
template <typename T, int MF>
__host__ __device__ inline void bv_add(const Phys<T, MF>& ph, T s, T* F) {
  if (ph.bv_r < MF) F[ph.bv_r] -= s;
  F[0] -= ph.bv_z * s;
}

// the test-trace combination that the electrode terms are tested with
template <typename T, int MF>
__host__ __device__ inline T bv_weight(const Phys<T, MF>& ph, const T* wv) {
  return (ph.bv_r < MF ? wv[ph.bv_r] : T(0)) + ph.bv_z * wv[0];
}

// ----------------------------------------------------------------------------
// Boundary faces (outward normal).  cbc: concentration kind of the face,
// phid: potential Dirichlet flag, gd[f]: data (gd[0] potential, gd[k] c_k).
template <typename T, int MF>
__host__ __device__ inline void bnd_res(const Phys<T, MF>& ph, const T* v, const T* g, T un, int cbc,
                                        bool phid, const T* gd, T* F, T* G) {
  T kap = T(0);
  for (int k = 1; k < MF; ++k) kap += ph.b[k - 1] * v[k];
  F[0] = T(0);
  G[0] = T(0);
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Q = un - zD * g[0];
    F[k] = T(0);
    G[k] = T(0);
    if (cbc == BC_DIRICHLET) {
      T jc = v[k] - gd[k];
      F[k] = -D * g[k] + D * ph.delta * jc + pos(Q) * v[k] + neg(Q) * gd[k];
      G[k] = -D * jc;
      G[0] -= ph.a[k - 1] * jc;
    } else if (cbc == BC_INFLOW) {
      F[k] = un * gd[k];
    } else if (cbc == BC_OUTFLOW) {
      F[k] = Q * v[k];
    }
  }
  if (phid) {
    T cur = kap * g[0];
    for (int k = 1; k < MF; ++k) cur += ph.a[k - 1] * g[k];
    T jp = v[0] - gd[0];
    F[0] = -cur + kap * ph.delta * jp;
    G[0] -= kap * jp;
  }
  if (cbc == BC_ELECTRODE) bv_add(ph, bv_rate(ph, v, gd).g, F);
}

template <typename T, int MF>
__host__ __device__ inline void bnd_jac(const Phys<T, MF>& ph, const T* v, const T* g, const T* tv,
                                        const T* tg, T un, int cbc, bool phid, const T* gd, T* F,
                                        T* G) {
  T kap = T(0), dkap = T(0);
  for (int k = 1; k < MF; ++k) {
    kap += ph.b[k - 1] * v[k];
    dkap += ph.b[k - 1] * tv[k];
  }
  F[0] = T(0);
  G[0] = T(0);
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Q = un - zD * g[0];
    T dQ = -zD * tg[0];
    F[k] = T(0);
    G[k] = T(0);
    if (cbc == BC_DIRICHLET) {
      T s = sgn(Q);
      F[k] = -D * tg[k] + D * ph.delta * tv[k] + pos(Q) * tv[k] +
             T(0.5) * (T(1) + s) * dQ * v[k] + T(0.5) * (T(1) - s) * dQ * gd[k];
      G[k] = -D * tv[k];
      G[0] -= ph.a[k - 1] * tv[k];
    } else if (cbc == BC_OUTFLOW) {
      F[k] = dQ * v[k] + Q * tv[k];
    }
  }
  if (phid) {
    T dcur = dkap * g[0] + kap * tg[0];
    for (int k = 1; k < MF; ++k) dcur += ph.a[k - 1] * tg[k];
    T jp = v[0] - gd[0];
    F[0] = -dcur + dkap * ph.delta * jp + kap * ph.delta * tv[0];
    G[0] += -dkap * jp - kap * tv[0];
  }
  if (cbc == BC_ELECTRODE) {
    const BvRate<T> r = bv_rate(ph, v, gd);
    bv_add(ph, r.dphi * tv[0] + r.dc * bv_conc(ph, tv), F);
  }
}

template <typename T, int MF>
__host__ __device__ inline void bnd_jacT(const Phys<T, MF>& ph, const T* v, const T* g, const T* wv,
                                         const T* wg, T un, int cbc, bool phid, const T* gd, T* Tv,
                                         T* Tg) {
  T kap = T(0);
  for (int k = 1; k < MF; ++k) kap += ph.b[k - 1] * v[k];
  Tv[0] = T(0);
  Tg[0] = T(0);
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Q = un - zD * g[0];
    Tv[k] = T(0);
    Tg[k] = T(0);
    if (cbc == BC_DIRICHLET) {
      T s = sgn(Q);
      Tv[k] = (D * ph.delta + pos(Q)) * wv[k] - D * wg[k] - ph.a[k - 1] * wg[0];
      Tg[k] = -D * wv[k];
      Tg[0] += -zD * (T(0.5) * (T(1) + s) * v[k] + T(0.5) * (T(1) - s) * gd[k]) * wv[k];
    } else if (cbc == BC_OUTFLOW) {
      Tv[k] = Q * wv[k];
      Tg[0] += -zD * v[k] * wv[k];
    }
  }
  if (phid) {
    T jp = v[0] - gd[0];
    for (int k = 1; k < MF; ++k) {
      Tg[k] += -ph.a[k - 1] * wv[0];
      Tv[k] += ph.b[k - 1] * (-g[0] + ph.delta * jp) * wv[0] - ph.b[k - 1] * jp * wg[0];
    }
    Tg[0] += -kap * wv[0];
    Tv[0] += kap * ph.delta * wv[0] - kap * wg[0];
  }
  if (cbc == BC_ELECTRODE) {
    const BvRate<T> r = bv_rate(ph, v, gd);
    const T W = bv_weight(ph, wv);
    Tv[0] -= r.dphi * W;
    for (int k = 1; k < MF; ++k) Tv[k] -= r.dc * ph.bv_dc[k - 1] * W;
  }
}

template <typename T, int MF>
__host__ __device__ inline void bnd_dpe(const Phys<T, MF>& ph, const T* v, const T* g, T un, T uhn,
                                        int cbc, const T* gd, T* F, T* G) {
  for (int f = 0; f < MF; ++f) {
    F[f] = T(0);
    G[f] = T(0);
  }
  for (int k = 1; k < MF; ++k) {
    T Q = un - ph.zD[k - 1] * g[0];
    if (cbc == BC_DIRICHLET) {
      T s = sgn(Q);
      F[k] = (T(0.5) * (T(1) + s) * v[k] + T(0.5) * (T(1) - s) * gd[k]) * uhn;
    } else if (cbc == BC_INFLOW) {
      F[k] = gd[k] * uhn;
    } else if (cbc == BC_OUTFLOW) {
      F[k] = v[k] * uhn;
    }
  }
}

// lambda^T dR/d(data): coefficient of the concentration data gd[k] at one point,
// given the adjoint traces (wv, wg); on an electrode face the coefficients of
// the applied potential (out[0]) and of the exchange current (out[1], per unit
// of the point value gd[1])
template <typename T, int MF>
__host__ __device__ inline void bnd_dataT(const Phys<T, MF>& ph, const T* v, const T* g, const T* wv,
                                          const T* wg, T un, int cbc, const T* gd, T* out) {
  out[0] = T(0);
  if (cbc == BC_ELECTRODE) {
    const BvRate<T> r = bv_rate(ph, v, gd);
    const T W = bv_weight(ph, wv);
    for (int k = 1; k < MF; ++k) out[k] = T(0);
    out[0] = -r.dpa * W;
    out[1] = -r.dj0 * W;
    return;
  }
  for (int k = 1; k < MF; ++k) {
    const T D = ph.D[k - 1], zD = ph.zD[k - 1];
    T Q = un - zD * g[0];
    out[k] = T(0);
    if (cbc == BC_DIRICHLET)
      out[k] = (-D * ph.delta + neg(Q)) * wv[k] + D * wg[k] + ph.a[k - 1] * wg[0];
    else if (cbc == BC_INFLOW)
      out[k] = un * wv[k];
  }
}

}  // namespace dgnp
