// Host-side tables: 1-D reference rules, structured-box mesh and face tables,
// boundary data at the face Gauss points, manufactured-solution data.
//
// Basis: Lagrange polynomials on the p+1 Gauss-Lobatto points per axis;
// quadrature: p+2 Gauss points per axis, i.e. integration of higher order than
// the polynomial degree on tensor-product elements (paper Sec. 4 intro).
#include <cmath>

#include "context.hpp"

namespace dgnp {

// Legendre polynomial P_n and its derivative by the three-term recurrence.
static void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

RefTables make_ref_tables(int p) {
  RefTables t;
  t.p = p;
  t.nn = p + 1;
  t.nq = p + 2;
  const int nq = t.nq, nn = t.nn;
  // Gauss-Legendre: Newton on P_nq from the Chebyshev-like initial guesses
  t.xq.resize(nq);
  t.wq.resize(nq);
  for (int i = 0; i < nq; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(nq, x, P, dP);
      double dx = P / dP;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double P, dP;
    legendre(nq, x, P, dP);
    t.xq[i] = x;
    t.wq[i] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  // Gauss-Lobatto: -1, roots of P_p', +1.  Newton on P_p' using
  // (1 - x^2) P_p'' = 2 x P_p' - p (p + 1) P_p.
  t.xn.resize(nn);
  t.xn[0] = -1.0;
  t.xn[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t.xn[i] = x;
  }
  // Lagrange values / derivatives (product formula)
  auto lag = [&](int j, double x, double& v, double& d) {
    v = 1.0;
    d = 0.0;
    for (int i = 0; i < nn; ++i)
      if (i != j) v *= (x - t.xn[i]) / (t.xn[j] - t.xn[i]);
    for (int k = 0; k < nn; ++k) {
      if (k == j) continue;
      double term = 1.0 / (t.xn[j] - t.xn[k]);
      for (int i = 0; i < nn; ++i)
        if (i != j && i != k) term *= (x - t.xn[i]) / (t.xn[j] - t.xn[i]);
      d += term;
    }
  };
  t.B.resize(nq * nn);
  t.Dq.resize(nq * nn);
  for (int q = 0; q < nq; ++q)
    for (int j = 0; j < nn; ++j) lag(j, t.xq[q], t.B[q * nn + j], t.Dq[q * nn + j]);
  for (int s = 0; s < 2; ++s) {
    t.Dend[s].resize(nn);
    for (int j = 0; j < nn; ++j) {
      double v, d;
      lag(j, s == 0 ? -1.0 : 1.0, v, d);
      t.Dend[s][j] = d;
    }
  }
  return t;
}

// ---- manufactured solutions (m = 2) --------------------------------------
// TRIG2D: c = 1 + sin(pi x) sin(pi y) / 2,   phi = cos(pi x) cos(pi y) / 10
// PAPER3D: c = cos x + sin y + 3,            phi = sin x + cos y + 3
// Sources S_c = -D1 lap c + u.grad c + c div u - z1 D1 (grad c.grad phi + c lap phi)
//         S_phi = -a1 lap c - b1 (grad c.grad phi + c lap phi)
// (every built-in velocity is divergence free).
struct MmsPoint {
  double c, gc[3], lc, ph, gp[3], lp;
};

static MmsPoint mms_eval(int kind, const double* x) {
  MmsPoint r{};
  if (kind == DGNP_MMS_TRIG2D) {
    const double sx = std::sin(M_PI * x[0]), cx = std::cos(M_PI * x[0]);
    const double sy = std::sin(M_PI * x[1]), cy = std::cos(M_PI * x[1]);
    r.c = 1.0 + 0.5 * sx * sy;
    r.gc[0] = 0.5 * M_PI * cx * sy;
    r.gc[1] = 0.5 * M_PI * sx * cy;
    r.lc = -M_PI * M_PI * sx * sy;
    r.ph = 0.1 * cx * cy;
    r.gp[0] = -0.1 * M_PI * sx * cy;
    r.gp[1] = -0.1 * M_PI * cx * sy;
    r.lp = -0.2 * M_PI * M_PI * cx * cy;
  } else {
    r.c = std::cos(x[0]) + std::sin(x[1]) + 3.0;
    r.gc[0] = -std::sin(x[0]);
    r.gc[1] = std::cos(x[1]);
    r.lc = -std::cos(x[0]) - std::sin(x[1]);
    r.ph = std::sin(x[0]) + std::cos(x[1]) + 3.0;
    r.gp[0] = std::cos(x[0]);
    r.gp[1] = -std::sin(x[1]);
    r.lp = -std::sin(x[0]) - std::cos(x[1]);
  }
  return r;
}

static void vel_hat_host(const dgnp_ctx& c, const double* x, double* uh) {
  uh[0] = uh[1] = uh[2] = 0.0;
  if (c.vel.kind == DGNP_VEL_VORTEX) {
    uh[0] = std::sin(M_PI * x[0]) * std::cos(M_PI * x[1]);
    uh[1] = -std::cos(M_PI * x[0]) * std::sin(M_PI * x[1]);
  } else if (c.vel.kind == DGNP_VEL_POISEUILLE_X) {
    const double H = c.hi[1] - c.lo[1], yy = x[1] - c.lo[1];
    uh[0] = 6.0 * yy * (H - yy) / (H * H);
  } else {
    for (int i = 0; i < c.dim; ++i) uh[i] = c.vel.param[i];
  }
}

void mms_exact(const dgnp_ctx& c, const double* x, double* phi, double* c1) {
  MmsPoint r = mms_eval(c.mms, x);
  *phi = r.ph;
  *c1 = r.c;
}

void mms_source(const dgnp_ctx& c, const double* x, double* s_phi, double* s_c1) {
  MmsPoint r = mms_eval(c.mms, x);
  double uh[3];
  vel_hat_host(c, x, uh);
  double ugc = 0.0, gcgp = 0.0;
  for (int i = 0; i < c.dim; ++i) {
    ugc += c.vel.Pe * uh[i] * r.gc[i];
    gcgp += r.gc[i] * r.gp[i];
  }
  const double zD = c.z[0] * c.D[0];
  *s_c1 = -c.D[0] * r.lc + ugc - zD * (gcgp + r.c * r.lp);
  *s_phi = -c.a[0] * r.lc - c.b[0] * (gcgp + r.c * r.lp);
}

// ---- mesh tables -------------------------------------------------------------
void build_tables(dgnp_ctx& c) {
  const int d = c.dim;
  int64_t stride[3] = {1, c.n[0], int64_t(c.n[0]) * c.n[1]};
  c.nbr.assign(size_t(c.E) * 2 * d, -1);
  for (int64_t e = 0; e < c.E; ++e) {
    int id[3] = {int(e % c.n[0]), int((e / c.n[0]) % c.n[1]), d == 3 ? int(e / stride[2]) : 0};
    for (int a = 0; a < d; ++a) {
      if (id[a] > 0) c.nbr[e * 2 * d + 2 * a] = int(e - stride[a]);
      if (id[a] < c.n[a] - 1) c.nbr[e * 2 * d + 2 * a + 1] = int(e + stride[a]);
    }
  }
  c.face_elems.clear();
  c.face_axis.clear();
  for (int a = 0; a < d; ++a)
    for (int64_t e = 0; e < c.E; ++e) {
      int up = c.nbr[e * 2 * d + 2 * a + 1];
      if (up >= 0) {
        c.face_elems.push_back(int(e));
        c.face_elems.push_back(up);
        c.face_axis.push_back(a);
      }
    }
  c.F = int64_t(c.face_axis.size());
  // boundary faces: tag t = 2a + side, ordered by element index within a tag
  int64_t off = 0, noff = 0;
  const int64_t nfn = c.nfn;
  for (int t = 0; t < 2 * d; ++t) {
    const int a = t / 2;
    int64_t cnt = c.E / c.n[a];
    c.btag_off[t] = off;
    off += cnt;
    if (c.c_bc[t] == DGNP_C_DIRICHLET || c.c_bc[t] == DGNP_C_INFLOW) {
      c.bnode_off[t] = noff;
      noff += cnt * nfn;
    } else {
      c.bnode_off[t] = -1;
    }
  }
  c.n_bface = off;
  c.n_bnode = noff;
}

}  // namespace dgnp
