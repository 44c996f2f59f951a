// Host checks of the mesh and reference tables (tables.cpp), built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py:
//   reference tables, p = 1..3: Gauss weights sum to 2 and integrate x^(2p+2)
//   exactly, interpolation rows sum to 1, derivative rows to 0, and the
//   derivative of the GLL interpolant of x^p is p x^(p-1) at every Gauss point;
//   mesh tables on 2-D and 3-D boxes: neighbours are mutual, every interior face
//   appears once, boundary faces and nodes are counted per tag.
#include <cmath>
#include <cstdio>

#include "context.hpp"

using namespace dgnp;

// the context's destructor releases solver and preconditioner storage, which
// this driver never creates
namespace dgnp {
void krylov_destroy(Krylov*) {}
void precond_destroy(Precond*) {}
}  // namespace dgnp

static int fails = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++fails;
  }
}

static void ref_checks(int p) {
  const RefTables R = make_ref_tables(p);
  expect(R.nn == p + 1 && R.nq == p + 2, "table sizes");
  double ws = 0.0, mom = 0.0;
  for (int q = 0; q < R.nq; ++q) {
    ws += R.wq[q];
    mom += R.wq[q] * std::pow(R.xq[q], 2 * p + 2);
  }
  expect(std::fabs(ws - 2.0) < 1e-14, "weights sum to 2");
  expect(std::fabs(mom - 2.0 / (2 * p + 3)) < 1e-14, "moment 2p+2 exact");
  for (int q = 0; q < R.nq; ++q) {
    double sb = 0.0, sd = 0.0, dxp = 0.0;
    for (int a = 0; a < R.nn; ++a) {
      sb += R.B[q * R.nn + a];
      sd += R.Dq[q * R.nn + a];
      dxp += R.Dq[q * R.nn + a] * std::pow(R.xn[a], p);
    }
    expect(std::fabs(sb - 1.0) < 1e-13, "interpolation rows sum to 1");
    expect(std::fabs(sd) < 1e-12, "derivative rows sum to 0");
    expect(std::fabs(dxp - p * std::pow(R.xq[q], p - 1)) < 1e-12, "derivative of x^p");
  }
}

static void mesh_checks(int dim, int n0, int n1, int n2) {
  dgnp_ctx c;
  c.dim = dim;
  c.n[0] = n0;
  c.n[1] = n1;
  c.n[2] = dim == 3 ? n2 : 1;
  c.E = int64_t(n0) * n1 * c.n[2];
  c.nfn = dim == 3 ? 9 : 3;  // p = 2 face nodes
  for (int t = 0; t < 6; ++t) c.c_bc[t] = t % 3 == 0 ? DGNP_C_DIRICHLET : DGNP_C_OUTFLOW;
  build_tables(c);
  const int d = dim;
  int64_t expect_int = 0, expect_bnd = 0;
  for (int a = 0; a < d; ++a) {
    expect_int += c.E / c.n[a] * (c.n[a] - 1);
    expect_bnd += 2 * (c.E / c.n[a]);
  }
  expect(c.F == expect_int, "interior face count");
  expect(c.n_bface == expect_bnd, "boundary face count");
  for (int64_t e = 0; e < c.E; ++e)
    for (int a = 0; a < d; ++a) {
      const int up = c.nbr[e * 2 * d + 2 * a + 1];
      if (up >= 0) expect(c.nbr[int64_t(up) * 2 * d + 2 * a] == e, "neighbours are mutual");
    }
  int64_t nodes = 0;
  for (int t = 0; t < 2 * d; ++t)
    if (c.bnode_off[t] >= 0) nodes += (c.E / c.n[t / 2]) * c.nfn;
  expect(c.n_bnode == nodes, "boundary node count");
}

int main() {
  for (int p = 1; p <= 3; ++p) ref_checks(p);
  mesh_checks(3, 4, 3, 2);
  mesh_checks(2, 5, 3, 1);
  mesh_checks(3, 1, 1, 1);
  std::printf(fails ? "FAIL %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
