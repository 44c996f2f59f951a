/* Host driver of the C ABI (plain C, include/dgnp.h only), run under the
 * address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py:
 * every argument error that dgnp_setup reports before touching a device, NULL
 * arguments of the other entry points, and one valid set-up, which either
 * succeeds (a GPU is present) or reports DGNP_E_HIP (none is). */
#include <stdio.h>
#include <string.h>

#include "dgnp.h"

static int fails = 0;
#define EXPECT(cond, what)                                      \
  do {                                                          \
    if (!(cond)) {                                              \
      printf("FAIL %s (%s)\n", what, dgnp_last_error());        \
      ++fails;                                                  \
    }                                                           \
  } while (0)

int main(void) {
  const double z[3] = {1.0, -1.0, 2.0}, D[3] = {1.0, 1.5, 0.7}, zbad[3] = {1.0, -1.0, 0.0};
  dgnp_mesh m;
  memset(&m, 0, sizeof m);
  m.dim = 3;
  m.n[0] = m.n[1] = m.n[2] = 2;
  for (int i = 0; i < 3; ++i) m.hi[i] = 1.0;
  for (int t = 0; t < 6; ++t) {
    m.c_bc[t] = DGNP_C_OUTFLOW;
    m.phi_bc[t] = DGNP_PHI_DIRICHLET;
  }
  m.c_bc[0] = DGNP_C_INFLOW;
  dgnp_species sp = {3, z, D};
  dgnp_velocity vel;
  memset(&vel, 0, sizeof vel);
  vel.kind = DGNP_VEL_CONST;
  vel.Pe = 1.0;
  vel.param[0] = 1.0;
  double bc[2 * 6 * 9];
  for (int i = 0; i < 2 * 6 * 9; ++i) bc[i] = 1.0;
  dgnp_options opt;
  memset(&opt, 0, sizeof opt);
  opt.c_ip = 10.0;
  opt.bc_conc = bc;
  dgnp_ctx* ctx = NULL;

  EXPECT(dgnp_setup(NULL, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "NULL mesh");
  EXPECT(dgnp_setup(&m, 2, &sp, &vel, &opt, NULL, NULL) == DGNP_E_ARG, "NULL out");
  EXPECT(dgnp_setup(&m, 4, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "order 4");
  dgnp_mesh bad = m;
  bad.dim = 1;
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "dim 1");
  bad = m;
  bad.n[1] = 0;
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "empty axis");
  bad = m;
  bad.hi[2] = bad.lo[2];
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "empty box");
  bad = m;
  bad.c_bc[3] = 9;
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "unknown boundary kind");
  bad = m;
  for (int t = 0; t < 6; ++t) bad.phi_bc[t] = DGNP_PHI_NEUMANN0;
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "potential not fixed");
  bad = m;
  bad.c_bc[4] = DGNP_C_ELECTRODE;
  EXPECT(dgnp_setup(&bad, 2, &sp, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "electrode with fixed potential");
  dgnp_species sp2 = {3, zbad, D};
  EXPECT(dgnp_setup(&m, 2, &sp2, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "uncharged eliminated ion");
  dgnp_species sp3 = {4, z, D};
  EXPECT(dgnp_setup(&m, 2, &sp3, &vel, &opt, NULL, &ctx) == DGNP_E_ARG, "four ions");
  dgnp_velocity vbad = vel;
  vbad.kind = 7;
  EXPECT(dgnp_setup(&m, 2, &sp, &vbad, &opt, NULL, &ctx) == DGNP_E_ARG, "velocity kind");
  dgnp_options obad = opt;
  obad.phi_mg = 99;
  EXPECT(dgnp_setup(&m, 2, &sp, &vel, &obad, NULL, &ctx) == DGNP_E_ARG, "phi_mg");
  EXPECT(ctx == NULL, "no context after errors");

  EXPECT(dgnp_residual(NULL, NULL, NULL, NULL) != DGNP_OK, "residual NULL");
  EXPECT(dgnp_solve(NULL, NULL, NULL, NULL) != DGNP_OK, "solve NULL");
  dgnp_destroy(NULL);

  const int rc = dgnp_setup(&m, 2, &sp, &vel, &opt, NULL, &ctx);
  EXPECT(rc == DGNP_OK || rc == DGNP_E_HIP, "valid set-up");
  if (rc == DGNP_OK) {
    EXPECT(ctx != NULL, "context");
    dgnp_destroy(ctx);
  }
  printf(fails ? "FAIL %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
