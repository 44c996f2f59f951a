// Host check of the one-sided face linearisation (face_jac_own) against the
// two-sided one (face_jac) of the same interior-face flux: for the own element
// as the minus side (o = 0) and as the plus side (o = 1), with the normal
// quantities of the one-sided form taken along the own outward normal, the
// value coefficients agree and the normal-derivative coefficient is sign_o
// times face_jac's d/dx_axis coefficient.  Random states, trial traces and
// physical constants; prints "ok" and the largest relative difference.
#include <cmath>
#include <cstdio>
#include <random>

#include "pointwise.hpp"

using namespace dgnp;

template <int MF>
static double check(std::mt19937_64& rng) {
  std::uniform_real_distribution<double> U(-1.0, 1.0), P(0.2, 2.0);
  Phys<double, MF> ph{};
  for (int k = 0; k < MF - 1; ++k) {
    ph.D[k] = P(rng);
    ph.zD[k] = U(rng) * 2.0;
    ph.a[k] = U(rng);
    ph.b[k] = P(rng);
  }
  ph.delta = 10.0 * P(rng);
  double worst = 0.0;
  for (int rep = 0; rep < 2000; ++rep) {
    double v[2][MF], g[2][MF], tv[2][MF], tg[2][MF];
    for (int s = 0; s < 2; ++s)
      for (int f = 0; f < MF; ++f) {
        v[s][f] = f == 0 ? U(rng) : P(rng);
        g[s][f] = U(rng);
        tv[s][f] = U(rng);
        tg[s][f] = U(rng);
      }
    // exact zeros of the upwind velocity are a case of their own
    const double un = rep % 50 == 0 ? 0.5 * ph.zD[0] * (g[0][0] + g[1][0]) : 3.0 * U(rng);
    for (int o = 0; o < 2; ++o) {
      double Fo[MF], Go[MF], Fs[MF], Gs[MF];
      face_jac<double, MF>(ph, v, g, tv, tg, un, o, Fo, Go);
      const int n = 1 - o;
      const double sg = o == 0 ? 1.0 : -1.0;
      double tgo[MF], tgn[MF];
      for (int f = 0; f < MF; ++f) {
        tgo[f] = sg * tg[o][f];
        tgn[f] = sg * tg[n][f];
      }
      face_jac_own<double, MF>(ph, v[o], v[n], sg * g[o][0], sg * g[n][0], tv[o], tv[n], tgo, tgn, sg * un, Fs,
                               Gs);
      double scale = 1e-300;
      for (int f = 0; f < MF; ++f) scale = std::fmax(scale, std::fmax(std::fabs(Fo[f]), std::fabs(Go[f])));
      for (int f = 0; f < MF; ++f) {
        worst = std::fmax(worst, std::fabs(Fs[f] - Fo[f]) / scale);
        worst = std::fmax(worst, std::fabs(sg * Gs[f] - Go[f]) / scale);
      }
    }
  }
  return worst;
}

int main() {
  std::mt19937_64 rng(20211217);
  const double w3 = check<3>(rng), w4 = check<4>(rng), w2 = check<2>(rng);
  const double w = std::fmax(w3, std::fmax(w4, w2));
  std::printf("%s max_rel %.3e (m=2 %.3e, m=3 %.3e, m=4 %.3e)\n", w <= 1e-13 ? "ok" : "FAIL", w, w2, w3, w4);
  return w <= 1e-13 ? 0 : 1;
}
