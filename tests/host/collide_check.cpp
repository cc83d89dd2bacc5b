// Host-side check of the device collision (csrc/d2q9.hpp compiled for the CPU)
// against the FP64 oracle, one node at a time, for every equilibrium and
// collision, FP64 and shifted FP32.  Prints the worst errors; the pytest
// wrapper asserts them.
#include <cmath>
#include <cstdio>
#include <random>

#include "d2q9.hpp"

extern "C" void orc_collide_cell(int eq, int coll, double tau, double theta, const double f[9],
                                 double fpost[9]);
extern "C" void orc_equilibrium(int eq, double theta, double rho, double ux, double uy,
                                double feq[9]);

using namespace oreg;

template <int EQ, int COLL>
void run(double theta, double tau, unsigned seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(-1, 1);
  const double th = EQ == LB_EQ_POLY2 ? 1.0 / 3.0 : theta;
  Coef64 c{th, 1 - th, 0.5 * th, (1 - 1 / tau) / (2 * th * th), 1 / tau, 0.0};
  double w64 = 0, w32 = 0, ww = 0;
  for (int t = 0; t < 5000; ++t) {
    const double rho = 1 + 0.2 * U(g), ux = 0.1 * U(g), uy = 0.1 * U(g);
    double feq[9], f[9], ref[9];
    orc_equilibrium(EQ, theta, rho, ux, uy, feq);
    for (int i = 0; i < 9; ++i) f[i] = feq[i] * (1 + 0.05 * U(g));
    orc_collide_cell(EQ, COLL, tau, theta, f, ref);
    c.rho0 = 0.0;
    double h[9];
    for (int i = 0; i < 9; ++i) h[i] = f[i];
    collide<EQ, COLL, false>(h, Coeffs<double>(c));
    for (int i = 0; i < 9; ++i) w64 = std::fmax(w64, std::fabs(h[i] - ref[i]) / std::fabs(ref[i]));
    c.rho0 = 1.1;
    double w[9];
    float s[9];
    for (int i = 0; i < 9; ++i) {
      w[i] = (cx_of(i) == 0 ? c.a0 : c.a1) * (cy_of(i) == 0 ? c.a0 : c.a1) * c.rho0;
      s[i] = (float)(f[i] - w[i]);
    }
    float sw[9];
    for (int i = 0; i < 9; ++i) sw[i] = s[i];
    collide<EQ, COLL, true>(s, Coeffs<float>(c));
    for (int i = 0; i < 9; ++i) w32 = std::fmax(w32, std::fabs((double)s[i] + w[i] - ref[i]));
    // shifted FP32 with u formed from drho / rho (the F32S storage)
    collide<EQ, COLL, true, true>(sw, Coeffs<float>(c));
    for (int i = 0; i < 9; ++i) ww = std::fmax(ww, std::fabs((double)sw[i] + w[i] - ref[i]));
  }
  std::printf("eq=%d coll=%d theta=%.4f tau=%.3f f64_rel=%.3e f32s_abs=%.3e f32u_abs=%.3e\n", EQ,
              COLL, theta, tau, w64, w32, ww);
}

int main() {
  run<LB_EQ_GUIDED, LB_COLL_OREG>(1.0 / 3.0, 0.8, 1);
  run<LB_EQ_GUIDED, LB_COLL_OREG>(0.35, 0.51, 2);
  run<LB_EQ_GUIDED, LB_COLL_OREG>(0.4, 1.3, 3);
  run<LB_EQ_POLY2, LB_COLL_OREG>(1.0 / 3.0, 0.6, 4);
  run<LB_EQ_GUIDED, LB_COLL_BGK>(0.35, 0.7, 5);
  run<LB_EQ_POLY2, LB_COLL_BGK>(1.0 / 3.0, 0.9, 6);
  return 0;
}
