// Host-side check of the D3Q27 device collision (csrc/d3q27.hpp compiled for
// the CPU) against the FP64 D3Q27 oracle, one node at a time, for every
// equilibrium and collision, FP64 and shifted FP32.  Prints the worst
// errors; the pytest wrapper asserts them.
#include <cmath>
#include <cstdio>
#include <random>

#include "d3q27.hpp"

extern "C" void orc3_collide_cell(int eq, int coll, double tau, double theta, const double f[27],
                                  double fpost[27]);
extern "C" void orc3_equilibrium(int eq, double theta, double rho, const double u[3],
                                 double feq[27]);

using namespace oreg;

template <int EQ, int COLL>
void run(double theta, double tau, unsigned seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(-1, 1);
  const double th = EQ == LB_EQ_POLY2 ? 1.0 / 3.0 : theta;
  Coef64 c{th, 1 - th, 0.5 * th, (1 - 1 / tau) / (2 * th * th), 1 / tau, 0.0};
  double w64 = 0, w32 = 0;
  for (int t = 0; t < 5000; ++t) {
    const double rho = 1 + 0.2 * U(g);
    const double u[3] = {0.1 * U(g), 0.1 * U(g), 0.1 * U(g)};
    double feq[27], f[27], ref[27];
    orc3_equilibrium(EQ, theta, rho, u, feq);
    for (int i = 0; i < 27; ++i) f[i] = feq[i] * (1 + 0.05 * U(g));
    orc3_collide_cell(EQ, COLL, tau, theta, f, ref);
    c.rho0 = 0.0;
    double h[27];
    for (int i = 0; i < 27; ++i) h[i] = f[i];
    d3::collide<EQ, COLL, false>(h, Coeffs<double>(c));
    for (int i = 0; i < 27; ++i) w64 = std::fmax(w64, std::fabs(h[i] - ref[i]) / std::fabs(ref[i]));
    c.rho0 = 1.1;
    double w[27];
    float s[27];
    for (int i = 0; i < 27; ++i) {
      w[i] = d3::shift64(d3::cx(i), d3::cy(i), d3::cz(i), c);
      s[i] = (float)(f[i] - w[i]);
    }
    d3::collide<EQ, COLL, true>(s, Coeffs<float>(c));
    for (int i = 0; i < 27; ++i) w32 = std::fmax(w32, std::fabs((double)s[i] + w[i] - ref[i]));
  }
  std::printf("eq=%d coll=%d theta=%.4f tau=%.3f f64_rel=%.3e f32s_abs=%.3e\n", EQ, COLL, theta,
              tau, w64, w32);
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
