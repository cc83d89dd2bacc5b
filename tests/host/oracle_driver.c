/* Exercises every entry point of both CPU oracles on small and degenerate
   shapes, for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
   test suite.  Exit status 0 and no sanitizer report is the pass. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oreg_oracle.h"
#include "oreg_oracle3.h"

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return ((*s >> 8) & 0xffffff) / 16777216.0 - 0.5;
}

static int run2(int nx, int ny, int eq, int coll, int bc, double theta, double tau,
                unsigned seed) {
  const size_t n = (size_t)nx * ny;
  double* rho = malloc(n * sizeof *rho);
  double* ux = malloc(n * sizeof *ux);
  double* uy = malloc(n * sizeof *uy);
  double* f = malloc(9 * n * sizeof *f);
  double* tmp = malloc(9 * n * sizeof *tmp);
  double* m = malloc(3 * n * sizeof *m);
  double d[6];
  for (size_t i = 0; i < n; ++i) {
    rho[i] = 1.0 + 0.1 * urand(&seed);
    ux[i] = 0.05 * urand(&seed);
    uy[i] = 0.05 * urand(&seed);
  }
  orc_init(nx, ny, eq, theta, rho, ux, uy, f);
  orc_run(nx, ny, eq, coll, bc, tau, theta, 7, f, tmp, 1);
  orc_moments(nx, ny, f, m);
  orc_diagnostics(nx, ny, theta, f, d);
  int bad = !(isfinite(d[0]) && d[5] == 0.0);
  free(rho), free(ux), free(uy), free(f), free(tmp), free(m);
  return bad;
}

static int run3(int nx, int ny, int nz, int eq, int coll, double theta, double tau,
                unsigned seed) {
  const size_t n = (size_t)nx * ny * nz;
  double* rho = malloc(n * sizeof *rho);
  double* u[3];
  for (int a = 0; a < 3; ++a) u[a] = malloc(n * sizeof(double));
  double* f = malloc(27 * n * sizeof *f);
  double* tmp = malloc(27 * n * sizeof *tmp);
  double* m = malloc(4 * n * sizeof *m);
  double d[7];
  for (size_t i = 0; i < n; ++i) {
    rho[i] = 1.0 + 0.1 * urand(&seed);
    for (int a = 0; a < 3; ++a) u[a][i] = 0.05 * urand(&seed);
  }
  orc3_init(nx, ny, nz, eq, theta, rho, u[0], u[1], u[2], f);
  orc3_run(nx, ny, nz, eq, coll, tau, theta, 4, f, tmp, 1);
  orc3_moments(nx, ny, nz, f, m);
  orc3_diagnostics(nx, ny, nz, theta, f, d);
  int bad = !(isfinite(d[0]) && d[6] == 0.0);
  free(rho), free(f), free(tmp), free(m);
  for (int a = 0; a < 3; ++a) free(u[a]);
  return bad;
}

int main(void) {
  static const int shapes[][2] = {{1, 1}, {1, 7}, {9, 1}, {2, 2}, {8, 8}, {13, 5}};
  int bad = 0;
  for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
    for (int eq = 0; eq < 2; ++eq)
      for (int coll = 0; coll < 2; ++coll)
        for (int bc = 0; bc < 2; ++bc)
          bad |= run2(shapes[s][0], shapes[s][1], eq, coll, bc, eq ? 1.0 / 3.0 : 0.35, 0.7,
                      (unsigned)(s * 8 + eq * 4 + coll * 2 + bc + 1));
  for (int eq = 0; eq < 2; ++eq)
    for (int coll = 0; coll < 2; ++coll) {
      bad |= run3(1, 1, 1, eq, coll, 1.0 / 3.0, 0.8, 3u);
      bad |= run3(5, 3, 4, eq, coll, 1.0 / 3.0, 0.6, 5u);
    }
  /* single-cell entry points */
  double f[9], fo[9], S[2][2], r, vx, vy;
  orc_equilibrium(0, 0.35, 1.1, 0.02, -0.03, f);
  orc_moments_cell(f, &r, &vx, &vy);
  orc_stress(f, S);
  orc_oreg_cell(0, 0.35, f, fo);
  orc_collide_cell(1, 0, 0.9, 1.0 / 3.0, f, fo);
  int c2[9][2], c3[27][3];
  orc_velocities(c2);
  orc3_velocities(c3);
  printf("oracle driver: %s\n", bad ? "non-finite result" : "ok");
  return bad;
}
