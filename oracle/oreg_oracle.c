/*
 * Plain FP64 CPU oracle of the Onsager-regularized (OReg) lattice Boltzmann
 * method on the D2Q9 lattice (arXiv 2501.16000).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU baseline of the benchmark, never by the GPU library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every function evaluates the paper's formulas as printed, in its notation,
 * with no algebraic simplification, blocking or fusion:
 *   Eq. (11)  guided equilibrium, the literal product over alpha = x, y with
 *             the (1 - 2 c^2) / 2^(c^2) prefactors;
 *   Sec. III.D  second-order polynomial equilibrium with tensor-product weights
 *             W_{+-1} = theta0/2, W_0 = 1 - theta0 at theta0 = 1/3.  As printed
 *             the bracket lacks the -u^2/(2 theta0) term, without which the
 *             density is not reproduced (sum f^eq = rho (1 + 3u^2/2)); the
 *             oracle includes it (the form the paper calls "popular");
 *   Eq. (6)   f^OReg from f^neq = f - f^eq, literal double sums over alpha,
 *             beta and over k, with D = 2;
 *   Eq. (7)   post-collision state f^eq + (1 - 1/tau) f^OReg, pushed to x + c_i;
 *   Eq. (1)   lattice-BGK collision f - (f - f^eq)/tau (comparison scheme).
 *   Full-way bounce-back (Sec. IV, shocktube): wall nodes reverse every
 *   population instead of colliding.
 * Delta t = 1 throughout (lattice units).
 */
#include "oreg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9
#define D 2

/* D2Q9 velocities of Fig. 1a in the order of the header. */
static const int CVEL[Q][D] = {
    {0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};

void orc_velocities(int c[9][2]) {
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < D; ++a) c[i][a] = CVEL[i][a];
}

/* Eq. (11): f_i^eq = rho prod_alpha (1 - 2 c_ia^2) / 2^(c_ia^2)
                          [c_ia^2 - 1 + c_ia u_a + u_a^2 + theta]. */
static void feq_guided(double theta, double rho, const double u[D], double feq[Q]) {
  for (int i = 0; i < Q; ++i) {
    double prod = 1.0;
    for (int a = 0; a < D; ++a) {
      const double c = (double)CVEL[i][a];
      const double c2 = c * c;
      const double pref = (1.0 - 2.0 * c2) / pow(2.0, c2);
      prod *= pref * (c2 - 1.0 + c * u[a] + u[a] * u[a] + theta);
    }
    feq[i] = rho * prod;
  }
}

/* Sec. III.D: f_i^eq = rho W_i [1 + (u.c_i)/theta0 + (u.c_i)^2/(2 theta0^2)
                                   - u^2/(2 theta0)],  theta0 = 1/3. */
static void feq_poly2(double rho, const double u[D], double feq[Q]) {
  const double theta0 = 1.0 / 3.0;
  for (int i = 0; i < Q; ++i) {
    double W = 1.0, cu = 0.0, uu = 0.0;
    for (int a = 0; a < D; ++a) {
      W *= (CVEL[i][a] == 0) ? (1.0 - theta0) : theta0 / 2.0;
      cu += u[a] * (double)CVEL[i][a];
      uu += u[a] * u[a];
    }
    feq[i] = rho * W *
             (1.0 + cu / theta0 + cu * cu / (2.0 * theta0 * theta0) - uu / (2.0 * theta0));
  }
}

void orc_equilibrium(int eq, double theta, double rho, double ux, double uy, double feq[9]) {
  const double u[D] = {ux, uy};
  if (eq == ORC_EQ_POLY2)
    feq_poly2(rho, u, feq);
  else
    feq_guided(theta, rho, u, feq);
}

/* Eq. (2a): rho = <f, 1>, rho u = <f, c>. */
void orc_moments_cell(const double f[9], double* rho, double* ux, double* uy) {
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < Q; ++i) {
    r += f[i];
    jx += (double)CVEL[i][0] * f[i];
    jy += (double)CVEL[i][1] * f[i];
  }
  *rho = r;
  *ux = jx / r;
  *uy = jy / r;
}

/* Inner sum of Eq. (6): S_ab = sum_k (c_ka c_kb - c_k^2/D delta_ab) f_k^neq. */
void orc_stress(const double fneq[9], double S[2][2]) {
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int k = 0; k < Q; ++k) {
        const double ck2 = (double)(CVEL[k][0] * CVEL[k][0] + CVEL[k][1] * CVEL[k][1]);
        const double t = (double)(CVEL[k][a] * CVEL[k][b]) - (a == b ? ck2 / D : 0.0);
        s += t * fneq[k];
      }
      S[a][b] = s;
    }
}

/* Eq. (6) given f, f^eq and the moments of the cell. */
static void oreg_from(double theta, double rho, const double u[D], const double f[Q],
                      const double feq[Q], double fo[Q]) {
  double fneq[Q], S[D][D];
  for (int k = 0; k < Q; ++k) fneq[k] = f[k] - feq[k];
  orc_stress(fneq, S);
  for (int i = 0; i < Q; ++i) {
    double C[D], C2 = 0.0;
    for (int a = 0; a < D; ++a) {
      C[a] = (double)CVEL[i][a] - u[a];
      C2 += C[a] * C[a];
    }
    double acc = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        acc += (C[a] * C[b] - (a == b ? C2 / D : 0.0)) * S[a][b];
    fo[i] = feq[i] / (2.0 * rho * theta * theta) * acc;
  }
}

static double eq_theta(int eq, double theta) { return eq == ORC_EQ_POLY2 ? 1.0 / 3.0 : theta; }

void orc_oreg_cell(int eq, double theta, const double f[9], double fo[9]) {
  double rho, u[D], feq[Q];
  orc_moments_cell(f, &rho, &u[0], &u[1]);
  orc_equilibrium(eq, theta, rho, u[0], u[1], feq);
  oreg_from(eq_theta(eq, theta), rho, u, f, feq, fo);
}

void orc_collide_cell(int eq, int coll, double tau, double theta, const double f[9],
                      double fpost[9]) {
  double rho, u[D], feq[Q];
  orc_moments_cell(f, &rho, &u[0], &u[1]);
  orc_equilibrium(eq, theta, rho, u[0], u[1], feq);
  if (coll == ORC_COLL_BGK) {
    /* Eq. (1) */
    for (int i = 0; i < Q; ++i) fpost[i] = f[i] - (f[i] - feq[i]) / tau;
    return;
  }
  double fo[Q];
  oreg_from(eq_theta(eq, theta), rho, u, f, feq, fo);
  /* Eq. (7) */
  for (int i = 0; i < Q; ++i) fpost[i] = feq[i] + (1.0 - 1.0 / tau) * fo[i];
}

void orc_init(int nx, int ny, int eq, double theta, const double* rho, const double* ux,
              const double* uy, double* f) {
  const size_t n = (size_t)nx * (size_t)ny;
  for (size_t c = 0; c < n; ++c) {
    double feq[Q];
    orc_equilibrium(eq, theta, rho[c], ux[c], uy[c], feq);
    for (int i = 0; i < Q; ++i) f[(size_t)i * n + c] = feq[i];
  }
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Opposite direction of velocity i: the j with c_j = -c_i. */
static int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (CVEL[j][0] == -CVEL[i][0] && CVEL[j][1] == -CVEL[i][1]) return j;
  return i;
}

/* One time step: collide every node, then write f_i^post(x) to x + c_i. */
static void step_once(int nx, int ny, int eq, int coll, int bc_x, double tau, double theta,
                      const double* f, double* fn, int nthreads) {
  const size_t n = (size_t)nx * (size_t)ny;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      const size_t c = (size_t)y * nx + x;
      double fc[Q], fp[Q];
      for (int i = 0; i < Q; ++i) fc[i] = f[(size_t)i * n + c];
      const int wall = (bc_x == ORC_BC_BOUNCEBACK) && (x == 0 || x == nx - 1);
      if (wall) {
        for (int i = 0; i < Q; ++i) fp[i] = fc[opposite(i)];
      } else {
        orc_collide_cell(eq, coll, tau, theta, fc, fp);
      }
      for (int i = 0; i < Q; ++i) {
        const int xd = wrap(x + CVEL[i][0], nx);
        const int yd = wrap(y + CVEL[i][1], ny);
        fn[(size_t)i * n + (size_t)yd * nx + xd] = fp[i];
      }
    }
  }
}

void orc_run(int nx, int ny, int eq, int coll, int bc_x, double tau, double theta,
             int64_t nsteps, double* f, double* tmp, int nthreads) {
  const size_t bytes = (size_t)Q * nx * ny * sizeof(double);
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
  nthreads = 1;
#endif
  double* a = f;
  double* b = tmp;
  for (int64_t t = 0; t < nsteps; ++t) {
    step_once(nx, ny, eq, coll, bc_x, tau, theta, a, b, nthreads);
    double* s = a;
    a = b;
    b = s;
  }
  if (a != f) memcpy(f, a, bytes);
}

void orc_moments(int nx, int ny, const double* f, double* out) {
  const size_t n = (size_t)nx * (size_t)ny;
  for (size_t c = 0; c < n; ++c) {
    double fc[Q];
    for (int i = 0; i < Q; ++i) fc[i] = f[(size_t)i * n + c];
    orc_moments_cell(fc, &out[c], &out[n + c], &out[2 * n + c]);
  }
}

/* Conserved-moment sums of Eq. (2a) and E = (D p + rho u^2)/2 with p = rho theta. */
void orc_diagnostics(int nx, int ny, double theta, const double* f, double out[6]) {
  const size_t n = (size_t)nx * (size_t)ny;
  double mass = 0.0, jx = 0.0, jy = 0.0, ke = 0.0, etot = 0.0, bad = 0.0;
  for (size_t c = 0; c < n; ++c) {
    double fc[Q];
    int finite = 1;
    for (int i = 0; i < Q; ++i) {
      fc[i] = f[(size_t)i * n + c];
      if (!isfinite(fc[i])) finite = 0;
    }
    if (!finite) {
      bad += 1.0;
      continue;
    }
    double rho, ux, uy;
    orc_moments_cell(fc, &rho, &ux, &uy);
    mass += rho;
    jx += rho * ux;
    jy += rho * uy;
    ke += 0.5 * rho * (ux * ux + uy * uy);
    etot += 0.5 * (D * rho * theta + rho * (ux * ux + uy * uy));
  }
  out[0] = mass;
  out[1] = jx;
  out[2] = jy;
  out[3] = ke;
  out[4] = etot;
  out[5] = bad;
}
