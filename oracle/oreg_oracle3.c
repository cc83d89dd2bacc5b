/*
 * Plain FP64 CPU oracle of the Onsager-regularized (OReg) lattice Boltzmann
 * method on the D3Q27 lattice (arXiv 2501.16000).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite and the CPU baseline of
 * the benchmark, never by the GPU library.  It shares no code, header, table
 * or constant with the GPU library (nor with the D2Q9 oracle).
 *
 * The formulas are those of the D2Q9 oracle with a third axis, evaluated as
 * printed with no simplification:
 *   Eq. (11)  guided equilibrium as a product over alpha = x, y, z of one
 *             factor per axis.  The printed D2Q9 factor
 *             (1 - 2 c^2) / 2^(c^2) [c^2 - 1 + c u + u^2 + theta] is minus a
 *             1D distribution over c in {-1, 0, 1} (its three values sum to
 *             -1); the two minus signs cancel in the printed 2D product, but
 *             three would not, so each 3D factor is the printed one negated,
 *             (2 c^2 - 1) / 2^(c^2) [c^2 - 1 + c u + u^2 + theta].  On D2Q9
 *             the product of these factors is the printed Eq. (11) exactly;
 *   Sec. III.D  polynomial equilibrium with tensor-product weights and the
 *             -u^2/(2 theta0) term, theta0 = 1/3;
 *   Eq. (6)   literal double sums over alpha, beta and over k, D = 3;
 *   Eq. (7)   f^eq + (1 - 1/tau) f^OReg pushed to x + c_i (periodic box);
 *   Eq. (1)   lattice BGK.
 */
#include "oreg_oracle3.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27
#define D 3

static int CV[Q][D];
static int cv_ready = 0;

/* i = 9 (cz + 1) + 3 (cy + 1) + (cx + 1). */
static void make_velocities(void) {
  if (cv_ready) return;
  for (int i = 0; i < Q; ++i) {
    CV[i][0] = i % 3 - 1;
    CV[i][1] = (i / 3) % 3 - 1;
    CV[i][2] = i / 9 - 1;
  }
  cv_ready = 1;
}

void orc3_velocities(int c[27][3]) {
  make_velocities();
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < D; ++a) c[i][a] = CV[i][a];
}

static void feq_guided(double theta, double rho, const double u[D], double feq[Q]) {
  for (int i = 0; i < Q; ++i) {
    double prod = 1.0;
    for (int a = 0; a < D; ++a) {
      const double c = (double)CV[i][a];
      const double c2 = c * c;
      const double pref = (2.0 * c2 - 1.0) / pow(2.0, c2);
      prod *= pref * (c2 - 1.0 + c * u[a] + u[a] * u[a] + theta);
    }
    feq[i] = rho * prod;
  }
}

static void feq_poly2(double rho, const double u[D], double feq[Q]) {
  const double theta0 = 1.0 / 3.0;
  for (int i = 0; i < Q; ++i) {
    double W = 1.0, cu = 0.0, uu = 0.0;
    for (int a = 0; a < D; ++a) {
      W *= (CV[i][a] == 0) ? (1.0 - theta0) : theta0 / 2.0;
      cu += u[a] * (double)CV[i][a];
      uu += u[a] * u[a];
    }
    feq[i] = rho * W *
             (1.0 + cu / theta0 + cu * cu / (2.0 * theta0 * theta0) - uu / (2.0 * theta0));
  }
}

void orc3_equilibrium(int eq, double theta, double rho, const double u[3], double feq[27]) {
  make_velocities();
  if (eq == ORC3_EQ_POLY2)
    feq_poly2(rho, u, feq);
  else
    feq_guided(theta, rho, u, feq);
}

void orc3_moments_cell(const double f[27], double* rho, double u[3]) {
  make_velocities();
  double r = 0.0, j[D] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    r += f[i];
    for (int a = 0; a < D; ++a) j[a] += (double)CV[i][a] * f[i];
  }
  *rho = r;
  for (int a = 0; a < D; ++a) u[a] = j[a] / r;
}

void orc3_stress(const double fneq[27], double S[3][3]) {
  make_velocities();
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int k = 0; k < Q; ++k) {
        double ck2 = 0.0;
        for (int g = 0; g < D; ++g) ck2 += (double)(CV[k][g] * CV[k][g]);
        const double t = (double)(CV[k][a] * CV[k][b]) - (a == b ? ck2 / D : 0.0);
        s += t * fneq[k];
      }
      S[a][b] = s;
    }
}

static void oreg_from(double theta, double rho, const double u[D], const double f[Q],
                      const double feq[Q], double fo[Q]) {
  double fneq[Q], S[D][D];
  for (int k = 0; k < Q; ++k) fneq[k] = f[k] - feq[k];
  orc3_stress(fneq, S);
  for (int i = 0; i < Q; ++i) {
    double C[D], C2 = 0.0;
    for (int a = 0; a < D; ++a) {
      C[a] = (double)CV[i][a] - u[a];
      C2 += C[a] * C[a];
    }
    double acc = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        acc += (C[a] * C[b] - (a == b ? C2 / D : 0.0)) * S[a][b];
    fo[i] = feq[i] / (2.0 * rho * theta * theta) * acc;
  }
}

static double eq_theta(int eq, double theta) { return eq == ORC3_EQ_POLY2 ? 1.0 / 3.0 : theta; }

void orc3_oreg_cell(int eq, double theta, const double f[27], double fo[27]) {
  double rho, u[D], feq[Q];
  orc3_moments_cell(f, &rho, u);
  orc3_equilibrium(eq, theta, rho, u, feq);
  oreg_from(eq_theta(eq, theta), rho, u, f, feq, fo);
}

void orc3_collide_cell(int eq, int coll, double tau, double theta, const double f[27],
                       double fpost[27]) {
  double rho, u[D], feq[Q];
  orc3_moments_cell(f, &rho, u);
  orc3_equilibrium(eq, theta, rho, u, feq);
  if (coll == ORC3_COLL_BGK) {
    for (int i = 0; i < Q; ++i) fpost[i] = f[i] - (f[i] - feq[i]) / tau;
    return;
  }
  double fo[Q];
  oreg_from(eq_theta(eq, theta), rho, u, f, feq, fo);
  for (int i = 0; i < Q; ++i) fpost[i] = feq[i] + (1.0 - 1.0 / tau) * fo[i];
}

void orc3_init(int nx, int ny, int nz, int eq, double theta, const double* rho,
               const double* ux, const double* uy, const double* uz, double* f) {
  const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
  for (size_t c = 0; c < n; ++c) {
    double feq[Q];
    const double u[D] = {ux[c], uy[c], uz[c]};
    orc3_equilibrium(eq, theta, rho[c], u, feq);
    for (int i = 0; i < Q; ++i) f[(size_t)i * n + c] = feq[i];
  }
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

static void step_once(int nx, int ny, int nz, int eq, int coll, double tau, double theta,
                      const double* f, double* fn, int nthreads) {
  const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        const size_t c = ((size_t)z * ny + y) * nx + x;
        double fc[Q], fp[Q];
        for (int i = 0; i < Q; ++i) fc[i] = f[(size_t)i * n + c];
        orc3_collide_cell(eq, coll, tau, theta, fc, fp);
        for (int i = 0; i < Q; ++i) {
          const int xd = wrap(x + CV[i][0], nx);
          const int yd = wrap(y + CV[i][1], ny);
          const int zd = wrap(z + CV[i][2], nz);
          fn[(size_t)i * n + ((size_t)zd * ny + yd) * nx + xd] = fp[i];
        }
      }
    }
  }
}

void orc3_run(int nx, int ny, int nz, int eq, int coll, double tau, double theta,
              int64_t nsteps, double* f, double* tmp, int nthreads) {
  make_velocities();
  const size_t bytes = (size_t)Q * nx * ny * nz * sizeof(double);
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
  nthreads = 1;
#endif
  double* a = f;
  double* b = tmp;
  for (int64_t t = 0; t < nsteps; ++t) {
    step_once(nx, ny, nz, eq, coll, tau, theta, a, b, nthreads);
    double* s = a;
    a = b;
    b = s;
  }
  if (a != f) memcpy(f, a, bytes);
}

void orc3_moments(int nx, int ny, int nz, const double* f, double* out) {
  const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
  for (size_t c = 0; c < n; ++c) {
    double fc[Q], rho, u[D];
    for (int i = 0; i < Q; ++i) fc[i] = f[(size_t)i * n + c];
    orc3_moments_cell(fc, &rho, u);
    out[c] = rho;
    for (int a = 0; a < D; ++a) out[(size_t)(a + 1) * n + c] = u[a];
  }
}

void orc3_diagnostics(int nx, int ny, int nz, double theta, const double* f, double out[7]) {
  const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
  double mass = 0.0, j[D] = {0.0, 0.0, 0.0}, ke = 0.0, etot = 0.0, bad = 0.0;
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
    double rho, u[D], uu = 0.0;
    orc3_moments_cell(fc, &rho, u);
    mass += rho;
    for (int a = 0; a < D; ++a) {
      j[a] += rho * u[a];
      uu += u[a] * u[a];
    }
    ke += 0.5 * rho * uu;
    etot += 0.5 * (D * rho * theta + rho * uu);
  }
  out[0] = mass;
  out[1] = j[0];
  out[2] = j[1];
  out[3] = j[2];
  out[4] = ke;
  out[5] = etot;
  out[6] = bad;
}
