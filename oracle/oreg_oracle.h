/*
 * Plain FP64 CPU oracle of the Onsager-regularized (OReg) lattice Boltzmann
 * method on the D2Q9 lattice (Jonnalagadda, Agrawal, Sharma, Rocchia, Succi,
 * "Towards nonlinear thermohydrodynamic simulations via the Onsager-Regularized
 * Lattice Boltzmann Method", arXiv 2501.16000).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library, and the GPU library never calls it.
 *
 * Conventions (the paper fixes none of them):
 *   velocity order i = 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 *                      5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
 *   populations f[i][y][x] (x fastest), nodes at integer (x, y),
 *   0 <= x < nx, 0 <= y < ny; the state is the pre-collision f(x, t).
 */
#ifndef OREG_ORACLE_H
#define OREG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EQ_GUIDED = 0, ORC_EQ_POLY2 = 1 };
enum { ORC_COLL_OREG = 0, ORC_COLL_BGK = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_BOUNCEBACK = 1 };

/* The velocity table above, as c[i][alpha]. */
void orc_velocities(int c[9][2]);

/* Equilibrium populations of one cell: Eq. (11) (eq = ORC_EQ_GUIDED) or the
   second-order polynomial equilibrium of Sec. III.D (eq = ORC_EQ_POLY2, which
   ignores theta and uses theta0 = 1/3). */
void orc_equilibrium(int eq, double theta, double rho, double ux, double uy,
                     double feq[9]);

/* Moments of one cell: rho = sum f, u = (sum c f) / rho. */
void orc_moments_cell(const double f[9], double* rho, double* ux, double* uy);

/* Trace-free non-equilibrium stress S[a][b] of Eq. (6) for given f^neq. */
void orc_stress(const double fneq[9], double S[2][2]);

/* Eq. (6): f^OReg of one cell from its populations f (f^neq = f - f^eq). */
void orc_oreg_cell(int eq, double theta, const double f[9], double fo[9]);

/* One collision of one cell: Eq. (7) (ORC_COLL_OREG) or Eq. (1) (ORC_COLL_BGK). */
void orc_collide_cell(int eq, int coll, double tau, double theta,
                      const double f[9], double fpost[9]);

/* f(x, 0) = f^eq(rho(x), u(x)); fields are [ny][nx], f is [9][ny][nx]. */
void orc_init(int nx, int ny, int eq, double theta, const double* rho,
              const double* ux, const double* uy, double* f);

/* n applications of Eq. (7) (or Eq. (1)) with streaming to x + c_i.
   bc_x selects periodic wrap or full-way bounce-back wall nodes in the first
   and last columns (y is always periodic).  f is updated in place; tmp is a
   caller buffer of the same size.  nthreads <= 0 uses every OpenMP thread. */
void orc_run(int nx, int ny, int eq, int coll, int bc_x, double tau,
             double theta, int64_t nsteps, double* f, double* tmp,
             int nthreads);

/* rho, ux, uy of every cell: out[3][ny][nx]. */
void orc_moments(int nx, int ny, const double* f, double* out);

/* mass, jx, jy, kinetic energy, total energy (rho*theta + rho|u|^2/2),
   count of cells holding a non-finite population. */
void orc_diagnostics(int nx, int ny, double theta, const double* f,
                     double out[6]);

#ifdef __cplusplus
}
#endif
#endif
