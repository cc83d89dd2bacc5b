/*
 * Plain FP64 CPU oracle of the Onsager-regularized (OReg) lattice Boltzmann
 * method on the D3Q27 lattice (arXiv 2501.16000, Fig. 1b).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite and the CPU baseline of the
 * benchmark load this library.  It shares no code, header, table or constant
 * with the GPU library, and the GPU library never calls it.
 *
 * The paper writes Eq. (6) for any stencil with dimension constant D and the
 * guided equilibrium of Eq. (11) as a product over the Cartesian axes of
 * D2Q9; on D3Q27 the product has a third factor and D = 3.  It does not print
 * the 3D equilibrium, so this extension is a reading, not a transcription:
 * each axis factor is the 1D distribution (1 - theta - u^2 at c = 0,
 * (theta + c u + u^2)/2 at c = +-1) whose product over two axes is the
 * printed Eq. (11).
 *
 * Conventions (the paper fixes none of them):
 *   velocity order i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1), c in {-1,0,1}^3
 *   (the rest velocity is i = 13, the opposite of i is 26 - i);
 *   populations f[i][z][y][x] (x fastest), nodes at integer (x, y, z);
 *   the state is the pre-collision f(x, t).
 */
#ifndef OREG_ORACLE3_H
#define OREG_ORACLE3_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC3_EQ_GUIDED = 0, ORC3_EQ_POLY2 = 1 };
enum { ORC3_COLL_OREG = 0, ORC3_COLL_BGK = 1 };

/* The velocity table above, as c[i][alpha]. */
void orc3_velocities(int c[27][3]);

/* Equilibrium of one cell: Eq. (11) with three axis factors (guided), or the
   second-order polynomial equilibrium of Sec. III.D with tensor-product
   weights (poly2, theta0 = 1/3, theta ignored). */
void orc3_equilibrium(int eq, double theta, double rho, const double u[3],
                      double feq[27]);

/* rho = sum f, u = (sum c f) / rho. */
void orc3_moments_cell(const double f[27], double* rho, double u[3]);

/* Trace-free non-equilibrium stress S[a][b] of Eq. (6), D = 3. */
void orc3_stress(const double fneq[27], double S[3][3]);

/* Eq. (6): f^OReg of one cell (f^neq = f - f^eq). */
void orc3_oreg_cell(int eq, double theta, const double f[27], double fo[27]);

/* One collision: Eq. (7) (ORC3_COLL_OREG) or Eq. (1) (ORC3_COLL_BGK). */
void orc3_collide_cell(int eq, int coll, double tau, double theta,
                       const double f[27], double fpost[27]);

/* f(x, 0) = f^eq(rho(x), u(x)); fields [nz][ny][nx], f [27][nz][ny][nx]. */
void orc3_init(int nx, int ny, int nz, int eq, double theta, const double* rho,
               const double* ux, const double* uy, const double* uz, double* f);

/* n time steps on a periodic box with streaming to x + c_i; f in place, tmp
   a caller buffer of the same size, nthreads <= 0 uses every OpenMP thread. */
void orc3_run(int nx, int ny, int nz, int eq, int coll, double tau,
              double theta, int64_t nsteps, double* f, double* tmp,
              int nthreads);

/* rho, ux, uy, uz of every cell: out[4][nz][ny][nx]. */
void orc3_moments(int nx, int ny, int nz, const double* f, double* out);

/* mass, jx, jy, jz, kinetic energy, total energy (3/2 rho theta + rho|u|^2/2),
   count of cells holding a non-finite population. */
void orc3_diagnostics(int nx, int ny, int nz, double theta, const double* f,
                      double out[7]);

#ifdef __cplusplus
}
#endif
#endif
