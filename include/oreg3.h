/*
 * oreg3.h -- C ABI of the D3Q27 lattices of liboreg.so (MI355X, gfx950).
 *
 * The paper (arXiv 2501.16000) states the OReg update of Eq. (6) for any
 * stencil, with the dimension constant D in the trace-free projection, and
 * shows the D3Q27 lattice in Fig. 1b, but only writes its equilibria for
 * D2Q9.  These entry points apply the same per-node update on a periodic
 * D3Q27 box:
 *
 *   rho = <f, 1>, rho u = <f, c>                               (Eq. 2a)
 *   f^eq = rho Psi(c_x, u_x) Psi(c_y, u_y) Psi(c_z, u_z)      (Eq. 11, one
 *          factor per axis: Psi(0, u) = 1 - theta - u^2,
 *          Psi(+-1, u) = (theta +- u + u^2)/2)
 *          or the second-order polynomial equilibrium with tensor-product
 *          weights at theta0 = 1/3                             (Sec. III.D)
 *   f^OReg = f^eq/(2 rho theta^2) (C C - C^2/3 I) : S,
 *          S = sum_k (c_k c_k - c_k^2/3 I) f^neq_k, C = c - u   (Eq. 6, D = 3)
 *   f_i(x + c_i, t + 1) = f_i^eq + (1 - 1/tau) f_i^OReg        (Eq. 7)
 *
 * or the lattice-BGK update of Eq. (1).  Delta t = 1, nu = theta (tau - 1/2).
 *
 * Conventions shared by every lb3_ entry point:
 *   - velocity index i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1), c in {-1,0,1}^3
 *     (rest velocity i = 13; the opposite of i is 26 - i);
 *   - node (x, y, z), 0 <= x < nx, ..., stored x fastest, then y, then z;
 *   - fields are double [nz][ny][nx]; populations are double [27][nz][ny][nx];
 *   - the observable state is the pre-collision f(x, t) of Eq. (7).
 * Ownership, errors, stream semantics and threading are those of oreg.h: a
 * lattice owns its device memory, host arrays are copied and never kept,
 * device arrays are the caller's and must stay valid until lb3_sync, every
 * call returns an lb_status and nothing throws across the ABI.
 */
#ifndef OREG3_H
#define OREG3_H

#include <stdint.h>

#include "oreg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb3_lattice lb3_lattice;

typedef struct lb3_options {
  int nx, ny, nz;             /* box size, each >= 1                              */
  double tau;                 /* relaxation time, > 1/2                            */
  double theta;               /* reduced temperature; 1/3 for LB_EQ_POLY2         */
  lb_equilibrium equilibrium;
  lb_storage storage;         /* LB_F64, or shifted LB_F32S / LB_F16S / LB_BF16S
                                 (f_i - w_i rho0 stored, FP32 collision)          */
  lb_collision collision;     /* LB_COLL_OREG (Eqs. 6, 7) or LB_COLL_BGK (Eq. 1)   */
  double rho0;                /* reference density of shifted storage, > 0        */
  void* stream;               /* hipStream_t to enqueue on when use_stream         */
  int use_stream;             /* 0: own non-blocking stream; 1: `stream` (NULL =
                                 the null stream), kept alive by the caller       */
  int device;                 /* HIP device ordinal; -1: current device            */
} lb3_options;

/* Defaults: 0 x 0 x 0, tau 1, theta 1/3, guided, LB_F64, OReg, rho0 1, own
   stream, current device.  NULL-safe. */
void lb3_options_init(lb3_options* opt);

/* Allocate a D3Q27 lattice (two population buffers of
   27 * nx * ny * nz * sizeof(storage) bytes).  LB_EINVAL: NULL pointer, a
   size < 1 or too large for one launch, tau or theta not finite, tau <= 1/2,
   guided with theta outside (0, 1), polynomial with |theta - 1/3| > 1e-12,
   rho0 not finite or <= 0 with shifted storage, unknown enum, device out of
   range.  LB_ENOMEM / LB_EDEVICE from HIP. */
lb_status lb3_create(const lb3_options* opt, lb3_lattice** out);

/* f(x, 0) = f^eq(rho(x), u(x)) and t = 0.  Host double [nz][ny][nx] each.
   LB_EINVAL for a NULL pointer, a non-finite value or rho <= 0.  Synchronous. */
lb_status lb3_init(lb3_lattice* h, const double* rho, const double* ux, const double* uy,
                   const double* uz);

/* lb3_init from device arrays; waits for the lattice's stream to validate
   them (LB_EINVAL leaves the lattice uninitialized).  The arrays must be
   completely written when the lattice's stream reaches the init: work on
   other streams is not waited for (synchronize the producer first). */
lb_status lb3_init_device(lb3_lattice* h, const double* rho, const double* ux,
                          const double* uy, const double* uz);

/* Enqueue n time steps (one sweep launch each) and return.  n == 0 is a
   no-op; LB_EINVAL for n < 0, LB_ESTATE before init. */
lb_status lb3_step(lb3_lattice* h, int64_t n);

/* rho, ux, uy, uz of the current state into host double [4][nz][ny][nx].
   Synchronous.  LB_ESTATE before init. */
lb_status lb3_moments(lb3_lattice* h, double* out);

/* The same into a device array of 4 * nx * ny * nz doubles, enqueued on the
   lattice's stream (asynchronous). */
lb_status lb3_moments_device(lb3_lattice* h, double* out_dev);

/* Pre-collision populations, unshifted FP64, into host double
   [27][nz][ny][nx] (checkpoint).  Synchronous. */
lb_status lb3_populations(lb3_lattice* h, double* out);

/* Replace the state by host populations [27][nz][ny][nx] (rounded to the
   storage format) and set t = 0.  LB_EINVAL for a non-finite value or a node
   with sum_i f_i <= 0.  Synchronous. */
lb_status lb3_set_populations(lb3_lattice* h, const double* in);

/* FP64 sums over the box, in a fixed order (deterministic): out[0] mass,
   out[1..3] momentum, out[4] kinetic energy, out[5] total energy
   sum (3/2 rho theta + rho |u|^2 / 2), out[6] the number of nodes holding a
   non-finite population (they are left out of the other sums).  Synchronous. */
lb_status lb3_diagnostics(lb3_lattice* h, double out[7]);

/* Wait for the lattice's stream. */
lb_status lb3_sync(lb3_lattice* h);

/* Time steps since the last init (-1 for NULL). */
int64_t lb3_time(const lb3_lattice* h);

/* Device bytes held by the lattice (0 for NULL). */
int64_t lb3_device_bytes(const lb3_lattice* h);

/* Wait for outstanding work, free everything.  NULL-safe. */
lb_status lb3_destroy(lb3_lattice* h);

/* Message of the last failing call on h (NULL: on the calling thread). */
const char* lb3_last_error(const lb3_lattice* h);

#ifdef __cplusplus
}
#endif
#endif
