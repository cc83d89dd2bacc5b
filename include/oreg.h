/*
 * oreg.h -- C ABI of the MI355X (gfx950) Onsager-regularized lattice
 * Boltzmann library (liboreg.so).
 *
 * The library advances periodic D2Q9 lattices with the OReg method of
 * Jonnalagadda, Agrawal, Sharma, Rocchia and Succi (arXiv 2501.16000):
 * every time step applies, to every node x independently,
 *
 *   rho = <f, 1>, rho u = <f, c>                              (Eq. 2a)
 *   f^eq(rho, u): guided equilibrium                          (Eq. 11)
 *                 or second-order polynomial equilibrium      (Sec. III.D)
 *   f^neq = f - f^eq;  f^OReg from f^neq                      (Eq. 6)
 *   f_i(x + c_i, t + 1) = f_i^eq + (1 - 1/tau) f_i^OReg       (Eq. 7)
 *
 * with Delta t = 1.  The lattice-BGK update of Eq. (1) is available as a
 * comparison scheme, and full-way bounce-back wall columns (Sec. IV,
 * shocktube) as a boundary option.
 *
 * Conventions shared by every entry point:
 *   - velocity order i = 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 *                        5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1);
 *   - node (x, y), 0 <= x < nx, 0 <= y < ny, stored x fastest;
 *   - fields are double [ny][nx]; populations are double [9][ny][nx];
 *   - the observable state is the pre-collision f(x, t) of Eq. (7), with
 *     t counted from the last lb_init / lb_set_populations.
 *
 * Ownership: a lattice owns its device memory for its whole life.  Host
 * arrays passed in or out are owned by the caller, copied and never kept.
 * Device pointers (the *_device calls) are owned by the caller, must be HIP
 * device allocations on the lattice's device, and must stay valid until the
 * work enqueued on the lattice's stream has completed (lb_sync).
 *
 * Errors: every call returns an lb_status; nothing throws or aborts across
 * the ABI.  lb_last_error() gives a message for the last failing call on a
 * lattice (or, for NULL, on the calling thread).
 *
 * Threading: calls on one lattice must not overlap (one lattice per thread,
 * or external locking); distinct lattices are independent.
 */
#ifndef OREG_H
#define OREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_lattice lb_lattice;

/* Equilibrium of the collision: Eq. (11) (any 0 < theta < 1) or the
   second-order polynomial form of Sec. III.D at theta0 = 1/3. */
typedef enum lb_equilibrium { LB_EQ_GUIDED = 0, LB_EQ_POLY2 = 1 } lb_equilibrium;

/* Population storage in device memory.  LB_F64 keeps f_i in FP64 and
   computes in FP64.  The shifted formats keep f_i - w_i rho0 (w_i the rest
   equilibrium weights of the chosen equilibrium, rho0 the reference density
   of lb_options) rounded to nearest-even in FP32, FP16 or BF16, and collide
   in FP32 registers; LB_F32S forms u = j / rho as (j - j e) / rho0 with
   e = (rho - rho0) / rho, so that the FP32 rounding of rho near rho0 (a
   smooth error that biases the momentum every step) enters u only through
   the small e. */
typedef enum lb_storage {
  LB_F64 = 0,
  LB_F32S = 1,
  LB_F16S = 2,
  LB_BF16S = 3
} lb_storage;

/* Collision: OReg (Eqs. 6, 7) or lattice BGK (Eq. 1). */
typedef enum lb_collision { LB_COLL_OREG = 0, LB_COLL_BGK = 1 } lb_collision;

/* Boundary in x: periodic, or full-way bounce-back wall nodes in columns
   x = 0 and x = nx - 1 (they reverse every population instead of colliding;
   the wall sits half-way to the first fluid column).  y is always periodic. */
typedef enum lb_boundary { LB_BC_PERIODIC = 0, LB_BC_BOUNCEBACK = 1 } lb_boundary;

typedef enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,      /* invalid argument (see each call)                    */
  LB_ENOMEM = -2,      /* a device allocation failed                          */
  LB_EDEVICE = -3,     /* any other HIP error, or no usable device            */
  LB_ESTATE = -4,      /* call not valid in the lattice's state (not inited)  */
  LB_ENONFINITE = -5,  /* lb_step with check_nonfinite found NaN/Inf          */
  LB_EAGAIN = -6       /* server: no room / nothing ready now; retry later    */
} lb_status;

typedef struct lb_options {
  int nx, ny;                 /* lattice size, both >= 1                        */
  double tau;                 /* relaxation time, > 1/2 (nu = theta (tau - 1/2)) */
  double theta;               /* reduced temperature; 1/3 for LB_EQ_POLY2       */
  lb_equilibrium equilibrium;
  lb_storage storage;
  lb_collision collision;
  lb_boundary boundary_x;
  double rho0;                /* reference density of shifted storage, > 0     */
  void* stream;               /* hipStream_t to enqueue on when use_stream      */
  int use_stream;             /* 0: the lattice creates and owns a non-blocking
                                 stream; 1: enqueue on `stream` (NULL = the
                                 device's null stream), owned by the caller and
                                 kept alive until lb_destroy returns           */
  int device;                 /* HIP device ordinal; -1: current device         */
  int check_nonfinite;        /* nonzero: lb_step scans for NaN/Inf afterwards  */
  int fuse_steps;             /* 0: lb_step advances K time steps per launch
                                 (register-resident multi-step sweep; same
                                 result bit for bit; K = 7 for LB_F64, 6 for
                                 the shifted formats) on lattices of at least
                                 48^2 nodes, where it is faster, a remainder of
                                 2 .. K-1 steps in one shorter fused launch
                                 (periodic OReg lattices) and one step per
                                 launch below that size and otherwise;
                                 1: one sweep launch per time step;
                                 2: fused launches whatever the size           */
} lb_options;

/* Defaults: 0 x 0, tau 1, theta 1/3, guided, LB_F64, OReg, periodic, rho0 1,
   own stream (use_stream 0), current device, no checks, fused steps.
   NULL-safe. */
void lb_options_init(lb_options* opt);

/* FP64 periodic OReg lattice on the current device with its own stream.
   LB_EINVAL: nx or ny < 1, too large, tau or theta not finite, tau <= 1/2,
   guided with theta outside (0, 1), polynomial with |theta - 1/3| > 1e-12,
   unknown enum, fuse_steps not 0, 1 or 2, out == NULL.  LB_ENOMEM / LB_EDEVICE
   from HIP. */
lb_status lb_create(int nx, int ny, double tau, double theta, lb_equilibrium eq,
                    lb_lattice** out);

/* Same as lb_create with every option; additionally LB_EINVAL for rho0 not
   finite or <= 0 with shifted storage, or a device ordinal out of range. */
lb_status lb_create_ex(const lb_options* opt, lb_lattice** out);

/* Initial state (Sec. II; equilibrium of Eq. (11), or of Sec. III.D for
   LB_EQ_POLY2): f(x, 0) = f^eq(rho(x), u(x)), with no non-equilibrium part,
   and t = 0.  rho, ux, uy: host double [ny][nx].
   LB_EINVAL for a NULL pointer, a non-finite value or rho <= 0.  Synchronous. */
lb_status lb_init(lb_lattice* h, const double* rho, const double* ux, const double* uy);

/* lb_init from device arrays (e.g. torch tensors).  Enqueued on the
   lattice's stream; waits for it to validate the fields (LB_EINVAL as in
   lb_init, in which case the state is left uninitialized).  The arrays must
   be completely written when the lattice's stream reaches the init: work
   that produces them on another stream is not waited for, so synchronize
   that stream first (or create the lattice on it with use_stream). */
lb_status lb_init_device(lb_lattice* h, const double* rho, const double* ux,
                         const double* uy);

/* Eq. (7) applied n times: every step streams the populations and replaces
   them by f^eq + (1 - 1/tau) f^OReg (Eq. 6), or by the lattice-BGK update of
   Eq. (1).  Enqueue n time steps on the lattice's stream and return
   (asynchronous).
   n == 0 is a no-op.  LB_EINVAL for n < 0, LB_ESTATE before init.  With
   check_nonfinite set, waits and returns LB_ENONFINITE if a node holds a
   non-finite population. */
lb_status lb_step(lb_lattice* h, int64_t n);

/* Moments of Eq. (2a): rho = sum_i f_i and u = (sum_i c_i f_i) / rho of the
   pre-collision f(x, t): host double out[3][ny][nx] = rho, ux, uy.
   Waits for the stream. */
lb_status lb_moments(lb_lattice* h, double* out);

/* Same into a device array out_dev[3][ny][nx]; enqueued, asynchronous: the
   values are there once the lattice's stream has reached this point
   (lb_sync, or an event on that stream). */
lb_status lb_moments_device(lb_lattice* h, double* out_dev);

/* Pre-collision populations f(x, t), unshifted, FP64: host double
   out[9][ny][nx].  Waits for the stream. */
lb_status lb_populations(lb_lattice* h, double* out);

/* Replace the state by host populations in[9][ny][nx] (pre-collision, FP64,
   unshifted; shifted storage rounds them) and set t = 0.  LB_EINVAL for a
   non-finite value or a node with sum_i f_i <= 0.  Synchronous. */
lb_status lb_set_populations(lb_lattice* h, const double* in);

/* FP64 sums over all nodes of the pre-collision state, in a fixed reduction
   order (bit-reproducible for a given lattice size):
   out[0] mass sum rho, out[1..2] momentum sum rho u, out[3] kinetic energy
   sum rho |u|^2 / 2, out[4] total energy sum (rho theta + rho |u|^2 / 2)
   (E of Eq. 2a with p = rho theta, D = 2), out[5] number of nodes holding a
   non-finite population (those nodes are left out of out[0..4]).
   Waits for the stream. */
lb_status lb_diagnostics(lb_lattice* h, double out[6]);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
   lb_diagnostics, bit for bit, enqueued into the caller's device array
   out_dev[6] on the lattice's stream, asynchronously (no host transfer, no
   synchronization, no hipMalloc/hipFree, no memset).  The reduction's
   partial sums go to a 48 KiB (1024 x 6 doubles) device array that the
   library holds statically, one per GPU, for the life of the process: its
   size is fixed and covers every lattice size.  Every call on a GPU shares
   that GPU's array, so calls that overlap on one GPU (lattices on different
   streams, or threads) race and must be ordered by the caller; the array
   keeps the last call's partials.  The lattice itself must have been created
   (and initialized) beforehand.  LB_EINVAL for NULL arguments, LB_ESTATE
   before init, LB_EDEVICE if the array cannot be located on the device. */
lb_status lb_diagnostics_device_noalloc(lb_lattice* h, double* out_dev);

/* y-average of rho(x) of the pre-collision state: host double out[nx].
   Waits for the stream. */
lb_status lb_density_profile(lb_lattice* h, double* out);

/* Wait for all work enqueued on the lattice's stream. */
lb_status lb_sync(lb_lattice* h);

/* Time steps taken since the last init (-1 for NULL). */
int64_t lb_time(const lb_lattice* h);

/* Options the lattice was created with (NULL-safe: LB_EINVAL). */
lb_status lb_get_options(const lb_lattice* h, lb_options* out);

/* Bytes of device memory held by the lattice. */
int64_t lb_device_bytes(const lb_lattice* h);

/* Free the lattice and its device memory after its stream drains.
   NULL-safe (returns LB_OK). */
lb_status lb_destroy(lb_lattice* h);

/* Measurement helper, not a step of the method: copy `bytes` bytes from src
   to dst (caller-owned device memory of the current device, 16-byte
   aligned, not overlapping) with a plain streaming kernel, every byte read
   once and written once, enqueued on hip_stream (NULL: the null stream) and
   asynchronous.  Timed by the caller, it gives the practical HBM ceiling
   that the sweeps' achieved bandwidth is set against.  LB_EINVAL for a NULL
   buffer, a size that is negative or not a multiple of 16, misaligned or
   overlapping buffers; LB_EDEVICE (or LB_ENOMEM) if the launch fails.
   bytes == 0 is a no-op. */
lb_status lb_copy_device(const void* src, void* dst, int64_t bytes, void* hip_stream);

/* Static text for a status code. */
const char* lb_status_string(lb_status s);

/* Message of the last failing call on h, or of the calling thread's last
   failing call when h is NULL; "" if none.  Valid until the next call. */
const char* lb_last_error(const lb_lattice* h);

/* ------------------------------------------------------------------------
 * Serving: many independent lattices resident on one GPU (continuous
 * batching).
 *
 * A server owns a device arena of `memory_budget` bytes.  lb_server_submit
 * admits a request at once when a slot and arena space are free (its
 * footprint is 2 * 9 * sizeof(storage) + 24 bytes per node) and returns
 * LB_EAGAIN otherwise, so the caller keeps the queue and retries as lattices
 * retire.  lb_server_step issues batched launches; one launch covers every
 * resident lattice and advances each by up to K time steps (K as for
 * lb_step: 7 for LB_F64, 6 for the shifted formats; fewer in a
 * lattice's last launch), running the same per-node update as lb_step (Eqs. (6), (7) with the
 * server's equilibrium and storage and the request's tau).  Each lattice is
 * retired after its requested number of steps: its moments are gathered and
 * copied to pinned host memory asynchronously.  lb_server_poll reports finished results,
 * lb_server_fetch hands their moments to the caller.  A result does not depend
 * on which other lattices shared the launches: the per-node arithmetic is that
 * of a lattice running alone.
 * ------------------------------------------------------------------------ */
typedef struct lb_server lb_server;

typedef struct lb_server_options {
  int64_t memory_budget;      /* device bytes for resident lattices, > 0       */
  int64_t pinned_bytes;       /* pinned host bytes for field uploads and
                                 results (each side), > 0                      */
  int max_active;             /* resident lattices at most, 1 .. 65536         */
  lb_equilibrium equilibrium;
  lb_storage storage;
  double theta;               /* as in lb_options                              */
  double rho0;                /* reference density of shifted storage          */
  int device;                 /* -1: current device                            */
} lb_server_options;

typedef struct lb_request {
  int64_t tag;                /* caller's identifier, reported with the result */
  int nx, ny;                 /* lattice size, >= 1                            */
  double tau;                 /* > 1/2                                         */
  int64_t steps;              /* time steps to run, >= 1                       */
  const double* rho;          /* host [ny][nx] initial fields (f = f^eq),     */
  const double* ux;           /* copied during the call                        */
  const double* uy;
} lb_request;

typedef struct lb_result {
  int64_t tag;
  int nx, ny;
  int64_t steps;
  double t_submit, t_done;    /* server clock (seconds, monotonic) at admission
                                 and when the moments reached host memory      */
} lb_result;

typedef struct lb_server_stats {
  int active;                 /* resident lattices being stepped               */
  int retiring;               /* finished, moments in flight to the host       */
  int ready;                  /* results waiting for lb_server_fetch           */
  int64_t device_bytes_used;  /* arena bytes held                              */
  int64_t launches;           /* batched launches issued                       */
  int64_t node_updates;       /* node updates done (nodes x steps)             */
  double clock;               /* server clock now (seconds)                    */
} lb_server_stats;

/* Defaults: 16 GiB arena, 1 GiB pinned per side, 256 slots, guided, F32S,
   theta 1/3, rho0 1, current device. */
void lb_server_options_init(lb_server_options* opt);

/* LB_EINVAL for invalid options (as lb_create_ex for the equilibrium, storage,
   theta and rho0); LB_ENOMEM / LB_EDEVICE from HIP. */
lb_status lb_server_create(const lb_server_options* opt, lb_server** out);

/* Admit one request now.  LB_EAGAIN: no free slot, arena or pinned space at
   the moment (nothing was kept; retry after lb_server_step / lb_server_poll).
   LB_EINVAL: invalid request, non-finite field or rho <= 0, or a footprint
   larger than the whole arena. */
lb_status lb_server_submit(lb_server* s, const lb_request* req);

/* Issue up to n batched launches (fewer if no lattice is resident); retires
   lattices as they finish.  Asynchronous: returns once the launches are
   enqueued. */
lb_status lb_server_step(lb_server* s, int64_t n);

/* Oldest finished result whose moments are in host memory: fills *out and
   returns LB_OK, or LB_EAGAIN if none is ready. */
lb_status lb_server_poll(lb_server* s, lb_result* out);

/* Copy the moments rho, ux, uy (host double out[3][ny][nx]) of the ready
   result `tag` and release it.  LB_EINVAL if no ready result has that tag. */
lb_status lb_server_fetch(lb_server* s, int64_t tag, double* out);

lb_status lb_server_stats_get(lb_server* s, lb_server_stats* out);

/* Wait for all enqueued work. */
lb_status lb_server_sync(lb_server* s);

/* Free the server (waits for its work).  NULL-safe. */
lb_status lb_server_destroy(lb_server* s);

/* Message of the last failing call on s ("" if none); for NULL, of the
   calling thread's last failure that had no server handle (lb_server_create). */
const char* lb_server_last_error(const lb_server* s);

#ifdef __cplusplus
}
#endif

#endif /* OREG_H */
