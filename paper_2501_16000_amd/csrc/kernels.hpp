// kernels.hpp -- host-side launchers of the D2Q9 OReg kernels (gfx950).
//
// Internal storage convention of a lattice buffer: plane i holds the
// post-collision, not yet streamed populations g_i, so that the observable
// pre-collision state of Eq. (7) is f_i(x, t) = g_i(x - c_i) (periodic).
// A sweep pulls g_i(x - c_i) from one buffer, collides, and stores g_i(x)
// into the other; streaming is the pull.  Shifted storage keeps g_i - w_i rho0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d2q9.hpp"

namespace oreg {

struct Geometry {
  int nx, ny;
  int64_t plane;  // nx * ny
};

// Number of workgroups of the diagnostics reduction (fixed: the reduction
// order, hence the FP64 result, depends only on the lattice size).
constexpr int kDiagBlocks = 1024;

// One time step: src -> dst.
hipError_t launch_sweep(int eq, int coll, int bc, int st, const void* src, void* dst,
                        const Geometry& g, const Coef64& c, hipStream_t s);

// Work-items (threads) of the single-step sweep launch for storage st on an
// nx x ny lattice: nodes per row rounded up to the workgroup's tile, times
// ny, divided by the nodes per thread.  HIP launches stay below 2^32.
int64_t sweep_work_items(int st, int nx, int ny);

// Time steps one fused launch advances for a storage format.
int fused_levels(int st);

// Wavefronts that sweep one strip of a fused launch together (1 or 4).
int fused_wavefronts(int st);

// Whether fused launches beat single-step launches for this lattice size.
bool fused_worthwhile(int st, int nx, int ny);

// Whether a fused launch of `levels` steps (2 .. fused_levels(st)) is
// compiled for this collision and boundary: the full count always, fewer
// steps for periodic OReg lattices.
bool fused_levels_available(int coll, int bc, int st, int levels);

// `levels` time steps in one launch: src -> dst; each column strip (of one
// wavefront, or of a whole workgroup: fused_wavefronts) produces `rows` (a
// multiple of 3) output rows.
hipError_t launch_fused_sweep(int eq, int coll, int bc, int st, const void* src, void* dst,
                              const Geometry& g, const Coef64& c, int rows, int levels,
                              hipStream_t s);

// SIMDs of the current device and wavefronts of the `levels`-step fused sweep
// for storage st that one SIMD holds at once (zeros if the query fails).
struct FusedShape {
  int simds;
  int waves_per_simd;
};
FusedShape fused_shape(int st, int levels);

// Modelled time of one K-step fused launch on an nx x ny lattice with H
// output rows per strip, in row-collision units of one wavefront.
double fused_cost(int st, int nx, int ny, int H, const FusedShape& sh, int K);

// Output rows per strip (a multiple of 3) that minimise fused_cost.
int fused_rows(int st, int nx, int ny, const FusedShape& sh, int levels);

// g from fields (device FP64 [ny][nx] each); counts invalid input nodes
// (non-finite value or rho <= 0) into *bad.
hipError_t launch_init(int eq, int st, const double* rho, const double* ux, const double* uy,
                       void* dst, const Geometry& g, const Coef64& c, unsigned int* bad,
                       hipStream_t s);

// Plane i of g from plane i of pre-collision FP64 populations (device).
hipError_t launch_import_plane(int st, int i, const double* fin, void* dst, const Geometry& g,
                               const Coef64& c, hipStream_t s);

// Plane i of the pre-collision FP64 populations (device) from g.
hipError_t launch_export_plane(int st, int i, const void* src, double* fout, const Geometry& g,
                               const Coef64& c, hipStream_t s);

// rho, ux, uy of the pre-collision state into out[3][ny][nx] (device FP64).
hipError_t launch_moments(int st, const void* src, double* out, const Geometry& g,
                          const Coef64& c, hipStream_t s);

// Diagnostics of the pre-collision state: partials[kDiagBlocks][6] scratch,
// out[6] result (device FP64).
hipError_t launch_diagnostics(int st, const void* src, double* partials, double* out,
                              const Geometry& g, const Coef64& c, double theta_energy,
                              hipStream_t s);

// y-average of rho(x): out[nx] (device FP64).
hipError_t launch_profile(int st, const void* src, double* out, const Geometry& g,
                          const Coef64& c, hipStream_t s);

// ------------------------------------------------------------ serving --
// One resident lattice of a server, as the batched sweep reads it.
struct LatticeDesc {
  void* buf[2];        // A/B population buffers
  double* fields;      // 3 * plane FP64: initial fields, later the result moments
  int nx, ny;
  int64_t plane;       // nx * ny
  int64_t admit_T;     // server launch counter at admission; the state is in
                       // buf[(T - admit_T) % 2] before launch T
  int64_t tile_begin;  // first work item of this lattice
  int kl;              // fused launches: time steps this launch advances the lattice
  int rows;            // fused launches: output rows per work item
  int strips;          // fused launches: column strips
  Coef64 coef;
};

// tile_map[b] = index of the lattice that owns work item b (after the
// descriptors are in device memory).
hipError_t launch_tile_map(const LatticeDesc* d, int n, int* tile_map, int64_t tiles,
                           hipStream_t s);

// Fused batched launches: up to fused_levels(st) steps per lattice per launch
// (d[i].kl each), one wavefront per work item (a column strip x a row block).
// Column strip width of the fused sweep for storage st.
int fused_strip_width(int st);
hipError_t launch_batched_fused(int eq, int st, const LatticeDesc* d, const int* item_map,
                                int64_t items, int64_t T, hipStream_t s);

// Plain streaming copy of bytes / 16 16-byte words (copy.hip).
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);

}  // namespace oreg
