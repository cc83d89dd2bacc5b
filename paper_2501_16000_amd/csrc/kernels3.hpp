// kernels3.hpp -- host-side launchers of the D3Q27 kernels (gfx950).
//
// Storage convention (as on D2Q9): plane i of a buffer holds the
// post-collision, not yet streamed populations g_i, so the observable state
// is f_i(x, t) = g_i(x - c_i) (periodic); a sweep pulls g_i(x - c_i) from one
// buffer, collides and stores g_i(x) into the other.  Shifted storage keeps
// g_i - w_i rho0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3q27.hpp"

namespace oreg {

struct Geometry3 {
  int nx, ny, nz;
  int64_t cells;  // nx * ny * nz
};

// Workgroups of the diagnostics reduction (fixed, so the FP64 sums depend
// only on the box size).
constexpr int kDiag3Blocks = 1024;

// Wavefront tasks of one sweep: 64-node segments of every x-row.
int64_t sweep3_tasks(const Geometry3& g);

// One time step src -> dst.
hipError_t launch_sweep3(int eq, int coll, int st, const void* src, void* dst, const Geometry3& g,
                         const Coef64& c, hipStream_t s);

// g from device FP64 fields [nz][ny][nx]; invalid nodes are counted in *bad.
hipError_t launch_init3(int eq, int st, const double* rho, const double* ux, const double* uy,
                        const double* uz, void* dst, const Geometry3& g, const Coef64& c,
                        unsigned int* bad, hipStream_t s);

// Plane i of pre-collision FP64 populations in/out of a buffer.
hipError_t launch_import3(int st, int i, const double* fin, void* dst, const Geometry3& g,
                          const Coef64& c, hipStream_t s);
hipError_t launch_export3(int st, int i, const void* src, double* fout, const Geometry3& g,
                          const Coef64& c, hipStream_t s);

// rho, ux, uy, uz into out[4][cells].
hipError_t launch_moments3(int st, const void* src, double* out, const Geometry3& g,
                           const Coef64& c, hipStream_t s);

// The seven FP64 sums of lb3_diagnostics into out[7]; partials holds
// kDiag3Blocks * 7 doubles.
hipError_t launch_diagnostics3(int st, const void* src, double* partials, double* out,
                               const Geometry3& g, const Coef64& c, double theta_energy,
                               hipStream_t s);

}  // namespace oreg
