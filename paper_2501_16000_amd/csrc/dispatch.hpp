// dispatch.hpp -- helpers shared by the D2Q9 kernel translation units
// (kernels.hip and the per-storage fused_*.hip): runtime-to-template
// dispatch, periodic index wrap, the XCD-aware workgroup order, and the shape
// of the fused multi-step sweep for each storage format.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace oreg {
namespace detail {

constexpr int kThreads = 256;

template <int V>
using IC = std::integral_constant<int, V>;

// ------------------------------------------------------------- dispatch --
template <class F>
hipError_t with_storage(int st, F&& f) {
  switch (st) {
    case LB_F64: return f(IC<LB_F64>{});
    case LB_F32S: return f(IC<LB_F32S>{});
    case LB_F16S: return f(IC<LB_F16S>{});
    case LB_BF16S: return f(IC<LB_BF16S>{});
    default: return hipErrorInvalidValue;
  }
}
template <class F>
hipError_t with_eq(int eq, F&& f) {
  switch (eq) {
    case LB_EQ_GUIDED: return f(IC<LB_EQ_GUIDED>{});
    case LB_EQ_POLY2: return f(IC<LB_EQ_POLY2>{});
    default: return hipErrorInvalidValue;
  }
}
template <class F>
hipError_t with_coll(int coll, F&& f) {
  switch (coll) {
    case LB_COLL_OREG: return f(IC<LB_COLL_OREG>{});
    case LB_COLL_BGK: return f(IC<LB_COLL_BGK>{});
    default: return hipErrorInvalidValue;
  }
}
template <class F>
hipError_t with_bc(int bc, F&& f) {
  switch (bc) {
    case LB_BC_PERIODIC: return f(IC<LB_BC_PERIODIC>{});
    case LB_BC_BOUNCEBACK: return f(IC<LB_BC_BOUNCEBACK>{});
    default: return hipErrorInvalidValue;
  }
}

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v == n - 1 ? 0 : v + 1; }
__device__ __forceinline__ int wrap_sub(int v, int c, int n) {
  return c == 0 ? v : (c > 0 ? wrap_dec(v, n) : wrap_inc(v, n));
}

// Workgroups go to the 8 XCDs of the chip round-robin (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  xcd_block() renumbers them (a
// bijection on 0 .. gridDim.x - 1) so that every XCD takes one contiguous
// range: neighbouring tiles, which share cache lines at their edges, run on
// the same XCD.  Used by the fused sweeps, whose strips share 2K halo
// columns (their HBM reads fell from 1.27-1.62 to 1.16-1.19 times the
// algorithmic bytes).
__device__ __forceinline__ int xcd_block() {
  const int nwg = gridDim.x, b = blockIdx.x, xcd = b % 8, per = nwg / 8, extra = nwg % 8;
  return xcd * per + (xcd < extra ? xcd : extra) + b / 8;
}

// Fused launches per storage.  K: steps per launch.  FP64: seven.  Its
// launch time is set by the memory traffic of the strip pipeline (a
// streaming-only copy of the kernel, with the collision removed, ran within
// 2 % of it at K = 6, and launches of 2 to 6 steps all took 0.57-0.61 ms on
// 4096^2), so a further level is nearly free: 4096^2 ran at 169 (K = 6), 178
// (K = 7) and 179 (K = 8) GLUPS, and K = 7 wastes fewer halo columns and
// splits short step counts better.  The FP32 formats are bound by their
// collisions at K = 6 (0.44 ms per launch against 0.30 ms for two steps in
// F32S) and keep six.
// NW: wavefronts per strip.  F32S shares one
// 256-column strip per workgroup (measured 9 % faster than a strip per
// wavefront: 12 % fewer instructions per node update against six workgroup
// barriers per row step); in F64 the same layout measured 2 % slower, and
// the 16-bit formats pre-shift their windows inside the wavefront.
template <int ST> struct FusedLevels { static constexpr int K = 6, NW = 1; };
template <> struct FusedLevels<LB_F64> { static constexpr int K = 7, NW = 1; };
template <> struct FusedLevels<LB_F32S> { static constexpr int K = 6, NW = 4; };

// Fused launches of fewer than FusedLevels<ST>::K steps (lb_step's remainder)
// are compiled for periodic OReg lattices, the configuration the benchmark
// and the server use; other configurations run a remainder one step per
// launch.
constexpr bool short_fused(int coll, int bc) {
  return coll == LB_COLL_OREG && bc == LB_BC_PERIODIC;
}

}  // namespace detail

// The fused sweeps of one storage format (fused_*.hip, one translation unit
// per format so that they compile in parallel).
template <int ST>
hipError_t fused_launch_st(int eq, int coll, int bc, const void* src, void* dst, const Geometry& g,
                           const Coef64& c, int rows, int levels, hipStream_t s);
template <int ST>
hipError_t fused_occupancy_st(int levels, int* blocks);
template <int ST>
hipError_t batched_fused_launch_st(int eq, const LatticeDesc* d, const int* item_map, int64_t items,
                                   int64_t T, hipStream_t s);

}  // namespace oreg
