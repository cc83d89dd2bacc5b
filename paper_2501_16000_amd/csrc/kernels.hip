// kernels.hip -- D2Q9 OReg kernels for gfx950 and their launchers.
//
// The sweep is one fused pass per time step: pull the nine populations of a
// node from their upwind neighbours (periodic wrap), collide in registers
// (d2q9.hpp), store the node's nine post-collision populations.  Every plane
// element of the source is read by exactly one node, so the pass moves
// 2 * 9 * sizeof(storage) bytes per node and is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dispatch.hpp"

namespace oreg {
namespace {
using namespace detail;

// Output rows per strip of a fused launch when the device query fails.
constexpr int kFusedRowsDefault = 66;

// ---------------------------------------------------------------- sweep --
// Launch shape per storage: nodes per thread (VX) and workgroup size.  One
// node per thread keeps the FP64 and FP32 collisions at high occupancy; two
// nodes per thread give the 16-bit formats 4-byte loads per lane.
template <int ST> struct SweepShape { static constexpr int VX = 1, BS = 256; };
template <> struct SweepShape<LB_F32S> { static constexpr int VX = 1, BS = 512; };
template <> struct SweepShape<LB_F16S> { static constexpr int VX = 2, BS = 256; };
template <> struct SweepShape<LB_BF16S> { static constexpr int VX = 2, BS = 256; };

// Unaligned vector load (gfx950 global loads accept any 2-byte alignment).
template <typename V, typename T>
__device__ __forceinline__ V load_vec(const T* p) {
  V v;
  __builtin_memcpy(&v, p, sizeof(V));
  return v;
}

// Pull f_i(x) = g_i(x - c_i) for VX consecutive nodes x0 .. x0+VX-1 of row y.
// Threads away from the x edges use one vector load per plane; edge threads
// wrap node by node.
template <int ST, int VX>
__device__ __forceinline__ void pull(const typename Storage<ST>::T* __restrict__ src,
                                     const Geometry& g, int x0, int64_t r0, int64_t rm,
                                     int64_t rp, typename Storage<ST>::R (&f)[VX][9]) {
  using S = Storage<ST>;
  using T = typename S::T;
  typedef T V __attribute__((ext_vector_type(VX)));
  const int64_t P = g.plane;
  const int nx = g.nx;
  if (x0 >= 1 && x0 + VX < nx) {
    const V v0 = load_vec<V>(src + 0 * P + r0 + x0);
    const V v1 = load_vec<V>(src + 1 * P + r0 + x0 - 1);
    const V v2 = load_vec<V>(src + 2 * P + rm + x0);
    const V v3 = load_vec<V>(src + 3 * P + r0 + x0 + 1);
    const V v4 = load_vec<V>(src + 4 * P + rp + x0);
    const V v5 = load_vec<V>(src + 5 * P + rm + x0 - 1);
    const V v6 = load_vec<V>(src + 6 * P + rm + x0 + 1);
    const V v7 = load_vec<V>(src + 7 * P + rp + x0 + 1);
    const V v8 = load_vec<V>(src + 8 * P + rp + x0 - 1);
#pragma unroll
    for (int q = 0; q < VX; ++q) {
      f[q][0] = S::load(v0[q]);
      f[q][1] = S::load(v1[q]);
      f[q][2] = S::load(v2[q]);
      f[q][3] = S::load(v3[q]);
      f[q][4] = S::load(v4[q]);
      f[q][5] = S::load(v5[q]);
      f[q][6] = S::load(v6[q]);
      f[q][7] = S::load(v7[q]);
      f[q][8] = S::load(v8[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < VX; ++q) {
      const int x = (x0 + q < nx) ? x0 + q : nx - 1;  // nodes past nx are not stored
      const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
      f[q][0] = S::load(src[0 * P + r0 + x]);
      f[q][1] = S::load(src[1 * P + r0 + xm]);
      f[q][2] = S::load(src[2 * P + rm + x]);
      f[q][3] = S::load(src[3 * P + r0 + xp]);
      f[q][4] = S::load(src[4 * P + rp + x]);
      f[q][5] = S::load(src[5 * P + rm + xm]);
      f[q][6] = S::load(src[6 * P + rm + xp]);
      f[q][7] = S::load(src[7 * P + rp + xp]);
      f[q][8] = S::load(src[8 * P + rp + xm]);
    }
  }
}

// Store the post-collision populations of VX nodes at x0.. (nontemporal: the
// next sweep reads them back only after the whole lattice has streamed by).
template <int ST, int VX>
__device__ __forceinline__ void push_local(typename Storage<ST>::T* __restrict__ dst,
                                           const Geometry& g, int x0, int64_t r0,
                                           const typename Storage<ST>::R (&f)[VX][9]) {
  using S = Storage<ST>;
  using T = typename S::T;
  typedef T V __attribute__((ext_vector_type(VX)));
  const int64_t P = g.plane;
  // Vector stores need sizeof(V) alignment: an even row length (VX = 2).
  const bool aligned = (VX == 1) || ((((r0 + x0) | P) & (VX - 1)) == 0);
  if (x0 + VX <= g.nx && aligned) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      V v;
#pragma unroll
      for (int q = 0; q < VX; ++q) v[q] = S::store(f[q][i]);
      __builtin_nontemporal_store(v, reinterpret_cast<V*>(dst + i * P + r0 + x0));
    }
  } else {
#pragma unroll
    for (int q = 0; q < VX; ++q) {
      if (x0 + q < g.nx) {
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * P + r0 + x0 + q] = S::store(f[q][i]);
      }
    }
  }
}

template <int EQ, int COLL, int BC, int ST>
__global__ __launch_bounds__(SweepShape<ST>::BS) void sweep_kernel(
    const typename Storage<ST>::T* __restrict__ src, typename Storage<ST>::T* __restrict__ dst,
    Geometry g, Coef64 c, int nseg) {
  using S = Storage<ST>;
  using R = typename S::R;
  constexpr int VX = SweepShape<ST>::VX, BS = SweepShape<ST>::BS;
  // Plain block order: renumbering the blocks per XCD (xcd_block) removed
  // the 4 % of reads that straddle two blocks' x ranges but made this
  // HBM-bound sweep 5 % slower (measured), so it is not used here.
  const int y = blockIdx.x / nseg;
  const int x0 = ((blockIdx.x - y * nseg) * BS + threadIdx.x) * VX;
  if (x0 >= g.nx) return;
  const int ym = wrap_dec(y, g.ny), yp = wrap_inc(y, g.ny);
  const int64_t r0 = (int64_t)y * g.nx, rm = (int64_t)ym * g.nx, rp = (int64_t)yp * g.nx;
  R f[VX][9];
  pull<ST, VX>(src, g, x0, r0, rm, rp, f);
  const Coeffs<R> k(c);
#pragma unroll
  for (int q = 0; q < VX; ++q) {
    if (BC == LB_BC_BOUNCEBACK && (x0 + q == 0 || x0 + q == g.nx - 1)) {
      // Full-way bounce-back wall node: reverse every population.
      R r[9];
      unroll<0, 9>([&](auto I) { r[I.value] = f[q][opp_of(I.value)]; });
      unroll<0, 9>([&](auto I) { f[q][I.value] = r[I.value]; });
    } else {
      collide<EQ, COLL, S::shifted, S::delta_u>(f[q], k);
    }
  }
  push_local<ST, VX>(dst, g, x0, r0, f);
}

// ----------------------------------------------------------------- init --
template <int EQ, int ST>
__global__ __launch_bounds__(kThreads) void init_kernel(const double* __restrict__ rho,
                                                        const double* __restrict__ ux,
                                                        const double* __restrict__ uy,
                                                        typename Storage<ST>::T* __restrict__ dst,
                                                        Geometry g, Coef64 c,
                                                        unsigned int* __restrict__ bad) {
  using S = Storage<ST>;
  using R = typename S::R;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.plane) return;
  const int y = (int)(idx / g.nx);
  const int x = (int)(idx - (int64_t)y * g.nx);
  double r = rho[idx], vx = ux[idx], vy = uy[idx];
  if (!(isfinite(r) && isfinite(vx) && isfinite(vy) && r > 0.0)) {
    atomicAdd(bad, 1u);
    r = 1.0;
    vx = vy = 0.0;
  }
  const Coeffs<double> k(c);
  double feq[9], deq[9];
  equilibrium<EQ, S::shifted>(S::shifted ? r - c.rho0 : r, r, vx, vy, vx * vx, vy * vy, k, feq, deq);
  // f_i(x, 0) = f^eq_i(x) is stored as g_i(x - c_i).
  unroll<0, 9>([&](auto I) {
    constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
    const int xd = wrap_sub(x, cx, g.nx), yd = wrap_sub(y, cy, g.ny);
    dst[I.value * g.plane + (int64_t)yd * g.nx + xd] = S::store((R)deq[I.value]);
  });
}

// ------------------------------------------------------- import / export --
template <int ST>
__global__ __launch_bounds__(kThreads) void import_kernel(int i, const double* __restrict__ fin,
                                                          typename Storage<ST>::T* __restrict__ dst,
                                                          Geometry g, Coef64 c) {
  using S = Storage<ST>;
  using R = typename S::R;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.plane) return;
  const int y = (int)(idx / g.nx);
  const int x = (int)(idx - (int64_t)y * g.nx);
  const int cx = cx_of(i), cy = cy_of(i);
  const double w = S::shifted ? shift64(cx, cy, c) : 0.0;
  const int xd = wrap_sub(x, cx, g.nx), yd = wrap_sub(y, cy, g.ny);
  dst[i * g.plane + (int64_t)yd * g.nx + xd] = S::store((R)(fin[idx] - w));
}

template <int ST>
__global__ __launch_bounds__(kThreads) void export_kernel(int i,
                                                          const typename Storage<ST>::T* __restrict__ src,
                                                          double* __restrict__ fout, Geometry g,
                                                          Coef64 c) {
  using S = Storage<ST>;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.plane) return;
  const int y = (int)(idx / g.nx);
  const int x = (int)(idx - (int64_t)y * g.nx);
  const int cx = cx_of(i), cy = cy_of(i);
  const double w = S::shifted ? shift64(cx, cy, c) : 0.0;
  const int xs = wrap_sub(x, cx, g.nx), ys = wrap_sub(y, cy, g.ny);
  fout[idx] = (double)S::load(src[i * g.plane + (int64_t)ys * g.nx + xs]) + w;
}

// Pre-collision populations of node (x, y) in FP64, still shifted by w_i rho0.
template <int ST>
__device__ __forceinline__ void gather64(const typename Storage<ST>::T* __restrict__ src,
                                         const Geometry& g, int x, int y, double (&d)[9]) {
  using S = Storage<ST>;
  const int xm = wrap_dec(x, g.nx), xp = wrap_inc(x, g.nx);
  const int ym = wrap_dec(y, g.ny), yp = wrap_inc(y, g.ny);
  const int64_t P = g.plane;
  const int64_t r0 = (int64_t)y * g.nx, rm = (int64_t)ym * g.nx, rp = (int64_t)yp * g.nx;
  d[0] = (double)S::load(src[0 * P + r0 + x]);
  d[1] = (double)S::load(src[1 * P + r0 + xm]);
  d[2] = (double)S::load(src[2 * P + rm + x]);
  d[3] = (double)S::load(src[3 * P + r0 + xp]);
  d[4] = (double)S::load(src[4 * P + rp + x]);
  d[5] = (double)S::load(src[5 * P + rm + xm]);
  d[6] = (double)S::load(src[6 * P + rm + xp]);
  d[7] = (double)S::load(src[7 * P + rp + xp]);
  d[8] = (double)S::load(src[8 * P + rp + xm]);
}

// rho - rho0 and j of shifted populations (sum w_i = 1, sum w_i c_i = 0).
__device__ __forceinline__ void moments64(const double (&d)[9], double& drho, double& jx,
                                          double& jy) {
  drho = d[0] + ((d[1] + d[3]) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]));
  jx = (d[1] - d[3]) + (d[5] - d[7]) + (d[8] - d[6]);
  jy = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
}

template <int ST>
__global__ __launch_bounds__(kThreads) void moments_kernel(const typename Storage<ST>::T* __restrict__ src,
                                                           double* __restrict__ out, Geometry g,
                                                           Coef64 c) {
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.plane) return;
  const int y = (int)(idx / g.nx);
  const int x = (int)(idx - (int64_t)y * g.nx);
  double d[9], drho, jx, jy;
  gather64<ST>(src, g, x, y, d);
  moments64(d, drho, jx, jy);
  const double rho = c.rho0 + drho;
  out[idx] = rho;
  out[g.plane + idx] = jx / rho;
  out[2 * g.plane + idx] = jy / rho;
}

// ---------------------------------------------------------- diagnostics --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Fixed-order block sum of 6 values; result valid in thread 0.
__device__ __forceinline__ void block_sum6(double (&v)[6]) {
  __shared__ double part[kThreads / 64][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) part[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double s = part[0][k];
      for (int w = 1; w < kThreads / 64; ++w) s += part[w][k];
      v[k] = s;
    }
  }
}

template <int ST>
__global__ __launch_bounds__(kThreads) void diag_kernel(const typename Storage<ST>::T* __restrict__ src,
                                                        double* __restrict__ partials, Geometry g,
                                                        Coef64 c, double theta) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < g.plane; idx += stride) {
    const int y = (int)(idx / g.nx);
    const int x = (int)(idx - (int64_t)y * g.nx);
    double d[9], drho, jx, jy;
    gather64<ST>(src, g, x, y, d);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 9; ++i) finite = finite && isfinite(d[i]);
    if (!finite) {
      acc[5] += 1.0;
      continue;
    }
    moments64(d, drho, jx, jy);
    const double rho = c.rho0 + drho;
    const double ke = 0.5 * (jx * jx + jy * jy) / rho;
    acc[0] += rho;
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += ke;
    acc[4] += rho * theta + ke;
  }
  block_sum6(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) partials[blockIdx.x * 6 + k] = acc[k];
  }
}

__global__ __launch_bounds__(kThreads) void diag_final_kernel(const double* __restrict__ partials,
                                                              int nblocks, double* __restrict__ out) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kThreads) {
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += partials[b * 6 + k];
  }
  block_sum6(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = acc[k];
  }
}

template <int ST>
__global__ __launch_bounds__(kThreads) void profile_kernel(const typename Storage<ST>::T* __restrict__ src,
                                                           double* __restrict__ out, Geometry g,
                                                           Coef64 c) {
  const int x = blockIdx.x * kThreads + threadIdx.x;
  if (x >= g.nx) return;
  double sum = 0.0;
  for (int y = 0; y < g.ny; ++y) {
    double d[9], drho, jx, jy;
    gather64<ST>(src, g, x, y, d);
    moments64(d, drho, jx, jy);
    sum += c.rho0 + drho;
  }
  out[x] = sum / g.ny;
}

// ------------------------------------------------------ batched sweep --
__global__ __launch_bounds__(kThreads) void tile_map_kernel(const LatticeDesc* __restrict__ d,
                                                            int n, int* __restrict__ map,
                                                            int64_t tiles) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= tiles) return;
  int lo = 0, hi = n - 1;  // last lattice whose first tile is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  map[b] = lo;
}

unsigned int blocks_for(int64_t n) { return (unsigned int)((n + kThreads - 1) / kThreads); }

}  // namespace
using namespace detail;

// ------------------------------------------------------------ launchers --
hipError_t launch_sweep(int eq, int coll, int bc, int st, const void* src, void* dst,
                        const Geometry& g, const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    constexpr int tile = SweepShape<ST.value>::VX * SweepShape<ST.value>::BS;
    const int nseg = (g.nx + tile - 1) / tile;
    const unsigned int nblocks = (unsigned int)nseg * (unsigned int)g.ny;
    return with_eq(eq, [&](auto EQ) {
      return with_coll(coll, [&](auto CO) {
        return with_bc(bc, [&](auto BC) {
          sweep_kernel<EQ.value, CO.value, BC.value, ST.value>
              <<<nblocks, SweepShape<ST.value>::BS, 0, s>>>(
              static_cast<const T*>(src), static_cast<T*>(dst), g, c, nseg);
          return hipGetLastError();
        });
      });
    });
  });
}

int64_t sweep_work_items(int st, int nx, int ny) {
  int64_t items = -1;
  (void)with_storage(st, [&](auto ST) {
    constexpr int VX = SweepShape<ST.value>::VX, BS = SweepShape<ST.value>::BS;
    const int64_t nseg = ((int64_t)nx + VX * BS - 1) / (VX * BS);
    items = nseg * BS * (int64_t)ny;
    return hipSuccess;
  });
  return items;
}

int fused_levels(int st) {
  switch (st) {
    case LB_F64: return FusedLevels<LB_F64>::K;
    case LB_F32S: return FusedLevels<LB_F32S>::K;
    case LB_F16S: return FusedLevels<LB_F16S>::K;
    case LB_BF16S: return FusedLevels<LB_BF16S>::K;
    default: return 1;
  }
}

bool fused_levels_available(int coll, int bc, int st, int levels) {
  const int K = fused_levels(st);
  if (K < 2 || levels < 2 || levels > K) return false;
  return levels == K || short_fused(coll, bc);
}

hipError_t launch_fused_sweep(int eq, int coll, int bc, int st, const void* src, void* dst,
                              const Geometry& g, const Coef64& c, int rows, int levels,
                              hipStream_t s) {
  if (rows < 3 || rows % 3 != 0) return hipErrorInvalidValue;
  if (!fused_levels_available(coll, bc, st, levels)) return hipErrorInvalidValue;
  return with_storage(st, [&](auto ST) {
    return fused_launch_st<ST.value>(eq, coll, bc, src, dst, g, c, rows, levels, s);
  });
}

FusedShape fused_shape(int st, int levels) {
  FusedShape sh{0, 0};
  int dev = 0, cus = 0, blocks = 0;
  if (hipGetDevice(&dev) != hipSuccess) return sh;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return sh;
  const hipError_t e =
      with_storage(st, [&](auto ST) { return fused_occupancy_st<ST.value>(levels, &blocks); });
  if (e != hipSuccess) return sh;
  sh.simds = cus * 4;
  sh.waves_per_simd = blocks;  // 256-thread workgroups: one wavefront per SIMD each
  return sh;
}

int fused_wavefronts(int st) {
  switch (st) {
    case LB_F64: return FusedLevels<LB_F64>::NW;
    case LB_F32S: return FusedLevels<LB_F32S>::NW;
    case LB_F16S: return FusedLevels<LB_F16S>::NW;
    case LB_BF16S: return FusedLevels<LB_BF16S>::NW;
    default: return 1;
  }
}

double fused_cost(int st, int nx, int ny, int H, const FusedShape& sh, int K) {
  const int NW = fused_wavefronts(st), W = 64 * NW - 2 * K;
  const int64_t strips = (nx + W - 1) / W;
  // a work item takes NW wavefronts, one on each of NW SIMDs
  const int64_t items = strips * ((ny + H - 1) / H) * NW;
  const int64_t w = (items + sh.simds - 1) / sh.simds;
  const int64_t resident = w < sh.waves_per_simd ? w : sh.waves_per_simd;
  const double work = K * (double)(H + 2 * K) - K * (K + 1) + 2 * K;
  return (double)w / (1.0 + 0.08 * (double)(resident - 1)) * work;
}

int fused_rows(int st, int nx, int ny, const FusedShape& sh, int levels) {
  if (sh.simds <= 0 || sh.waves_per_simd <= 0) return kFusedRowsDefault;
  // One wavefront per SIMD already runs the pipeline near the SIMD's issue
  // limit (measured: a second one adds 6-11 %), so a launch takes about w
  // wavefront-times, w = ceil(work items / SIMDs), and one wavefront's time
  // follows its row collisions, K (H + 2K) - K (K + 1), plus a start-up of
  // about 2K.  H (a multiple of 3) minimises the modelled launch time.
  const int hmax = ny < 3 * 1024 ? (ny + 2) / 3 * 3 : 3 * 1024;
  int best = 3;
  double best_cost = -1;
  for (int H = 3; H <= hmax; H += 3) {
    const double c = fused_cost(st, nx, ny, H, sh, levels);
    if (best_cost < 0 || c < best_cost) {
      best_cost = c;
      best = H;
    }
  }
  return best;
}

hipError_t launch_init(int eq, int st, const double* rho, const double* ux, const double* uy,
                       void* dst, const Geometry& g, const Coef64& c, unsigned int* bad,
                       hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    return with_eq(eq, [&](auto EQ) {
      init_kernel<EQ.value, ST.value><<<blocks_for(g.plane), kThreads, 0, s>>>(
          rho, ux, uy, static_cast<T*>(dst), g, c, bad);
      return hipGetLastError();
    });
  });
}

hipError_t launch_import_plane(int st, int i, const double* fin, void* dst, const Geometry& g,
                               const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    import_kernel<ST.value><<<blocks_for(g.plane), kThreads, 0, s>>>(i, fin, static_cast<T*>(dst),
                                                                      g, c);
    return hipGetLastError();
  });
}

hipError_t launch_export_plane(int st, int i, const void* src, double* fout, const Geometry& g,
                               const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    export_kernel<ST.value><<<blocks_for(g.plane), kThreads, 0, s>>>(
        i, static_cast<const T*>(src), fout, g, c);
    return hipGetLastError();
  });
}

hipError_t launch_moments(int st, const void* src, double* out, const Geometry& g,
                          const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    moments_kernel<ST.value><<<blocks_for(g.plane), kThreads, 0, s>>>(static_cast<const T*>(src),
                                                                       out, g, c);
    return hipGetLastError();
  });
}

hipError_t launch_diagnostics(int st, const void* src, double* partials, double* out,
                              const Geometry& g, const Coef64& c, double theta_energy,
                              hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    diag_kernel<ST.value><<<kDiagBlocks, kThreads, 0, s>>>(static_cast<const T*>(src), partials, g,
                                                           c, theta_energy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, kThreads, 0, s>>>(partials, kDiagBlocks, out);
    return hipGetLastError();
  });
}

hipError_t launch_tile_map(const LatticeDesc* d, int n, int* tile_map, int64_t tiles,
                           hipStream_t s) {
  tile_map_kernel<<<blocks_for(tiles), kThreads, 0, s>>>(d, n, tile_map, tiles);
  return hipGetLastError();
}

int fused_strip_width(int st) { return 64 - 2 * fused_levels(st); }

bool fused_worthwhile(int st, int nx, int ny) {
  // With the row count chosen per lattice (fused_rows), fused launches beat
  // single-step ones on MI355X from 64^2 nodes up in every storage format
  // (1.1-1.3x at 64^2..192^2, 2-3x at 384^2..1024^2, 3.6x for F64 at
  // 4096^2) and tie at 32^2.
  return fused_levels(st) > 1 && (int64_t)nx * ny >= 48 * 48;
}

hipError_t launch_batched_fused(int eq, int st, const LatticeDesc* d, const int* item_map,
                                int64_t items, int64_t T, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  return with_storage(st, [&](auto ST) {
    return batched_fused_launch_st<ST.value>(eq, d, item_map, items, T, s);
  });
}

hipError_t launch_profile(int st, const void* src, double* out, const Geometry& g,
                          const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    profile_kernel<ST.value><<<blocks_for(g.nx), kThreads, 0, s>>>(static_cast<const T*>(src),
                                                                    out, g, c);
    return hipGetLastError();
  });
}

}  // namespace oreg
