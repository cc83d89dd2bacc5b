// kernels3.hip -- D3Q27 kernels for gfx950 and their launchers.
//
// The sweep is one pass per time step: every node pulls its 27 populations
// from the upwind neighbours (periodic wrap), collides in registers
// (d3q27.hpp) and stores 27 post-collision populations.  Every element of
// the source is read by exactly one node, so the pass moves
// 2 * 27 * sizeof(storage) bytes per node and is bound by HBM bandwidth.
//
// Work split: one wavefront per 64-node segment of an x-row, four per
// workgroup.  A segment's (y, z) is uniform across the wavefront, so the 27
// source rows are scalar base addresses and each lane adds only its own
// column (x, x - 1 or x + 1 with the periodic wrap).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels3.hpp"

namespace oreg {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <int V>
using IC = std::integral_constant<int, V>;

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

// (v - c) mod n for c in {-1, 0, 1} and 0 <= v < n.
__host__ __device__ __forceinline__ int wrap_sub(int v, int c, int n) {
  if (c == 0) return v;
  if (c > 0) return v == 0 ? n - 1 : v - 1;
  return v == n - 1 ? 0 : v + 1;
}

// ---------------------------------------------------------------- sweep --
// Wavefronts per workgroup of the sweep, per storage (measured on 256^3:
// 8 for F64 and 16 for F32S beat 4 by 2 %; 4 is best for the 16-bit formats).
template <int ST> struct Sweep3Waves { static constexpr int N = 4; };
template <> struct Sweep3Waves<LB_F64> { static constexpr int N = 8; };
template <> struct Sweep3Waves<LB_F32S> { static constexpr int N = 16; };

template <int EQ, int COLL, int ST>
__global__ __launch_bounds__(64 * Sweep3Waves<ST>::N) void sweep3_kernel(
    const typename Storage<ST>::T* __restrict__ src, typename Storage<ST>::T* __restrict__ dst,
    Geometry3 g, Coef64 c, unsigned int nseg, unsigned int tasks) {
  using S = Storage<ST>;
  using R = typename S::R;
  using T = typename S::T;
  const unsigned int task = blockIdx.x * Sweep3Waves<ST>::N +
                            (unsigned int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (task >= tasks) return;
  const unsigned int row = task / nseg;
  const unsigned int seg = task - row * nseg;
  const int y = (int)(row % (unsigned int)g.ny);
  const int z = (int)(row / (unsigned int)g.ny);
  const int x = (int)(seg * 64u) + (int)(threadIdx.x & 63);
  const bool active = x < g.nx;
  const int xc = active ? x : g.nx - 1;  // lanes past the row end load a valid node
  const int xm = xc == 0 ? g.nx - 1 : xc - 1;
  const int xp = xc == g.nx - 1 ? 0 : xc + 1;
  const int64_t P = g.cells;
  // Start of the source row of g_i(x - c_i) for each (c_y, c_z).
  int64_t rows[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      rows[a][b] = ((int64_t)wrap_sub(z, b - 1, g.nz) * g.ny + wrap_sub(y, a - 1, g.ny)) * g.nx;
  R f[27];
  unroll<0, 27>([&](auto I) {
    constexpr int vx = d3::cx(I.value), vy = d3::cy(I.value), vz = d3::cz(I.value);
    const T* p = src + I.value * P + rows[vy + 1][vz + 1];
    f[I.value] = S::load(p[vx == 0 ? xc : (vx > 0 ? xm : xp)]);
  });
  const Coeffs<R> k(c);
  d3::collide<EQ, COLL, S::shifted>(f, k);
  if (active) {
    T* q = dst + rows[1][1] + x;
    unroll<0, 27>([&](auto I) { __builtin_nontemporal_store(S::store(f[I.value]), q + I.value * P); });
  }
}

// ---------------------------------------------------------- per node --
struct Node {
  int x, y, z;
};
__device__ __forceinline__ Node node_of(int64_t idx, const Geometry3& g) {
  const int64_t r = idx / g.nx;
  Node n;
  n.x = (int)(idx - r * g.nx);
  n.y = (int)(r % g.ny);
  n.z = (int)(r / g.ny);
  return n;
}
__device__ __forceinline__ int64_t cell_of(int x, int y, int z, const Geometry3& g) {
  return ((int64_t)z * g.ny + y) * g.nx + x;
}
// Cell that holds g_i(x - c_i) for node n.
__device__ __forceinline__ int64_t upwind(const Node& n, int i, const Geometry3& g) {
  return cell_of(wrap_sub(n.x, d3::cx(i), g.nx), wrap_sub(n.y, d3::cy(i), g.ny),
                 wrap_sub(n.z, d3::cz(i), g.nz), g);
}

template <int EQ, int ST>
__global__ __launch_bounds__(kThreads) void init3_kernel(const double* __restrict__ rho,
                                                         const double* __restrict__ ux,
                                                         const double* __restrict__ uy,
                                                         const double* __restrict__ uz,
                                                         typename Storage<ST>::T* __restrict__ dst,
                                                         Geometry3 g, Coef64 c,
                                                         unsigned int* __restrict__ bad) {
  using S = Storage<ST>;
  using R = typename S::R;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.cells) return;
  double r = rho[idx];
  double u[3] = {ux[idx], uy[idx], uz[idx]};
  if (!(isfinite(r) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && r > 0.0)) {
    atomicAdd(bad, 1u);
    r = 1.0;
    u[0] = u[1] = u[2] = 0.0;
  }
  const double u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
  const Coeffs<double> k(c);
  double feq[27], deq[27];
  d3::equilibrium<EQ, S::shifted>(S::shifted ? r - c.rho0 : r, r, u, u2, k, feq, deq);
  // f_i(x, 0) = f^eq_i(x) is stored as g_i(x - c_i).
  const Node n = node_of(idx, g);
  unroll<0, 27>([&](auto I) { dst[I.value * g.cells + upwind(n, I.value, g)] = S::store((R)deq[I.value]); });
}

template <int ST>
__global__ __launch_bounds__(kThreads) void import3_kernel(int i, const double* __restrict__ fin,
                                                           typename Storage<ST>::T* __restrict__ dst,
                                                           Geometry3 g, Coef64 c) {
  using S = Storage<ST>;
  using R = typename S::R;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.cells) return;
  const double w = S::shifted ? d3::shift64(d3::cx(i), d3::cy(i), d3::cz(i), c) : 0.0;
  dst[i * g.cells + upwind(node_of(idx, g), i, g)] = S::store((R)(fin[idx] - w));
}

template <int ST>
__global__ __launch_bounds__(kThreads) void export3_kernel(int i,
                                                           const typename Storage<ST>::T* __restrict__ src,
                                                           double* __restrict__ fout, Geometry3 g,
                                                           Coef64 c) {
  using S = Storage<ST>;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.cells) return;
  const double w = S::shifted ? d3::shift64(d3::cx(i), d3::cy(i), d3::cz(i), c) : 0.0;
  fout[idx] = (double)S::load(src[i * g.cells + upwind(node_of(idx, g), i, g)]) + w;
}

// Pre-collision populations of a node in FP64, still shifted by w_i rho0.
template <int ST>
__device__ __forceinline__ void gather3(const typename Storage<ST>::T* __restrict__ src,
                                        const Geometry3& g, const Node& n, double (&d)[27]) {
  using S = Storage<ST>;
  unroll<0, 27>([&](auto I) { d[I.value] = (double)S::load(src[I.value * g.cells + upwind(n, I.value, g)]); });
}

template <int ST>
__global__ __launch_bounds__(kThreads) void moments3_kernel(const typename Storage<ST>::T* __restrict__ src,
                                                            double* __restrict__ out, Geometry3 g,
                                                            Coef64 c) {
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.cells) return;
  double d[27], drho, j[3], M[6];
  gather3<ST>(src, g, node_of(idx, g), d);
  d3::moments(d, drho, j, M);
  const double rho = c.rho0 + drho;
  out[idx] = rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[(a + 1) * g.cells + idx] = j[a] / rho;
}

// ---------------------------------------------------------- diagnostics --
constexpr int kSums = 7;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Fixed-order block sum; result valid in thread 0.
__device__ __forceinline__ void block_sum(double (&v)[kSums]) {
  __shared__ double part[kWaves][kSums];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kSums; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) part[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) {
      double s = part[0][k];
      for (int w = 1; w < kWaves; ++w) s += part[w][k];
      v[k] = s;
    }
  }
}

template <int ST>
__global__ __launch_bounds__(kThreads) void diag3_kernel(const typename Storage<ST>::T* __restrict__ src,
                                                         double* __restrict__ partials, Geometry3 g,
                                                         Coef64 c, double theta) {
  double acc[kSums] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < g.cells; idx += stride) {
    double d[27], drho, j[3], M[6];
    gather3<ST>(src, g, node_of(idx, g), d);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 27; ++i) finite = finite && isfinite(d[i]);
    if (!finite) {
      acc[6] += 1.0;
      continue;
    }
    d3::moments(d, drho, j, M);
    const double rho = c.rho0 + drho;
    const double ke = 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
    acc[0] += rho;
    acc[1] += j[0];
    acc[2] += j[1];
    acc[3] += j[2];
    acc[4] += ke;
    acc[5] += 1.5 * rho * theta + ke;
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) partials[blockIdx.x * kSums + k] = acc[k];
  }
}

__global__ __launch_bounds__(kThreads) void diag3_final_kernel(const double* __restrict__ partials,
                                                               int nblocks, double* __restrict__ out) {
  double acc[kSums] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kThreads) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) acc[k] += partials[b * kSums + k];
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kSums; ++k) out[k] = acc[k];
  }
}

unsigned int blocks_for(int64_t n) { return (unsigned int)((n + kThreads - 1) / kThreads); }

}  // namespace

// ------------------------------------------------------------ launchers --
int64_t sweep3_tasks(const Geometry3& g) {
  return (int64_t)((g.nx + 63) / 64) * g.ny * g.nz;
}

hipError_t launch_sweep3(int eq, int coll, int st, const void* src, void* dst, const Geometry3& g,
                         const Coef64& c, hipStream_t s) {
  const unsigned int nseg = (unsigned int)((g.nx + 63) / 64);
  const unsigned int tasks = (unsigned int)sweep3_tasks(g);
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    constexpr int W = Sweep3Waves<ST.value>::N;
    const unsigned int nblocks = (tasks + W - 1) / W;
    return with_eq(eq, [&](auto EQ) {
      return with_coll(coll, [&](auto CO) {
        sweep3_kernel<EQ.value, CO.value, ST.value><<<nblocks, 64 * W, 0, s>>>(
            static_cast<const T*>(src), static_cast<T*>(dst), g, c, nseg, tasks);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_init3(int eq, int st, const double* rho, const double* ux, const double* uy,
                        const double* uz, void* dst, const Geometry3& g, const Coef64& c,
                        unsigned int* bad, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    return with_eq(eq, [&](auto EQ) {
      init3_kernel<EQ.value, ST.value><<<blocks_for(g.cells), kThreads, 0, s>>>(
          rho, ux, uy, uz, static_cast<T*>(dst), g, c, bad);
      return hipGetLastError();
    });
  });
}

hipError_t launch_import3(int st, int i, const double* fin, void* dst, const Geometry3& g,
                          const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    import3_kernel<ST.value><<<blocks_for(g.cells), kThreads, 0, s>>>(i, fin, static_cast<T*>(dst), g, c);
    return hipGetLastError();
  });
}

hipError_t launch_export3(int st, int i, const void* src, double* fout, const Geometry3& g,
                          const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    export3_kernel<ST.value><<<blocks_for(g.cells), kThreads, 0, s>>>(i, static_cast<const T*>(src),
                                                                       fout, g, c);
    return hipGetLastError();
  });
}

hipError_t launch_moments3(int st, const void* src, double* out, const Geometry3& g,
                           const Coef64& c, hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    moments3_kernel<ST.value><<<blocks_for(g.cells), kThreads, 0, s>>>(static_cast<const T*>(src),
                                                                        out, g, c);
    return hipGetLastError();
  });
}

hipError_t launch_diagnostics3(int st, const void* src, double* partials, double* out,
                               const Geometry3& g, const Coef64& c, double theta_energy,
                               hipStream_t s) {
  return with_storage(st, [&](auto ST) {
    using T = typename Storage<ST.value>::T;
    diag3_kernel<ST.value><<<kDiag3Blocks, kThreads, 0, s>>>(static_cast<const T*>(src), partials, g,
                                                             c, theta_energy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag3_final_kernel<<<1, kThreads, 0, s>>>(partials, kDiag3Blocks, out);
    return hipGetLastError();
  });
}

}  // namespace oreg
