// kernels.hip -- D2Q9 OReg kernels for gfx950 and their launchers.
//
// The sweep is one fused pass per time step: pull the nine populations of a
// node from their upwind neighbours (periodic wrap), collide in registers
// (d2q9.hpp), store the node's nine post-collision populations.  Every plane
// element of the source is read by exactly one node, so the pass moves
// 2 * 9 * sizeof(storage) bytes per node and is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace oreg {
namespace {

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
      collide<EQ, COLL, S::shifted>(f[q], k);
    }
  }
  push_local<ST, VX>(dst, g, x0, r0, f);
}

// ------------------------------------------------ multi-step (fused) sweep --
// K time steps per launch.  Each wavefront owns a strip of 64 columns (in
// F32S each workgroup one of 256, see fused_strip) and marches down H output
// rows; lane l holds column X0 - K + l.  The rows of
// time level 0 come from memory; level k + 1 of row y is computed from the
// last three rows of level k (a sliding window kept in registers), the x
// neighbours arrive by one-lane shifts (DPP, or ds_bpermute for window rows
// of the 16-bit formats).  Every level loses one column on
// each side, so the 64 - 2K (256 - 2K) middle columns of level K are stored.  The rows
// needed above and below the strip's H rows (K on each side) are recomputed
// by the neighbouring strips.  Between levels the populations are rounded
// through the storage format, so the result equals K single-step sweeps bit
// for bit.  The 2K pipeline-fill rows are unrolled, so that which levels
// produce is known at compile time, and the steady-state loop (three rows
// per trip) has no branches apart from the store predicate.  H is a runtime
// multiple of 3 chosen per lattice (fused_rows).
constexpr int kFusedRowsDefault = 66;  // output rows per wavefront of fused_sweep_kernel

// Fused launches per storage.  K: steps per launch (six in every format).
// NW: wavefronts per strip.  F32S shares one
// 256-column strip per workgroup (measured 9 % faster than a strip per
// wavefront: 12 % fewer instructions per node update against six workgroup
// barriers per row step); in F64 the same layout measured 2 % slower, and
// the 16-bit formats pre-shift their windows inside the wavefront.
template <int ST> struct FusedLevels { static constexpr int K = 6, NW = 1; };
template <> struct FusedLevels<LB_F32S> { static constexpr int K = 6, NW = 4; };

// lane l <- lane l - 1 (wave_shr:1) and lane l <- lane l + 1 (wave_shl:1).
// Lanes without a source are outside the valid region of the next level: in
// FP32 they read zero (bound_ctrl), which lets the compiler fold the shift
// into the arithmetic instruction that consumes it; in FP64 (two 32-bit
// moves, no folding) they keep their own value.
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double from_left(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_right(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xF, 0xF, false));
}

// The same shifts, with lane 0 (from_left_or) or lane 63 (from_right_or)
// taking `e` instead: the value of the column beyond the wavefront's edge,
// handed over by the neighbouring wavefront of the workgroup.
__device__ __forceinline__ float from_left_or(float v, float e) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(e), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_right_or(float v, float e) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(e), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_left_or(double v, double e) {
  return __hiloint2double(
      __builtin_amdgcn_update_dpp(__double2hiint(e), __double2hiint(v), 0x138, 0xF, 0xF, false),
      __builtin_amdgcn_update_dpp(__double2loint(e), __double2loint(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_right_or(double v, double e) {
  return __hiloint2double(
      __builtin_amdgcn_update_dpp(__double2hiint(e), __double2hiint(v), 0x130, 0xF, 0xF, false),
      __builtin_amdgcn_update_dpp(__double2loint(e), __double2loint(v), 0x130, 0xF, 0xF, false));
}

// The same shifts through the LDS crossbar (ds_bpermute: no LDS memory, no
// VALU issue slot), for values that are needed a step after they are
// shifted: the latency is hidden and the VALU keeps its slots for the
// collision.  src_byte is 4 x the source lane (wrapped, so edge lanes read
// a value from the other edge; they are outside the valid region).
__device__ __forceinline__ float lane_perm(float v, int src_byte) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_byte, __float_as_int(v)));
}

// One strip: K time steps over the rows Y0 .. Y0 + H - 1 of the columns
// X0 .. X0 + 64 NW - 1 - 2 KS.  Lane l of wavefront w holds column
// X0 - KS + 64 w + l; KS >= K is the strip's halo width, so strip columns
// KS .. 64 NW - 1 - KS are stored.  NW = 1: one wavefront per strip.  NW = 4
// (SHARE): the four wavefronts of a workgroup sweep one 256-column strip
// together and hand each other the populations that cross their edges
// through LDS, so only the workgroup's outer edges carry a halo.
template <int K, int KS, int EQ, int COLL, int BC, int ST, bool SHARE = false>
__device__ __forceinline__ void fused_strip(const typename Storage<ST>::T* __restrict__ src,
                                            typename Storage<ST>::T* __restrict__ dst, int nx,
                                            int ny, int64_t P, int X0, int Y0, int H,
                                            const Coeffs<typename Storage<ST>::R>& k, int lane,
                                            int wv = 0) {
  using S = Storage<ST>;
  using R = typename S::R;
  using Tt = typename S::T;
  constexpr int NW = SHARE ? 4 : 1;
  const int J = H + 2 * K;  // rows of level 0 read (H is a multiple of 3)
  const int cs = 64 * wv + lane;  // column within the strip, halo included
  int col = (X0 - KS + cs) % nx;
  if (col < 0) col += nx;
  const bool store_lane = cs >= KS && cs < 64 * NW - KS && X0 - KS + cs < nx;
  const int left_byte = ((lane - 1) & 63) << 2, right_byte = ((lane + 1) & 63) << 2;
  // Window shifts through ds_bpermute for the 16-bit formats (measured 16 %
  // faster for F16S and 7 % for BF16S); F64 and F32S keep all shifts on DPP
  // (no gain there).
  constexpr bool PERM = ST == LB_F16S || ST == LB_BF16S;
  static_assert(!(SHARE && PERM), "pre-shifted windows take their edge values in-wave");
  // A window population as stored (pre-shifted with PERM) and as pulled at
  // the gather (shifted there without PERM).
  auto enter = [&](R v, int src_byte) -> R {
    if constexpr (PERM) return lane_perm(v, src_byte);
    else return v;
  };
  auto pull_left = [&](R v) -> R {
    if constexpr (PERM) return v;
    else return from_left(v);
  };
  auto pull_right = [&](R v) -> R {
    if constexpr (PERM) return v;
    else return from_right(v);
  };
  const bool wall = BC == LB_BC_BOUNCEBACK && (col == 0 || col == nx - 1);
  // Window of level lv: row j of the level lives in slot j % 3 and holds
  // pops 0, 1, 2, 3, 5, 6 (pops 4, 7, 8 of a row are used as soon as it
  // arrives).  With three slots and the row loop unrolled by three, a new row
  // always goes to the slot of a row that is no longer read, so the slot
  // roles are compile-time constants and the window slides without register
  // moves.
  R Sl[K][3][6];
  // Edge exchange (SHARE): edge[lv][q][e][w] holds pops 1, 5, 8, 3, 6, 7 of
  // the row of level lv in ring slot q at the left (e = 0: lane 0) or right
  // (e = 1: lane 63) edge of wavefront w.  Lane 0 of w pulls pops 1, 5, 8 from
  // the right edge of w - 1, lane 63 pops 3, 6, 7 from the left edge of w + 1.
  // A row is published when it arrives at its level; the barrier after each
  // publication orders it before the other wavefronts' reads, and a slot is
  // rewritten three rows later, after the barriers of the steps that read it.
  __shared__ R edge[SHARE ? K : 1][3][2][4][6];
  const bool at_edge = lane == 0 || lane == 63;
  const int side = lane == 63 ? 1 : 0;
  const int wl = (wv + 3) & 3, wr = (wv + 1) & 3;  // neighbours (wrapped ones feed halo lanes)
  auto publish = [&](int lv, int q, const R(&v)[9]) {
    if constexpr (SHARE) {
      if (at_edge) {
        R* e = edge[lv][q][side][wv];
        e[0] = v[1];
        e[1] = v[5];
        e[2] = v[8];
        e[3] = v[3];
        e[4] = v[6];
        e[5] = v[7];
      }
      __syncthreads();
    }
  };
  int row = (Y0 - K) % ny;
  if (row < 0) row += ny;
  Tt nb[3][9];  // level-0 rows: row j is loaded into nb[j % 3] one row ahead
#pragma unroll
  for (int i = 0; i < 9; ++i) nb[0][i] = src[i * P + (int64_t)row * nx + col];
  // Output row y is stored one step after it is computed, before that step's
  // prefetch: the wait for the prefetched row then covers only stores issued
  // a whole step earlier, never the ones just issued.
  Tt pend[9];
  auto store_row = [&](int y) {
    if (store_lane && y >= Y0 && y < ny) {
#pragma unroll
      for (int i = 0; i < 9; ++i)
        __builtin_nontemporal_store(pend[i], dst + i * P + (int64_t)y * nx + col);
    }
  };

  // One row step: row j of level 0 arrives and the first NP levels (those
  // whose three source rows are complete, NP = min(K, j / 2)) produce a row
  // of the next level.  NP is a compile-time constant: the fill steps are
  // unrolled and the steady steps have NP = K.
  auto one_row = [&](int j, auto SLOT, auto NPROD) {
    constexpr int q = decltype(SLOT)::value;  // j % 3
    constexpr int qa = (q + 1) % 3;           // slot of row j - 2
    constexpr int qb = (q + 2) % 3;           // slot of row j - 1
    constexpr int NP = decltype(NPROD)::value;
    R C[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) C[i] = S::load(nb[q][i]);
    // Keep the first use of the row that arrives here at this step: without
    // the ordering point the compiler hoists it into the previous step, right
    // behind the load, and the wavefront waits for memory.
    __asm__ volatile("" : "+v"(C[0]), "+v"(C[1]), "+v"(C[2]), "+v"(C[3]), "+v"(C[4]), "+v"(C[5]),
                     "+v"(C[6]), "+v"(C[7]), "+v"(C[8]));
    if constexpr (NP == K) store_row(Y0 + j - 1 - 2 * K);  // the previous step's output row
    publish(0, q, C);
    // Prefetch the next row of level 0.  The last step reloads its own row
    // (a cache hit) instead of skipping the load: an unconditional load
    // leaves nothing of the old buffer alive.
    if (j + 1 < J) row = wrap_inc(row, ny);
#pragma unroll
    for (int i = 0; i < 9; ++i) nb[qa][i] = src[i * P + (int64_t)row * nx + col];
#pragma unroll
    for (int lv = 0; lv < K; ++lv) {
      // Slot q held row j - 3 of the level, which is no longer read.  With
      // PERM, pops 1, 3, 5 and 6 enter the window already shifted to the
      // lane that pulls them (they are read one and two steps later).
      Sl[lv][q][0] = C[0];
      Sl[lv][q][1] = enter(C[1], left_byte);
      Sl[lv][q][2] = C[2];
      Sl[lv][q][3] = enter(C[3], right_byte);
      Sl[lv][q][4] = enter(C[5], left_byte);
      Sl[lv][q][5] = enter(C[6], right_byte);
      if (lv >= NP) break;  // no rows of level lv + 1 yet
      R N[9];
      const R(&A)[6] = Sl[lv][qa];  // row j - 2 (pops 2, 5, 6 used)
      const R(&B)[6] = Sl[lv][qb];  // row j - 1 (pops 0, 1, 3 used)
      N[0] = B[0];
      N[2] = A[2];
      N[4] = C[4];
      if constexpr (SHARE) {
        N[1] = from_left_or(B[1], edge[lv][qb][1][wl][0]);
        N[5] = from_left_or(A[4], edge[lv][qa][1][wl][1]);
        N[8] = from_left_or(C[8], edge[lv][q][1][wl][2]);
        N[3] = from_right_or(B[3], edge[lv][qb][0][wr][3]);
        N[6] = from_right_or(A[5], edge[lv][qa][0][wr][4]);
        N[7] = from_right_or(C[7], edge[lv][q][0][wr][5]);
      } else {
        N[1] = pull_left(B[1]);
        N[3] = pull_right(B[3]);
        N[5] = pull_left(A[4]);
        N[6] = pull_right(A[5]);
        N[7] = from_right(C[7]);
        N[8] = from_left(C[8]);
      }
      if (wall) {
        R r[9];
        unroll<0, 9>([&](auto I) { r[I.value] = N[opp_of(I.value)]; });
        unroll<0, 9>([&](auto I) { N[I.value] = r[I.value]; });
      } else {
        collide<EQ, COLL, S::shifted>(N, k);
      }
      if (lv + 1 == K) {
#pragma unroll
        for (int i = 0; i < 9; ++i) pend[i] = S::store(N[i]);  // output row Y0 + j - 2K
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) C[i] = S::load(S::store(N[i]));
        // Materialise the level's row here: without this ordering point the
        // compiler interleaves the collisions of the straight-line steady
        // loop and runs out of registers.
        __asm__ volatile("" : "+v"(C[0]), "+v"(C[1]), "+v"(C[2]), "+v"(C[3]), "+v"(C[4]),
                         "+v"(C[5]), "+v"(C[6]), "+v"(C[7]), "+v"(C[8]));
        publish(lv + 1, q, C);
      }
    }
  };
  // Pipeline fill: rows 0 .. 2K - 1, level lv + 1 starting at row 2 (lv + 1).
  unroll<0, 2 * K>([&](auto JJ) { one_row(JJ.value, IC<JJ.value % 3>{}, IC<JJ.value / 2>{}); });
  // Steady state: every level produces a row per step.
  for (int j = 2 * K; j < J; j += 3) {
    one_row(j, IC<(2 * K) % 3>{}, IC<K>{});
    one_row(j + 1, IC<(2 * K + 1) % 3>{}, IC<K>{});
    one_row(j + 2, IC<(2 * K + 2) % 3>{}, IC<K>{});
  }
  store_row(Y0 + J - 1 - 2 * K);
}

template <int K, int EQ, int COLL, int BC, int ST>
__global__ __launch_bounds__(256) void fused_sweep_kernel(
    const typename Storage<ST>::T* __restrict__ src, typename Storage<ST>::T* __restrict__ dst,
    Geometry g, Coef64 c, int strips, int items, int H) {
  constexpr int NW = FusedLevels<ST>::NW;
  constexpr int W = 64 * NW - 2 * K;
  // Neighbouring strips share their halo columns, which then come from the
  // XCD's L2 instead of HBM a second time.  The wavefront index is uniform:
  // keep it (and every row base derived from it) in scalar registers.
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const Coeffs<typename Storage<ST>::R> k(c);
  if constexpr (NW == 4) {
    const int item = xcd_block();  // one work item per workgroup
    if (item >= items) return;     // the whole workgroup leaves together
    const int strip = item % strips, seg = item / strips;
    fused_strip<K, K, EQ, COLL, BC, ST, true>(src, dst, g.nx, g.ny, g.plane, strip * W, seg * H,
                                              H, k, lane, wv);
  } else {
    const int wave = xcd_block() * 4 + wv;
    if (wave >= items) return;  // whole wavefronts leave together
    const int strip = wave % strips, seg = wave / strips;
    fused_strip<K, K, EQ, COLL, BC, ST>(src, dst, g.nx, g.ny, g.plane, strip * W, seg * H, H, k,
                                        lane);
  }
}

// Batched form of fused_sweep_kernel for the server: each wavefront takes one
// work item (lattice, column strip, row block) of a descriptor table and runs
// the same pipeline with that lattice's own step count kl <= KMAX and row
// block height.  Strips are KMAX-wide at every kl, so the item layout of a
// lattice does not change when its last launch has fewer steps.
template <int KMAX, int EQ, int ST>
__global__ __launch_bounds__(256) void batched_fused_kernel(const LatticeDesc* __restrict__ d,
                                                            const int* __restrict__ map,
                                                            int64_t items, int64_t T) {
  using S = Storage<ST>;
  using Tt = typename S::T;
  constexpr int W = 64 - 2 * KMAX;
  const int64_t item = (int64_t)xcd_block() * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= items) return;  // whole wavefronts leave together
  const LatticeDesc& L = d[map[item]];
  const int local = (int)(item - L.tile_begin);
  const int strip = local % L.strips, seg = local / L.strips;
  const int H = L.rows;
  const int64_t t = T - L.admit_T;
  const Tt* __restrict__ src = static_cast<const Tt*>(L.buf[t & 1]);
  Tt* __restrict__ dst = static_cast<Tt*>(L.buf[(t + 1) & 1]);
  const Coeffs<typename S::R> k(L.coef);
  // The step count is uniform over the wavefront: branch to the pipeline
  // compiled for it.
  unroll<1, KMAX + 1>([&](auto KL) {
    if (L.kl == KL.value)
      fused_strip<KL.value, KMAX, EQ, LB_COLL_OREG, LB_BC_PERIODIC, ST>(
          src, dst, L.nx, L.ny, L.plane, strip * W, seg * H, H, k, lane);
  });
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

// Each workgroup updates kBatchTile consecutive nodes (row-major) of one
// lattice, kBatchTile / kThreads nodes per thread, one node at a time with
// per-node periodic wrap; the collision is the one of sweep_kernel.
template <int EQ, int ST>
__global__ __launch_bounds__(kThreads) void batched_sweep_kernel(const LatticeDesc* __restrict__ d,
                                                                 const int* __restrict__ map,
                                                                 int64_t T) {
  using S = Storage<ST>;
  using R = typename S::R;
  using Tt = typename S::T;
  const LatticeDesc& L = d[map[blockIdx.x]];
  const int64_t first = ((int64_t)blockIdx.x - L.tile_begin) * kBatchTile;
  const int64_t t = T - L.admit_T;
  const Tt* __restrict__ src = static_cast<const Tt*>(L.buf[t & 1]);
  Tt* __restrict__ dst = static_cast<Tt*>(L.buf[(t + 1) & 1]);
  const Geometry g{L.nx, L.ny, L.plane};
  const Coeffs<R> k(L.coef);
#pragma unroll 1
  for (int j = 0; j < kBatchTile / kThreads; ++j) {
    const int64_t c = first + j * kThreads + threadIdx.x;
    if (c >= g.plane) break;
    const int y = (int)(c / g.nx);
    const int x = (int)(c - (int64_t)y * g.nx);
    const int ym = wrap_dec(y, g.ny), yp = wrap_inc(y, g.ny);
    const int64_t r0 = (int64_t)y * g.nx, rm = (int64_t)ym * g.nx, rp = (int64_t)yp * g.nx;
    R f[1][9];
    pull<ST, 1>(src, g, x, r0, rm, rp, f);
    collide<EQ, LB_COLL_OREG, S::shifted>(f[0], k);
    push_local<ST, 1>(dst, g, x, r0, f);
  }
}

unsigned int blocks_for(int64_t n) { return (unsigned int)((n + kThreads - 1) / kThreads); }

}  // namespace

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

int fused_levels(int st) {
  switch (st) {
    case LB_F64: return FusedLevels<LB_F64>::K;
    case LB_F32S: return FusedLevels<LB_F32S>::K;
    case LB_F16S: return FusedLevels<LB_F16S>::K;
    case LB_BF16S: return FusedLevels<LB_BF16S>::K;
    default: return 1;
  }
}

hipError_t launch_fused_sweep(int eq, int coll, int bc, int st, const void* src, void* dst,
                              const Geometry& g, const Coef64& c, int rows, hipStream_t s) {
  if (rows < 3 || rows % 3 != 0) return hipErrorInvalidValue;
  return with_storage(st, [&](auto ST) -> hipError_t {
    using T = typename Storage<ST.value>::T;
    constexpr int K = FusedLevels<ST.value>::K;
    if constexpr (K < 2) {
      return hipErrorInvalidValue;  // single-step storage: use launch_sweep
    } else {
    constexpr int NW = FusedLevels<ST.value>::NW;
    constexpr int W = 64 * NW - 2 * K;
    const int strips = (g.nx + W - 1) / W;
    const int segs = (g.ny + rows - 1) / rows;
    const int items = strips * segs;
    const unsigned int nblocks = (unsigned int)((items + 4 / NW - 1) / (4 / NW));
    return with_eq(eq, [&](auto EQ) {
      return with_coll(coll, [&](auto CO) {
        return with_bc(bc, [&](auto BC) {
          fused_sweep_kernel<K, EQ.value, CO.value, BC.value, ST.value><<<nblocks, 256, 0, s>>>(
              static_cast<const T*>(src), static_cast<T*>(dst), g, c, strips, items, rows);
          return hipGetLastError();
        });
      });
    });
    }
  });
}

FusedShape fused_shape(int st) {
  FusedShape sh{0, 0};
  int dev = 0, cus = 0, blocks = 0;
  if (hipGetDevice(&dev) != hipSuccess) return sh;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return sh;
  const hipError_t e = with_storage(st, [&](auto ST) -> hipError_t {
    constexpr int K = FusedLevels<ST.value>::K;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks,
        reinterpret_cast<const void*>(
            &fused_sweep_kernel<K, LB_EQ_GUIDED, LB_COLL_OREG, LB_BC_PERIODIC, ST.value>),
        256, 0);
  });
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

double fused_cost(int st, int nx, int ny, int H, const FusedShape& sh) {
  const int K = fused_levels(st), NW = fused_wavefronts(st), W = 64 * NW - 2 * K;
  const int64_t strips = (nx + W - 1) / W;
  // a work item takes NW wavefronts, one on each of NW SIMDs
  const int64_t items = strips * ((ny + H - 1) / H) * NW;
  const int64_t w = (items + sh.simds - 1) / sh.simds;
  const int64_t resident = w < sh.waves_per_simd ? w : sh.waves_per_simd;
  const double work = K * (double)(H + 2 * K) - K * (K + 1) + 2 * K;
  return (double)w / (1.0 + 0.08 * (double)(resident - 1)) * work;
}

int fused_rows(int st, int nx, int ny, const FusedShape& sh) {
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
    const double c = fused_cost(st, nx, ny, H, sh);
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

hipError_t launch_batched_sweep(int eq, int st, const LatticeDesc* d, const int* tile_map,
                                int64_t tiles, int64_t T, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  return with_storage(st, [&](auto ST) {
    return with_eq(eq, [&](auto EQ) {
      batched_sweep_kernel<EQ.value, ST.value><<<(unsigned int)tiles, kThreads, 0, s>>>(
          d, tile_map, T);
      return hipGetLastError();
    });
  });
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
  return with_storage(st, [&](auto ST) -> hipError_t {
    constexpr int K = FusedLevels<ST.value>::K;
    if constexpr (K < 2) {
      return hipErrorInvalidValue;
    } else {
      return with_eq(eq, [&](auto EQ) {
        batched_fused_kernel<K, EQ.value, ST.value>
            <<<(unsigned int)((items + 3) / 4), 256, 0, s>>>(d, item_map, items, T);
        return hipGetLastError();
      });
    }
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
