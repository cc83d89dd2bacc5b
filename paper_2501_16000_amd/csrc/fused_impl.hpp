// fused_impl.hpp -- the fused multi-step D2Q9 sweep (K time steps per
// launch, register-resident row pipeline) and its batched serving form, with
// their host launchers as templates over the storage format.  Included only
// by fused_f64.hip, fused_f32s.hip, fused_f16s.hip and fused_bf16s.hip, which
// instantiate them for one format each.
#pragma once

#include "dispatch.hpp"

namespace oreg {
namespace {
using namespace detail;

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

// Access to element (plane i, row r, column col) of the source and
// destination population buffers.  Global form: a 64-bit address per plane
// and row.  Buffer form (BUF): one resource descriptor per buffer, the plane
// offset i * P in a scalar register and the 32-bit in-plane byte offset per
// lane, so no 64-bit address arithmetic per access (3-5 fewer VALU
// instructions per collision; measured 1-2 % faster on 4096^2 in every
// format).  The buffer form needs the buffer below 2 GiB (its byte offsets
// and the descriptor's record count are 32-bit); the hardware range check
// returns zero for, and drops, any access beyond it.
template <typename Tt, bool BUF>
struct PlaneIO {
  const Tt* __restrict__ src;
  Tt* __restrict__ dst;
  int64_t P;
  int nx;
  __device__ PlaneIO(const Tt* s, Tt* d, int64_t p, int n) : src(s), dst(d), P(p), nx(n) {}
  __device__ Tt load(int i, int r, int col) const { return src[i * P + (int64_t)r * nx + col]; }
  __device__ void store(int i, int r, int col, Tt v) const {
    dst[i * P + (int64_t)r * nx + col] = v;
  }
};
template <typename Tt>
struct PlaneIO<Tt, true> {
  static constexpr int kDword3 = 0x00020000;  // raw buffer access, gfx9 family
  __amdgpu_buffer_rsrc_t rs, rd;
  uint32_t plane_bytes;
  int nx;
  __device__ PlaneIO(const Tt* s, Tt* d, int64_t p, int n)
      : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<Tt*>(s), 0,
                                             (int)(9 * p * (int64_t)sizeof(Tt)), kDword3)),
        rd(__builtin_amdgcn_make_buffer_rsrc(d, 0, (int)(9 * p * (int64_t)sizeof(Tt)), kDword3)),
        plane_bytes((uint32_t)(p * (int64_t)sizeof(Tt))),
        nx(n) {}
  __device__ uint32_t off(int r, int col) const {
    return ((uint32_t)r * (uint32_t)nx + (uint32_t)col) * (uint32_t)sizeof(Tt);
  }
  __device__ Tt load(int i, int r, int col) const {
    const uint32_t o = off(r, col), so = (uint32_t)i * plane_bytes;
    if constexpr (sizeof(Tt) == 8)
      return __builtin_bit_cast(Tt, __builtin_amdgcn_raw_buffer_load_b64(rs, o, so, 0));
    else if constexpr (sizeof(Tt) == 4)
      return __builtin_bit_cast(Tt, __builtin_amdgcn_raw_buffer_load_b32(rs, o, so, 0));
    else
      return __builtin_bit_cast(Tt, __builtin_amdgcn_raw_buffer_load_b16(rs, o, so, 0));
  }
  __device__ void store(int i, int r, int col, Tt v) const {
    const uint32_t o = off(r, col), so = (uint32_t)i * plane_bytes;
    if constexpr (sizeof(Tt) == 8)
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(unsigned int __attribute__((ext_vector_type(2))), v), rd, o, so, 0);
    else if constexpr (sizeof(Tt) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rd, o, so, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), rd, o, so, 0);
  }
};

// Largest population buffer (both A/B halves use the same size) that the
// buffer form of PlaneIO addresses.
constexpr int64_t kBufferFormBytes = 0x7fffffff;

// One strip: K time steps over the rows Y0 .. Y0 + H - 1 of the columns
// X0 .. X0 + 64 NW - 1 - 2 KS.  Lane l of wavefront w holds column
// X0 - KS + 64 w + l; KS >= K is the strip's halo width, so strip columns
// KS .. 64 NW - 1 - KS are stored.  NW = 1: one wavefront per strip.  NW = 4
// (SHARE): the four wavefronts of a workgroup sweep one 256-column strip
// together and hand each other the populations that cross their edges
// through LDS, so only the workgroup's outer edges carry a halo.
template <int K, int KS, int EQ, int COLL, int BC, int ST, bool SHARE = false, bool BUF = false>
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
  const PlaneIO<Tt, BUF> io(src, dst, P, nx);
  int row = (Y0 - K) % ny;
  if (row < 0) row += ny;
  Tt nb[3][9];  // level-0 rows: row j is loaded into nb[j % 3] one row ahead
#pragma unroll
  for (int i = 0; i < 9; ++i) nb[0][i] = io.load(i, row, col);
  // Output row y is stored one step after it is computed, before that step's
  // prefetch: the wait for the prefetched row then covers only stores issued
  // a whole step earlier, never the ones just issued.  Plain stores, not
  // nontemporal ones: a strip's row piece shares its end cache lines with
  // the neighbouring strips (same XCD, same time), which the L2 then merges;
  // measured on 4096^2, nontemporal stores made the fused sweep 6 % (F64),
  // 4 % (F16S) and 2 % (BF16S) slower and the served FP64 stream 7 % slower
  // (F32S unchanged).  The single-step sweep keeps nontemporal stores (3-6 %
  // faster there).
  Tt pend[9];
  auto store_row = [&](int y) {
    if (store_lane && y >= Y0 && y < ny) {
#pragma unroll
      for (int i = 0; i < 9; ++i) io.store(i, y, col, pend[i]);
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
    for (int i = 0; i < 9; ++i) nb[qa][i] = io.load(i, row, col);
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
        collide<EQ, COLL, S::shifted, S::delta_u>(N, k);
      }
      if (lv + 1 == K) {
#pragma unroll
        for (int i = 0; i < 9; ++i) pend[i] = S::store(N[i]);  // output row Y0 + j - 2K
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) C[i] = N[i];
        S::round2(C[0], C[1]);
        S::round2(C[2], C[3]);
        S::round2(C[4], C[5]);
        S::round2(C[6], C[7]);
        C[8] = S::load(S::store(C[8]));
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

template <int K, int EQ, int COLL, int BC, int ST, bool BUF = false>
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
    fused_strip<K, K, EQ, COLL, BC, ST, true, BUF>(src, dst, g.nx, g.ny, g.plane, strip * W,
                                                   seg * H, H, k, lane, wv);
  } else {
    const int wave = xcd_block() * 4 + wv;
    if (wave >= items) return;  // whole wavefronts leave together
    const int strip = wave % strips, seg = wave / strips;
    fused_strip<K, K, EQ, COLL, BC, ST, false, BUF>(src, dst, g.nx, g.ny, g.plane, strip * W,
                                                    seg * H, H, k, lane);
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
  // The wavefront index is uniform: with readfirstlane the descriptor loads
  // become scalar loads and the lattice's parameters stay in scalar
  // registers (without it they took 26-30 VGPRs, one wavefront per SIMD
  // fewer in F32S, F16S and BF16S).
  const int64_t item =
      (int64_t)xcd_block() * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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

}  // namespace

template <int ST>
hipError_t fused_launch_st(int eq, int coll, int bc, const void* src, void* dst, const Geometry& g,
                           const Coef64& c, int rows, int levels, hipStream_t s) {
  using T = typename Storage<ST>::T;
  constexpr int K = FusedLevels<ST>::K;
  constexpr int NW = FusedLevels<ST>::NW;
  return with_eq(eq, [&](auto EQ) {
    return with_coll(coll, [&](auto CO) {
      return with_bc(bc, [&](auto BC) -> hipError_t {
        // The buffer form of the plane access (PlaneIO) for the guided
        // periodic OReg sweep, the configuration of the benchmark, when the
        // population buffer is below 2 GiB.
        constexpr bool buf_config = EQ.value == LB_EQ_GUIDED && short_fused(CO.value, BC.value);
        const bool buf = buf_config && 9 * g.plane * (int64_t)sizeof(T) <= kBufferFormBytes;
        auto go = [&](auto L) -> hipError_t {
          constexpr int W = 64 * NW - 2 * L.value;
          const int strips = (g.nx + W - 1) / W;
          const int segs = (g.ny + rows - 1) / rows;
          const int items = strips * segs;
          const unsigned int nblocks = (unsigned int)((items + 4 / NW - 1) / (4 / NW));
          if constexpr (buf_config) {
            if (buf) {
              fused_sweep_kernel<L.value, EQ.value, CO.value, BC.value, ST, true>
                  <<<nblocks, 256, 0, s>>>(static_cast<const T*>(src), static_cast<T*>(dst), g, c,
                                           strips, items, rows);
              return hipGetLastError();
            }
          }
          fused_sweep_kernel<L.value, EQ.value, CO.value, BC.value, ST><<<nblocks, 256, 0, s>>>(
              static_cast<const T*>(src), static_cast<T*>(dst), g, c, strips, items, rows);
          return hipGetLastError();
        };
        if (levels == K) return go(IC<K>{});
        hipError_t e = hipErrorInvalidValue;
        if constexpr (short_fused(CO.value, BC.value)) {
          unroll<2, K>([&](auto L) {
            if (levels == L.value) e = go(L);
          });
        }
        return e;
      });
    });
  });
}

template <int ST>
hipError_t fused_occupancy_st(int levels, int* blocks) {
  auto occ = [&](auto L) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks,
        reinterpret_cast<const void*>(
            &fused_sweep_kernel<L.value, LB_EQ_GUIDED, LB_COLL_OREG, LB_BC_PERIODIC, ST>),
        256, 0);
  };
  hipError_t e = hipErrorInvalidValue;
  unroll<2, FusedLevels<ST>::K + 1>([&](auto L) {
    if (levels == L.value) e = occ(L);
  });
  return e;
}

template <int ST>
hipError_t batched_fused_launch_st(int eq, const LatticeDesc* d, const int* item_map, int64_t items,
                                   int64_t T, hipStream_t s) {
  constexpr int K = FusedLevels<ST>::K;
  return with_eq(eq, [&](auto EQ) {
    batched_fused_kernel<K, EQ.value, ST><<<(unsigned int)((items + 3) / 4), 256, 0, s>>>(
        d, item_map, items, T);
    return hipGetLastError();
  });
}

}  // namespace oreg
