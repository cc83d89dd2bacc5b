// d2q9.hpp -- device-side D2Q9 lattice, storage codecs and the OReg collision.
//
// One node's collision in registers, written for gfx950 VALU arithmetic:
//   moments rho, j (Eq. 2a); equilibrium factors of Eq. (11) or the
//   polynomial equilibrium of Sec. III.D; the trace-free non-equilibrium
//   stress S of Eq. (6) from second moments; f^OReg and the update of Eq. (7)
//   (or Eq. (1) for lattice BGK).
//
// Algebraic forms used here instead of the printed ones (identical in exact
// arithmetic):
//   * the guided equilibrium factorizes into per-axis factors
//     Psi(0, u) = 1 - theta - u^2 and Psi(+-1, u) = (theta +- u + u^2)/2,
//     f^eq_i = rho Psi(c_ix, u_x) Psi(c_iy, u_y);
//   * both equilibria reproduce Pi^eq = rho theta delta + rho u u exactly, so
//     the trace-free stress of f^neq is taken from second moments of f:
//       S_xx = -S_yy = s = ((f1 + f3) - (f2 + f4) - rho (ux^2 - uy^2)) / 2,
//       S_xy = (f5 + f7) - (f6 + f8) - rho ux uy;
//   * with a trace-free S, (C C - C^2/2 I):S = s (Cx^2 - Cy^2) + 2 S_xy Cx Cy,
//     C = c_i - u, and f^post_i = f^eq_i + f^eq_i kappa b_i with
//     kappa = (1 - 1/tau) / (2 rho theta^2); kappa b_i is assembled from
//     per-axis factors (3 x-values, 3 y-values);
//   * shifted storage carries df_i = f_i - w_i rho0; the axis and diagonal
//     weights are equal in pairs, so s and S_xy need no shift, and
//     f^eq_i - w_i rho0 is formed from small differences to keep FP32
//     cancellation out of the update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "oreg.h"

namespace oreg {

// Velocity components in the order of the public header, and the index of
// the opposite velocity (c_opp = -c_i).
__host__ __device__ constexpr int cx_of(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
}
__host__ __device__ constexpr int cy_of(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp_of(int i) {
  return (i == 0) ? 0 : (i <= 4) ? ((i + 1) % 4 + 1) : ((i - 5 + 2) % 4 + 5);
}
static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(3) == 1 && opp_of(4) == 2, "axis");
static_assert(opp_of(5) == 7 && opp_of(6) == 8 && opp_of(7) == 5 && opp_of(8) == 6, "diag");

// Compile-time loop over the nine populations.
template <int I, int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll<I + 1, N>(f);
  }
}

// ---------------------------------------------------------------- storage --
template <int S> struct Storage;
template <> struct Storage<LB_F64> {
  using T = double;
  using R = double;
  static constexpr bool shifted = false;
  static constexpr bool delta_u = false;  // u from drho / rho (see moments_delta)
  __host__ __device__ static R load(T v) { return v; }
  __host__ __device__ static T store(R v) { return v; }
  // a, b <- load(store(a)), load(store(b)): the round trip through the
  // storage format (see the 16-bit formats).
  __host__ __device__ static void round2(R&, R&) {}
};
template <> struct Storage<LB_F32S> {
  using T = float;
  using R = float;
  static constexpr bool shifted = true;
  static constexpr bool delta_u = true;
  __host__ __device__ static R load(T v) { return v; }
  __host__ __device__ static T store(R v) { return v; }
  __host__ __device__ static void round2(R&, R&) {}
};
template <> struct Storage<LB_F16S> {
  using T = _Float16;
  using R = float;
  static constexpr bool shifted = true;
  static constexpr bool delta_u = false;
  __host__ __device__ static R load(T v) { return (float)v; }
  // Round the FP32 value to nearest even.  The empty asm pins v in a VGPR
  // first: without it the compiler may merge the FP32 FMA that produced v
  // with the conversion into v_fma_mixlo_f16, which rounds the exact FMA
  // result once to FP16 and so differs from FP32-then-FP16 rounding in about
  // 6 of 100000 values (measured), and only in the kernels where it chose to
  // merge.
  __host__ __device__ static T store(R v) {
#if defined(__HIP_DEVICE_COMPILE__)
    __asm__ volatile("" : "+v"(v));
#endif
    return (_Float16)v;
  }
  // Two round trips, one value at a time: the packed form (v_cvt_pk_f16_f32
  // and two v_cvt_f32_f16, one instruction fewer per pair) made the fused
  // F16S sweep 4 % slower (measured on 4096^2), where BF16S gains from it.
  __host__ __device__ static void round2(R& a, R& b) {
    a = load(store(a));
    b = load(store(b));
  }
};
template <> struct Storage<LB_BF16S> {
  using T = __bf16;
  using R = float;
  static constexpr bool shifted = true;
  static constexpr bool delta_u = false;
  __host__ __device__ static R load(T v) { return (float)v; }
  __host__ __device__ static T store(R v) { return (__bf16)v; }  // v_cvt_pk_bf16_f32, RNE
  // Two round trips in one packed conversion (v_cvt_pk_bf16_f32, then a
  // shift and a mask): three instructions instead of four, the same values;
  // the fused BF16S sweep ran 6 % faster with it (4096^2).
  __host__ __device__ static void round2(R& a, R& b) {
    typedef float F2 __attribute__((ext_vector_type(2)));
    typedef __bf16 B2 __attribute__((ext_vector_type(2)));
    const F2 w = __builtin_convertvector(__builtin_convertvector(F2{a, b}, B2), F2);
    a = w[0];
    b = w[1];
  }
};

// Per-lattice constants of the collision, precomputed on the host in FP64.
struct Coef64 {
  double theta;   // theta (exactly 1/3 for the polynomial equilibrium)
  double a0, a1;  // rest per-axis factors 1 - theta and theta/2 (w_i = a_cx a_cy)
  double kappa0;  // (1 - 1/tau) / (2 theta^2)
  double omega;   // 1 / tau (lattice BGK)
  double rho0;    // reference density of shifted storage (0 when unshifted)
};

// The same constants in the register type R.
template <typename R>
struct Coeffs {
  R theta, a0, a1, kappa0, omega, rho0;
  R r0a0, r0a1;        // rho0 a0, rho0 a1
  R kappa_h, kappa_2;  // kappa0 / 2 and 2 kappa0 (exact scalings of kappa0 in R)
  R inv0;              // 1 / rho0 (0 when rho0 = 0: unshifted storage never uses it)
  // a1 = (1 - a0) / 2 is formed in R from the rounded a0, exactly (1 - a0
  // and the halving do not round for 0 < a0 < 1), so that a0 + 2 a1 = 1
  // holds exactly in R: the per-axis rest factors then sum to one and the
  // equilibrium carries the momentum rho u with no spurious factor.
  // Rounding 1 - theta and theta / 2 separately instead gives, at theta =
  // 1/3 in FP32, a0 + 2 a1 = 1 + 3e-8, which scales the momentum by that
  // factor at every collision and made the decay of a shear wave in
  // shifted FP32 storage 2e-4 too slow over 1500 steps (CPU run of this
  // collision); with the exact partition it is unbiased.
  __host__ __device__ explicit Coeffs(const Coef64& c)
      : theta((R)c.theta), a0((R)c.a0), a1((R(1) - (R)c.a0) * R(0.5)), kappa0((R)c.kappa0),
        omega((R)c.omega), rho0((R)c.rho0), r0a0((R)c.rho0 * a0), r0a1((R)c.rho0 * a1),
        kappa_h(R(0.5) * (R)c.kappa0), kappa_2(R(2) * (R)c.kappa0),
        inv0(c.rho0 != 0.0 ? (R)(1.0 / c.rho0) : R(0)) {}
};

// Per-axis factor selected by the velocity component c (-1, 0, +1).
template <int c, typename R>
__host__ __device__ __forceinline__ R pick(R m, R z, R p) {
  if constexpr (c == 0) return z;
  else if constexpr (c == 1) return p;
  else return m;
}

// Peculiar velocity component C = c - u, formed without multiplying by c.
template <int c, typename R>
__host__ __device__ __forceinline__ R peculiar(R u) {
  if constexpr (c == 0) return -u;
  else if constexpr (c == 1) return R(1) - u;
  else return R(-1) - u;
}

// a * b + c with one rounding.  The collision spells out every fused
// multiply-add and is compiled with contraction off, so every kernel that
// inlines it (plain sweep, multi-step sweep, batched serving sweep) rounds
// identically and their results agree bit for bit.
__host__ __device__ __forceinline__ double fmadd(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__host__ __device__ __forceinline__ float fmadd(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// 1 / x from the hardware reciprocal refined by Newton-Raphson steps
// r <- r + r (1 - x r): two in FP64, one in FP32 (each step doubles the
// correct bits).  v_rcp_f64 alone is good to about 2^-24 relative on gfx950;
// after two steps the result matched the IEEE quotient exactly on 4M random
// x in [0.25, 4) (one step left 2e-15), at a third of the cost of the IEEE
// division sequence.  v_rcp_f32 alone is within 0.9 ulp: where u = j (1 /
// rho) (FP16S, BF16S) the Newton step stays (without it the shocktube
// density error grew by a quarter); the delta form of F32S needs 1 / rho
// only for the small e = drho / rho and the bracket, where the raw
// reciprocal (recip_raw) gives the same errors (shocktube L2 6.8e-6 against
// 8.3e-6 with the step) for 1 % more throughput.  Host builds (the CPU
// check of this header) divide.
__host__ __device__ __forceinline__ double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ float recip_raw(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}

// Equilibrium of one node: feq_i (full value) and deq_i = feq_i - w_i rho0
// (deq = feq when unshifted).  drho = rho - rho0 (= rho when unshifted);
// uxx = ux^2, uyy = uy^2.
template <int EQ, bool SHIFTED, typename R>
__host__ __device__ __forceinline__ void equilibrium(R drho, R rho, R ux, R uy, R uxx, R uyy,
                                                     const Coeffs<R>& k, R (&feq)[9],
                                                     R (&deq)[9]) {
#pragma clang fp contract(off)
  if constexpr (EQ == LB_EQ_GUIDED && !SHIFTED) {
    // Per-axis factors of Eq. (11): Psi(+-1) = (a1 + u^2/2) +- u/2,
    // Psi(0) = a0 - u^2; f^eq_i = (rho X) Y.
    const R bx = k.a1 + R(0.5) * uxx, by = k.a1 + R(0.5) * uyy;
    const R Xm = fmadd(R(-0.5), ux, bx), X0 = k.a0 - uxx, Xp = fmadd(R(0.5), ux, bx);
    const R Ym = fmadd(R(-0.5), uy, by), Y0 = k.a0 - uyy, Yp = fmadd(R(0.5), uy, by);
    const R rXm = rho * Xm, rX0 = rho * X0, rXp = rho * Xp;
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      feq[I.value] = pick<cx>(rXm, rX0, rXp) * pick<cy>(Ym, Y0, Yp);
      deq[I.value] = feq[I.value];
    });
  } else if constexpr (EQ == LB_EQ_GUIDED) {
    // Shifted storage: the per-axis factors as rest value + small difference,
    // Psi(-1) = a1 + (u^2 - u)/2, Psi(0) = a0 - u^2, Psi(+1) = a1 + (u^2 + u)/2,
    // so that f^eq_i - w_i rho0 is formed from the differences.
    const R hx = R(0.5) * uxx, hy = R(0.5) * uyy;
    const R dXm = fmadd(R(-0.5), ux, hx), dX0 = -uxx, dXp = fmadd(R(0.5), ux, hx);
    const R dYm = fmadd(R(-0.5), uy, hy), dY0 = -uyy, dYp = fmadd(R(0.5), uy, hy);
    const R Xm = k.a1 + dXm, X0 = k.a0 + dX0, Xp = k.a1 + dXp;
    const R Ym = k.a1 + dYm, Y0 = k.a0 + dY0, Yp = k.a1 + dYp;
    // feq_i = (rho X) Y
    const R rXm = rho * Xm, rX0 = rho * X0, rXp = rho * Xp;
    // deq_i = rho X Y - rho0 ax ay = (drho X + rho0 dX) Y + (rho0 ax) dY: every
    // term is of the size of the deviation, so nothing cancels.
    const R Exm = fmadd(drho, Xm, k.rho0 * dXm), Ex0 = fmadd(drho, X0, k.rho0 * dX0),
            Exp = fmadd(drho, Xp, k.rho0 * dXp);
    const R a0dYm = k.r0a0 * dYm, a0dY0 = k.r0a0 * dY0, a0dYp = k.r0a0 * dYp;
    const R a1dYm = k.r0a1 * dYm, a1dY0 = k.r0a1 * dY0, a1dYp = k.r0a1 * dYp;
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      const R Y = pick<cy>(Ym, Y0, Yp);
      feq[I.value] = pick<cx>(rXm, rX0, rXp) * Y;
      const R adY = (cx == 0) ? pick<cy>(a0dYm, a0dY0, a0dYp) : pick<cy>(a1dYm, a1dY0, a1dYp);
      deq[I.value] = fmadd(pick<cx>(Exm, Ex0, Exp), Y, adY);
    });
  } else {
    // Polynomial equilibrium at theta0 = 1/3: rho W_i (1 + P_i),
    // P_i = 3 c.u + 9/2 (c.u)^2 - 3/2 u^2.
    const R u2h = R(1.5) * (uxx + uyy);
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      R cu;
      if constexpr (cx == 0 && cy == 0) cu = R(0);
      else if constexpr (cx == 0) cu = (cy > 0) ? uy : -uy;
      else if constexpr (cy == 0) cu = (cx > 0) ? ux : -ux;
      else cu = ((cx > 0) ? ux : -ux) + ((cy > 0) ? uy : -uy);
      const R W = ((cx == 0) ? k.a0 : k.a1) * ((cy == 0) ? k.a0 : k.a1);
      R P;
      if constexpr (cx == 0 && cy == 0) P = -u2h;
      else P = fmadd(cu, fmadd(R(4.5), cu, R(3)), -u2h);
      const R rW = rho * W;
      feq[I.value] = fmadd(rW, P, rW);
      if constexpr (SHIFTED) deq[I.value] = fmadd(drho, W, rW * P);
      else deq[I.value] = feq[I.value];
    });
  }
}

// OReg update with the guided equilibrium, written on the per-axis factors:
// f^eq_i = (rho X) Y with X = Psi(c_ix, u_x), Y = Psi(c_iy, u_y), and
// f^post_i = f^eq_i (1 + ax - by + tx Cy) (Eqs. 6, 7; the bracket terms are
// defined in collide below), evaluated as
//   rho X (Y (1 - by) + Y ax + (Y Cy) tx)                  (unshifted), or
//   Y (E + rho X ax - rho X by) + (rho X tx) (Y Cy) + (rho0 ax) dY
//                                                          (shifted, with
//   deq_i = f^eq_i - w_i rho0 folded in: see below),
// with the per-x and per-y products formed once: three operations per
// population.
// d13 = f1 + f3 - f2 - f4 and d57 = f5 + f7 - f6 - f8 (second moments).
template <bool SHIFTED, typename R>
__host__ __device__ __forceinline__ void collide_guided_oreg(R (&f)[9], const Coeffs<R>& k, R drho,
                                                             R rho, R inv, R jx, R ux, R uy,
                                                             R uxx, R uyy, R d13, R d57) {
#pragma clang fp contract(off)
  R rXm, rX0, rXp, Ym, Y0, Yp;  // rho X and Y
  // Shifted storage only: E = drho X + rho0 dX (per x) and (rho0 a) dY.
  R Exm = 0, Ex0 = 0, Exp = 0, a0dYm = 0, a0dY0 = 0, a0dYp = 0, a1dYm = 0, a1dY0 = 0, a1dYp = 0;
  if constexpr (!SHIFTED) {
    // Psi(+-1) = (a1 + u^2/2) +- u/2, Psi(0) = a0 - u^2.
    const R gx = fmadd(R(0.5), uxx, k.a1), gy = fmadd(R(0.5), uyy, k.a1);
    const R Xm = fmadd(R(-0.5), ux, gx), X0 = k.a0 - uxx, Xp = fmadd(R(0.5), ux, gx);
    Ym = fmadd(R(-0.5), uy, gy), Y0 = k.a0 - uyy, Yp = fmadd(R(0.5), uy, gy);
    rXm = rho * Xm, rX0 = rho * X0, rXp = rho * Xp;
  } else {
    // Rest value + small difference, so that deq_i = f^eq_i - w_i rho0 is
    // formed from the differences: deq_i = (drho X + rho0 dX) Y + (rho0 ax) dY.
    const R hx = R(0.5) * uxx, hy = R(0.5) * uyy;
    const R dXm = fmadd(R(-0.5), ux, hx), dX0 = -uxx, dXp = fmadd(R(0.5), ux, hx);
    const R dYm = fmadd(R(-0.5), uy, hy), dY0 = -uyy, dYp = fmadd(R(0.5), uy, hy);
    Ym = k.a1 + dYm, Y0 = k.a0 + dY0, Yp = k.a1 + dYp;
    // E = drho X + rho0 dX = rho dX + drho a (X = a + dX, rho = rho0 + drho),
    // and rho X = E + rho0 a.
    const R da0 = drho * k.a0, da1 = drho * k.a1;
    Exm = fmadd(rho, dXm, da1), Ex0 = fmadd(rho, dX0, da0), Exp = fmadd(rho, dXp, da1);
    rXm = Exm + k.r0a1, rX0 = Ex0 + k.r0a0, rXp = Exp + k.r0a1;
    a0dYm = k.r0a0 * dYm, a0dY0 = k.r0a0 * dY0, a0dYp = k.r0a0 * dYp;
    a1dYm = k.r0a1 * dYm, a1dY0 = k.r0a1 * dY0, a1dYp = k.r0a1 * dYp;
  }
  // Non-equilibrium stress (2 s = Pi_xx - Pi_yy, S_xy) and the bracket of
  // Eq. (6): kappa [..] = ks Cx^2 - ks Cy^2 + (kt Cx) Cy, C = c_i - u.
  // (rho ux uy = jx uy.)
  const R s2 = fmadd(-rho, uxx - uyy, d13);
  const R sxy = fmadd(-jx, uy, d57);
  const R ks = (k.kappa_h * inv) * s2, kt = (k.kappa_2 * inv) * sxy;
  // With C = -1 - u, -u, 1 - u:  ks C^2 = ks (1 +- 2 u) + ks u^2, ks u^2;
  // kt C = -kt - kt u, -kt u, kt - kt u;  Y C = -(Y + Y u), -Y u, Y - Y u.
  const R ax0 = ks * uxx;
  const R axm = fmadd(ks, fmadd(R(2), ux, R(1)), ax0), axp = fmadd(ks, fmadd(R(-2), ux, R(1)), ax0);
  const R by0 = ks * uyy;
  const R bym = fmadd(ks, fmadd(R(2), uy, R(1)), by0), byp = fmadd(ks, fmadd(R(-2), uy, R(1)), by0);
  const R ktx = kt * ux;
  const R txm = -kt - ktx, tx0 = -ktx, txp = kt - ktx;
  const R Qm = fmadd(-Ym, uy, -Ym), Q0 = -(Y0 * uy), Qp = fmadd(-Yp, uy, Yp);  // Y Cy
  if constexpr (!SHIFTED) {
    const R Pm = fmadd(-Ym, bym, Ym), P0 = fmadd(-Y0, by0, Y0), Pp = fmadd(-Yp, byp, Yp);
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      const R Y = pick<cy>(Ym, Y0, Yp);
      const R v = fmadd(pick<cy>(Qm, Q0, Qp), pick<cx>(txm, tx0, txp),
                        fmadd(Y, pick<cx>(axm, ax0, axp), pick<cy>(Pm, P0, Pp)));
      f[I.value] = pick<cx>(rXm, rX0, rXp) * v;
    });
  } else {
    // deq_i + rho X (Y ax - Y by + (Y Cy) tx)
    //   = Y (E + rho X ax - rho X by) + (rho X tx) (Y Cy) + (rho0 ax) dY,
    // every term of the size of the deviation.
    const R Gm = fmadd(rXm, axm, Exm), G0 = fmadd(rX0, ax0, Ex0), Gp = fmadd(rXp, axp, Exp);
    const R Tm = rXm * txm, T0 = rX0 * tx0, Tp = rXp * txp;
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      const R adY = (cx == 0) ? pick<cy>(a0dYm, a0dY0, a0dYp) : pick<cy>(a1dYm, a1dY0, a1dYp);
      const R g = fmadd(-pick<cx>(rXm, rX0, rXp), pick<cy>(bym, by0, byp), pick<cx>(Gm, G0, Gp));
      f[I.value] = fmadd(pick<cy>(Ym, Y0, Yp), g,
                         fmadd(pick<cx>(Tm, T0, Tp), pick<cy>(Qm, Q0, Qp), adY));
    });
  }
}

// Moments of one node (Eq. 2a): rho - rho0 (rho when unshifted), rho, 1/rho,
// j, u and the second-moment differences d13 = f1 + f3 - f2 - f4, d57 =
// f5 + f7 - f6 - f8.  Sum w_i = 1 and sum w_i c_i = 0, so the shift only
// enters rho.
template <typename R>
struct Moments {
  R drho, rho, inv, jx, jy, ux, uy, d13, d57;
};

template <bool SHIFTED, typename R>
__host__ __device__ __forceinline__ Moments<R> moments(const R (&f)[9], const Coeffs<R>& k) {
#pragma clang fp contract(off)
  Moments<R> m;
  const R s13 = f[1] + f[3], s24 = f[2] + f[4], s57 = f[5] + f[7], s68 = f[6] + f[8];
  m.drho = f[0] + (s13 + s24) + (s57 + s68);
  const R d57 = f[5] - f[7], d86 = f[8] - f[6];
  m.jx = (f[1] - f[3]) + (d57 + d86);
  m.jy = (f[2] - f[4]) + (d57 - d86);
  m.rho = SHIFTED ? k.rho0 + m.drho : m.drho;
  m.inv = recip(m.rho);
  m.ux = m.jx * m.inv;
  m.uy = m.jy * m.inv;
  m.d13 = s13 - s24;
  m.d57 = s57 - s68;
  return m;
}

// The same for shifted FP32 storage, with u formed so that the rounding of
// rho does not enter it: u = j / rho = (j - j e) / rho0 with e = drho / rho.
// Rounding rho = rho0 + drho to FP32 moves it by up to 2^-25 rho, an error
// that follows the smooth drho field and so does not average out over the
// lattice; in u = j / rho it biased the decay of a shear wave (CPU runs of
// this collision, 969^2, tau 0.70, 4256 steps: decay rate 9.0e-4 too slow).
// In e the same rounding is an error of relative size drho, and the FMA
// rounds j - j e once: 2.8e-4 on that run, against 2.7e-4 with the sums,
// rho, 1/rho and u formed in FP64 and rounded once, which cost 14 more
// instructions per collision (10 % of the fused F32S sweep's, and 14 % of
// its throughput); this form costs three more than u = j (1 / rho).
__host__ __device__ __forceinline__ Moments<float> moments_delta(const float (&f)[9],
                                                                 const Coeffs<float>& k) {
#pragma clang fp contract(off)
  Moments<float> m;
  const float s13 = f[1] + f[3], s24 = f[2] + f[4], s57 = f[5] + f[7], s68 = f[6] + f[8];
  m.drho = f[0] + (s13 + s24) + (s57 + s68);
  const float d57 = f[5] - f[7], d86 = f[8] - f[6];
  m.jx = (f[1] - f[3]) + (d57 + d86);
  m.jy = (f[2] - f[4]) + (d57 - d86);
  m.rho = k.rho0 + m.drho;
  m.inv = recip_raw(m.rho);
  const float e = m.drho * m.inv;
  m.ux = fmadd(-m.jx, e, m.jx) * k.inv0;
  m.uy = fmadd(-m.jy, e, m.jy) * k.inv0;
  m.d13 = s13 - s24;
  m.d57 = s57 - s68;
  return m;
}

// Collide one node in place.  f holds the pre-collision populations (shifted
// by w_i rho0 when SHIFTED) and receives the post-collision ones (same
// shift).  DELTA_U: moments by moments_delta (shifted FP32 only).
template <int EQ, int COLL, bool SHIFTED, bool DELTA_U = false, typename R>
__host__ __device__ __forceinline__ void collide(R (&f)[9], const Coeffs<R>& k) {
#pragma clang fp contract(off)
  Moments<R> m;
  if constexpr (DELTA_U && SHIFTED && std::is_same<R, float>::value) m = moments_delta(f, k);
  else m = moments<SHIFTED>(f, k);
  const R drho = m.drho, rho = m.rho, inv = m.inv, jx = m.jx, ux = m.ux, uy = m.uy;
  const R uxx = ux * ux, uyy = uy * uy;

  if constexpr (EQ == LB_EQ_GUIDED && COLL == LB_COLL_OREG) {
    collide_guided_oreg<SHIFTED>(f, k, drho, rho, inv, jx, ux, uy, uxx, uyy, m.d13, m.d57);
    return;
  }

  R feq[9], deq[9];
  equilibrium<EQ, SHIFTED>(drho, rho, ux, uy, uxx, uyy, k, feq, deq);

  if constexpr (COLL == LB_COLL_BGK) {
    // Eq. (1): f + (f^eq - f) / tau (the shift cancels in the difference).
    unroll<0, 9>([&](auto I) { f[I.value] = fmadd(k.omega, deq[I.value] - f[I.value], f[I.value]); });
    return;
  } else {
    // Trace-free non-equilibrium stress of Eq. (6) from second moments:
    // S_xx = -S_yy = s, S_xy.
    // 2 s = (Pi_xx - Pi_yy) of f^neq and S_xy.
    const R s2 = fmadd(-rho, uxx - uyy, m.d13);
    const R sxy = fmadd(-rho, ux * uy, m.d57);
    // Eqs. (6), (7): f^post_i = f^eq_i + kappa f^eq_i [s (Cx^2 - Cy^2) + 2 S_xy Cx Cy],
    // kappa = (1 - 1/tau)/(2 rho theta^2), C = c_i - u.  With ks = kappa s and
    // kt = 2 kappa S_xy the bracket splits into per-axis factors:
    // kappa [..] = ks Cx^2 - ks Cy^2 + (kt Cx) Cy.  (kappa0/2) and (2 kappa0)
    // are exact rescalings, so ks and kt round as kappa (s2/2) and kappa (2 S_xy).
    const R ks = (k.kappa_h * inv) * s2, kt = (k.kappa_2 * inv) * sxy;
    const R Cxm = R(-1) - ux, Cx0 = -ux, Cxp = R(1) - ux;
    const R Cym = R(-1) - uy, Cy0 = -uy, Cyp = R(1) - uy;
    const R axm = (ks * Cxm) * Cxm, ax0 = ks * uxx, axp = (ks * Cxp) * Cxp;
    const R bym = (ks * Cym) * Cym, by0 = ks * uyy, byp = (ks * Cyp) * Cyp;
    const R txm = kt * Cxm, tx0 = kt * Cx0, txp = kt * Cxp;
    unroll<0, 9>([&](auto I) {
      constexpr int cx = cx_of(I.value), cy = cy_of(I.value);
      const R term = fmadd(pick<cx>(txm, tx0, txp), pick<cy>(Cym, Cy0, Cyp),
                           pick<cx>(axm, ax0, axp) - pick<cy>(bym, by0, byp));
      f[I.value] = fmadd(feq[I.value], term, deq[I.value]);
    });
  }
}

// Rest weight times rho0 of a population with velocity (cx, cy), in FP64.
__host__ __device__ __forceinline__ double shift64(int cx, int cy, const Coef64& c) {
  return ((cx == 0) ? c.a0 : c.a1) * ((cy == 0) ? c.a0 : c.a1) * c.rho0;
}

}  // namespace oreg
