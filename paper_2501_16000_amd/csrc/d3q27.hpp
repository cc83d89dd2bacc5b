// d3q27.hpp -- device-side D3Q27 collision (OReg of Eq. (6) with D = 3, or
// lattice BGK of Eq. (1)) of one node in registers.
//
// The storage codecs, Coef64/Coeffs constants and helpers are those of the
// D2Q9 lattice (d2q9.hpp).  Algebraic forms used instead of the printed ones
// (identical in exact arithmetic):
//   * moments by lines: for each (c_y, c_z) the three populations along x
//     give their sum, difference and outer sum; planes of constant c_z
//     combine lines, the box combines planes (66 additions for rho, j and
//     the six second moments);
//   * both equilibria reproduce Pi^eq = rho theta I + rho u u, so the
//     trace-free stress of f^neq is the trace-free part of Pi - rho u u
//     (the shift w_i rho0 adds rho0 theta I, which has no trace-free part);
//   * with a trace-free S, (C C - C^2/3 I):S = sum_ab C_a C_b S_ab, and
//     kappa times it is assembled from per-axis tables:
//       A_a[c] = kappa S_aa C_a(c)^2,  T_ab[c] = 2 kappa S_ab C_a(c),
//       kappa b_i = (A_x + A_y + T_xy C_y) + A_z + (T_xz + T_yz) C_z;
//   * the guided equilibrium is rho X(c_x) Y(c_y) Z(c_z) with rest value +
//     small difference per axis factor, and in shifted storage
//     f^eq_i - w_i rho0 = drho XYZ + rho0 (dX YZ + a_x dY Z + a_x a_y dZ).
#pragma once

#include "d2q9.hpp"

namespace oreg {
namespace d3 {

// i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1).
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
static_assert(cx(13) == 0 && cy(13) == 0 && cz(13) == 0, "rest velocity");
static_assert(cx(0) == -1 && cy(0) == -1 && cz(0) == -1 && cx(26) == 1 && cz(26) == 1, "corners");

// Rest weight of an axis component: a0 (c = 0) or a1 (c = +-1).
template <int c, typename R>
__host__ __device__ __forceinline__ R axis_w(const Coeffs<R>& k) {
  return c == 0 ? k.a0 : k.a1;
}

// rho - rho0 (rho when unshifted), j and the raw second moments
// M_ab = sum_i c_ia c_ib f_i of one node.
template <typename R>
__host__ __device__ __forceinline__ void moments(const R (&f)[27], R& drho, R (&j)[3],
                                                 R (&M)[6]) {
#pragma clang fp contract(off)
  R L0[9], L1[9], L2[9];  // per line l = 3 (c_z + 1) + (c_y + 1)
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    L2[l] = f[3 * l + 2] + f[3 * l];
    L0[l] = L2[l] + f[3 * l + 1];
    L1[l] = f[3 * l + 2] - f[3 * l];
  }
  R P0[3], Py[3], Pyy[3], Px[3], Pxy[3], Pxx[3];  // per plane p = c_z + 1
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    Pyy[p] = L0[3 * p + 2] + L0[3 * p];
    P0[p] = Pyy[p] + L0[3 * p + 1];
    Py[p] = L0[3 * p + 2] - L0[3 * p];
    Px[p] = (L1[3 * p + 2] + L1[3 * p]) + L1[3 * p + 1];
    Pxy[p] = L1[3 * p + 2] - L1[3 * p];
    Pxx[p] = (L2[3 * p + 2] + L2[3 * p]) + L2[3 * p + 1];
  }
  const R Mzz = P0[2] + P0[0];
  drho = Mzz + P0[1];
  j[0] = (Px[2] + Px[0]) + Px[1];
  j[1] = (Py[2] + Py[0]) + Py[1];
  j[2] = P0[2] - P0[0];
  M[0] = (Pxx[2] + Pxx[0]) + Pxx[1];  // xx
  M[1] = (Pyy[2] + Pyy[0]) + Pyy[1];  // yy
  M[2] = Mzz;                         // zz
  M[3] = (Pxy[2] + Pxy[0]) + Pxy[1];  // xy
  M[4] = Px[2] - Px[0];               // xz
  M[5] = Py[2] - Py[0];               // yz
}

// Equilibrium: feq_i (full value) and deq_i = feq_i - w_i rho0 (deq = feq
// when unshifted).  u2[a] = u_a^2.
template <int EQ, bool SHIFTED, typename R>
__host__ __device__ __forceinline__ void equilibrium(R drho, R rho, const R (&u)[3],
                                                     const R (&u2)[3], const Coeffs<R>& k,
                                                     R (&feq)[27], R (&deq)[27]) {
#pragma clang fp contract(off)
  if constexpr (EQ == LB_EQ_GUIDED) {
    // Per-axis factors Psi(-1) = a1 + (u^2 - u)/2, Psi(0) = a0 - u^2,
    // Psi(+1) = a1 + (u^2 + u)/2, as rest value + difference d[a][c + 1].
    R d[3][3], F[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R h = R(0.5) * u2[a];
      d[a][0] = fmadd(R(-0.5), u[a], h);
      d[a][1] = -u2[a];
      d[a][2] = fmadd(R(0.5), u[a], h);
      F[a][0] = k.a1 + d[a][0];
      F[a][1] = k.a0 + d[a][1];
      F[a][2] = k.a1 + d[a][2];
    }
    R rXY[3][3];
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
      const R rX = rho * F[0][ix];
#pragma unroll
      for (int iy = 0; iy < 3; ++iy) rXY[ix][iy] = rX * F[1][iy];
    }
    if constexpr (SHIFTED) {
      R YZ[3][3];
#pragma unroll
      for (int iy = 0; iy < 3; ++iy)
#pragma unroll
        for (int iz = 0; iz < 3; ++iz) YZ[iy][iz] = F[1][iy] * F[2][iz];
      unroll<0, 27>([&](auto I) {
        constexpr int ix = cx(I.value) + 1, iy = cy(I.value) + 1, iz = cz(I.value) + 1;
        const R ax = ix == 1 ? k.a0 : k.a1, ay = iy == 1 ? k.a0 : k.a1;
        feq[I.value] = rXY[ix][iy] * F[2][iz];
        const R XYZ = F[0][ix] * YZ[iy][iz];
        const R t3 = ((k.rho0 * ax) * ay) * d[2][iz];
        const R t2 = fmadd((k.rho0 * ax) * d[1][iy], F[2][iz], t3);
        deq[I.value] = fmadd(drho, XYZ, fmadd(k.rho0 * d[0][ix], YZ[iy][iz], t2));
      });
    } else {
      unroll<0, 27>([&](auto I) {
        constexpr int ix = cx(I.value) + 1, iy = cy(I.value) + 1, iz = cz(I.value) + 1;
        feq[I.value] = rXY[ix][iy] * F[2][iz];
        deq[I.value] = feq[I.value];
      });
    }
  } else {
    // Polynomial equilibrium at theta0 = 1/3: rho W_i (1 + P_i),
    // P_i = 3 c.u + 9/2 (c.u)^2 - 3/2 u^2.
    const R u2h = R(1.5) * ((u2[0] + u2[1]) + u2[2]);
    unroll<0, 27>([&](auto I) {
      constexpr int ccx = cx(I.value), ccy = cy(I.value), ccz = cz(I.value);
      R cu = R(0);
      if constexpr (ccx != 0) cu = ccx > 0 ? u[0] : -u[0];
      if constexpr (ccy != 0) cu = cu + (ccy > 0 ? u[1] : -u[1]);
      if constexpr (ccz != 0) cu = cu + (ccz > 0 ? u[2] : -u[2]);
      const R W = (axis_w<ccx>(k) * axis_w<ccy>(k)) * axis_w<ccz>(k);
      const R P = fmadd(cu, fmadd(R(4.5), cu, R(3)), -u2h);
      const R rW = rho * W;
      feq[I.value] = fmadd(rW, P, rW);
      if constexpr (SHIFTED) deq[I.value] = fmadd(drho, W, rW * P);
      else deq[I.value] = feq[I.value];
    });
  }
}

// Collide one node in place: f holds the pre-collision populations (shifted
// by w_i rho0 when SHIFTED) and receives the post-collision ones.
template <int EQ, int COLL, bool SHIFTED, typename R>
__host__ __device__ __forceinline__ void collide(R (&f)[27], const Coeffs<R>& k) {
#pragma clang fp contract(off)
  R drho, j[3], M[6];
  moments(f, drho, j, M);
  const R rho = SHIFTED ? k.rho0 + drho : drho;
  const R inv = recip(rho);
  const R u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
  const R u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};

  R feq[27], deq[27];
  equilibrium<EQ, SHIFTED>(drho, rho, u, u2, k, feq, deq);

  if constexpr (COLL == LB_COLL_BGK) {
    unroll<0, 27>([&](auto I) { f[I.value] = fmadd(k.omega, deq[I.value] - f[I.value], f[I.value]); });
  } else {
    // Trace-free part of Pi - rho u u (Pi^eq = rho theta I + rho u u).
    const R Dxx = fmadd(-rho, u2[0], M[0]);
    const R Dyy = fmadd(-rho, u2[1], M[1]);
    const R Dzz = fmadd(-rho, u2[2], M[2]);
    const R tr3 = ((Dxx + Dyy) + Dzz) * R(1.0 / 3.0);
    const R Sxx = Dxx - tr3, Syy = Dyy - tr3, Szz = Dzz - tr3;
    const R Sxy = fmadd(-rho, u[0] * u[1], M[3]);
    const R Sxz = fmadd(-rho, u[0] * u[2], M[4]);
    const R Syz = fmadd(-rho, u[1] * u[2], M[5]);
    const R kappa = k.kappa0 * inv;
    const R kxx = kappa * Sxx, kyy = kappa * Syy, kzz = kappa * Szz;
    const R txy = kappa * (Sxy + Sxy), txz = kappa * (Sxz + Sxz), tyz = kappa * (Syz + Syz);
    R Cx[3], Cy[3], Cz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cx[c] = R(c - 1) - u[0];
      Cy[c] = R(c - 1) - u[1];
      Cz[c] = R(c - 1) - u[2];
    }
    R Az[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) Az[c] = (kzz * Cz[c]) * Cz[c];
    R B[3][3], U[3][3];
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
      const R Ax = (kxx * Cx[ix]) * Cx[ix];
      const R Txy = txy * Cx[ix], Txz = txz * Cx[ix];
#pragma unroll
      for (int iy = 0; iy < 3; ++iy) {
        const R Ay = (kyy * Cy[iy]) * Cy[iy];
        B[ix][iy] = fmadd(Txy, Cy[iy], Ax + Ay);
        U[ix][iy] = Txz + tyz * Cy[iy];
      }
    }
    unroll<0, 27>([&](auto I) {
      constexpr int ix = cx(I.value) + 1, iy = cy(I.value) + 1, iz = cz(I.value) + 1;
      const R term = fmadd(U[ix][iy], Cz[iz], B[ix][iy] + Az[iz]);
      f[I.value] = fmadd(feq[I.value], term, deq[I.value]);
    });
  }
}

// Rest weight times rho0 of a population with velocity (cx, cy, cz), FP64.
__host__ __device__ __forceinline__ double shift64(int vx, int vy, int vz, const Coef64& c) {
  auto w = [&](int v) { return v == 0 ? c.a0 : c.a1; };
  return w(vx) * w(vy) * w(vz) * c.rho0;
}

}  // namespace d3
}  // namespace oreg
