// Per-site arithmetic of the KT D2V9 finite-difference LB step, shared by every
// kernel of the library (single grid, batched, every launch shape) so that they
// all execute the same instruction sequence per site and agree bitwise.
//
// Every fused multiply-add is written out with fma(); the library is compiled
// with -ffp-contract=off so the compiler adds no other contraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbkt {

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_WALL = 2, BC_INFLOW = 3, BC_SHOCK = 4 };

// Everything a step needs about one grid, precomputed on the host in float64.
struct KTConsts {
  int32_t nx, ny;
  int64_t pitch, plane;   // row pitch and plane stride in elements
  // Linear part of the step, Eq. (SEC-VON-11) with Eqs. (SEC-VON-2a/2b):
  //   f_i' = Wc f(x) + sum over the 4 neighbours of (coefficient) f(neighbour) + inv_tau f_i^eq
  // Per velocity group (rest 0; axis 1..4 with speed c1; diagonal 5..8 with
  // component speed s) the coefficients are
  //   centre     wc = 1 - 1/tau - 4 l - (number of moving axes) r v (1 - 2 beta)
  //   upstream   up = l + r v (1 - beta)     (neighbour the velocity comes from)
  //   downstream dn = l - r v beta
  //   along a zero velocity component: l
  // with r = dt/dx, v the component speed and l = dt lambda / dx^2.
  double wc0, l0;            // i = 0
  double wca, upa, dna, la;  // i = 1..4
  double wcd, upd, dnd, ld;  // i = 5..8
  double inv_tau;
  // velocity set, Eq. (e14): c1 on the axes, s = c2/sqrt(2) per diagonal component
  double c1, s;
  // energy weights |v_i|^2 + eta_i^2 of Eq. (e7): eta0^2 (i=0), c1^2 (1..4), c2^2 (5..8)
  double eta0sq, c1sq, c2sq;
  double inv_b;           // 1/b, b = 2/(gamma-1)
  double bval;            // b
  // Eqs. (e17)-(e18) in the paper's grouping, one quotient per coefficient:
  //   A_0 = a0T T
  //   A_1..4 = (-c2^2 + k1T T + k1u usq) / k1d,  k1T = (b-2) c2^2/eta0^2 + 2, k1u = c2^2/c1^2, k1d = 4 (c1^2 - c2^2)
  //   A_5..8 = (-c1^2 + k5T T + k5u usq) / k5d,  (c1 <-> c2)
  //   B_1..4 = (-c2^2 + bT T + usq) / b1d,       bT = b + 2, b1d = 2 c1^2 (c1^2 - c2^2)
  //   B_5..8 = (-c1^2 + bT T + usq) / b5d,       b5d = 2 c2^2 (c2^2 - c1^2)
  //   D = d1 = 1/(2 c1^4), d5 = 1/(2 c2^4)
  // with usq = u.u; r* are the rounded reciprocals of the divisors.
  double a0T;
  double k1u, k1T, k1d, r1d, k5u, k5T, k5d, r5d, bT, b1d, rb1d, b5d, rb5d;
  double d1, d5;
  // derivatives for the adjoint: dA/dT, dA/dusq, dB/dT, dB/dusq per group
  double a1T, a1u, a5T, a5u, b1T, b1u, b5T, b5u;
  // boundary edges x-, x+, y-, y+
  int32_t kind[4], split[4];
  double ga[4][9], gb[4][9];  // f^eq of edge states a and b
};

// Velocity components of plane i (Eq. (e14) with the (cos, sin) reading).
__host__ __device__ inline double vel_x(const KTConsts& K, int i) {
  switch (i) {
    case 1: return -K.c1;
    case 3: return K.c1;
    case 5: return -K.s;
    case 6: return K.s;
    case 7: return K.s;
    case 8: return -K.s;
    default: return 0.0;
  }
}
__host__ __device__ inline double vel_y(const KTConsts& K, int i) {
  switch (i) {
    case 2: return -K.c1;
    case 4: return K.c1;
    case 5: return -K.s;
    case 6: return -K.s;
    case 7: return K.s;
    case 8: return K.s;
    default: return 0.0;
  }
}

// a / b given rb = 1/b rounded: one Newton-type correction of a * rb with the
// exact FMA residual gives the correctly rounded quotient in all but rare
// cases (Markstein), and never a systematic bias, for three operations
// instead of a full division sequence.
__host__ __device__ __forceinline__ double div_cr(double a, double b, double rb) {
  const double q = a * rb;
  const double r = fma(-q, b, a);
  return fma(r, rb, q);
}

// 1/x within about an ulp: the hardware reciprocal refined by two Newton steps
// (each squares the relative error), 5 instructions instead of the IEEE
// division sequence. It only feeds div_cr's corrections (and the adjoint's chain
// rule), whose quotients stay correctly rounded with a reciprocal that is off by
// an ulp: the residual is exact, and the correction's error is second order in it.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

// Macroscopic fields, Eqs. (e4), (e5), (e7): rho, u = j/rho, T = (E/rho - u.u)/b.
struct Prim { double rho, ux, uy, T, rinv, usq; };

// RCP: the quotients as products with 1/rho (recip) and the host-rounded 1/b,
// within two ulps of the corrected ones (the kernels with FP32 storage; see site_update).
template <bool RCP = false>
__device__ inline Prim moments9(const KTConsts& K, const double f[9]) {
  const double s14 = (f[1] + f[2]) + (f[3] + f[4]);
  const double s58 = (f[5] + f[6]) + (f[7] + f[8]);
  const double rho = (f[0] + s14) + s58;
  const double jx = fma(K.c1, f[3] - f[1], K.s * ((f[6] + f[7]) - (f[5] + f[8])));
  const double jy = fma(K.c1, f[4] - f[2], K.s * ((f[7] + f[8]) - (f[5] + f[6])));
  const double E = fma(K.eta0sq, f[0], fma(K.c1sq, s14, K.c2sq * s58));
  Prim P;
  P.rho = rho;
  P.rinv = recip(rho);
  if constexpr (RCP) {
    P.ux = jx * P.rinv;
    P.uy = jy * P.rinv;
    P.usq = fma(P.ux, P.ux, P.uy * P.uy);
    P.T = (E * P.rinv - P.usq) * K.inv_b;
  } else {
    P.ux = div_cr(jx, rho, P.rinv);
    P.uy = div_cr(jy, rho, P.rinv);
    P.usq = fma(P.ux, P.ux, P.uy * P.uy);
    P.T = div_cr(div_cr(E, rho, P.rinv) - P.usq, K.bval, K.inv_b);
  }
  return P;
}

// Group coefficients of Eqs. (e17)-(e18) at (T, usq).
struct Coef { double A0, A1, A5, B1, B5; };

template <bool RCP = false>
__host__ __device__ inline Coef coef(const KTConsts& K, double T, double usq) {
  Coef C;
  C.A0 = K.a0T * T;
  if constexpr (RCP) {
    C.A1 = fma(K.k1u, usq, fma(K.k1T, T, -K.c2sq)) * K.r1d;
    C.A5 = fma(K.k5u, usq, fma(K.k5T, T, -K.c1sq)) * K.r5d;
    C.B1 = (fma(K.bT, T, usq) - K.c2sq) * K.rb1d;
    C.B5 = (fma(K.bT, T, usq) - K.c1sq) * K.rb5d;
  } else {
    C.A1 = div_cr(fma(K.k1u, usq, fma(K.k1T, T, -K.c2sq)), K.k1d, K.r1d);
    C.A5 = div_cr(fma(K.k5u, usq, fma(K.k5T, T, -K.c1sq)), K.k5d, K.r5d);
    C.B1 = div_cr(fma(K.bT, T, usq) - K.c2sq, K.b1d, K.rb1d);
    C.B5 = div_cr(fma(K.bT, T, usq) - K.c1sq, K.b5d, K.rb5d);
  }
  return C;
}

// Equilibrium, Eq. (e16): f_i^eq = rho (A_i + B_i (v_i.u) + D_i (v_i.u)^2).
// Axis planes: v.u = -/+ c1 ux (1, 3), -/+ c1 uy (2, 4);
// diagonal planes: v.u = -/+ s (ux+uy) (5, 7), +/- s (ux-uy) (6, 8).
template <bool RCP = false>
__host__ __device__ inline void feq9(const KTConsts& K, double rho, double ux, double uy, double T,
                                     double usq, double fe[9]) {
  const Coef C = coef<RCP>(K, T, usq);
  const double ex = K.c1 * ux, ey = K.c1 * uy;
  const double dp = K.s * (ux + uy), dm = K.s * (ux - uy);
  const double px = fma(K.d1 * ex, ex, C.A1);
  const double py = fma(K.d1 * ey, ey, C.A1);
  const double pp = fma(K.d5 * dp, dp, C.A5);
  const double pm = fma(K.d5 * dm, dm, C.A5);
  fe[0] = rho * C.A0;
  fe[1] = rho * fma(-C.B1, ex, px);
  fe[3] = rho * fma(C.B1, ex, px);
  fe[2] = rho * fma(-C.B1, ey, py);
  fe[4] = rho * fma(C.B1, ey, py);
  fe[5] = rho * fma(-C.B5, dp, pp);
  fe[7] = rho * fma(C.B5, dp, pp);
  fe[6] = rho * fma(C.B5, dm, pm);
  fe[8] = rho * fma(-C.B5, dm, pm);
}

// Stencil coefficient of plane i for neighbour k (0 centre, 1 x+dx, 2 x-dx,
// 3 y+dy, 4 y-dy). With i and k compile-time constants this folds to one field.
__host__ __device__ __forceinline__ double wcoef(const KTConsts& K, int i, int k) {
  if (i == 0) return k == 0 ? K.wc0 : K.l0;
  if (i <= 4) {
    if (k == 0) return K.wca;
    // i = 1 (-c1,0): x+ upstream; 3 (c1,0): x- upstream; 2 (0,-c1): y+ upstream; 4 (0,c1): y- upstream
    const bool xaxis = (i == 1 || i == 3);
    if ((k == 1 || k == 2) != xaxis) return K.la;
    const bool up = (i == 1 && k == 1) || (i == 3 && k == 2) || (i == 2 && k == 3) || (i == 4 && k == 4);
    return up ? K.upa : K.dna;
  }
  if (k == 0) return K.wcd;
  // diagonal i: sign of vx (5,8 negative) and vy (5,6 negative)
  const bool vxneg = (i == 5 || i == 8), vyneg = (i == 5 || i == 6);
  bool up;
  if (k == 1) up = vxneg;
  else if (k == 2) up = !vxneg;
  else if (k == 3) up = vyneg;
  else up = !vyneg;
  return up ? K.upd : K.dnd;
}

// Linear part and relaxation of plane i at one site (the fixed operation order
// every kernel uses); fe_tau = f_i^eq / tau.
__host__ __device__ __forceinline__ double plane_update(const KTConsts& K, int i, double fe_tau, double c, double xp,
                                                        double xm, double yp, double ym) {
  double acc = fe_tau;
  acc = fma(wcoef(K, i, 4), ym, acc);
  acc = fma(wcoef(K, i, 3), yp, acc);
  acc = fma(wcoef(K, i, 2), xm, acc);
  acc = fma(wcoef(K, i, 1), xp, acc);
  return fma(wcoef(K, i, 0), c, acc);
}

// One site of the step: centre values c, neighbours at x+dx, x-dx, y+dy, y-dy.
// RCP (the kernels with FP32 storage): quotients as products with reciprocals,
// within two ulps of the corrected ones, far below the storage's rounding (FP32
// two-step pass 2%, the batched four-step pass 5% faster); the FP64-storage
// kernels keep the corrected quotients of the oracle's divisions. Every kernel of
// one storage type takes the same form, so they agree bitwise.
template <bool RCP = false>
__device__ __forceinline__ void site_update(const KTConsts& K, const double c[9], const double xp[9],
                                                     const double xm[9], const double yp[9], const double ym[9],
                                                     double out[9]) {
  const Prim P = moments9<RCP>(K, c);
  // f^eq / tau, with 1/tau applied to rho once instead of to each f_i^eq (the
  // equilibrium is linear in rho; exact for tau = 1)
  double fe[9];
  feq9<RCP>(K, P.rho * K.inv_tau, P.ux, P.uy, P.T, P.usq, fe);
#pragma unroll
  for (int i = 0; i < 9; ++i) out[i] = plane_update(K, i, fe[i], c[i], xp[i], xm[i], yp[i], ym[i]);
}

// Mirror maps of a reflecting wall: x-normal swaps 1<->3, 5<->6, 7<->8;
// y-normal swaps 2<->4, 5<->8, 6<->7.
__host__ __device__ inline int mirror_x(int i) {
  const int m[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};
  return m[i];
}
__host__ __device__ inline int mirror_y(int i) {
  const int m[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
  return m[i];
}

// Adjoint of the collision part at one site. Given g (= dL/df' at the site) and the
// primitive state of f at the site, returns c_j = (1/tau) sum_i g_i d f_i^eq / d f_j.
// f^eq depends on f only through m = (rho, jx, jy, E) with d m_k / d f_j =
// psi_k(j) = (1, v_jx, v_jy, |v_j|^2 + eta_j^2).
__host__ __device__ inline void collision_adjoint(const KTConsts& K, const Prim& P, const double g[9],
                                                  double out[9]) {
  const double rho = P.rho, ux = P.ux, uy = P.uy, T = P.T, usq = P.usq;
  const Coef C = coef(K, T, usq);
  // d/dT and d/d(usq) of the group coefficients
  const double A0T = K.a0T, A1T = K.a1T, A5T = K.a5T, B1T = K.b1T, B5T = K.b5T;
  const double A1u = K.a1u, A5u = K.a5u, B1u = K.b1u, B5u = K.b5u;
  double Gr = 0.0, GT = 0.0, Gx = 0.0, Gy = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double vx = vel_x(K, i), vy = vel_y(K, i);
    const double vu = fma(vx, ux, vy * uy);
    double A, B, D, AT, BT, Au, Bu;
    if (i == 0) {
      A = C.A0; B = 0.0; D = 0.0; AT = A0T; BT = 0.0; Au = 0.0; Bu = 0.0;
    } else if (i <= 4) {
      A = C.A1; B = C.B1; D = K.d1; AT = A1T; BT = B1T; Au = A1u; Bu = B1u;
    } else {
      A = C.A5; B = C.B5; D = K.d5; AT = A5T; BT = B5T; Au = A5u; Bu = B5u;
    }
    const double phi = fma(fma(D, vu, B), vu, A);         // A + B vu + D vu^2
    const double dphidT = fma(BT, vu, AT);
    const double dphidusq = fma(Bu, vu, Au);
    const double dphidvu = fma(2.0 * D, vu, B);
    // d phi / d ux = dphi/dusq * 2 ux + dphi/dvu * vx
    const double dphidux = fma(dphidusq, 2.0 * ux, dphidvu * vx);
    const double dphiduy = fma(dphidusq, 2.0 * uy, dphidvu * vy);
    Gr = fma(g[i], phi, Gr);
    GT = fma(g[i], dphidT, GT);
    Gx = fma(g[i], dphidux, Gx);
    Gy = fma(g[i], dphiduy, Gy);
  }
  GT *= rho;
  Gx *= rho;
  Gy *= rho;
  // chain rule to m = (rho, jx, jy, E): u = j/rho, T = (E/rho - u.u)/b
  const double rinv = P.rinv;
  const double brinv = K.inv_b * rinv;
  const double s_r = Gr - (ux * Gx + uy * Gy) * rinv + GT * (usq - K.bval * T) * brinv;
  const double s_jx = Gx * rinv - 2.0 * ux * GT * brinv;
  const double s_jy = Gy * rinv - 2.0 * uy * GT * brinv;
  const double s_E = GT * brinv;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const double w = (j == 0) ? K.eta0sq : ((j <= 4) ? K.c1sq : K.c2sq);
    const double sj = s_r + vel_x(K, j) * s_jx + vel_y(K, j) * s_jy + w * s_E;
    out[j] = K.inv_tau * sj;
  }
}

// d f_i^eq(rho, u, p/rho) / d rho at fixed u and p: phi_i - T dphi_i/dT  (T = p/rho).
__host__ __device__ inline double init_adjoint_site(const KTConsts& K, double rho, double ux, double uy,
                                                    double p, const double g[9]) {
  const double T = p / rho;
  const double usq = fma(ux, ux, uy * uy);
  const Coef C = coef(K, T, usq);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double vu = fma(vel_x(K, i), ux, vel_y(K, i) * uy);
    double A, B, D, AT, BT;
    if (i == 0) {
      A = C.A0; B = 0.0; D = 0.0; AT = K.a0T; BT = 0.0;
    } else if (i <= 4) {
      A = C.A1; B = C.B1; D = K.d1; AT = K.a1T; BT = K.b1T;
    } else {
      A = C.A5; B = C.B5; D = K.d5; AT = K.a5T; BT = K.b5T;
    }
    const double phi = fma(fma(D, vu, B), vu, A);
    const double dphidT = fma(BT, vu, AT);
    acc = fma(g[i], fma(-T, dphidT, phi), acc);
  }
  return acc;
}

}  // namespace lbkt
