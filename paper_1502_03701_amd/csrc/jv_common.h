// Shared pieces of the operator kernels: stencil coefficients, per-point
// derivative data and the pointwise tangent-linear algebra.  The discrete
// operator is described at the top of jv.hip.
#pragma once

#include "sa_internal.h"

namespace sa {

template <typename R, int ND>
struct Pt {
  R q[ND + 3];        // p, u_1..u_ND, s, T
  R D[ND + 3][ND];    // D_a of each of them
  R Lu[ND];           // sum_a D2_a u_i
  R G[ND];            // D2_i u_i + sum_{j != i} D_i D_j u_j
  R LT;               // sum_a D2_a T
};

// Stencil coefficients of one axis at one point.
template <typename R>
struct Axis {
  R c1[3];   // multiplies f(+m) - f(-m)
  R c0;      // second-derivative centre
  R c2[3];   // multiplies f(+m) + f(-m)
};

template <typename R>
__device__ __forceinline__ Axis<R> axis_coefs(int order) {
  Axis<R> a;
  if (order == 6) {
    a.c1[0] = R(3.0 / 4.0); a.c1[1] = R(-3.0 / 20.0); a.c1[2] = R(1.0 / 60.0);
    a.c0 = R(-49.0 / 18.0);
    a.c2[0] = R(3.0 / 2.0); a.c2[1] = R(-3.0 / 20.0); a.c2[2] = R(1.0 / 90.0);
  } else if (order == 4) {
    a.c1[0] = R(2.0 / 3.0); a.c1[1] = R(-1.0 / 12.0); a.c1[2] = R(0);
    a.c0 = R(-5.0 / 2.0);
    a.c2[0] = R(4.0 / 3.0); a.c2[1] = R(-1.0 / 12.0); a.c2[2] = R(0);
  } else if (order == 2) {
    a.c1[0] = R(1.0 / 2.0); a.c1[1] = R(0); a.c1[2] = R(0);
    a.c0 = R(-2.0);
    a.c2[0] = R(1.0); a.c2[1] = R(0); a.c2[2] = R(0);
  } else {
    a.c1[0] = a.c1[1] = a.c1[2] = R(0);
    a.c0 = R(0);
    a.c2[0] = a.c2[1] = a.c2[2] = R(0);
  }
  return a;
}

// v, or +0 where z (the wall rows' output): a bitwise mask instead of a
// select, so that the compiler does not put the computation of v under a
// branch on z (whose register copies would wait for pending loads)
__device__ __forceinline__ double zero_on(bool z, double v) {
  const long long m = (long long)z - 1;   // z: 0, else all ones
  return __longlong_as_double(__double_as_longlong(v) & m);
}
__device__ __forceinline__ float zero_on(bool z, float v) {
  const int m = (int)z - 1;
  return __int_as_float(__float_as_int(v) & m);
}

__device__ __forceinline__ int wall_row_order(int j, int ny, int bcy) {
  if (bcy == 0) return 6;
  if (j <= 0 || j >= ny - 1) return 0;
  if (j == 1 || j == ny - 2) return 2;
  if (j == 2 || j == ny - 3) return 4;
  return 6;
}

// Pointwise tangent-linear algebra: out = N'(q0; v) given base and
// perturbation data at one point.
template <typename R, int ND>
__device__ __forceinline__ void tangent(const Pt<R, ND>& b, const Pt<R, ND>& v, const OpParams& op,
                                        R rho, R ip0, R mu0, R muT, R muTT, R out[ND + 2]) {
  const R gam = R(op.gamma);
  const R cp = R(op.cp);
  const R cpr = R(op.cp / op.pr);
  const R p0 = b.q[0];
  const R T0 = b.q[ND + 2];
  const R pp = v.q[0];
  const R sp = v.q[ND + 1];
  const R Tpr = v.q[ND + 2];
  const R rhop = rho * (pp * ip0 * R(1.0 / op.gamma) - sp * R(1.0 / op.cp));   // rho_p p' + rho_s s'

  R th0 = R(0), thp = R(0);
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    th0 += b.D[1 + k][k];
    thp += v.D[1 + k][k];
  }
  R S00 = R(0), S0p = R(0);
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const R s0 = R(0.5) * (b.D[1 + i][j] + b.D[1 + j][i]);
      const R s1 = R(0.5) * (v.D[1 + i][j] + v.D[1 + j][i]);
      S00 += s0 * s0;
      S0p += s0 * s1;
    }
  R g2 = R(0), g1 = R(0);
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    g2 += b.D[ND + 2][j] * b.D[ND + 2][j];
    g1 += b.D[ND + 2][j] * v.D[ND + 2][j];
  }
  const R lam0 = cpr * mu0, lamT = cpr * muT, lamTT = cpr * muTT;
  const R phiS = R(2) * S00 - R(2.0 / 3.0) * th0 * th0;
  const R Phi0 = mu0 * phiS;
  const R Phip = muT * Tpr * phiS + mu0 * (R(4) * S0p - R(4.0 / 3.0) * th0 * thp);
  const R Q0 = lam0 * b.LT + lamT * g2;
  const R Qp = lamT * Tpr * b.LT + lam0 * v.LT + lamTT * Tpr * g2 + R(2) * lamT * g1;
  const R H0 = Q0 + Phi0;
  const R Hp = Qp + Phip;

  // pressure
  R adv = R(0);
#pragma unroll
  for (int j = 0; j < ND; ++j) adv += v.q[1 + j] * b.D[0][j] + b.q[1 + j] * v.D[0][j];
  out[0] = -adv - gam * (pp * th0 + p0 * thp) + (gam - R(1)) * Hp;

  // velocity
  const R irho = R(op.R) * T0 * ip0;   // 1/rho = R T0/p0
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    R c0 = R(0), cpert = R(0), advu = R(0);
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const R s0 = b.D[1 + i][j] + b.D[1 + j][i];   // 2 s0_ij
      const R s1 = v.D[1 + i][j] + v.D[1 + j][i];   // 2 s'_ij
      c0 += b.D[ND + 2][j] * s0;
      cpert += v.D[ND + 2][j] * s0 + b.D[ND + 2][j] * s1;
      advu += v.q[1 + j] * b.D[1 + i][j] + b.q[1 + j] * v.D[1 + i][j];
    }
    const R visc0 = b.Lu[i] + b.G[i] * R(1.0 / 3.0);
    const R viscp = v.Lu[i] + v.G[i] * R(1.0 / 3.0);
    const R bT0 = c0 - R(2.0 / 3.0) * b.D[ND + 2][i] * th0;
    const R V0 = mu0 * visc0 + muT * bT0;
    const R Vp = muT * Tpr * visc0 + mu0 * viscp + muTT * Tpr * bT0 +
                 muT * (cpert - R(2.0 / 3.0) * (v.D[ND + 2][i] * th0 + b.D[ND + 2][i] * thp));
    out[1 + i] = -advu + (Vp - v.D[0][i]) * irho - rhop * (V0 - b.D[0][i]) * irho * irho;
  }

  // entropy
  R advs = R(0);
#pragma unroll
  for (int j = 0; j < ND; ++j) advs += v.q[1 + j] * b.D[ND + 1][j] + b.q[1 + j] * v.D[ND + 1][j];
  const R irT = R(op.R) * ip0;   // 1/(rho T0), since rho T0 = p0/R
  out[ND + 1] = -advs + Hp * irT - H0 * (rhop * T0 + rho * Tpr) * (irT * irT);
}


// Base thermodynamics at the point (T0 from the stored field) and the algebra.
template <typename R, int ND>
__device__ __forceinline__ void tangent_point(const Pt<R, ND>& b, const Pt<R, ND>& v, const OpParams& op,
                                              R out[ND + 2]) {
  const R T0 = b.q[ND + 2];
  const R S = R(op.suth);
  const R iT = R(1) / T0;
  const R iTS = R(1) / (T0 + S);
  const R ip0 = R(1) / b.q[0];
  const R rho = b.q[0] * iT * R(1.0 / op.R);
  const R mu0 = R(op.mu_ref) * T0 * sqrt(T0) * (R(1) + S) * iTS;
  const R f1 = R(1.5) * iT - iTS;
  const R muT = mu0 * f1;
  const R muTT = muT * f1 + mu0 * (R(-1.5) * iT * iT + iTS * iTS);
  tangent<R, ND>(b, v, op, rho, ip0, mu0, muT, muTT, out);
}

}  // namespace sa
