// Gas-kinetic BGK flux at one face Gauss point (Pan & Xu, Sec. 3), written
// for one GPU lane.  Templated on the arithmetic type T (double or float).
//
// Everything is in the local frame of the Gauss point: u along the face
// normal n_x, v along n_y, w along n_z.  A Maxwellian with density rho,
// velocity (U, V, W) and lambda = rho / (2 p) has the one-dimensional
// moments
//   <u^0> = 1, <u^1> = U, <u^{k+1}> = U <u^k> + k/(2 lambda) <u^{k-1}>
// (likewise v, w), the internal-energy moments <xi^2> = K/(2 lambda),
// <xi^4> = K (K+2) / (4 lambda^2), K = (5 - 3 gamma)/(gamma - 1), and the
// half-line moments over u > 0 (u < 0) start from (1/2) erfc(-+ sqrt(lambda) U)
// and U <u^0> +- exp(-lambda U^2) / (2 sqrt(pi lambda)) with the same
// recurrence.
//
// The flux of Eq. (15), read with H(u) on the left state g_l and 1 - H(u) on
// the right state g_r (the compatibility condition that follows the equation
// takes u > 0 from the left), integrated over [0, delta]:
//   Fhat(delta) = T1 <u psi>_0 + T2 <u (abar.u) psi>_0 + T3 <u Abar psi>_0
//               + T4 (<u psi>_{l,u>0} + <u psi>_{r,u<0})
//               - T5 (<u (a^l.u) psi>_{l,u>0} + <u (a^r.u) psi>_{r,u<0})
//               - tau T4 (<u A^l psi>_{l,u>0} + <u A^r psi>_{r,u<0})
// where a.u = a_1 u + a_2 v + a_3 w with each a_j a polynomial
// a_j1 + a_j2 u + a_j3 v + a_j4 w + a_j5 (u^2+v^2+w^2+xi^2)/2 (the
// micro-slopes), T1..T5 the time integrals of the five time factors of
// Eq. (15).  F and dF/dt come from the linear-in-time fit of Eq. (16) to
// Fhat(dt) and Fhat(dt/2): F = (4 Fhat(dt/2) - Fhat(dt)) / dt and
// dF = 4 (Fhat(dt) - 2 Fhat(dt/2)) / dt^2, applied term by term.
#pragma once

#include "common.h"

namespace hgks {

// Constants of the gas and of the collision time, in the arithmetic type.
template <typename T>
struct GasParams {
  T gm1;      // gamma - 1
  T K;        // internal degrees of freedom
  T K3;       // K + 3
  T KK2;      // K (K + 2)
  T mu;       // viscosity (0: inviscid collision time)
  T tau_eps, tau_C;
  int viscous;
};

// One-dimensional moments of a normalised Maxwellian.
template <typename T>
struct Maxw {
  T u[7];  // <u^0..u^6>, full line or a half line
  T v[6];  // <v^0..v^5>
  T w[6];  // <w^0..w^5>
  T x[3];  // <xi^0>, <xi^2>, <xi^4>
};

template <int N, typename T>
__device__ __forceinline__ void gauss_line(T U, T h, T (&m)[N]) {
  // h = 1 / (2 lambda)
  m[0] = T(1);
  m[1] = U;
#pragma unroll
  for (int k = 1; k < N - 1; ++k) m[k + 1] = U * m[k] + T(k) * h * m[k - 1];
}

// Half-line u-moments; SIDE = +1: u > 0, SIDE = -1: u < 0.
template <int SIDE, typename T>
__device__ __forceinline__ void half_line(T U, T lam, T h, T (&m)[7]) {
  const T sl = d_sqrt(lam);
  const T inv_sqrt_pi = T(0.56418958354775628694807945156077259);
  m[0] = T(0.5) * d_erfc(T(-SIDE) * sl * U);
  m[1] = U * m[0] + T(SIDE) * T(0.5) * inv_sqrt_pi * d_exp(-lam * U * U) / sl;
#pragma unroll
  for (int k = 1; k < 6; ++k) m[k + 1] = U * m[k] + T(k) * h * m[k - 1];
}

template <typename T>
__device__ __forceinline__ void full_maxwellian(Maxw<T>& M, T U, T V, T W, T h, const GasParams<T>& g) {
  gauss_line(U, h, M.u);
  gauss_line(V, h, M.v);
  gauss_line(W, h, M.w);
  M.x[0] = T(1);
  M.x[1] = g.K * h;
  M.x[2] = g.KK2 * h * h;
}

#define HGKS_E(p, q, r, s) (M.u[p] * M.v[q] * M.w[r] * M.x[s])
#define HGKS_E5(p, q, r) \
  (T(0.5) * (HGKS_E((p) + 2, q, r, 0) + HGKS_E(p, (q) + 2, r, 0) + HGKS_E(p, q, (r) + 2, 0) + HGKS_E(p, q, r, 1)))
#define HGKS_E55(p, q, r)                                                                  \
  (T(0.25) * (HGKS_E((p) + 4, q, r, 0) + HGKS_E(p, (q) + 4, r, 0) + HGKS_E(p, q, (r) + 4, 0) + \
              HGKS_E(p, q, r, 2) +                                                         \
              T(2) * (HGKS_E((p) + 2, (q) + 2, r, 0) + HGKS_E((p) + 2, q, (r) + 2, 0) +      \
                      HGKS_E(p, (q) + 2, (r) + 2, 0) + HGKS_E((p) + 2, q, r, 1) +           \
                      HGKS_E(p, (q) + 2, r, 1) + HGKS_E(p, q, (r) + 2, 1))))

// out = < u^EU v^EV w^EW psi >
template <int EU, int EV, int EW, typename T>
__device__ __forceinline__ void psi_mom(const Maxw<T>& M, T (&out)[5]) {
  out[0] = HGKS_E(EU, EV, EW, 0);
  out[1] = HGKS_E(EU + 1, EV, EW, 0);
  out[2] = HGKS_E(EU, EV + 1, EW, 0);
  out[3] = HGKS_E(EU, EV, EW + 1, 0);
  out[4] = HGKS_E5(EU, EV, EW);
}

// out (+)= < u^EU v^EV w^EW (a . psi) psi >
template <int EU, int EV, int EW, bool ACC, typename T>
__device__ __forceinline__ void apsi(const Maxw<T>& M, const T (&a)[5], T (&out)[5]) {
  const T m0 = HGKS_E(EU, EV, EW, 0);
  const T mu = HGKS_E(EU + 1, EV, EW, 0), mv = HGKS_E(EU, EV + 1, EW, 0), mw = HGKS_E(EU, EV, EW + 1, 0);
  const T muu = HGKS_E(EU + 2, EV, EW, 0), mvv = HGKS_E(EU, EV + 2, EW, 0), mww = HGKS_E(EU, EV, EW + 2, 0);
  const T muv = HGKS_E(EU + 1, EV + 1, EW, 0), muw = HGKS_E(EU + 1, EV, EW + 1, 0);
  const T mvw = HGKS_E(EU, EV + 1, EW + 1, 0);
  const T e5 = HGKS_E5(EU, EV, EW);
  const T e5u = HGKS_E5(EU + 1, EV, EW), e5v = HGKS_E5(EU, EV + 1, EW), e5w = HGKS_E5(EU, EV, EW + 1);
  const T e55 = HGKS_E55(EU, EV, EW);
  T r0 = a[0] * m0 + a[1] * mu + a[2] * mv + a[3] * mw + a[4] * e5;
  T r1 = a[0] * mu + a[1] * muu + a[2] * muv + a[3] * muw + a[4] * e5u;
  T r2 = a[0] * mv + a[1] * muv + a[2] * mvv + a[3] * mvw + a[4] * e5v;
  T r3 = a[0] * mw + a[1] * muw + a[2] * mvw + a[3] * mww + a[4] * e5w;
  T r4 = a[0] * e5 + a[1] * e5u + a[2] * e5v + a[3] * e5w + a[4] * e55;
  if (ACC) {
    out[0] += r0; out[1] += r1; out[2] += r2; out[3] += r3; out[4] += r4;
  } else {
    out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3; out[4] = r4;
  }
}
#undef HGKS_E
#undef HGKS_E5
#undef HGKS_E55

// Micro-slope: the a with <a psi> = b for the Maxwellian (U, V, W, lambda),
// b already divided by rho.  Closed-form inverse of the 5x5 moment matrix
// with q = U^2 + V^2 + W^2 + (K+3)/(2 lambda), h = 1/(2 lambda).
template <typename T>
__device__ __forceinline__ void micro_slope(const T (&b)[5], T U, T V, T W, T h, T q, T K3, T (&a)[5]) {
  const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = b[3] - W * b[0];
  const T R5 = T(2) * b[4] - q * b[0];
  const T il = T(1) / h;  // 2 lambda
  a[4] = (R5 - T(2) * (U * R2 + V * R3 + W * R4)) / (K3 * h * h);
  a[3] = il * R4 - W * a[4];
  a[2] = il * R3 - V * a[4];
  a[1] = il * R2 - U * a[4];
  a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - T(0.5) * a[4] * q;
}

// Running sums over the two sides of the interface.
template <typename T>
struct FluxAcc {
  T Q0[5];
  T dQ0[3][5];
  T X4[5], X5[5], X6[5];
  T p[2];
};

template <typename T>
__device__ __forceinline__ void acc_zero(FluxAcc<T>& A) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    A.Q0[i] = T(0); A.X4[i] = T(0); A.X5[i] = T(0); A.X6[i] = T(0);
    A.dQ0[0][i] = T(0); A.dQ0[1][i] = T(0); A.dQ0[2][i] = T(0);
  }
}

template <typename T>
__device__ __forceinline__ void axpy5(T s, const T (&x)[5], T (&y)[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) y[i] += s * x[i];
}

// Contributions of one side (SIDE = +1: left state, particles with u > 0;
// SIDE = -1: right state, u < 0).  W: conservative variables in the local
// frame; dW[j]: their derivatives along n_x, n_y, n_z.
template <int SIDE, typename T>
__device__ __forceinline__ void side_terms(const T (&W)[5], const T (&dW)[3][5], const GasParams<T>& g,
                                           FluxAcc<T>& A) {
  const T rho = W[0];
  const T ir = T(1) / rho;
  const T U = W[1] * ir, V = W[2] * ir, Wv = W[3] * ir;
  const T p = g.gm1 * (W[4] - T(0.5) * rho * (U * U + V * V + Wv * Wv));
  const T h = p * ir;                // 1 / (2 lambda)
  const T lam = T(0.5) / h;
  const T q = U * U + V * V + Wv * Wv + g.K3 * h;
  Maxw<T> M;
  full_maxwellian(M, U, V, Wv, h, g);

  T a[3][5];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) b[i] = dW[j][i] * ir;
    micro_slope(b, U, V, Wv, h, q, g.K3, a[j]);
  }
  // <a_1 u + a_2 v + a_3 w + A> = 0
  T t[5];
  apsi<1, 0, 0, false>(M, a[0], t);
  apsi<0, 1, 0, true>(M, a[1], t);
  apsi<0, 0, 1, true>(M, a[2], t);
#pragma unroll
  for (int i = 0; i < 5; ++i) t[i] = -t[i];
  T Acoef[5];
  micro_slope(t, U, V, Wv, h, q, g.K3, Acoef);

  half_line<SIDE>(U, lam, h, M.u);
  T m[5];
  psi_mom<0, 0, 0>(M, m);
  axpy5(rho, m, A.Q0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    apsi<0, 0, 0, false>(M, a[j], m);
    axpy5(rho, m, A.dQ0[j]);
  }
  psi_mom<1, 0, 0>(M, m);
  axpy5(rho, m, A.X4);
  apsi<2, 0, 0, false>(M, a[0], m);
  apsi<1, 1, 0, true>(M, a[1], m);
  apsi<1, 0, 1, true>(M, a[2], m);
  axpy5(rho, m, A.X5);
  apsi<1, 0, 0, false>(M, Acoef, m);
  axpy5(rho, m, A.X6);
  A.p[SIDE > 0 ? 0 : 1] = p;
}

// Time integrals over [0, delta] of the five time factors of Eq. (15).
template <typename T>
__device__ __forceinline__ void time_integrals(T delta, T tau, T (&Tc)[5]) {
  const T E = d_exp(-delta / tau);
  const T om = T(1) - E;
  Tc[0] = delta - tau * om;
  Tc[1] = T(2) * tau * tau * om - tau * delta * (T(1) + E);
  Tc[2] = T(0.5) * delta * delta - tau * delta + tau * tau * om;
  Tc[3] = tau * om;
  Tc[4] = T(2) * tau * tau * om - tau * delta * E;
}

// Equilibrium part, collision time and the time fit.  On return F and dF
// hold the flux and its time derivative in the local frame and Q0 the
// conservative variables of g_0.
template <typename T>
__device__ __forceinline__ void finish_flux(FluxAcc<T>& A, const GasParams<T>& g, T dt, T (&F)[5],
                                            T (&dF)[5]) {
  const T r0 = A.Q0[0];
  const T ir0 = T(1) / r0;
  const T U = A.Q0[1] * ir0, V = A.Q0[2] * ir0, W = A.Q0[3] * ir0;
  const T p0 = g.gm1 * (A.Q0[4] - T(0.5) * r0 * (U * U + V * V + W * W));
  const T h = p0 * ir0;
  const T q = U * U + V * V + W * W + g.K3 * h;
  Maxw<T> M;
  full_maxwellian(M, U, V, W, h, g);

  T ab[3][5];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) b[i] = A.dQ0[j][i] * ir0;
    micro_slope(b, U, V, W, h, q, g.K3, ab[j]);
  }
  T t[5];
  apsi<1, 0, 0, false>(M, ab[0], t);
  apsi<0, 1, 0, true>(M, ab[1], t);
  apsi<0, 0, 1, true>(M, ab[2], t);
#pragma unroll
  for (int i = 0; i < 5; ++i) t[i] = -t[i];
  T Ab[5];
  micro_slope(t, U, V, W, h, q, g.K3, Ab);

  T X1[5], X2[5], X3[5];
  psi_mom<1, 0, 0>(M, X1);
  apsi<2, 0, 0, false>(M, ab[0], X2);
  apsi<1, 1, 0, true>(M, ab[1], X2);
  apsi<1, 0, 1, true>(M, ab[2], X2);
  apsi<1, 0, 0, false>(M, Ab, X3);

  const T jump = d_abs((A.p[0] - A.p[1]) / (A.p[0] + A.p[1])) * dt;
  const T tau = g.viscous ? g.mu / p0 + g.tau_C * jump : g.tau_eps * dt + g.tau_C * jump;

  T Tf[5], Th[5];
  time_integrals(dt, tau, Tf);
  time_integrals(T(0.5) * dt, tau, Th);
  const T idt = T(1) / dt;
  const T idt2 = T(4) * idt * idt;
  T c[5], d[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    c[i] = (T(4) * Th[i] - Tf[i]) * idt;
    d[i] = (Tf[i] - T(2) * Th[i]) * idt2;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const T e1 = r0 * X1[i], e2 = r0 * X2[i], e3 = r0 * X3[i];
    F[i] = c[0] * e1 + c[1] * e2 + c[2] * e3 + c[3] * A.X4[i] - c[4] * A.X5[i] - tau * c[3] * A.X6[i];
    dF[i] = d[0] * e1 + d[1] * e2 + d[2] * e3 + d[3] * A.X4[i] - d[4] * A.X5[i] - tau * d[3] * A.X6[i];
  }
}

}  // namespace hgks
