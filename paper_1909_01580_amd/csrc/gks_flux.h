// Gas-kinetic BGK flux at one face Gauss point (Pan & Xu, Sec. 3), written
// for one GPU lane.  Templated on the arithmetic type T (double or float).
//
// Everything is in the local frame of the Gauss point: u along the face
// normal n_x, v along n_y, w along n_z.  A Maxwellian with density rho,
// velocity (U, V, W) and lambda = rho / (2 p) is normalised to unit mass;
// h = 1/(2 lambda) = p / rho and K = (5 - 3 gamma)/(gamma - 1).
//
// Moments against psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2).  Only the
// normal velocity u is ever integrated over a half line, so the tangential
// and internal velocities are integrated out analytically.  With the
// peculiar velocities c = v - V, d = w - W (Gaussian, variance h) and
// e = (v^2 + w^2 + xi^2)/2 with mean ebar = (V^2 + W^2 + (K+2) h)/2 and
// variance se = (V^2 + W^2) h + (K+2) h^2 / 2, a micro-slope
// a.psi = a1 + a2 u + a3 v + a4 w + a5 (u^2/2 + e) has the tangential mean
// alpha(u) = (a1 + a3 V + a4 W + a5 ebar) + a2 u + (a5/2) u^2, and
//   E_t[a.psi]                  = alpha
//   E_t[(a.psi) v]              = V alpha + t3,     t3 = h (a3 + a5 V)
//   E_t[(a.psi) w]              = W alpha + t4,     t4 = h (a4 + a5 W)
//   E_t[(a.psi) e]              = ebar alpha + s5,  s5 = h (a3 V + a4 W) + a5 se
//   E_t[(a.psi) v v]            = (V^2 + h) alpha + 2 V t3 + a5 h^2
//   E_t[(a.psi) v w]            = V W alpha + V t4 + W t3
//   E_t[(a.psi) v e]            = ebar (V alpha + t3) + V h alpha + C5v,
//     C5v = V h (a3 V + a4 W) + a5 V (se + 2 h^2) + a3 h^2   (w: V <-> W, a3 <-> a4)
// so every moment <u^k (a.psi) psi>, <u^k v (a.psi) psi>, <u^k w (a.psi) psi>
// is a short combination of G_n = <u^n alpha(u)> and of the u-moments m_n,
// full line or half line.  The u-moments obey
//   m_0 = 1, m_1 = U, m_{k+1} = U m_k + k h m_{k-1}
// on the full line, and over u > 0 (u < 0) start from
//   m_0 = erfc(-+ sqrt(lambda) U)/2, m_1 = U m_0 +- exp(-lambda U^2)/(2 sqrt(pi lambda)).
//
// The flux of Eq. (15), read with H(u) on the left state g_l and 1 - H(u) on
// the right state g_r (the compatibility condition that follows the equation
// takes u > 0 from the left), integrated over [0, delta]:
//   Fhat(delta) = T1 <u psi>_0 + T2 <u (abar.u) psi>_0 + T3 <u Abar psi>_0
//               + T4 (<u psi>_{l,u>0} + <u psi>_{r,u<0})
//               - T5 (<u (a^l.u) psi>_{l,u>0} + <u (a^r.u) psi>_{r,u<0})
//               - tau T4 (<u A^l psi>_{l,u>0} + <u A^r psi>_{r,u<0})
// where a.u = (a_1.psi) u + (a_2.psi) v + (a_3.psi) w for the micro-slopes
// a_j along n_x, n_y, n_z, and T1..T5 are the time integrals of the five
// time factors of Eq. (15).  F and dF/dt come from the linear-in-time fit of
// Eq. (16) to Fhat(dt) and Fhat(dt/2): F = (4 Fhat(dt/2) - Fhat(dt)) / dt,
// dF = 4 (Fhat(dt) - 2 Fhat(dt/2)) / dt^2, applied term by term.
#pragma once

#include "common.h"

namespace hgks {

// Constants of the gas and of the collision time, in the arithmetic type.
template <typename T>
struct GasParams {
  T gm1;      // gamma - 1
  T K;        // internal degrees of freedom
  T K2;       // K + 2
  T K3;       // K + 3
  T inv_K3;   // 1 / (K + 3)
  T two_gm1;  // 2 / (gamma - 1)
  T mu;       // viscosity (0: inviscid collision time)
  T tau_eps, tau_C;
  int viscous;
  T mu_exp;   // viscosity law mu (T / T0)^mu_exp on the viscous branch (0: constant)
  T mu_iT0;   // 1 / T0
  T pr_fix;   // 1 / Pr - 1: weight of the heat flux added to the energy flux
  double gamma;  // ratio of specific heats (characteristic projection)
};

// Gaussian moments of the tangential and internal velocities of one state.
template <typename T>
struct Tang {
  T V, W, h, e, se;
};

template <typename T>
HGKS_FN void tang_init(Tang<T>& t, T V, T W, T h, const GasParams<T>& g) {
  t.V = V;
  t.W = W;
  t.h = h;
  const T vw = V * V + W * W;
  t.e = T(0.5) * (vw + g.K2 * h);
  t.se = vw * h + T(0.5) * g.K2 * h * h;
}

template <typename T>
HGKS_FN void full_line(T U, T h, T (&m)[7]) {
  m[0] = T(1);
  m[1] = U;
#pragma unroll
  for (int k = 1; k < 6; ++k) m[k + 1] = U * m[k] + T(k) * h * m[k - 1];
}

// Half-line u-moments; sg = +1: u > 0, sg = -1: u < 0.  il = 2 lambda
// = 1/h; 1/sqrt(lambda) = 2 h sqrt(lambda), so no division is needed.
template <typename T>
HGKS_FN void half_line_s(T U, T h, T il, T sg, T (&m)[7]) {
  const T lam = T(0.5) * il;
  const T sl = d_sqrt(lam);
  const T inv_sqrt_pi = T(0.56418958354775628694807945156077259);
  m[0] = T(0.5) * d_erfc(-sg * sl * U);
  m[1] = U * m[0] + sg * inv_sqrt_pi * h * sl * d_exp(-lam * U * U);
#pragma unroll
  for (int k = 1; k < 6; ++k) m[k + 1] = U * m[k] + T(k) * h * m[k - 1];
}

template <int SIDE, typename T>
HGKS_FN void half_line(T U, T h, T il, T (&m)[7]) {
  half_line_s(U, h, il, T(SIDE), m);
}

// A micro-slope prepared for moments: tangential mean alpha(u) = c0 + a2 u +
// h5 u^2 and the constants of the expectations listed above.
template <typename T>
struct Slope {
  T c0, a2, h5;  // alpha(u)
  T a5;
  T t3, t4, s5;
  T c5v, c5w;  // only for the v / w multiplied moments
};

template <typename T>
HGKS_FN void slope_prep(const T (&a)[5], const Tang<T>& t, Slope<T>& s) {
  const T avw = a[2] * t.V + a[3] * t.W;
  s.c0 = a[0] + avw + a[4] * t.e;
  s.a2 = a[1];
  s.h5 = T(0.5) * a[4];
  s.a5 = a[4];
  s.t3 = t.h * (a[2] + a[4] * t.V);
  s.t4 = t.h * (a[3] + a[4] * t.W);
  s.s5 = t.h * avw + a[4] * t.se;
  const T hh = t.h * t.h;
  const T q = t.h * avw + a[4] * (t.se + T(2) * hh);
  s.c5v = t.V * q + a[2] * hh;
  s.c5w = t.W * q + a[3] * hh;
}

template <int N, typename T>
HGKS_FN T Gn(const Slope<T>& s, const T (&m)[7]) {
  return s.c0 * m[N] + s.a2 * m[N + 1] + s.h5 * m[N + 2];
}

template <bool ACC, typename T>
HGKS_FN void put5(T (&out)[5], T r0, T r1, T r2, T r3, T r4) {
  if (ACC) {
    out[0] += r0; out[1] += r1; out[2] += r2; out[3] += r3; out[4] += r4;
  } else {
    out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3; out[4] = r4;
  }
}

// out (+)= < u^k (a.psi) psi >
template <int k, bool ACC, typename T>
HGKS_FN void mom_a(const Slope<T>& s, const Tang<T>& t, const T (&m)[7], T (&out)[5]) {
  const T g0 = Gn<k>(s, m), g1 = Gn<k + 1>(s, m), g2 = Gn<k + 2>(s, m);
  const T r0 = g0, r1 = g1;
  const T r2 = t.V * g0 + s.t3 * m[k];
  const T r3 = t.W * g0 + s.t4 * m[k];
  const T r4 = T(0.5) * g2 + t.e * g0 + s.s5 * m[k];
  put5<ACC>(out, r0, r1, r2, r3, r4);
}

// out (+)= < u^k v (a.psi) psi >
template <int k, bool ACC, typename T>
HGKS_FN void mom_av(const Slope<T>& s, const Tang<T>& t, const T (&m)[7], T (&out)[5]) {
  const T g0 = Gn<k>(s, m), g1 = Gn<k + 1>(s, m), g2 = Gn<k + 2>(s, m);
  const T A0 = t.V * g0 + s.t3 * m[k];
  put5<ACC>(out, A0, t.V * g1 + s.t3 * m[k + 1],
            (t.V * t.V + t.h) * g0 + (T(2) * t.V * s.t3 + s.a5 * t.h * t.h) * m[k],
            t.V * t.W * g0 + (t.W * s.t3 + t.V * s.t4) * m[k],
            T(0.5) * (t.V * g2 + s.t3 * m[k + 2]) + t.e * A0 + t.V * t.h * g0 + s.c5v * m[k]);
}

// out (+)= < u^k w (a.psi) psi >
template <int k, bool ACC, typename T>
HGKS_FN void mom_aw(const Slope<T>& s, const Tang<T>& t, const T (&m)[7], T (&out)[5]) {
  const T g0 = Gn<k>(s, m), g1 = Gn<k + 1>(s, m), g2 = Gn<k + 2>(s, m);
  const T B0 = t.W * g0 + s.t4 * m[k];
  put5<ACC>(out, B0, t.W * g1 + s.t4 * m[k + 1],
            t.V * t.W * g0 + (t.V * s.t4 + t.W * s.t3) * m[k],
            (t.W * t.W + t.h) * g0 + (T(2) * t.W * s.t4 + s.a5 * t.h * t.h) * m[k],
            T(0.5) * (t.W * g2 + s.t4 * m[k + 2]) + t.e * B0 + t.W * t.h * g0 + s.c5w * m[k]);
}

// out = < u^k psi >
template <int k, typename T>
HGKS_FN void mom_psi(const Tang<T>& t, const T (&m)[7], T (&out)[5]) {
  out[0] = m[k];
  out[1] = m[k + 1];
  out[2] = t.V * m[k];
  out[3] = t.W * m[k];
  out[4] = T(0.5) * m[k + 2] + t.e * m[k];
}

// Micro-slope: the a with <a psi> = b for the unit-mass Maxwellian
// (U, V, W, lambda).  Closed-form inverse of the 5x5 moment matrix with
// q = U^2 + V^2 + W^2 + (K+3)/(2 lambda), il = 2 lambda and
// c5 = 4 lambda^2 / (K + 3).  The map is linear in b; the callers pass the
// derivatives of the conservative variables themselves (not divided by
// rho), so the result is rho times the micro-slope of Eq. (8) and every
// moment taken with it carries that factor rho.
template <typename T>
HGKS_FN void micro_slope(const T (&b)[5], T U, T V, T W, T il, T q, T c5, T (&a)[5]) {
  const T R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = b[3] - W * b[0];
  const T R5 = T(2) * b[4] - q * b[0];
  a[4] = c5 * (R5 - T(2) * (U * R2 + V * R3 + W * R4));
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
  // Prandtl correction only: the state moments of the slope and time
  // derivative terms of the initial distribution (X5, X6 without the
  // factor u), which the heat flux needs.
  T S5[5], S6[5];
};

// How the first side of a face enters the sums: assigned (true) or added to
// zeroed sums (false).  The values are the same; assigning issues about 35
// fewer adds and 45 fewer register clears per Gauss point.  Measured on
// gfx950 it shortens the FP64 flux launch by about 1% but lengthens the FP32
// one by about 3% (the compiler's schedule of the mixed kernel loses more
// than the instructions save), so the choice is per precision.
template <typename T>
inline constexpr bool kAssignFirst = sizeof(T) == 8;

template <typename T>
HGKS_FN void acc_zero(FluxAcc<T>& A) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    A.Q0[i] = T(0); A.X4[i] = T(0); A.X5[i] = T(0); A.X6[i] = T(0);
    A.dQ0[0][i] = T(0); A.dQ0[1][i] = T(0); A.dQ0[2][i] = T(0);
    A.S5[i] = T(0); A.S6[i] = T(0);
  }
}

// Ready the sums for the first side of a face: zeroed unless that side
// assigns them.
template <typename T>
HGKS_FN void acc_begin(FluxAcc<T>& A) {
  if constexpr (!kAssignFirst<T>) acc_zero(A);
}

// y (+)= s x
template <bool ACC = true, typename T>
HGKS_FN void axpy5(T s, const T (&x)[5], T (&y)[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) y[i] = ACC ? y[i] + s * x[i] : s * x[i];
}

// Primitive quantities of a state with conservative variables Q, from one
// reciprocal: with p2 = 2 rho E - |M|^2 = 2 rho p / (gamma - 1) and
// R = 1 / (rho p2), 1/rho = p2 R and 2 lambda = rho/p = (2/(gamma-1)) rho^2/p2.
template <typename T>
struct Prim {
  T rho, ir, U, V, W, p, h, il, q, c5;
};

template <typename T>
HGKS_FN void primitives(const T (&Q)[5], const GasParams<T>& g, Prim<T>& s) {
  const T rho = Q[0];
  const T p2 = T(2) * rho * Q[4] - (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]);
  const T R = d_rcp(rho * p2);
  const T ir = p2 * R;
  s.rho = rho;
  s.ir = ir;
  s.U = Q[1] * ir;
  s.V = Q[2] * ir;
  s.W = Q[3] * ir;
  s.p = T(0.5) * g.gm1 * p2 * ir;
  s.h = s.p * ir;                            // 1 / (2 lambda)
  s.il = g.two_gm1 * (rho * rho) * (rho * R);  // 2 lambda
  s.q = s.U * s.U + s.V * s.V + s.W * s.W + g.K3 * s.h;
  s.c5 = s.il * s.il * g.inv_K3;             // 4 lambda^2 / (K + 3)
}

// Contributions of one side (sg = +1: left state, particles with u > 0;
// sg = -1: right state, u < 0; sg may be a runtime value).  W: conservative
// variables in the local frame; dW[j]: their derivatives along n_x, n_y,
// n_z.  The three micro-slopes are formed and consumed one at a time, so
// that only one is live: each adds its full-line term to the compatibility
// residual (which gives A) and its half-line terms to dQ0[j] and X5.  The
// side's pressure goes to pside.  FIRST: the first side of the pair, whose
// terms are assigned to the sums rather than added to zeroed ones (the same
// values; an add to 0.0 cannot be dropped by the compiler, whereas here
// no zeroing or add is issued).
template <bool PR = false, bool FIRST = false, typename T>
HGKS_FN void side_terms_s(const T (&W)[5], const T (&dW)[3][5], const GasParams<T>& g, T sg, FluxAcc<T>& A,
                          T& pside) {
  constexpr bool ACC = !FIRST;
  Prim<T> P;
  primitives(W, g, P);
  const T rho = P.rho, U = P.U, V = P.V, Wv = P.W, p = P.p, h = P.h, il = P.il, q = P.q, c5 = P.c5;
  Tang<T> t;
  tang_init(t, V, Wv, h, g);
  T mf[7], mh[7];
  full_line(U, h, mf);
  half_line_s(U, h, il, sg, mh);

  // r = rho <(a_1 u + a_2 v + a_3 w) psi>, then A from <(a.u + A) psi> = 0.
  T r[5];
  {
    T a[5];
    Slope<T> s;
    micro_slope(dW[0], U, V, Wv, il, q, c5, a);
    slope_prep(a, t, s);
    mom_a<1, false>(s, t, mf, r);
    mom_a<0, ACC>(s, t, mh, A.dQ0[0]);
    mom_a<2, ACC>(s, t, mh, A.X5);
    if constexpr (PR) mom_a<1, ACC>(s, t, mh, A.S5);
  }
  {
    T a[5];
    Slope<T> s;
    micro_slope(dW[1], U, V, Wv, il, q, c5, a);
    slope_prep(a, t, s);
    mom_av<0, true>(s, t, mf, r);
    mom_a<0, ACC>(s, t, mh, A.dQ0[1]);
    mom_av<1, true>(s, t, mh, A.X5);
    if constexpr (PR) mom_av<0, true>(s, t, mh, A.S5);
  }
  {
    T a[5];
    Slope<T> s;
    micro_slope(dW[2], U, V, Wv, il, q, c5, a);
    slope_prep(a, t, s);
    mom_aw<0, true>(s, t, mf, r);
    mom_a<0, ACC>(s, t, mh, A.dQ0[2]);
    mom_aw<1, true>(s, t, mh, A.X5);
    if constexpr (PR) mom_aw<0, true>(s, t, mh, A.S5);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) r[i] = -r[i];
  {
    T a[5];
    Slope<T> s;
    micro_slope(r, U, V, Wv, il, q, c5, a);
    slope_prep(a, t, s);
    mom_a<1, ACC>(s, t, mh, A.X6);
    if constexpr (PR) mom_a<0, ACC>(s, t, mh, A.S6);
  }
  T v5[5];
  mom_psi<0>(t, mh, v5);
  axpy5<ACC>(rho, v5, A.Q0);
  mom_psi<1>(t, mh, v5);
  axpy5<ACC>(rho, v5, A.X4);
  pside = p;
}

template <int SIDE, bool PR = false, bool FIRST = false, typename T>
HGKS_FN void side_terms(const T (&W)[5], const T (&dW)[3][5], const GasParams<T>& g, FluxAcc<T>& A) {
  side_terms_s<PR, FIRST>(W, dW, g, T(SIDE), A, A.p[SIDE > 0 ? 0 : 1]);
}

// Register budget of the flux kernels: at least two waves per SIMD in FP64
// (three in FP32), so that one wave's memory and transcendental latency
// hides behind another's arithmetic.  Left to itself the compiler would
// keep one FP64 wave per SIMD (over 256 registers); a third FP64 wave does
// not fit without spilling the left side's sums.
#define HGKS_FLUX_OCCUPANCY __attribute__((amdgpu_waves_per_eu(sizeof(TC) == 8 ? 2 : 3)))

// Orders the loads of the right cell after the left side's terms.  The
// address gets a dependence on the left side's last results through an
// empty asm, so the compiler cannot hoist the right cell's coefficient
// loads into the left side's work, where both sides' values would be live
// at once.
template <typename T>
__device__ __forceinline__ void after_left_side(size_t& idx, const FluxAcc<T>& A) {
  asm volatile("" : "+v"(idx) : "v"(A.X6[0]), "v"(A.X6[4]), "v"(A.Q0[4]), "v"(A.X4[4]));
}

// Time integrals over [0, delta] of the five time factors of Eq. (15);
// E = exp(-delta / tau).
template <typename T>
HGKS_FN void time_integrals(T delta, T tau, T E, T (&Tc)[5]) {
  const T om = T(1) - E;
  Tc[0] = delta - tau * om;
  Tc[1] = T(2) * tau * tau * om - tau * delta * (T(1) + E);
  Tc[2] = T(0.5) * delta * delta - tau * delta + tau * tau * om;
  Tc[3] = tau * om;
  Tc[4] = T(2) * tau * tau * om - tau * delta * E;
}

// The state of g_0 and the coefficients of the time fit: everything the
// moments of the equilibrium part and the folding into F and dF need.
template <typename T>
struct EqState {
  T r0, U, V, W, h, il, q, c5, tau;
  T c[5], d[5];  // F- and dF-coefficients of the five time integrals
  Tang<T> t;
  T m[7];        // full-line u-moments of g_0
};

// Collision time and the time fit from the summed accumulators (A.Q0 the
// conservative variables of g_0, A.p the two sides' pressures).
// PR: the extended viscous model -- the viscosity law and the Prandtl
// correction (either may be trivial: mu_exp = 0, pr_fix = 0).
template <bool PR = false, typename T>
HGKS_FN void eq_state(const FluxAcc<T>& A, const GasParams<T>& g, T dt, T idt, EqState<T>& e) {
  Prim<T> P;
  primitives(A.Q0, g, P);
  e.r0 = P.rho;
  e.U = P.U;
  e.V = P.V;
  e.W = P.W;
  e.h = P.h;
  e.il = P.il;
  e.q = P.q;
  e.c5 = P.c5;
  const T jump = d_abs(A.p[0] - A.p[1]) * d_rcp(A.p[0] + A.p[1]) * dt;
  // mu / p_0 = mu (rho_0 / p_0) (1 / rho_0); mu = mu0 (T / T0)^omega with
  // T = p_0 / rho_0 when a viscosity law is set
  T mu = g.mu;
  if constexpr (PR) {
    if (g.mu_exp != T(0)) mu *= exp(g.mu_exp * log(P.h * g.mu_iT0));
  }
  e.tau = g.viscous ? mu * P.il * P.ir + g.tau_C * jump : g.tau_eps * dt + g.tau_C * jump;
  const T itau = T(1) / e.tau;
  {
    T Tf[5], Th[5];
    // exp(-dt / tau) as the square of exp(-dt / (2 tau))
    const T Eh = d_exp(T(-0.5) * dt * itau);
    time_integrals(dt, e.tau, Eh * Eh, Tf);
    time_integrals(T(0.5) * dt, e.tau, Eh, Th);
    const T idt2 = T(4) * idt * idt;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      e.c[i] = (T(4) * Th[i] - Tf[i]) * idt;
      e.d[i] = (Tf[i] - T(2) * Th[i]) * idt2;
    }
  }
  tang_init(e.t, e.V, e.W, e.h, g);
  full_line(e.U, e.h, e.m);
}

// Non-equilibrium part (T4, T5 and tau T4 terms) of the sums in A:
// F = c3 X4 - c4 X5 - tau c3 X6 (likewise dF).
template <typename T>
HGKS_FN void fold_noneq(const FluxAcc<T>& A, const EqState<T>& e, T (&F)[5], T (&dF)[5]) {
  const T c6 = e.tau * e.c[3], d6 = e.tau * e.d[3];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    F[i] = e.c[3] * A.X4[i] - e.c[4] * A.X5[i] - c6 * A.X6[i];
    dF[i] = e.d[3] * A.X4[i] - e.d[4] * A.X5[i] - d6 * A.X6[i];
  }
}

// T1 term: rho_0 <u psi>_0.
template <typename T>
HGKS_FN void fold_eq_mean(const EqState<T>& e, T (&F)[5], T (&dF)[5]) {
  T v5[5];
  mom_psi<1>(e.t, e.m, v5);
  const T c0 = e.c[0] * e.r0, d0 = e.d[0] * e.r0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    F[i] += c0 * v5[i];
    dF[i] += d0 * v5[i];
  }
}

// Micro-slope abar_J of g_0 from its moments b = dQ0[J] (carrying rho_0):
// its T2 term into F and dF, its part of the compatibility residual into r
// (assigned when ACC is false).
template <int J, bool ACC, typename T>
HGKS_FN void fold_abar(const EqState<T>& e, const T (&b)[5], T (&r)[5], T (&F)[5], T (&dF)[5]) {
  T a[5];
  Slope<T> s;
  micro_slope(b, e.U, e.V, e.W, e.il, e.q, e.c5, a);
  slope_prep(a, e.t, s);
  T v5[5];
  if constexpr (J == 0) {
    mom_a<1, ACC>(s, e.t, e.m, r);
    mom_a<2, false>(s, e.t, e.m, v5);
  } else if constexpr (J == 1) {
    mom_av<0, ACC>(s, e.t, e.m, r);
    mom_av<1, false>(s, e.t, e.m, v5);
  } else {
    mom_aw<0, ACC>(s, e.t, e.m, r);
    mom_aw<1, false>(s, e.t, e.m, v5);
  }
  axpy5(e.c[1], v5, F);
  axpy5(e.d[1], v5, dF);
}

// Time derivative Abar of g_0 from rA = rho_0 <Abar psi> (minus the
// compatibility residual): its T3 term into F and dF.
template <typename T>
HGKS_FN void fold_Abar(const EqState<T>& e, const T (&rA)[5], T (&F)[5], T (&dF)[5]) {
  T a[5];
  Slope<T> s;
  micro_slope(rA, e.U, e.V, e.W, e.il, e.q, e.c5, a);
  slope_prep(a, e.t, s);
  T v5[5];
  mom_a<1, false>(s, e.t, e.m, v5);
  axpy5(e.c[2], v5, F);
  axpy5(e.d[2], v5, dF);
}

// X_E - U.X_M + u2 X_rho for a moment vector X, the velocity U of g_0 and
// u2 = |U|^2/2: the heat-flux form of the Prandtl correction below.
template <typename T>
HGKS_FN T heat_form(const EqState<T>& e, T u2, const T (&X)[5]) {
  return X[4] - (e.U * X[1] + e.V * X[2] + e.W * X[3]) + u2 * X[0];
}

// Prandtl correction: the heat flux relative to the velocity (U, V, W) of
// g_0 is the moment of (u - U)(|c|^2 + xi^2)/2, which expands into the
// fluxes F and the state moments S of the same distribution:
//   q = F_E - U.F_M + |U|^2/2 F_rho - U (S_E - U.S_M + |U|^2/2 S_rho).
// S over time: g_0's moments Q0 (T1 and T4 terms), rho_0 <Abar psi> = rA
// (T3 - T2) and the initial slopes and time derivatives (-T5 S5,
// -tau T4 S6); fitted with the same coefficients as the flux.
template <typename T>
HGKS_FN void prandtl_fix(const FluxAcc<T>& A, const EqState<T>& e, const T (&rA)[5], const GasParams<T>& g,
                         T (&F)[5], T (&dF)[5]) {
  T S[5], dS[5];
  const T ce = e.c[0] + e.c[3], de = e.d[0] + e.d[3], cr = e.c[2] - e.c[1], dr = e.d[2] - e.d[1];
  const T c6 = e.tau * e.c[3], d6 = e.tau * e.d[3];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    S[i] = ce * A.Q0[i] + cr * rA[i] - e.c[4] * A.S5[i] - c6 * A.S6[i];
    dS[i] = de * A.Q0[i] + dr * rA[i] - e.d[4] * A.S5[i] - d6 * A.S6[i];
  }
  const T u2 = T(0.5) * (e.U * e.U + e.V * e.V + e.W * e.W);
  const T qf = heat_form(e, u2, F) - e.U * heat_form(e, u2, S);
  const T dq = heat_form(e, u2, dF) - e.U * heat_form(e, u2, dS);
  F[4] += g.pr_fix * qf;
  dF[4] += g.pr_fix * dq;
}

// Equilibrium part, collision time and the time fit.  On return F and dF
// hold the flux and its time derivative in the local frame.  The collision
// time and the coefficients of the time fit come first, so that every
// moment is folded into F and dF as soon as it is formed; the micro-slopes
// abar_j of g_0 are formed one at a time.
template <bool PR = false, typename T>
HGKS_FN void finish_flux(const FluxAcc<T>& A, const GasParams<T>& g, T dt, T idt, T (&F)[5], T (&dF)[5]) {
  EqState<T> e;
  eq_state<PR>(A, g, dt, idt, e);
  fold_noneq(A, e, F, dF);
  fold_eq_mean(e, F, dF);
  T r[5];
  fold_abar<0, false>(e, A.dQ0[0], r, F, dF);
  fold_abar<1, true>(e, A.dQ0[1], r, F, dF);
  fold_abar<2, true>(e, A.dQ0[2], r, F, dF);
#pragma unroll
  for (int i = 0; i < 5; ++i) r[i] = -r[i];
  fold_Abar(e, r, F, dF);
  if constexpr (PR) prandtl_fix(A, e, r, g, F, dF);
}

}  // namespace hgks
