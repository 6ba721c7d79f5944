// WENO-AO reconstruction of one conservative variable in one cell of a
// uniform box grid (Pan & Xu, Sec. 2), for one GPU lane.
//
// Coordinates: xi = (x - x_c) / Delta per axis (the unit cube [-1/2, 1/2]^3).
// The least-squares problems of Sec. 2 are invariant under this per-axis
// scaling (the same quadratic / linear polynomial is returned), and on the
// unit cube their normal equations have closed-form solutions:
//   big stencil S (18 neighbours o, differences d_o = Q_o - Q_c):
//     a_d  = (1/10) sum_{o_d != 0} o_d d_o
//     a_de = (1/4)  sum_{o_d o_e != 0} o_d o_e d_o        (d < e)
//     a_dd = (r_d - (2/9)(r_x + r_y + r_z)) / 6,  r_d = sum_{o_d != 0} d_o
//   for P_0 = Q_c + sum a_n (xi^n - mean(xi^n)), mean(xi_d^2) = 1/12;
//   sub-stencil {s_a e_a, s_b e_b, s_a e_a + s_b e_b, s_c e_c} of the axis
//   triple (a, b; c):
//     b_c = s_c d_{s_c e_c},  s_a b_a = (2 d_a - d_b + d_ab)/3,
//     s_b b_b = (2 d_b - d_a + d_ab)/3.
// Smoothness indicators (Eq. (4)) are evaluated in X = (x - x_c)/|Omega|^(1/3):
// with s_d = (|Omega|^(1/3) / Delta_d)^2,
//   beta_m = sum_d s_d b_d^2,
//   beta_0 = sum_d s_d a_d^2 + sum_d (s_d/3 + 4 s_d^2) a_dd^2
//            + sum_{d<e} (s_d s_e + (s_d + s_e)/12) a_de^2
// (on cubes: sum a_d^2 + 13/3 sum a_dd^2 + 7/6 sum a_de^2).
// Weights: tau = mean |beta_0 - beta_m| (Eq. (5)), omega_m = gamma_m
// (1 + tau/(beta_m + eps)) (Eq. (3)), normalised.  The reconstructed
// quadratic of Sec. 2, wbar_0 (P_0/gamma_0 - sum gamma_m/gamma_0 P_m) +
// sum wbar_m P_m, is stored as its nine coefficients in xi:
//   c = (wbar_0/gamma_0) a + sum_m (wbar_m - wbar_0 gamma_m/gamma_0) b^m.
#pragma once

#include "common.h"

namespace hgks {

template <typename T>
struct WenoParams {
  T gamma0, Gamma, eps;
  T kl[3];  // s_d
  T kq[3];  // s_d/3 + 4 s_d^2
  T km[3];  // (x,y), (y,z), (x,z): s_d s_e + (s_d + s_e)/12
};

// Offsets o in {-1,0,1}^3 are stored at index (o_z+1)*9 + (o_y+1)*3 + (o_x+1).
HGKS_FN constexpr int sidx(int ox, int oy, int oz) { return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1); }
HGKS_FN constexpr int sidx3(const int (&o)[3]) { return sidx(o[0], o[1], o[2]); }

// Coefficient order: x, y, z, xx, yy, zz, xy, yz, xz.
template <typename T>
struct BoxRecon {
  T c[9];      // combined quadratic
  T bound;     // max over the 25 polynomials and the 24 Gauss points of
               // |P_m(x_G) - Q_c| (a bound, see box_bound)
};

// Bound of |P - Q_c| over the 24 face Gauss points for a polynomial with
// linear coefficients l and (optional) quadratic coefficients: |xi_d| <= 1/2,
// |xi_d^2 - 1/12| <= 1/6, |xi_d xi_e| <= 1/(4 sqrt 3).
template <typename T>
HGKS_FN T lin_bound(T bx, T by, T bz) {
  return T(0.5) * (d_abs(bx) + d_abs(by) + d_abs(bz));
}

// Least-squares quadratic of the big stencil (closed form above).
template <typename T>
HGKS_FN void big_quadratic(const T (&d)[27], T (&a)[9]) {
  {
    T r[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      T s = T(0), rr = T(0);
      // the 10 neighbours with o_ax != 0: face (+-e_ax) and edges with one
      // other axis
#pragma unroll
      for (int sg = -1; sg <= 1; sg += 2) {
        int o[3] = {0, 0, 0};
        o[ax] = sg;
        T acc = d[sidx3(o)];
#pragma unroll
        for (int oth = 1; oth <= 2; ++oth) {
          const int e = (ax + oth) % 3;
#pragma unroll
          for (int se = -1; se <= 1; se += 2) {
            int oo[3] = {0, 0, 0};
            oo[ax] = sg;
            oo[e] = se;
            acc += d[sidx3(oo)];
          }
        }
        s += T(sg) * acc;
        rr += acc;
      }
      a[ax] = s * T(0.1);
      r[ax] = rr;
    }
    const T rs = T(2.0 / 9.0) * (r[0] + r[1] + r[2]);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) a[3 + ax] = (r[ax] - rs) * T(1.0 / 6.0);
    // mixed: (x,y), (y,z), (x,z)
    const int pd[3] = {0, 1, 0}, pe[3] = {1, 2, 2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T s = T(0);
#pragma unroll
      for (int s1 = -1; s1 <= 1; s1 += 2)
#pragma unroll
        for (int s2 = -1; s2 <= 1; s2 += 2) {
          int o[3] = {0, 0, 0};
          o[pd[k]] = s1;
          o[pe[k]] = s2;
          s += T(s1 * s2) * d[sidx3(o)];
        }
      a[6 + k] = T(0.25) * s;
    }
  }
}

template <typename T>
HGKS_FN void weno_box(const T (&d)[27], const WenoParams<T>& P, BoxRecon<T>& out) {
  T a[9];
  big_quadratic(d, a);
  const T beta0 = P.kl[0] * a[0] * a[0] + P.kl[1] * a[1] * a[1] + P.kl[2] * a[2] * a[2] +
                  P.kq[0] * a[3] * a[3] + P.kq[1] * a[4] * a[4] + P.kq[2] * a[5] * a[5] +
                  P.km[0] * a[6] * a[6] + P.km[1] * a[7] * a[7] + P.km[2] * a[8] * a[8];

  // One pass over the sub-stencils.  With r_m = 1/(beta_m + eps) and
  // r_0 = 1/(beta_0 + eps) the nonlinear weights are affine in tau:
  // omega_m = Gamma (1 + tau r_m), omega_0 / gamma_0 = 1 + tau r_0.  So the
  // weight sum is S = gamma_0 (1 + tau r_0) + Gamma (24 + tau sum_m r_m)
  // and the combined linear part sum_m (omega_m - Gamma omega_0 / gamma_0)
  // b^m / S is (Gamma tau / S) sum_m (r_m - r_0) b^m.  The pass gathers
  // sum |beta_0 - beta_m| (tau), sum r_m and sum (r_m - r_0) b^m; tau enters
  // afterwards, and no sub-stencil's indicator is kept.  Sub-stencils in the
  // order of the printed S_1..S_8 and their two cyclic permutations: triple
  // t, then s_c, s_b, s_a in (+, -).
  const T r0 = d_rcp(beta0 + P.eps);
  T tsum = T(0), rsum = T(0), db[3] = {T(0), T(0), T(0)};
  T bnd = T(0.5) * (d_abs(a[0]) + d_abs(a[1]) + d_abs(a[2])) +
          T(1.0 / 6.0) * (d_abs(a[3]) + d_abs(a[4]) + d_abs(a[5])) +
          T(0.14433756729740644113) * (d_abs(a[6]) + d_abs(a[7]) + d_abs(a[8]));
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int ea = t, eb = (t + 1) % 3, ec = (t + 2) % 3;
#pragma unroll
    for (int ic = 0; ic < 2; ++ic)
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int ia = 0; ia < 2; ++ia) {
          const int sa = ia ? -1 : 1, sb = ib ? -1 : 1, sc = ic ? -1 : 1;
          int oa[3] = {0, 0, 0}, ob[3] = {0, 0, 0}, oab[3] = {0, 0, 0}, oc[3] = {0, 0, 0};
          oa[ea] = sa; ob[eb] = sb; oab[ea] = sa; oab[eb] = sb; oc[ec] = sc;
          const T da = d[sidx3(oa)], db_ = d[sidx3(ob)], dab = d[sidx3(oab)], dc = d[sidx3(oc)];
          const T bc = T(sc) * dc;
          const T ba = T(sa) * (T(2) * da - db_ + dab) * T(1.0 / 3.0);
          const T bb = T(sb) * (T(2) * db_ - da + dab) * T(1.0 / 3.0);
          const T beta = P.kl[ea] * ba * ba + P.kl[eb] * bb * bb + P.kl[ec] * bc * bc;
          tsum += d_abs(beta0 - beta);
          const T rm = d_rcp(beta + P.eps);
          rsum += rm;
          const T dr = rm - r0;
          db[ea] += dr * ba;
          db[eb] += dr * bb;
          db[ec] += dr * bc;
          bnd = d_max(bnd, T(0.5) * (d_abs(ba) + d_abs(bb) + d_abs(bc)));
        }
  }
  const T tau = tsum * T(1.0 / 24.0);
  const T w0r = T(1) + tau * r0;  // omega_0 / gamma_0
  const T iS = d_rcp(P.gamma0 * w0r + P.Gamma * (T(24) + tau * rsum));
  const T w0g = w0r * iS;           // wbar_0 / gamma_0
  const T gl = P.Gamma * tau * iS;  // weight of sum (r_m - r_0) b^m
#pragma unroll
  for (int e = 0; e < 3; ++e) out.c[e] = w0g * a[e] + gl * db[e];
#pragma unroll
  for (int k = 3; k < 9; ++k) out.c[k] = w0g * a[k];
  out.bound = bnd;
}

// The alternative of Remark 1: big stencil S' = S plus the six cells two
// steps away along the axes (far differences f, order -2x, +2x, -2y, +2y,
// -2z, +2z), sub-stencils S'_m = the centre and one face neighbour per axis,
// one per sign octant (s_x, s_y, s_z).  Closed forms on the unit cube:
//   a_d  = (1/18) sum_{o in S'} o_d d_o
//   a_de = (1/4)  sum o_d o_e d_o                          (as for S)
//   a_dd = (r_d - (2/25)(r_x + r_y + r_z)) / 38,  r_d = sum o_d^2 d_o
// (the 24x9 normal equations: diagonal 18 for the linear terms, 4 for the
// mixed ones, 38 I + 4 (1 1^T) for the squares); each sub-stencil is
// interpolated, b_d = s_d d_{s_d e_d}.  Linear weights 1 - 8 Gamma and
// Gamma, tau the mean over the eight sub-stencils.
template <typename T>
HGKS_FN void big_quadratic_wide(const T (&d)[27], const T (&f)[6], T (&a)[9]) {
  T r[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    T s = T(0), rr = T(0);
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
      int o[3] = {0, 0, 0};
      o[ax] = sg;
      T acc = d[sidx3(o)];
#pragma unroll
      for (int oth = 1; oth <= 2; ++oth) {
        const int e = (ax + oth) % 3;
#pragma unroll
        for (int se = -1; se <= 1; se += 2) {
          int oo[3] = {0, 0, 0};
          oo[ax] = sg;
          oo[e] = se;
          acc += d[sidx3(oo)];
        }
      }
      const T far = f[2 * ax + (sg > 0 ? 1 : 0)];
      s += T(sg) * (acc + T(2) * far);
      rr += acc + T(4) * far;
    }
    a[ax] = s * T(1.0 / 18.0);
    r[ax] = rr;
  }
  const T rs = T(2.0 / 25.0) * (r[0] + r[1] + r[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) a[3 + ax] = (r[ax] - rs) * T(1.0 / 38.0);
  const int pd[3] = {0, 1, 0}, pe[3] = {1, 2, 2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T s = T(0);
#pragma unroll
    for (int s1 = -1; s1 <= 1; s1 += 2)
#pragma unroll
      for (int s2 = -1; s2 <= 1; s2 += 2) {
        int o[3] = {0, 0, 0};
        o[pd[k]] = s1;
        o[pe[k]] = s2;
        s += T(s1 * s2) * d[sidx3(o)];
      }
    a[6 + k] = T(0.25) * s;
  }
}

// Slopes of the octant sub-stencil m = 4 iz + 2 iy + ix (sign - for a set
// bit), in the order of the printed S'_1..S'_8 read as x fastest.
template <typename T>
HGKS_FN void octant_slopes(const T (&d)[27], int m, T (&b)[3]) {
  const int sx = (m & 1) ? -1 : 1, sy = (m & 2) ? -1 : 1, sz = (m & 4) ? -1 : 1;
  b[0] = T(sx) * d[sidx(sx, 0, 0)];
  b[1] = T(sy) * d[sidx(0, sy, 0)];
  b[2] = T(sz) * d[sidx(0, 0, sz)];
}

template <typename T>
HGKS_FN void weno_box_wide(const T (&d)[27], const T (&f)[6], const WenoParams<T>& P, BoxRecon<T>& out) {
  T a[9];
  big_quadratic_wide(d, f, a);
  const T beta0 = P.kl[0] * a[0] * a[0] + P.kl[1] * a[1] * a[1] + P.kl[2] * a[2] * a[2] +
                  P.kq[0] * a[3] * a[3] + P.kq[1] * a[4] * a[4] + P.kq[2] * a[5] * a[5] +
                  P.km[0] * a[6] * a[6] + P.km[1] * a[7] * a[7] + P.km[2] * a[8] * a[8];
  T beta[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    T b[3];
    octant_slopes(d, m, b);
    beta[m] = P.kl[0] * b[0] * b[0] + P.kl[1] * b[1] * b[1] + P.kl[2] * b[2] * b[2];
  }
  T tau = T(0);
#pragma unroll
  for (int m = 0; m < 8; ++m) tau += d_abs(beta0 - beta[m]);
  tau *= T(1.0 / 8.0);
  const T w0r = T(1) + tau * d_rcp(beta0 + P.eps);
  T wsum = P.gamma0 * w0r;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    beta[m] = P.Gamma * (T(1) + tau * d_rcp(beta[m] + P.eps));
    wsum += beta[m];
  }
  const T iw = d_rcp(wsum);
  const T w0g = w0r * iw;
  const T off = w0g * P.Gamma;
  T cl[3] = {w0g * a[0], w0g * a[1], w0g * a[2]};
  T bnd = T(0.5) * (d_abs(a[0]) + d_abs(a[1]) + d_abs(a[2])) +
          T(1.0 / 6.0) * (d_abs(a[3]) + d_abs(a[4]) + d_abs(a[5])) +
          T(0.14433756729740644113) * (d_abs(a[6]) + d_abs(a[7]) + d_abs(a[8]));
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    T b[3];
    octant_slopes(d, m, b);
    const T cm = beta[m] * iw - off;
    cl[0] += cm * b[0];
    cl[1] += cm * b[1];
    cl[2] += cm * b[2];
    const T bm = T(0.5) * (d_abs(b[0]) + d_abs(b[1]) + d_abs(b[2]));
    bnd = d_max(bnd, bm);
  }
  out.c[0] = cl[0];
  out.c[1] = cl[1];
  out.c[2] = cl[2];
#pragma unroll
  for (int k = 3; k < 9; ++k) out.c[k] = w0g * a[k];
  out.bound = bnd;
}

// Value and unit-cube gradient of a quadratic with coefficients c (order x,
// y, z, xx, yy, zz, xy, yz, xz) about the cell mean q at xi.
template <typename T>
HGKS_FN void quad_eval(T q, const T (&c)[9], T x, T y, T z, T& val, T& gx, T& gy, T& gz) {
  const T t12 = T(1.0 / 12.0);
  val = q + c[0] * x + c[1] * y + c[2] * z + c[3] * (x * x - t12) + c[4] * (y * y - t12) +
        c[5] * (z * z - t12) + c[6] * x * y + c[7] * y * z + c[8] * x * z;
  gx = c[0] + T(2) * c[3] * x + c[6] * y + c[8] * z;
  gy = c[1] + T(2) * c[4] * y + c[6] * x + c[7] * z;
  gz = c[2] + T(2) * c[5] * z + c[7] * y + c[8] * x;
}

}  // namespace hgks
