// Eigenvectors of the Euler Jacobian along a grid axis, for the
// reconstruction in characteristic variables (Pan & Xu, Sec. 4: the option
// stated after the limiting procedure).
#pragma once

#include "common.h"

namespace hgks {

// Eigenvectors of the Euler Jacobian along axis D at a state, in terms of a
// few scalars; rows of L = R^-1 and columns of R are formed on demand.
// Order of the fields: u_n - c, entropy, shear along axis D+1, shear along
// axis D+2 (cyclic), u_n + c.
struct CharBasis {
  double V[3], c, ic, H, q2, b1, b2;
  double un, vA, vC;  // velocity along D, D+1, D+2
  int D, A, C;
};

// v[i] for a lane-uniform runtime i, by selects (no indexed private array).
HGKS_FN double pick3(const double (&v)[3], int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }

HGKS_FN void char_basis(const double (&Qb)[5], int D, double gamma, CharBasis& B) {
  B.D = D;
  B.A = D == 2 ? 0 : D + 1;
  B.C = D == 0 ? 2 : D - 1;
  const double ir = 1.0 / Qb[0];
  for (int e = 0; e < 3; ++e) B.V[e] = Qb[1 + e] * ir;
  B.q2 = B.V[0] * B.V[0] + B.V[1] * B.V[1] + B.V[2] * B.V[2];
  const double p = (gamma - 1.0) * (Qb[4] - 0.5 * Qb[0] * B.q2);
  const double c2 = gamma * p * ir;
  B.c = sqrt(c2);
  B.ic = 1.0 / B.c;
  B.H = (Qb[4] + p) * ir;
  B.b1 = (gamma - 1.0) / c2;
  B.b2 = 0.5 * B.b1 * B.q2;
  B.un = pick3(B.V, D);
  B.vA = pick3(B.V, B.A);
  B.vC = pick3(B.V, B.C);
}

// Row f of L (acting on rho, rho u, rho v, rho w, rho E).
HGKS_FN void char_lrow(const CharBasis& B, int f, double (&l)[5]) {
  const double un = B.un;
  if (f == 0 || f == 4) {
    const double sg = f == 0 ? 1.0 : -1.0;
    l[0] = 0.5 * (B.b2 + sg * un * B.ic);
    for (int e = 0; e < 3; ++e) l[1 + e] = -0.5 * (B.b1 * B.V[e] + (e == B.D ? sg * B.ic : 0.0));
    l[4] = 0.5 * B.b1;
  } else if (f == 1) {
    l[0] = 1.0 - B.b2;
    for (int e = 0; e < 3; ++e) l[1 + e] = B.b1 * B.V[e];
    l[4] = -B.b1;
  } else {
    const int t = f == 2 ? B.A : B.C;
    l[0] = f == 2 ? -B.vA : -B.vC;
    for (int e = 0; e < 3; ++e) l[1 + e] = e == t ? 1.0 : 0.0;
    l[4] = 0.0;
  }
}

// Column f of R.
HGKS_FN void char_rcol(const CharBasis& B, int f, double (&r)[5]) {
  const double un = B.un;
  if (f == 0 || f == 4) {
    const double sg = f == 0 ? -1.0 : 1.0;
    r[0] = 1.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = B.V[e] + (e == B.D ? sg * B.c : 0.0);
    r[4] = B.H + sg * B.c * un;
  } else if (f == 1) {
    r[0] = 1.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = B.V[e];
    r[4] = 0.5 * B.q2;
  } else {
    const int t = f == 2 ? B.A : B.C;
    r[0] = 0.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = e == t ? 1.0 : 0.0;
    r[4] = f == 2 ? B.vA : B.vC;
  }
}

// The same eigenvectors along a general orthonormal frame (n, t1, t2): the
// normal n of a face and its tangential axes (hexahedral grids; the frame
// of the face flux at the face's centre).  Field order as above, the shear
// fields along t1 and t2.
struct CharFrame {
  double V[3], c, ic, H, q2, b1, b2;
  double n[3], t1[3], t2[3];
  double un, v1, v2;  // velocity along n, t1, t2
};

HGKS_FN void char_frame(const double (&Qb)[5], const double (&n)[3], const double (&t1)[3], const double (&t2)[3],
                        double gamma, CharFrame& B) {
  const double ir = 1.0 / Qb[0];
  for (int e = 0; e < 3; ++e) {
    B.V[e] = Qb[1 + e] * ir;
    B.n[e] = n[e];
    B.t1[e] = t1[e];
    B.t2[e] = t2[e];
  }
  B.q2 = B.V[0] * B.V[0] + B.V[1] * B.V[1] + B.V[2] * B.V[2];
  const double p = (gamma - 1.0) * (Qb[4] - 0.5 * Qb[0] * B.q2);
  const double c2 = gamma * p * ir;
  B.c = sqrt(c2);
  B.ic = 1.0 / B.c;
  B.H = (Qb[4] + p) * ir;
  B.b1 = (gamma - 1.0) / c2;
  B.b2 = 0.5 * B.b1 * B.q2;
  B.un = B.V[0] * n[0] + B.V[1] * n[1] + B.V[2] * n[2];
  B.v1 = B.V[0] * t1[0] + B.V[1] * t1[1] + B.V[2] * t1[2];
  B.v2 = B.V[0] * t2[0] + B.V[1] * t2[1] + B.V[2] * t2[2];
}

// Row f of L.
HGKS_FN void char_lrow(const CharFrame& B, int f, double (&l)[5]) {
  if (f == 0 || f == 4) {
    const double sg = f == 0 ? 1.0 : -1.0;
    l[0] = 0.5 * (B.b2 + sg * B.un * B.ic);
    for (int e = 0; e < 3; ++e) l[1 + e] = -0.5 * (B.b1 * B.V[e] + sg * B.n[e] * B.ic);
    l[4] = 0.5 * B.b1;
  } else if (f == 1) {
    l[0] = 1.0 - B.b2;
    for (int e = 0; e < 3; ++e) l[1 + e] = B.b1 * B.V[e];
    l[4] = -B.b1;
  } else {
    const bool a = f == 2;
    l[0] = a ? -B.v1 : -B.v2;
    for (int e = 0; e < 3; ++e) l[1 + e] = a ? B.t1[e] : B.t2[e];
    l[4] = 0.0;
  }
}

// Column f of R.
HGKS_FN void char_rcol(const CharFrame& B, int f, double (&r)[5]) {
  if (f == 0 || f == 4) {
    const double sg = f == 0 ? -1.0 : 1.0;
    r[0] = 1.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = B.V[e] + sg * B.c * B.n[e];
    r[4] = B.H + sg * B.c * B.un;
  } else if (f == 1) {
    r[0] = 1.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = B.V[e];
    r[4] = 0.5 * B.q2;
  } else {
    const bool a = f == 2;
    r[0] = 0.0;
    for (int e = 0; e < 3; ++e) r[1 + e] = a ? B.t1[e] : B.t2[e];
    r[4] = a ? B.v1 : B.v2;
  }
}

}  // namespace hgks
