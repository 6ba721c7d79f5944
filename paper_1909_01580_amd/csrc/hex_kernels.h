// Kernels of the HGKS stage on a periodic hexahedral (vertex) grid, static
// or moving (Pan & Xu, Sec. 2 final part; Sec. 3, Eqs. (10)-(11) and
// Remark 2).
//
// Geometry.  A cell is the trilinear image of [-1/2, 1/2]^3 of its eight
// vertices (corner 4a + 2b + c = vertex (i+a, j+b, k+c)); cell integrals use
// the 2x2x2 Gauss rule with |J|.  A face is the bilinear image of its four
// vertices, parameterised by the two other axes in cyclic order (a, b) =
// (d+1, d+2), so that X_a x X_b points towards increasing index along d;
// Gauss point g = 2 [a>0] + [b>0] of the 2x2 rule, weight 1/4.  Vertices
// move with the constant velocity (x^{n+1} - x^n)/dt; the stage geometry is
// at t_n (stage 1) and t_n + dt/2 (stage 2).
//
// Per-stage geometry record of a cell (doubles, SoA [kHexGeo][N]): volume,
// centroid (3), central second moments xx, yy, zz, xy, yz, xz (6), all by
// the 2x2x2 rule, then h = |Omega|^(1/3) and 1/h.  The average over neighbour cell o of the scaled
// monomials X^n, X = (x - c_i)/h_i, h_i = |Omega_i|^(1/3), follows from
// o's record: mean X = (c_o - c_i)/h_i, mean X_a X_b = (M_o,ab + (c_o -
// c_i)_a (c_o - c_i)_b)/h_i^2; this fills the rows of the least-squares
// systems of Sec. 2 (big stencil 18 x 9, sub-stencils 4 x 3), solved here by
// normal equations (Cholesky for 9 x 9, closed-form inverse for 3 x 3).
//
// Face flux.  At each face Gauss point the two reconstructions are
// evaluated, shifted to the frame moving with the grid velocity U^g of the
// point (M - rho U^g, E - M.U^g + rho |U^g|^2 / 2), rotated into the local
// frame, passed through the static gas-kinetic flux and transformed back.
// With a_G = X_a x X_b:
//   F_p   = sum_G (1/4) |a_G| F_G,
//   dF_p  = sum_G (1/4) (|a_G| dF_G - Q_0 (U^g . da_G/dt)),
//   R_V   = sum_G (1/4) U^g . a_G,       dR_V = sum_G (1/4) U^g . da_G/dt,
// and the stage update acts on |Omega| Q and |Omega| together.
#pragma once

#include <cstring>
#include <type_traits>

#include "box_kernels.h"
#include "char_basis.h"
#include "common.h"
#include "gks_flux.h"

namespace hgks {

constexpr int kHexGeo = 12;
// Face record: F (5) and dF (5) in the compute type; the volume rates R_V
// and dR_V in double in a side array of their own (the moving-mesh volume
// stays FP64 in every precision mode).
constexpr int kHexFace = 10;

struct HexGrid {
  int n[3];
  double period[3];
  const double* x0;  // vertices at t_n, [3][N]
  const double* x1;  // vertices at t_{n+1}, or null (or x0) for a static grid
  double alpha;      // stage time (t - t_n) / dt
  double inv_dt;
  BoxGrid box;       // the same extents (all periodic) for index splitting and flux block order
};

inline void hex_setup(HexGrid& H, const int n[3], const double period[3]) {
  for (int d = 0; d < 3; ++d) {
    H.n[d] = n[d];
    H.period[d] = period[d];
  }
  H.x0 = H.x1 = nullptr;
  H.alpha = 0.0;
  H.inv_dt = 0.0;
  std::memset(&H.box, 0, sizeof H.box);
  for (int d = 0; d < 3; ++d) {
    H.box.n[d] = H.box.nr[d] = n[d];
    H.box.per[d] = 1;
    for (int e = 0; e < 3; ++e) H.box.nf[d][e] = n[e];
  }
  set_index_split(H.box);
}

// Index within [0, n) of a periodic index c in [-n, 2n) and the number of
// periods w it was moved by (c = wrapped + w n).  Every caller stays within
// one period of the grid.
__device__ __forceinline__ int wrap_once(int c, int n, int& w) {
  w = c < 0 ? -1 : (c >= n ? 1 : 0);
  return c - w * n;
}

// Position and velocity of vertex (i, j, k) (indices may leave [0, n): the
// periodic image is shifted by the period along that axis).
__device__ __forceinline__ void hex_vertex(const HexGrid& H, int i, int j, int k, double (&x)[3], double (&u)[3]) {
  int c[3] = {i, j, k};
  double s[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int w;
    c[d] = wrap_once(c[d], H.n[d], w);
    s[d] = w * H.period[d];
  }
  const size_t N = (size_t)H.n[0] * H.n[1] * H.n[2];
  const size_t idx = ((size_t)c[2] * H.n[1] + c[1]) * H.n[0] + c[0];
  // A static grid reads its one vertex array twice (b - a = 0 exactly, so
  // x = a and u = 0): no branch between the loads, which lets all of them
  // be in flight at once.
  const double* __restrict__ x1 = H.x1 ? H.x1 : H.x0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double a = H.x0[e * N + idx] + s[e];
    const double b = x1[e * N + idx] + s[e];
    x[e] = a + H.alpha * (b - a);
    u[e] = (b - a) * H.inv_dt;
  }
}

__device__ __forceinline__ void cross3(const double (&a)[3], const double (&b)[3], double (&c)[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Bilinear face map (Eq. (10)) at parameters (sa, sb): position, the two
// parametric derivatives, and the same for the vertex velocities.
struct FacePoint {
  double x[3], xa[3], xb[3], u[3], ua[3], ub[3];
};

__device__ __forceinline__ void face_point(const double (&cx)[4][3], const double (&cu)[4][3], double sa, double sb,
                                           FacePoint& P) {
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    P.x[e] = P.xa[e] = P.xb[e] = P.u[e] = P.ua[e] = P.ub[e] = 0.0;
  }
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      const double ea = ia ? 1.0 : -1.0, eb = ib ? 1.0 : -1.0;
      const double fa = 1.0 + 2.0 * ea * sa, fb = 1.0 + 2.0 * eb * sb;
      const int m = 2 * ia + ib;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        P.x[e] += 0.25 * fa * fb * cx[m][e];
        P.xa[e] += 0.5 * ea * fb * cx[m][e];
        P.xb[e] += 0.5 * eb * fa * cx[m][e];
        P.u[e] += 0.25 * fa * fb * cu[m][e];
        P.ua[e] += 0.5 * ea * fb * cu[m][e];
        P.ub[e] += 0.5 * eb * fa * cu[m][e];
      }
    }
}

// Corners of the face normal to axis d on vertex plane (i, j, k) (the
// face's lowest vertex), corner 2*ia + ib along the cyclic axes (a, b).
__device__ __forceinline__ void face_corners(const HexGrid& H, int d, int i, int j, int k, double (&cx)[4][3],
                                             double (&cu)[4][3]) {
  const int a = (d + 1) % 3, b = (d + 2) % 3;
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      int c[3] = {i, j, k};
      c[a] += ia;
      c[b] += ib;
      hex_vertex(H, c[0], c[1], c[2], cx[2 * ia + ib], cu[2 * ia + ib]);
    }
}

// The four corners of the face normal to axis D whose lowest vertex is the
// lattice point c, every c[d] in [0, n_d) (the face flux's case): only the
// +1 neighbours along the face's own axes A and B can pass the last plane,
// where they wrap to 0 with their position shifted by the period.  Indices
// in 32-bit arithmetic and loads at 32-bit byte offsets from the arrays'
// uniform bases (the grid has fewer than 2^29 vertices); the same values as
// face_corners for such c.
template <int D>
__device__ __forceinline__ void face_corners_in(const HexGrid& H, const int (&c)[3], double (&cx)[4][3],
                                               double (&cu)[4][3]) {
  constexpr int A = (D + 1) % 3, B = (D + 2) % 3;
  const unsigned st[3] = {1u, (unsigned)H.n[0], (unsigned)H.n[0] * (unsigned)H.n[1]};
  const unsigned N = st[2] * (unsigned)H.n[2];
  const unsigned base = (unsigned)c[0] + (unsigned)c[1] * st[1] + (unsigned)c[2] * st[2];
  const bool wa = c[A] + 1 == H.n[A], wb = c[B] + 1 == H.n[B];
  const unsigned oa = wa ? 0u - (unsigned)c[A] * st[A] : st[A];
  const unsigned ob = wb ? 0u - (unsigned)c[B] * st[B] : st[B];
  const double sa = wa ? H.period[A] : 0.0, sb = wb ? H.period[B] : 0.0;
  const double* __restrict__ x1p = H.x1 ? H.x1 : H.x0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int ia = m >> 1, ib = m & 1;
    const unsigned off = (base + (ia ? oa : 0u) + (ib ? ob : 0u)) * 8u;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      // uniform base of coordinate e, per-lane 32-bit byte offset
      const char* __restrict__ x0 = (const char*)(H.x0 + (size_t)e * N);
      const char* __restrict__ x1 = (const char*)(x1p + (size_t)e * N);
      const double s = (e == A && ia) ? sa : ((e == B && ib) ? sb : 0.0);
      const double a = *(const double*)(x0 + off) + s;
      const double b = *(const double*)(x1 + off) + s;
      cx[m][e] = a + H.alpha * (b - a);
      cu[m][e] = (b - a) * H.inv_dt;
    }
  }
}

// The eight vertices of cell (i, j, k) with every index in [0, n) (vertex
// m = 4 a + 2 b + c at (i + a, j + b, k + c)): only the +1 neighbours can
// pass the last plane, where they wrap with a period shift.  32-bit indices
// and byte offsets as in face_corners_in; the same positions as hex_vertex.
struct CellVerts {
  unsigned base, o[3], N;
  double s[3];
};

__device__ __forceinline__ CellVerts cell_verts(const HexGrid& H, int i, int j, int k) {
  CellVerts V;
  const unsigned st[3] = {1u, (unsigned)H.n[0], (unsigned)H.n[0] * (unsigned)H.n[1]};
  V.N = st[2] * (unsigned)H.n[2];
  const int c[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool w = c[d] + 1 == H.n[d];
    V.o[d] = w ? 0u - (unsigned)c[d] * st[d] : st[d];
    V.s[d] = w ? H.period[d] : 0.0;
  }
  V.base = (unsigned)i + (unsigned)j * st[1] + (unsigned)k * st[2];
  return V;
}

// Position of vertex m of the cell at the stage time.
__device__ __forceinline__ void cell_vertex(const HexGrid& H, const CellVerts& V, int m, double (&x)[3]) {
  const int bit[3] = {(m >> 2) & 1, (m >> 1) & 1, m & 1};
  const unsigned off = (V.base + (bit[0] ? V.o[0] : 0u) + (bit[1] ? V.o[1] : 0u) + (bit[2] ? V.o[2] : 0u)) * 8u;
  const double* __restrict__ x1p = H.x1 ? H.x1 : H.x0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const char* __restrict__ x0 = (const char*)(H.x0 + (size_t)e * V.N);
    const char* __restrict__ x1 = (const char*)(x1p + (size_t)e * V.N);
    const double sh = bit[e] ? V.s[e] : 0.0;
    const double a = *(const double*)(x0 + off) + sh;
    const double b = *(const double*)(x1 + off) + sh;
    x[e] = a + H.alpha * (b - a);
  }
}

// ---------------------------------------------------------------- K1
// Cell geometry record at the stage time.
__global__ void __launch_bounds__(kBlock) k_geometry_hex(HexGrid H, double* __restrict__ geo, size_t N) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  int i, j, k;
  split_index((uint32_t)idx, H.n[0], H.n[1], H.box.inv_n[0], H.box.inv_n[1], i, j, k);
  double cx[8][3];
  {
    const CellVerts cv = cell_verts(H, i, j, k);
#pragma unroll
    for (int m = 0; m < 8; ++m) cell_vertex(H, cv, m, cx[m]);
  }
  const double g = kGaussNode;
  double xq[8][3], wq[8];
  double V = 0.0, c[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double xi = ((q >> 2) & 1) ? g : -g, et = ((q >> 1) & 1) ? g : -g, ze = (q & 1) ? g : -g;
    double X[3] = {0, 0, 0}, D0[3] = {0, 0, 0}, D1[3] = {0, 0, 0}, D2[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double sa = ((m >> 2) & 1) ? 1.0 : -1.0, sb = ((m >> 1) & 1) ? 1.0 : -1.0, sc = (m & 1) ? 1.0 : -1.0;
      const double fa = 1.0 + 2.0 * sa * xi, fb = 1.0 + 2.0 * sb * et, fc = 1.0 + 2.0 * sc * ze;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        X[e] += fa * fb * fc * 0.125 * cx[m][e];
        D0[e] += 2.0 * sa * fb * fc * 0.125 * cx[m][e];
        D1[e] += 2.0 * sb * fa * fc * 0.125 * cx[m][e];
        D2[e] += 2.0 * sc * fa * fb * 0.125 * cx[m][e];
      }
    }
    double cr[3];
    cross3(D1, D2, cr);
    const double J = D0[0] * cr[0] + D0[1] * cr[1] + D0[2] * cr[2];
    wq[q] = 0.125 * (J < 0 ? -J : J);
#pragma unroll
    for (int e = 0; e < 3; ++e) xq[q][e] = X[e];
    V += wq[q];
#pragma unroll
    for (int e = 0; e < 3; ++e) c[e] += wq[q] * X[e];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) c[e] /= V;
  double M[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double dx = xq[q][0] - c[0], dy = xq[q][1] - c[1], dz = xq[q][2] - c[2];
    M[0] += wq[q] * dx * dx;
    M[1] += wq[q] * dy * dy;
    M[2] += wq[q] * dz * dz;
    M[3] += wq[q] * dx * dy;
    M[4] += wq[q] * dy * dz;
    M[5] += wq[q] * dx * dz;
  }
  geo[idx] = V;
#pragma unroll
  for (int e = 0; e < 3; ++e) geo[(1 + e) * N + idx] = c[e];
#pragma unroll
  for (int e = 0; e < 6; ++e) geo[(4 + e) * N + idx] = M[e] / V;
  const double h = cbrt(V);
  geo[10 * N + idx] = h;
  geo[11 * N + idx] = 1.0 / h;
}

// ---------------------------------------------------------------- K2
// Neighbour access for the reconstruction of cell (i, j, k).
struct HexCell {
  double c[3];   // centroid
  double h, ih;  // |Omega|^(1/3) and its inverse
  double m[6];   // central second moments / h^2 (means of X_a X_b)
};

__device__ __forceinline__ size_t hex_index(const HexGrid& H, int i, int j, int k, double (&shift)[3]) {
  int c[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int w;
    c[d] = wrap_once(c[d], H.n[d], w);
    shift[d] = w * H.period[d];
  }
  return ((size_t)c[2] * H.n[1] + c[1]) * H.n[0] + c[0];
}

__device__ __forceinline__ void load_cell(const double* __restrict__ geo, size_t N, size_t idx, HexCell& C) {
  C.h = geo[10 * N + idx];
  C.ih = geo[11 * N + idx];
#pragma unroll
  for (int e = 0; e < 3; ++e) C.c[e] = geo[(1 + e) * N + idx];
  const double ih2 = C.ih * C.ih;
#pragma unroll
  for (int e = 0; e < 6; ++e) C.m[e] = geo[(4 + e) * N + idx] * ih2;
}

// Neighbour data of the least-squares rows of cell i: for the neighbour at
// offset o, the scaled centroid offset d = (c_o - c_i) / h_i, optionally
// the neighbour's central second moments over h_i^2, and q_o - q_i of the
// five variables.  Two sources with identical arithmetic: global memory
// (any cell) and a workgroup tile staged in LDS.
struct NbrGlobal {
  const HexGrid& H;
  const double* __restrict__ geo;
  const double* __restrict__ q;
  size_t N;
  int i, j, k;
  template <bool MOM>
  __device__ __forceinline__ void get(int ox, int oy, int oz, const HexCell& Ci, const double (&qc)[5],
                                      double (&d)[3], double (&mo)[6], double (&dq)[5]) const {
    double sh[3];
    const size_t io = hex_index(H, i + ox, j + oy, k + oz, sh);
#pragma unroll
    for (int e = 0; e < 3; ++e) d[e] = (geo[(1 + e) * N + io] + sh[e] - Ci.c[e]) * Ci.ih;
    if (MOM) {
      const double ih2 = Ci.ih * Ci.ih;
#pragma unroll
      for (int e = 0; e < 6; ++e) mo[e] = geo[(4 + e) * N + io] * ih2;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) dq[v] = q[v * N + io] - qc[v];
  }
};

// LDS tile of the reconstruction: a kTX x kTY x kTZ block of cells and one
// layer around it; per cell the centroid of its periodic image (shift
// included), the central second moments and the five variables.
constexpr int kTX = 8, kTY = 8, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2, kHalo = kHX * kHY * kHZ;

struct HexTile {
  double c[3][kHalo];
  double m[6][kHalo];
  double q[5][kHalo];
};

struct NbrTile {
  const HexTile& T;
  int base;  // tile index of the cell itself
  template <bool MOM>
  __device__ __forceinline__ void get(int ox, int oy, int oz, const HexCell& Ci, const double (&qc)[5],
                                      double (&d)[3], double (&mo)[6], double (&dq)[5]) const {
    const int s = base + (oz * kHY + oy) * kHX + ox;
#pragma unroll
    for (int e = 0; e < 3; ++e) d[e] = (T.c[e][s] - Ci.c[e]) * Ci.ih;
    if (MOM) {
      const double ih2 = Ci.ih * Ci.ih;
#pragma unroll
      for (int e = 0; e < 6; ++e) mo[e] = T.m[e][s] * ih2;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) dq[v] = T.q[v][s] - qc[v];
  }
};

// In-place Cholesky factorisation of a symmetric positive definite 9x9
// matrix stored as its lower triangle L[i*(i+1)/2 + j]; the diagonal
// entries are left as their reciprocals, which is all the solves need.
__device__ __forceinline__ void chol9(double (&L)[45]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    double s = L[j * (j + 1) / 2 + j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
    const double inv = d_rcp(sqrt(s));
    L[j * (j + 1) / 2 + j] = inv;
#pragma unroll
    for (int i = j + 1; i < 9; ++i) {
      double t = L[i * (i + 1) / 2 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = t * inv;
    }
  }
}

__device__ __forceinline__ void chol9_solve(const double (&L)[45], double (&x)[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double t = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i * (i + 1) / 2 + k] * x[k];
    x[i] = t * L[i * (i + 1) / 2 + i];
  }
#pragma unroll
  for (int i = 8; i >= 0; --i) {
    double t = x[i];
#pragma unroll
    for (int k = i + 1; k < 9; ++k) t -= L[k * (k + 1) / 2 + i] * x[k];
    x[i] = t * L[i * (i + 1) / 2 + i];
  }
}

// The 24 sub-stencils (Sec. 2): axis triple t = (a, b; c) in
// ((x,y;z), (y,z;x), (z,x;y)), signs s_c, s_b, s_a in (+,-): cells
// s_a e_a, s_b e_b, s_a e_a + s_b e_b, s_c e_c.
__device__ __forceinline__ void sub_offsets(int m, int (&o)[4][3]) {
  const int t = m / 8, r = m % 8;
  const int ea = t, eb = (t + 1) % 3, ec = (t + 2) % 3;
  const int sa = (r & 1) ? -1 : 1, sb = (r & 2) ? -1 : 1, sc = (r & 4) ? -1 : 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q][0] = o[q][1] = o[q][2] = 0;
  o[0][ea] = sa;
  o[1][eb] = sb;
  o[2][ea] = sa;
  o[2][eb] = sb;
  o[3][ec] = sc;
}

// The eight sub-stencils of Remark 1: the face neighbours s_x e_x, s_y e_y,
// s_z e_z of one sign octant (s_x fastest, + first).
__device__ __forceinline__ void sub_offsets_wide(int m, int (&o)[3][3]) {
  const int sx = (m & 1) ? -1 : 1, sy = (m & 2) ? -1 : 1, sz = (m & 4) ? -1 : 1;
#pragma unroll
  for (int q = 0; q < 3; ++q) o[q][0] = o[q][1] = o[q][2] = 0;
  o[0][0] = sx;
  o[1][1] = sy;
  o[2][2] = sz;
}

// Sums over rows of a sub-stencil's normal equations: A (xx, yy, zz, xy,
// yz, xz) and r[v] = sum d dq[v].
struct SubSums {
  double A[6];
  double r[5][3];
};

template <typename NB>
__device__ __forceinline__ void sub_add_row(const NB& nb, const HexCell& Ci, const double (&qc)[5], int ox, int oy,
                                            int oz, SubSums& S) {
  double d[3], mo[6], dq[5];
  nb.template get<false>(ox, oy, oz, Ci, qc, d, mo, dq);
  S.A[0] += d[0] * d[0];
  S.A[1] += d[1] * d[1];
  S.A[2] += d[2] * d[2];
  S.A[3] += d[0] * d[1];
  S.A[4] += d[1] * d[2];
  S.A[5] += d[0] * d[2];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int e = 0; e < 3; ++e) S.r[v][e] += d[e] * dq[v];
  }
}

// The linear fit from summed normal equations (closed-form 3x3 inverse).
__device__ __forceinline__ void sub_solve(const SubSums& S, double (&b)[5][3]) {
  const double* A = S.A;
  const double c00 = A[1] * A[2] - A[4] * A[4];
  const double c01 = A[5] * A[4] - A[3] * A[2];
  const double c02 = A[3] * A[4] - A[1] * A[5];
  const double c11 = A[0] * A[2] - A[5] * A[5];
  const double c12 = A[3] * A[5] - A[0] * A[4];
  const double c22 = A[0] * A[1] - A[3] * A[3];
  const double idet = d_rcp(A[0] * c00 + A[3] * c01 + A[5] * c02);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    b[v][0] = idet * (c00 * S.r[v][0] + c01 * S.r[v][1] + c02 * S.r[v][2]);
    b[v][1] = idet * (c01 * S.r[v][0] + c11 * S.r[v][1] + c12 * S.r[v][2]);
    b[v][2] = idet * (c02 * S.r[v][0] + c12 * S.r[v][1] + c22 * S.r[v][2]);
  }
}

// Linear least squares of a sub-stencil with NR neighbour rows at offsets
// o for all five variables of cell i: b[v][3] in the scaled basis (NR = 4:
// Sec. 2; NR = 3: Remark 1, where the square system is solved exactly).
template <int NR, typename NB>
__device__ __forceinline__ void sub_fit_rows(const NB& nb, const HexCell& Ci, const double (&qc)[5],
                                             const int (&o)[NR][3], double (&b)[5][3]) {
  SubSums S;
#pragma unroll
  for (int e = 0; e < 6; ++e) S.A[e] = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) S.r[v][0] = S.r[v][1] = S.r[v][2] = 0.0;
#pragma unroll
  for (int s = 0; s < NR; ++s) sub_add_row(nb, Ci, qc, o[s][0], o[s][1], o[s][2], S);
  sub_solve(S, b);
}

// Linear fit of sub-stencil m of the stencil family (WIDE: Remark 1).
template <bool WIDE, typename NB>
__device__ __forceinline__ void sub_fit(const NB& nb, const HexCell& Ci, const double (&qc)[5], int m,
                                        double (&b)[5][3]) {
  if constexpr (WIDE) {
    int o[3][3];
    sub_offsets_wide(m, o);
    sub_fit_rows<3>(nb, Ci, qc, o, b);
  } else {
    int o[4][3];
    sub_offsets(m, o);
    sub_fit_rows<4>(nb, Ci, qc, o, b);
  }
}

// Sub-stencils of the family: 24 (Sec. 2) or 8 (Remark 1).
template <bool WIDE>
constexpr int kHexSubs = WIDE ? 8 : 24;

// Calls take(b) with the fits of the 24 sub-stencils of Sec. 2 (the order
// t * 8 + r with r = 0, 4, 1, 5, ...).  Sub-stencils t * 8 + r come in pairs
// that differ only in the sign of their last row (the face neighbour along
// e_c, bit 2 of r): the three shared rows (the face neighbours along e_a
// and e_b and their edge neighbour) are summed once per pair, in the order
// of sub_fit, so every fit equals sub_fit's.
template <typename NB, typename F>
__device__ __forceinline__ void each_sub_fit(const NB& nb, const HexCell& Ci, const double (&qc)[5], F&& take) {
#pragma unroll 1
  for (int p = 0; p < 12; ++p) {
    const int t = p >> 2, ea = t, eb = (t + 1) % 3, ec = (t + 2) % 3;
    const int sa = (p & 1) ? -1 : 1, sb = (p & 2) ? -1 : 1;
    int oa[3] = {0, 0, 0}, ob[3] = {0, 0, 0}, oe[3] = {0, 0, 0};
    oa[ea] = sa;
    ob[eb] = sb;
    oe[ea] = sa;
    oe[eb] = sb;
    SubSums S3;
#pragma unroll
    for (int e = 0; e < 6; ++e) S3.A[e] = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) S3.r[v][0] = S3.r[v][1] = S3.r[v][2] = 0.0;
    sub_add_row(nb, Ci, qc, oa[0], oa[1], oa[2], S3);
    sub_add_row(nb, Ci, qc, ob[0], ob[1], ob[2], S3);
    sub_add_row(nb, Ci, qc, oe[0], oe[1], oe[2], S3);
#pragma unroll
    for (int sc = 1; sc >= -1; sc -= 2) {
      SubSums S = S3;
      sub_add_row(nb, Ci, qc, ec == 0 ? sc : 0, ec == 1 ? sc : 0, ec == 2 ? sc : 0, S);
      double b[5][3];
      sub_solve(S, b);
      take(b);
    }
  }
}

// Quadratic least squares of the big stencil for all five variables: the
// row of neighbour o is the mean over o of (X, X_x^2 - m_xx, ...,
// X_x X_z - m_xz) in the scaled basis of cell i.  The 18 rows of S come
// from nb; with WIDE (Remark 1) six more, the cells two steps away along
// the axes, from far.
template <bool WIDE, typename NB, typename NF>
__device__ __forceinline__ void big_fit(const NB& nb, const NF& far, const HexCell& Ci, const double (&qc)[5],
                                        double (&a)[5][9]) {
  double L[45];
#pragma unroll
  for (int e = 0; e < 45; ++e) L[e] = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int e = 0; e < 9; ++e) a[v][e] = 0.0;
  auto add_row = [&](const double (&d)[3], const double (&mo)[6], const double (&dq)[5]) {
    double r[9];
    r[0] = d[0];
    r[1] = d[1];
    r[2] = d[2];
    r[3] = mo[0] + d[0] * d[0] - Ci.m[0];
    r[4] = mo[1] + d[1] * d[1] - Ci.m[1];
    r[5] = mo[2] + d[2] * d[2] - Ci.m[2];
    r[6] = mo[3] + d[0] * d[1] - Ci.m[3];
    r[7] = mo[4] + d[1] * d[2] - Ci.m[4];
    r[8] = mo[5] + d[0] * d[2] - Ci.m[5];
#pragma unroll
    for (int p = 0; p < 9; ++p)
#pragma unroll
      for (int t = 0; t <= p; ++t) L[p * (p + 1) / 2 + t] += r[p] * r[t];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
#pragma unroll
      for (int e = 0; e < 9; ++e) a[v][e] += r[e] * dq[v];
    }
  };
#pragma unroll 1
  for (int s = 0; s < 27; ++s) {
    const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = s / 9 - 1;
    const int nz = (ox != 0) + (oy != 0) + (oz != 0);
    if (nz == 0 || nz == 3) continue;
    double d[3], mo[6], dq[5];
    nb.template get<true>(ox, oy, oz, Ci, qc, d, mo, dq);
    add_row(d, mo, dq);
  }
  if constexpr (WIDE) {
#pragma unroll 1
    for (int s = 0; s < 6; ++s) {
      const int ax = s >> 1, sg = (s & 1) ? 2 : -2;
      double d[3], mo[6], dq[5];
      far.template get<true>(ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0, Ci, qc, d, mo, dq);
      add_row(d, mo, dq);
    }
  }
  chol9(L);
#pragma unroll
  for (int v = 0; v < 5; ++v) chol9_solve(L, a[v]);
}

// Scaled coordinates of the 24 face Gauss points of cell (i,j,k), Gauss
// point 4 f + g with faces (-x, +x, -y, +y, -z, +z).
__device__ __forceinline__ void cell_gp(const HexGrid& H, const HexCell& Ci, int i, int j, int k, int bit,
                                        double (&X)[3]) {
  const int f = bit >> 2, gp = bit & 3, d = f >> 1;
  int c[3] = {i, j, k};
  c[d] += (f & 1);
  double cx[4][3], cu[4][3];
  face_corners(H, d, c[0], c[1], c[2], cx, cu);
  FacePoint P;
  face_point(cx, cu, (gp >> 1) ? kGaussNode : -kGaussNode, (gp & 1) ? kGaussNode : -kGaussNode, P);
#pragma unroll
  for (int e = 0; e < 3; ++e) X[e] = (P.x[e] - Ci.c[e]) * Ci.ih;
}

__device__ __forceinline__ double pbasis(int n, const double (&X)[3], const double (&m)[6]) {
  switch (n) {
    case 0: return X[0];
    case 1: return X[1];
    case 2: return X[2];
    case 3: return X[0] * X[0] - m[0];
    case 4: return X[1] * X[1] - m[1];
    case 5: return X[2] * X[2] - m[2];
    case 6: return X[0] * X[1] - m[3];
    case 7: return X[1] * X[2] - m[4];
    default: return X[0] * X[2] - m[5];
  }
}

// Stages the reconstruction tile with origin (o0, o1, o2) and one layer
// around it in LDS: per tile cell the centroid of its periodic image (shift
// included), the central second moments and the five variables.
__device__ __forceinline__ void stage_hex_tile(const HexGrid& H, const double* __restrict__ geo,
                                               const double* __restrict__ q, size_t N, int o0, int o1, int o2,
                                               HexTile& T) {
  // A tile with its layer reaches at most one period past either end when
  // every extent is at least the tile's (uniform test); a very small grid
  // may be passed several times and takes the general wrap.
  const bool one_period = H.n[0] >= kTX && H.n[1] >= kTY && H.n[2] >= kTZ;
  for (int t = threadIdx.x; t < kHalo; t += kBlock) {
    const int g[3] = {o0 + t % kHX - 1, o1 + (t / kHX) % kHY - 1, o2 + t / (kHX * kHY) - 1};
    int c[3];
    double sh[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int w;
      if (one_period)
        w = g[d] < 0 ? -1 : (g[d] >= H.n[d] ? 1 : 0);
      else
        w = g[d] >= 0 ? g[d] / H.n[d] : -((-g[d] + H.n[d] - 1) / H.n[d]);
      c[d] = g[d] - w * H.n[d];
      sh[d] = w * H.period[d];
    }
    // 32-bit byte offset from each array's uniform base (fewer than 2^29
    // cells on a hexahedral grid)
    const unsigned off = ((unsigned)c[0] + (unsigned)c[1] * (unsigned)H.n[0] +
                          (unsigned)c[2] * ((unsigned)H.n[0] * (unsigned)H.n[1])) * 8u;
    auto at = [&](const double* __restrict__ base) { return *(const double*)((const char*)base + off); };
#pragma unroll
    for (int e = 0; e < 3; ++e) T.c[e][t] = at(geo + (1 + e) * N) + sh[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) T.m[e][t] = at(geo + (4 + e) * N);
#pragma unroll
    for (int v = 0; v < 5; ++v) T.q[v][t] = at(q + v * N);
  }
}

// beta_0 of Eq. (4) in the scaled basis for the quadratic with coefficients
// c: mean |grad P|^2 over the cell (second moments m) plus the squared
// second derivatives, each multi-index once.
__device__ __forceinline__ double hex_beta0(const double (&c)[9], const HexCell& Ci) {
  const double Hs[3][3] = {{2 * c[3], c[6], c[8]}, {c[6], 2 * c[4], c[7]}, {c[8], c[7], 2 * c[5]}};
  const double Mm[3][3] = {{Ci.m[0], Ci.m[3], Ci.m[5]}, {Ci.m[3], Ci.m[1], Ci.m[4]}, {Ci.m[5], Ci.m[4], Ci.m[2]}};
  double tr = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double hh = 0.0;
#pragma unroll
      for (int t = 0; t < 3; ++t) hh += Hs[t][r] * Hs[t][s];
      tr += hh * Mm[s][r];
    }
  return c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + tr + 4.0 * (c[3] * c[3] + c[4] * c[4] + c[5] * c[5]) +
         c[6] * c[6] + c[7] * c[7] + c[8] * c[8];
}

// WENO-AO reconstruction on a hexahedral cell (always in double): the
// combined quadratic in the scaled basis, written as (mean, 9 coefficients)
// per variable, and the fallback pre-test.
//
// One workgroup per kTX x kTY x kTZ tile of cells (tiles x-fastest): the
// tile and one layer around it are staged in LDS first, so that the 18
// big-stencil rows and the 2 x 24 sub-stencil fits of every cell read their
// neighbours from LDS instead of issuing some 1,800 global loads per cell.
// Grid extents need not be multiples of the tile: the lanes of cells beyond
// the grid only help to fill the tile.
// WIDE: the stencils of Remark 1 (the six far cells of the big stencil are
// read from global memory, the tile holds one layer).
template <typename TS, bool WIDE = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_recon_hex(HexGrid H, const double* __restrict__ geo,
                                                      const double* __restrict__ q, TS* __restrict__ coef,
                                                      uint32_t* __restrict__ mask, WenoParams<double> P, double gm1,
                                                      size_t N, unsigned ntx, unsigned nty, unsigned ntiles) {
  static_assert(kTX * kTY * kTZ == kBlock, "one lane per tile cell");
  __shared__ HexTile T;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= ntiles) return;
  const int tx = (int)(b % ntx), ty = (int)((b / ntx) % nty), tz = (int)(b / (ntx * nty));
  const int o0 = tx * kTX, o1 = ty * kTY, o2 = tz * kTZ;
  stage_hex_tile(H, geo, q, N, o0, o1, o2, T);
  __syncthreads();
  const int lx = threadIdx.x % kTX, ly = (threadIdx.x / kTX) % kTY, lz = threadIdx.x / (kTX * kTY);
  const int i = o0 + lx, j = o1 + ly, k = o2 + lz;
  if (i >= H.n[0] || j >= H.n[1] || k >= H.n[2]) return;
  const size_t idx = ((size_t)k * H.n[1] + j) * H.n[0] + i;
  const NbrTile nb{T, ((lz + 1) * kHY + (ly + 1)) * kHX + (lx + 1)};
  const NbrGlobal far{H, geo, q, N, i, j, k};
  HexCell Ci;
  load_cell(geo, N, idx, Ci);
  double qc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qc[v] = q[v * N + idx];
  double a[5][9];
  big_fit<WIDE>(nb, far, Ci, qc, a);

  double beta0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) beta0[v] = hex_beta0(a[v], Ci);
  // Bounds of the basis magnitudes over the 24 face Gauss points, for the
  // bound of |P_m - Q| used by the fallback pre-test.  The Gauss points
  // are convex combinations of the cell's vertices (bilinear faces), so
  // |X_e| <= max over the vertices; then |X_e^2 - m_ee| <= max(Xmax_e^2,
  // m_ee) and |X_a X_b - m_ab| <= Xmax_a Xmax_b + |m_ab|.
  double pmax[9];
  {
    double xm[3] = {0.0, 0.0, 0.0};
    const CellVerts cv = cell_verts(H, i, j, k);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      double xv[3];
      cell_vertex(H, cv, m, xv);
#pragma unroll
      for (int e = 0; e < 3; ++e) xm[e] = fmax(xm[e], fabs((xv[e] - Ci.c[e]) * Ci.ih));
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      pmax[e] = xm[e];
      pmax[3 + e] = fmax(xm[e] * xm[e], Ci.m[e]);
    }
    pmax[6] = xm[0] * xm[1] + fabs(Ci.m[3]);
    pmax[7] = xm[1] * xm[2] + fabs(Ci.m[4]);
    pmax[8] = xm[0] * xm[2] + fabs(Ci.m[5]);
  }
  // One pass over the sub-stencils.  With r_m = 1/(beta_m + eps) and
  // r_0 = 1/(beta_0 + eps) the weights are affine in tau: omega_m =
  // Gamma (1 + tau r_m), omega_0 / gamma_0 = 1 + tau r_0.  So the weight
  // sum is gamma_0 (1 + tau r_0) + Gamma (24 + tau sum_m r_m), and the
  // combined linear part sum_m (omega_m - Gamma omega_0 / gamma_0) b^m =
  // Gamma tau sum_m (r_m - r_0) b^m.  The pass gathers sum |beta_0 -
  // beta_m| (tau), sum r_m and sum (r_m - r_0) b^m; tau enters afterwards.
  double tsum[5], rsum[5], db[5][3], bnd[5], r0[5];
  TS* const cout = coef + coef_cell<TS>(idx);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    r0[v] = d_rcp(beta0[v] + P.eps);
    tsum[v] = rsum[v] = 0.0;
    db[v][0] = db[v][1] = db[v][2] = 0.0;
    // the bound of |P_0 - Q| starts the bound over all polynomials
    double b0 = 0.0;
#pragma unroll
    for (int n = 0; n < 9; ++n) b0 += fabs(a[v][n]) * pmax[n];
    bnd[v] = b0;
    // P_0 is parked in this cell's coefficient rows (read back by this lane
    // below), so that its 45 values do not hold registers through the pass
    TS* cv = cout + v * 10 * kCB<TS>;
#pragma unroll
    for (int e = 0; e < 9; ++e) cv[(e + 1) * kCB<TS>] = TS(a[v][e]);
  }
  asm volatile("" ::: "memory");
  auto take = [&](const double (&b)[5][3]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double bm = b[v][0] * b[v][0] + b[v][1] * b[v][1] + b[v][2] * b[v][2];
      tsum[v] += fabs(beta0[v] - bm);
      const double rm = d_rcp(bm + P.eps);
      rsum[v] += rm;
      const double dr = rm - r0[v];
#pragma unroll
      for (int e = 0; e < 3; ++e) db[v][e] += dr * b[v][e];
      bnd[v] = fmax(bnd[v], fabs(b[v][0]) * pmax[0] + fabs(b[v][1]) * pmax[1] + fabs(b[v][2]) * pmax[2]);
    }
  };
  if constexpr (WIDE) {
#pragma unroll 1
    for (int m = 0; m < kHexSubs<WIDE>; ++m) {
      double b[5][3];
      sub_fit<WIDE>(nb, Ci, qc, m, b);
      take(b);
    }
  } else {
    each_sub_fit(nb, Ci, qc, take);
  }
  double S[5], wb[5][3], w0r[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double tau = tsum[v] * (1.0 / kHexSubs<WIDE>);
    w0r[v] = 1.0 + tau * r0[v];
    S[v] = P.gamma0 * w0r[v] + P.Gamma * (double(kHexSubs<WIDE>) + tau * rsum[v]);
#pragma unroll
    for (int e = 0; e < 3; ++e) wb[v][e] = P.Gamma * tau * db[v][e];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double iS = d_rcp(S[v]);
    const double w0g = w0r[v] * iS;  // wbar_0 / gamma_0
    TS* cv = cout + v * 10 * kCB<TS>;
    double c[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) c[e] = (double)cv[(e + 1) * kCB<TS>];
#pragma unroll
    for (int e = 0; e < 3; ++e) c[e] = w0g * c[e] + iS * wb[v][e];
#pragma unroll
    for (int e = 3; e < 9; ++e) c[e] = w0g * c[e];
    cv[0] = TS(qc[v]);
#pragma unroll
    for (int e = 0; e < 9; ++e) cv[(e + 1) * kCB<TS>] = TS(c[e]);
  }
  const double margin = 1e-10;
  const double rmin = qc[0] - bnd[0];
  bool safe = rmin > margin * qc[0];
  if (safe) {
    double msq = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double mm = fabs(qc[1 + d]) + bnd[1 + d];
      msq += mm * mm;
    }
    safe = gm1 * (qc[4] - bnd[4] - 0.5 * msq * d_rcp(rmin)) > margin * gm1 * (fabs(qc[4]) + bnd[4]);
  }
  mask[idx] = safe ? 0u : kNeedsCheck;
}

// Exact fallback test of Sec. 4 for the cells the pre-test flagged.
template <bool WIDE = false>
__global__ void __launch_bounds__(kBlock) k_posit_exact_hex(HexGrid H, const double* __restrict__ geo,
                                                            const double* __restrict__ q, uint32_t* __restrict__ mask,
                                                            double gm1, size_t N) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  if (mask[idx] != kNeedsCheck) return;
  int i, j, k;
  split_index((uint32_t)idx, H.n[0], H.n[1], H.box.inv_n[0], H.box.inv_n[1], i, j, k);
  HexCell Ci;
  load_cell(geo, N, idx, Ci);
  double qc[5];
  for (int v = 0; v < 5; ++v) qc[v] = q[v * N + idx];
  const NbrGlobal nb{H, geo, q, N, i, j, k};
  double a[5][9];
  big_fit<WIDE>(nb, nb, Ci, qc, a);
  uint32_t bits = 0;
  for (int bit = 0; bit < 24; ++bit) {
    double X[3];
    cell_gp(H, Ci, i, j, k, bit, X);
    bool bad = false;
    for (int m = 0; m <= kHexSubs<WIDE> && !bad; ++m) {
      double val[5];
      if (m == 0) {
        for (int v = 0; v < 5; ++v) {
          double s = qc[v];
          for (int n = 0; n < 9; ++n) s += a[v][n] * pbasis(n, X, Ci.m);
          val[v] = s;
        }
      } else {
        double b[5][3];
        sub_fit<WIDE>(nb, Ci, qc, m - 1, b);
        for (int v = 0; v < 5; ++v) val[v] = qc[v] + b[v][0] * X[0] + b[v][1] * X[1] + b[v][2] * X[2];
      }
      bad = !(val[0] > 0.0);
      if (!bad) bad = gm1 * (val[4] - 0.5 * (val[1] * val[1] + val[2] * val[2] + val[3] * val[3]) / val[0]) < 0.0;
    }
    if (bad) bits |= 1u << bit;
  }
  mask[idx] = bits;
}

// ---------------------------------------------------------------- K3
// Value and physical gradient of the five variables of cell idx at the
// physical point x (centroid shifted by `shift` for periodic images), in
// the compute type: the scaled coordinates are formed in double (absolute
// positions), the polynomial is evaluated in TC.  A first-order fallback
// point gives the cell mean and zero gradient (Sec. 4).  cv points at the
// cell's 50 rows, kCB values apart: in the coefficient array or in a staged
// copy with the same row stride.
template <typename TC>
__device__ __forceinline__ void eval_hex_rows(const TC* cv, const double* __restrict__ geo, size_t N, size_t idx,
                                              const double (&shift)[3], const double (&x)[3], bool fb, TC (&val)[5],
                                              TC (&grad)[5][3]) {
  HexCell C;
  load_cell(geo, N, idx, C);
  TC X[3], m[6];
#pragma unroll
  for (int e = 0; e < 3; ++e) X[e] = TC((x[e] - C.c[e] - shift[e]) * C.ih);
#pragma unroll
  for (int e = 0; e < 6; ++e) m[e] = TC(C.m[e]);
  const TC ih = TC(C.ih);
  constexpr int CB = kCB<TC>;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const TC* ck = cv + v * 10 * CB;
    TC c[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) c[e] = ck[(e + 1) * CB];
    const TC q0 = ck[0];
    val[v] = q0 + c[0] * X[0] + c[1] * X[1] + c[2] * X[2] + c[3] * (X[0] * X[0] - m[0]) +
             c[4] * (X[1] * X[1] - m[1]) + c[5] * (X[2] * X[2] - m[2]) + c[6] * (X[0] * X[1] - m[3]) +
             c[7] * (X[1] * X[2] - m[4]) + c[8] * (X[0] * X[2] - m[5]);
    grad[v][0] = (c[0] + TC(2) * c[3] * X[0] + c[6] * X[1] + c[8] * X[2]) * ih;
    grad[v][1] = (c[1] + TC(2) * c[4] * X[1] + c[6] * X[0] + c[7] * X[2]) * ih;
    grad[v][2] = (c[2] + TC(2) * c[5] * X[2] + c[8] * X[0] + c[7] * X[1]) * ih;
  }
  if (fb) {
    asm volatile("");
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      val[v] = cv[v * 10 * CB];
      grad[v][0] = grad[v][1] = grad[v][2] = TC(0);
    }
  }
}

template <typename TC>
__device__ __forceinline__ void eval_hex(const TC* __restrict__ coef, const double* __restrict__ geo, size_t N,
                                         size_t idx, const double (&shift)[3], const double (&x)[3], bool fb,
                                         TC (&val)[5], TC (&grad)[5][3]) {
  eval_hex_rows(coef + coef_cell<TC>(idx), geo, N, idx, shift, x, fb, val, grad);
}

// Frame of Sec. 3 at the face point P: n along X_a x X_b, t2 along X_b,
// t1 = t2 x n (the arithmetic of the face flux's Gauss-point frame).
__device__ __forceinline__ void face_frame(const FacePoint& P, double (&n)[3], double (&t1)[3], double (&t2)[3]) {
  double av[3];
  cross3(P.xa, P.xb, av);
  const double ia = d_rcp(sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]));
  const double ib = d_rcp(sqrt(P.xb[0] * P.xb[0] + P.xb[1] * P.xb[1] + P.xb[2] * P.xb[2]));
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    n[e] = av[e] * ia;
    t2[e] = P.xb[e] * ib;
  }
  cross3(t2, n, t1);
}

// Frame at the centre of the face normal to D on vertex plane c (its lowest
// vertex), at the stage time of H.
__device__ __forceinline__ void face_centre_frame(const HexGrid& H, int D, int c0, int c1, int c2, double (&n)[3],
                                                  double (&t1)[3], double (&t2)[3]) {
  double cx[4][3], cu[4][3];
  face_corners(H, D, c0, c1, c2, cx, cu);
  FacePoint P;
  face_point(cx, cu, 0.0, 0.0, P);
  face_frame(P, n, t1, t2);
}

// Value and physical gradient of the five conservative variables at the
// physical point x of the cell reconstructed in characteristic variables:
// cv points at the cell in its face array, B holds the face's eigenvectors.
// A first-order fallback point gives the cell mean and zero gradient.
template <typename TC>
__device__ __forceinline__ void eval_char_hex(const TC* __restrict__ cv, const double* __restrict__ geo, size_t N,
                                              size_t idx, const double (&shift)[3], const double (&x)[3], bool fb,
                                              const CharFrame& B, TC (&val)[5], TC (&grad)[5][3]) {
  HexCell C;
  load_cell(geo, N, idx, C);
  TC X[3], m[6];
#pragma unroll
  for (int e = 0; e < 3; ++e) X[e] = TC((x[e] - C.c[e] - shift[e]) * C.ih);
#pragma unroll
  for (int e = 0; e < 6; ++e) m[e] = TC(C.m[e]);
  const TC ih = TC(C.ih);
  constexpr int CB = kCB<TC>;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    val[v] = cv[10 * v * CB];
    grad[v][0] = grad[v][1] = grad[v][2] = TC(0);
  }
  if (fb) return;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const TC* ck = cv + 10 * f * CB;
    TC c[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) c[e] = ck[(e + 1) * CB];
    const TC du = c[0] * X[0] + c[1] * X[1] + c[2] * X[2] + c[3] * (X[0] * X[0] - m[0]) +
                  c[4] * (X[1] * X[1] - m[1]) + c[5] * (X[2] * X[2] - m[2]) + c[6] * (X[0] * X[1] - m[3]) +
                  c[7] * (X[1] * X[2] - m[4]) + c[8] * (X[0] * X[2] - m[5]);
    TC g[3];
    g[0] = (c[0] + TC(2) * c[3] * X[0] + c[6] * X[1] + c[8] * X[2]) * ih;
    g[1] = (c[1] + TC(2) * c[4] * X[1] + c[6] * X[0] + c[7] * X[2]) * ih;
    g[2] = (c[2] + TC(2) * c[5] * X[2] + c[8] * X[0] + c[7] * X[1]) * ih;
    double r[5];
    char_rcol(B, f, r);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const TC rv = TC(r[v]);
      val[v] += rv * du;
#pragma unroll
      for (int e = 0; e < 3; ++e) grad[v][e] += rv * g[e];
    }
  }
}

// Conservative variables seen from a frame moving with u (one vector, also
// applied to the gradients), then rotated into the frame (nx, ny, nz); in
// the compute type.
template <typename TC>
__device__ __forceinline__ void to_local(const TC (&val)[5], const TC (&grad)[5][3], const double (&ud)[3],
                                         const double (&nxd)[3], const double (&nyd)[3], const double (&nzd)[3],
                                         TC (&W)[5], TC (&dW)[3][5]) {
  TC u[3], n[3][3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    u[e] = TC(ud[e]);
    n[0][e] = TC(nxd[e]);
    n[1][e] = TC(nyd[e]);
    n[2][e] = TC(nzd[e]);
  }
  const TC uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  // shifted values
  TC s[5];
  s[0] = val[0];
  TC Mu = TC(0);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    s[1 + e] = val[1 + e] - val[0] * u[e];
    Mu += val[1 + e] * u[e];
  }
  s[4] = val[4] - Mu + TC(0.5) * val[0] * uu;
  W[0] = s[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) W[1 + j] = s[1] * n[j][0] + s[2] * n[j][1] + s[3] * n[j][2];
  W[4] = s[4];
  // gradients: derivative along n_j of the shifted variables
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    TC g[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) g[v] = grad[v][0] * n[j][0] + grad[v][1] * n[j][1] + grad[v][2] * n[j][2];
    TC gs[5];
    gs[0] = g[0];
    TC gMu = TC(0);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      gs[1 + e] = g[1 + e] - g[0] * u[e];
      gMu += g[1 + e] * u[e];
    }
    gs[4] = g[4] - gMu + TC(0.5) * g[0] * uu;
    dW[j][0] = gs[0];
#pragma unroll
    for (int r = 0; r < 3; ++r) dW[j][1 + r] = gs[1] * n[r][0] + gs[2] * n[r][1] + gs[3] * n[r][2];
    dW[j][4] = gs[4];
  }
}

// Local-frame flux vector back to global components and to the fixed frame.
__device__ __forceinline__ void to_global(const double (&f)[5], const double (&u)[3], const double (&nx)[3],
                                          const double (&ny)[3], const double (&nz)[3], double (&g)[5]) {
  double M[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) M[e] = nx[e] * f[1] + ny[e] * f[2] + nz[e] * f[3];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  g[0] = f[0];
#pragma unroll
  for (int e = 0; e < 3; ++e) g[1 + e] = M[e] + u[e] * f[0];
  g[4] = f[4] + (M[0] * u[0] + M[1] * u[1] + M[2] * u[2]) + 0.5 * uu * f[0];
}

// Rows of the flux kernel's per-lane LDS slot: the Gauss point's geometry
// (18), and with per-face reconstructions (characteristic variables) the
// face-centre frame (9) and the face's mean state (5).
template <bool FS>
constexpr int kHexStash = FS ? 32 : 18;

// One lane = one Gauss point of one face normal to axis D (uniform over the
// workgroup); lane l of block lb takes Gauss point l % 4 of face slot l / 4
// in the flux block order of the box kernels (face_of_block).
// PR: the extended viscous model (viscosity law, Prandtl correction); FS:
// per-face coefficient arrays (reconstruction in characteristic variables),
// H.box.fs_stride elements apart.
template <typename TC, bool PR = false, bool FS = false>
__device__ __forceinline__ void flux_hex_face(const HexGrid& H, const TC* __restrict__ coef,
                                              const double* __restrict__ geo, const uint32_t* __restrict__ mask,
                                              TC* __restrict__ face, double* __restrict__ vface,
                                              const GasParams<TC>& gp, TC dt, TC idt, size_t N, unsigned lb, int D,
                                              double (&stash)[kHexStash<FS>][kBlock], TC* stage = nullptr) {
  const int gpi = (int)(threadIdx.x & 3);
  int c[3];
  size_t f;
  const bool live = face_of_block(H.box, D, lb, threadIdx.x >> 2, c, f);
  // Face on the lower side of cell c along D: plane c[D] (c[d] in [0, n_d)
  // for every lane, dead ones included).
  double cx[4][3], cu[4][3];
  if (D == 0)
    face_corners_in<0>(H, c, cx, cu);
  else if (D == 1)
    face_corners_in<1>(H, c, cx, cu);
  else
    face_corners_in<2>(H, c, cx, cu);
  FacePoint Pt;
  face_point(cx, cu, (gpi >> 1) ? kGaussNode : -kGaussNode, (gpi & 1) ? kGaussNode : -kGaussNode, Pt);
  double av[3], adot[3], t1[3], t2[3];
  cross3(Pt.xa, Pt.xb, av);
  cross3(Pt.ua, Pt.xb, t1);
  cross3(Pt.xa, Pt.ub, t2);
#pragma unroll
  for (int e = 0; e < 3; ++e) adot[e] = t1[e] + t2[e];
  const double area = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
  double nx[3], ny[3], nz[3];
  const double iarea = d_rcp(area);
  const double ilb = d_rcp(sqrt(Pt.xb[0] * Pt.xb[0] + Pt.xb[1] * Pt.xb[1] + Pt.xb[2] * Pt.xb[2]));
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    nx[e] = av[e] * iarea;
    nz[e] = Pt.xb[e] * ilb;
  }
  cross3(nz, nx, ny);
  // The point's geometry is parked in LDS (one slot per lane, no sharing)
  // and read back where each side needs it, so that it does not occupy
  // registers across the two sides' gas-kinetic terms: x, u, the frame,
  // area, d|a|/dt rate and the volume rate.
  {
    double* g = &stash[0][threadIdx.x];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      g[(0 + e) * kBlock] = Pt.x[e];
      g[(3 + e) * kBlock] = Pt.u[e];
      g[(6 + e) * kBlock] = nx[e];
      g[(9 + e) * kBlock] = ny[e];
      g[(12 + e) * kBlock] = nz[e];
    }
    g[15 * kBlock] = area;
    g[16 * kBlock] = Pt.u[0] * adot[0] + Pt.u[1] * adot[1] + Pt.u[2] * adot[2];
    g[17 * kBlock] = 0.25 * (Pt.u[0] * av[0] + Pt.u[1] * av[1] + Pt.u[2] * av[2]);
    if constexpr (FS) {
      // the frame at the face centre, the projection frame of both cells'
      // reconstructions for this face
      FacePoint Pc;
      face_point(cx, cu, 0.0, 0.0, Pc);
      double fn[3], f1[3], f2[3];
      face_frame(Pc, fn, f1, f2);
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        g[(18 + e) * kBlock] = fn[e];
        g[(21 + e) * kBlock] = f1[e];
        g[(24 + e) * kBlock] = f2[e];
      }
    }
  }
  // The re-reads are plain LDS loads behind a compiler-only memory fence
  // (no instruction): the fence keeps the compiler from forwarding the
  // stored registers, and unlike a volatile access it leaves the loads
  // free to be issued together with the others.
  const double* gs = &stash[0][threadIdx.x];
  auto get3 = [&](int k, double (&v)[3]) {
#pragma unroll
    for (int e = 0; e < 3; ++e) v[e] = gs[(k + e) * kBlock];
  };

  // The two cells: c itself (in range, no shift) and its lower neighbour
  // along D, which wraps to the last plane, shifted back by the period,
  // where c[D] = 0.
  double shL[3] = {0.0, 0.0, 0.0}, shR[3] = {0.0, 0.0, 0.0};
  size_t iL, iR;
  {
    const unsigned s1 = (unsigned)H.n[0], s2 = s1 * (unsigned)H.n[1];
    const unsigned r = (unsigned)c[0] + (unsigned)c[1] * s1 + (unsigned)c[2] * s2;
    const unsigned sD = D == 0 ? 1u : (D == 1 ? s1 : s2);
    const int cD = D == 0 ? c[0] : (D == 1 ? c[1] : c[2]);
    const bool wrap = cD == 0;
    iR = r;
    iL = wrap ? r + (unsigned)(H.n[D] - 1) * sD : r - sD;
    const double sh = wrap ? -H.period[D] : 0.0;
    shL[0] = D == 0 ? sh : 0.0;
    shL[1] = D == 1 ? sh : 0.0;
    shL[2] = D == 2 ? sh : 0.0;
  }
  const bool fbL = (mask[iL] >> (4 * (2 * D + 1) + gpi)) & 1u;
  const bool fbR = (mask[iR] >> (4 * (2 * D) + gpi)) & 1u;
  // the left cell's reconstruction for its high face, the right cell's for
  // its low face (one array unless the faces have their own)
  const TC* coefL = FS ? coef + (size_t)(2 * D + 1) * H.box.fs_stride : coef;
  const TC* coefR = FS ? coef + (size_t)(2 * D) * H.box.fs_stride : coef;
  if constexpr (FS) {
    // the face's mean state: the two cells' conservative means
    constexpr int CB = kCB<TC>;
    const TC* mL = coefL + coef_cell<TC>(iL);
    const TC* mR = coefR + coef_cell<TC>(iR);
#pragma unroll
    for (int v = 0; v < 5; ++v)
      stash[27 + v][threadIdx.x] = 0.5 * ((double)mL[10 * v * CB] + (double)mR[10 * v * CB]);
  }
  auto eval_side = [&](const TC* cf, size_t icell, const double (&sh)[3], const double (&x)[3], bool fb,
                       TC (&val)[5], TC (&grad)[5][3]) {
    if constexpr (FS) {
      CharFrame B;
      {
        double fn[3], f1[3], f2[3], Qb[5];
        get3(18, fn);
        get3(21, f1);
        get3(24, f2);
#pragma unroll
        for (int v = 0; v < 5; ++v) Qb[v] = gs[(27 + v) * kBlock];
        char_frame(Qb, fn, f1, f2, gp.gamma, B);
      }
      eval_char_hex(cf + coef_cell<TC>(icell), geo, N, icell, sh, x, fb, B, val, grad);
    } else {
      eval_hex(cf, geo, N, icell, sh, x, fb, val, grad);
    }
  };

  FluxAcc<TC> acc;
  acc_begin(acc);
  if constexpr (std::is_same<TC, float>::value) {
    // FP32: both sides' local states first, then the side terms; the
    // accumulators are not live while the coefficients are loaded (113
    // registers, no spills, 7% faster).  In FP64 this order is 11% slower
    // than the sides one after the other with the right cell's loads
    // deferred, below.
    TC WL[5], dWL[3][5], WR[5], dWR[3][5];
    {
      asm volatile("" ::: "memory");
      double x[3], u[3], n0[3], n1[3], n2[3];
      get3(0, x);
      get3(3, u);
      get3(6, n0);
      get3(9, n1);
      get3(12, n2);
      TC val[5], grad[5][3];
      eval_side(coefL, iL, shL, x, fbL, val, grad);
      to_local(val, grad, u, n0, n1, n2, WL, dWL);
      eval_side(coefR, iR, shR, x, fbR, val, grad);
      to_local(val, grad, u, n0, n1, n2, WR, dWR);
    }
    side_terms<+1, PR, kAssignFirst<TC>>(WL, dWL, gp, acc);
    side_terms<-1, PR>(WR, dWR, gp, acc);
  } else if constexpr (!FS) {
    // FP64: the right cells' coefficients are staged in LDS by direct
    // loads issued after the left cell's values have arrived, as in the box
    // flux (the same [50 rows][8 faces] groups of 64-byte rows), and read
    // from there after the left side's terms; the right cell's geometry
    // comes from global memory as before.
    static_assert(sizeof(TC) == 8 && kCB<TC> == 8, "rows of 8 doubles");
    const unsigned l = threadIdx.x & 63u;
    TC* rs = stage + (threadIdx.x >> 6) * kStageWave;
    unsigned cell0 = __shfl((unsigned)iR, (int)(((l >> 1) & 7u) * 4u));
    unsigned cell1 = __shfl((unsigned)iR, (int)((8u + ((l >> 1) & 7u)) * 4u));
    {
      asm volatile("" ::: "memory");
      double x[3], u[3], n0[3], n1[3], n2[3];
      get3(0, x);
      get3(3, u);
      get3(6, n0);
      get3(9, n1);
      get3(12, n2);
      TC val[5], grad[5][3];
      eval_hex(coefL, geo, N, iL, shL, x, fbL, val, grad);
      TC W[5], dW[3][5];
      to_local(val, grad, u, n0, n1, n2, W, dW);
      asm volatile("" : "+v"(cell0), "+v"(cell1) : "v"(W[0]), "v"(dW[2][4]));
      const unsigned lane = (l >> 4) * 64 + (l & 1u) * 4;
      const GlobalPtr s0 = (GlobalPtr)((const char*)(coefR + coef_cell<TC>(cell0)) + lane);
      const GlobalPtr s1 = (GlobalPtr)((const char*)(coefR + coef_cell<TC>(cell1)) + lane);
      const LdsPtr d0 = (LdsPtr)rs;
      const LdsPtr d1 = (LdsPtr)(rs + kStageGroup);
      copy_pieces<0, 12>(s0, d0);
      copy_pieces<0, 12>(s1, d1);
      if (l < 32u) {
        copy_pieces<12, 13>(s0, d0);
        copy_pieces<12, 13>(s1, d1);
      }
      side_terms<+1, PR, kAssignFirst<TC>>(W, dW, gp, acc);
    }
    size_t iRt = iR;
    after_left_side(iRt, acc);
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    {
      const unsigned slot = threadIdx.x >> 2 & 15u;
      const TC* cv = rs + (slot >> 3) * kStageGroup + (slot & 7u);
      double x[3], u[3], n0[3], n1[3], n2[3];
      get3(0, x);
      get3(3, u);
      get3(6, n0);
      get3(9, n1);
      get3(12, n2);
      TC val[5], grad[5][3];
      eval_hex_rows(cv, geo, N, iRt, shR, x, fbR, val, grad);
      TC W[5], dW[3][5];
      to_local(val, grad, u, n0, n1, n2, W, dW);
      side_terms<-1, PR>(W, dW, gp, acc);
    }
  } else {
    {
      asm volatile("" ::: "memory");
      double x[3], u[3], n0[3], n1[3], n2[3];
      get3(0, x);
      get3(3, u);
      get3(6, n0);
      get3(9, n1);
      get3(12, n2);
      TC val[5], grad[5][3];
      eval_side(coefL, iL, shL, x, fbL, val, grad);
      TC W[5], dW[3][5];
      to_local(val, grad, u, n0, n1, n2, W, dW);
      side_terms<+1, PR, kAssignFirst<TC>>(W, dW, gp, acc);
    }
    size_t iRt = iR;
    after_left_side(iRt, acc);
    {
      asm volatile("" ::: "memory");
      double x[3], u[3], n0[3], n1[3], n2[3];
      get3(0, x);
      get3(3, u);
      get3(6, n0);
      get3(9, n1);
      get3(12, n2);
      TC val[5], grad[5][3];
      eval_side(coefR, iRt, shR, x, fbR, val, grad);
      TC W[5], dW[3][5];
      to_local(val, grad, u, n0, n1, n2, W, dW);
      side_terms<-1, PR>(W, dW, gp, acc);
    }
  }
  asm volatile("" ::: "memory");
  double u[3], n0[3], n1[3], n2[3];
  get3(3, u);
  get3(6, n0);
  get3(9, n1);
  get3(12, n2);
  const double area2 = gs[15 * kBlock], rate = gs[16 * kBlock], vrate = gs[17 * kBlock];
  TC Fl[5], dFl[5];
  finish_flux<PR>(acc, gp, dt, idt, Fl, dFl);
  double fl[5], dfl[5], q0l[5];
#pragma unroll
  for (int e = 0; e < 5; ++e) {
    fl[e] = (double)Fl[e];
    dfl[e] = (double)dFl[e];
    q0l[e] = (double)acc.Q0[e];
  }
  double F[5], dF[5], Q0[5];
  to_global(fl, u, n0, n1, n2, F);
  to_global(dfl, u, n0, n1, n2, dF);
  to_global(q0l, u, n0, n1, n2, Q0);
  double out[12];
#pragma unroll
  for (int e = 0; e < 5; ++e) {
    out[e] = 0.25 * area2 * F[e];
    out[5 + e] = 0.25 * (area2 * dF[e] - Q0[e] * rate);
  }
  out[10] = vrate;
  out[11] = 0.25 * rate;
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    out[e] = quad_xor_add<2>(quad_xor_add<1>(out[e]));
  }
  if (live && gpi == 0) {
#pragma unroll
    for (int e = 0; e < 10; ++e) face[(size_t)e * N + f] = TC(out[e]);
    vface[f] = out[10];
    vface[N + f] = out[11];
  }
}

// All faces of the three directions in one launch, nb blocks of 64 faces per
// direction, interleaved (flux_block).  Register budget: two waves per SIMD
// in FP64; four in FP32 (113 registers).
template <typename TC, bool PR = false, bool FS = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(TC) == 8 ? 2 : 4)))
    k_flux_hex(HexGrid H, const TC* __restrict__ coef, const double* __restrict__ geo,
               const uint32_t* __restrict__ mask, TC* __restrict__ fx, TC* __restrict__ fy, TC* __restrict__ fz,
               double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz, GasParams<TC> gp, TC dt,
               TC idt, size_t N, unsigned nb) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= 3 * nb) return;
  const unsigned nbs[3] = {nb, nb, nb};
  int D;
  unsigned lb;
  flux_block(b, nbs, D, lb);
  TC* face = D == 0 ? fx : (D == 1 ? fy : fz);
  double* vface = D == 0 ? vx : (D == 1 ? vy : vz);
  __shared__ double stash[kHexStash<FS>][kBlock];
  if constexpr (sizeof(TC) == 8 && !FS) {
    __shared__ double stage[kBlock / 64 * kStageWave];
    flux_hex_face<TC, PR, FS>(H, coef, geo, mask, face, vface, gp, dt, idt, N, lb, D, stash, stage);
  } else {
    flux_hex_face<TC, PR, FS>(H, coef, geo, mask, face, vface, gp, dt, idt, N, lb, D, stash);
  }
}

// ---------------------------------------------------------------- K4
// Stage update of U = |Omega| Q and |Omega|.
// mode 0: one-stage; mode 1: first stage (writes qs, acc, vacc);
// mode 2: second stage.
template <typename TF>
__global__ void __launch_bounds__(kBlock) k_update_hex(HexGrid H, double* __restrict__ q, double* __restrict__ qs,
                                                       double* __restrict__ acc, double* __restrict__ vacc,
                                                       const double* __restrict__ geo, const TF* __restrict__ fx,
                                                       const TF* __restrict__ fy, const TF* __restrict__ fz,
                                                       const double* __restrict__ vx, const double* __restrict__ vy,
                                                       const double* __restrict__ vz, double dt, int mode, size_t N) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  int c[3];
  split_index((uint32_t)idx, H.n[0], H.n[1], H.box.inv_n[0], H.box.inv_n[1], c[0], c[1], c[2]);
  const TF* fs[3] = {fx, fy, fz};
  const double* vs[3] = {vx, vy, vz};
  // byte offsets in 32 bits from each array's uniform base (fewer than 2^29
  // cells)
  const unsigned ob = (unsigned)idx * 8u;
  auto ld = [](const auto* base, unsigned off) { return *(const decltype(+*base)*)((const char*)base + off); };
  auto el = [&](double* a, int v) -> double& { return *(double*)((char*)(a + (size_t)v * N) + ob); };
  double R[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) R[e] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int hi[3] = {c[0], c[1], c[2]};
    hi[d] = hi[d] + 1 == H.n[d] ? 0 : hi[d] + 1;
    const unsigned hi_i = ((unsigned)hi[2] * (unsigned)H.n[1] + (unsigned)hi[1]) * (unsigned)H.n[0] + (unsigned)hi[0];
    const unsigned hf = hi_i * (unsigned)sizeof(TF), lf = (unsigned)idx * (unsigned)sizeof(TF);
#pragma unroll
    for (int e = 0; e < 10; ++e) R[e] -= (double)ld(fs[d] + e * N, hf) - (double)ld(fs[d] + e * N, lf);
    R[10] += ld(vs[d], hi_i * 8u) - ld(vs[d], ob);
    R[11] += ld(vs[d] + N, hi_i * 8u) - ld(vs[d] + N, ob);
  }
  if (mode == 2) {
    const double Vn = ld(vacc, ob) + dt * dt / 3.0 * R[11];
#pragma unroll
    for (int v = 0; v < 5; ++v) el(q, v) = (el(acc, v) + dt * dt / 3.0 * R[5 + v]) / Vn;
    return;
  }
  const double V = ld(geo, ob);
  if (mode == 0) {
    const double Vn = V + dt * R[10] + 0.5 * dt * dt * R[11];
#pragma unroll
    for (int v = 0; v < 5; ++v) el(q, v) = (V * el(q, v) + dt * R[v] + 0.5 * dt * dt * R[5 + v]) / Vn;
    return;
  }
  const double Vs = V + 0.5 * dt * R[10] + 0.125 * dt * dt * R[11];
  *(double*)((char*)vacc + ob) = V + dt * R[10] + dt * dt / 6.0 * R[11];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double U = V * el(q, v);
    el(qs, v) = (U + 0.5 * dt * R[v] + 0.125 * dt * dt * R[5 + v]) / Vs;
    el(acc, v) = U + dt * R[v] + dt * dt / 6.0 * R[5 + v];
  }
}

// ---------------------------------------------------------------- reductions
__global__ void __launch_bounds__(kBlock) k_dt_hex(HexGrid H, const double* __restrict__ q, double gamma,
                                                   double* __restrict__ part, size_t N) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double val = 1e300;
  if (idx < N) {
    int i, j, k;
  split_index((uint32_t)idx, H.n[0], H.n[1], H.box.inv_n[0], H.box.inv_n[1], i, j, k);
    double cx[8][3];
    for (int m = 0; m < 8; ++m) {
      double u[3];
      hex_vertex(H, i + ((m >> 2) & 1), j + ((m >> 1) & 1), k + (m & 1), cx[m], u);
    }
    double hmin = 1e300;
    for (int d = 0; d < 3; ++d) {
      const int bit = 4 >> d;
      double lo[3] = {0, 0, 0}, up[3] = {0, 0, 0};
      for (int m = 0; m < 8; ++m)
        for (int e = 0; e < 3; ++e) {
          if (m & bit) up[e] += 0.25 * cx[m][e];
          else lo[e] += 0.25 * cx[m][e];
        }
      const double dd = sqrt((up[0] - lo[0]) * (up[0] - lo[0]) + (up[1] - lo[1]) * (up[1] - lo[1]) +
                             (up[2] - lo[2]) * (up[2] - lo[2]));
      hmin = fmin(hmin, dd);
    }
    const double rho = q[idx];
    const double u = q[N + idx] / rho, v = q[2 * N + idx] / rho, w = q[3 * N + idx] / rho;
    const double p = (gamma - 1.0) * (q[4 * N + idx] - 0.5 * rho * (u * u + v * v + w * w));
    const double c = sqrt(gamma * p / rho);
    val = hmin / (sqrt(u * u + v * v + w * w) + c);
    if (!(val > 0.0)) val = -1.0;
  }
  const double r = block_reduce(val, sh, MinOp());
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_totals_hex(const double* __restrict__ q, const double* __restrict__ geo,
                                                       double* __restrict__ part, size_t N, int nblk) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  for (int v = 0; v < 5; ++v) {
    const double x = idx < N ? q[(size_t)v * N + idx] * geo[idx] : 0.0;
    const double r = block_reduce(x, sh, SumOp());
    if (threadIdx.x == 0) part[(size_t)v * nblk + blockIdx.x] = r;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- debug
// Gauss-point states of every cell (parity hook).  fs_stride != 0: per-face
// reconstructions in characteristic variables (arrays fs_stride apart),
// projected back with the face's eigenvectors.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_debug_gp_hex(HexGrid H, const TC* __restrict__ coef,
                                                         const double* __restrict__ geo,
                                                         const uint32_t* __restrict__ mask, size_t N, double gamma,
                                                         size_t fs_stride, double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  int i, j, k;
  split_index((uint32_t)idx, H.n[0], H.n[1], H.box.inv_n[0], H.box.inv_n[1], i, j, k);
  const double zero[3] = {0.0, 0.0, 0.0};
  for (int bit = 0; bit < 24; ++bit) {
    const int f = bit >> 2, gp = bit & 3, d = f >> 1;
    int c[3] = {i, j, k};
    c[d] += (f & 1);
    double cx[4][3], cu[4][3];
    face_corners(H, d, c[0], c[1], c[2], cx, cu);
    FacePoint P;
    face_point(cx, cu, (gp >> 1) ? kGaussNode : -kGaussNode, (gp & 1) ? kGaussNode : -kGaussNode, P);
    TC val[5], grad[5][3];
    const bool fb = (mask[idx] >> bit) & 1u;
    if (fs_stride) {
      // the neighbour across face f and its reconstruction for that face
      int nc[3] = {i, j, k};
      nc[d] += (f & 1) ? 1 : -1;
      double sh[3];
      const size_t in = hex_index(H, nc[0], nc[1], nc[2], sh);
      constexpr int CB = kCB<TC>;
      const TC* cv = coef + (size_t)f * fs_stride + coef_cell<TC>(idx);
      const TC* cn = coef + (size_t)(f ^ 1) * fs_stride + coef_cell<TC>(in);
      double Qb[5];
      for (int v = 0; v < 5; ++v) Qb[v] = 0.5 * ((double)cv[10 * v * CB] + (double)cn[10 * v * CB]);
      FacePoint Pc;
      face_point(cx, cu, 0.0, 0.0, Pc);
      double fn[3], f1[3], f2[3];
      face_frame(Pc, fn, f1, f2);
      CharFrame B;
      char_frame(Qb, fn, f1, f2, gamma, B);
      eval_char_hex(cv, geo, N, idx, zero, P.x, fb, B, val, grad);
    } else {
      eval_hex(coef, geo, N, idx, zero, P.x, fb, val, grad);
    }
    for (int v = 0; v < 5; ++v) {
      double* o = out + ((idx * 24 + bit) * 5 + v) * 4;
      o[0] = val[v];
      o[1] = grad[v][0];
      o[2] = grad[v][1];
      o[3] = grad[v][2];
    }
  }
}

template <typename TF>
__global__ void __launch_bounds__(kBlock) k_debug_face_hex(const TF* __restrict__ face, int d, size_t N,
                                                           double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  for (int k = 0; k < 10; ++k) out[((size_t)d * N + idx) * 10 + k] = (double)face[(size_t)k * N + idx];
}

}  // namespace hgks
