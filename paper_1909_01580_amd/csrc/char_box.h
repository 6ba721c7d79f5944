// Reconstruction in characteristic variables on box grids (Pan & Xu, Sec. 4:
// the option stated after the limiting procedure).
//
// For the face of a cell normal to axis D on side s (s = 0 the low face,
// s = 1 the high one) the stencil data are projected to U = L Q, L = R^-1,
// R the right eigenvectors of the Euler Jacobian along e_D, taken at the
// mean of the two cell averages that share the face.  The WENO-AO
// reconstruction of Sec. 2 runs on each component of U -- the least squares
// are linear, so its polynomials are the projected ones, while indicators
// and nonlinear weights belong to each characteristic field.  Each cell
// thus gets six reconstructions, one per face, stored as six coefficient
// arrays of the usual layout (array 2 D + s): row 10 v holds the
// conservative cell mean of variable v, rows 10 f + 1 .. 10 f + 9 the nine
// coefficients of characteristic field f.  The face flux reads the left
// cell's array 2 D + 1 and the right cell's array 2 D, forms R from the two
// means (the same mean state) and projects back at its Gauss point: value
// Q_c + R dU(x), gradient R grad U(x), dU the fields' deviation from their
// means.  The positivity fallback stays on the conservative polynomials
// (the mask of the component-wise reconstruction).
//
// The shear eigenvectors are the tangential axes D+1, D+2 in cyclic order,
// the frame of the face flux.
#pragma once

#include "box_kernels.h"

namespace hgks {

// Characteristic reconstruction of reconstruction-box cell idx for its face
// fs = 2 D + s, written into the face array `out` (coefficient layout).
template <typename TC>
__device__ __forceinline__ void char_recon_box_cell(const double* __restrict__ q, TC* out, const BoxGrid& G,
                                                    const WenoParams<TC>& P, double gamma, size_t idx, int D,
                                                    int side) {
  int ri, rj, rk;
  split_index((uint32_t)idx, G.nr[0], G.nr[1], G.inv_nr[0], G.inv_nr[1], ri, rj, rk);
  const int i = ri - G.g[0], j = rj - G.g[1], k = rk - G.g[2];
  int ix[3], iy[3], iz[3];
  double sx[3], sy[3], sz[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    ix[o] = bc_index(G, 0, i + o - 1, sx[o]);
    iy[o] = bc_index(G, 1, j + o - 1, sy[o]);
    iz[o] = bc_index(G, 2, k + o - 1, sz[o]);
  }
  const size_t nx = G.n[0], nxy = (size_t)G.n[0] * G.n[1], N = nxy * G.n[2];
  // value of variable v in the stencil cell at offset (ox, oy, oz), mirror
  // images with the normal momentum reversed
  auto at = [&](int v, int ox, int oy, int oz) -> double {
    const double s = v == 1 ? sx[ox + 1] : (v == 2 ? sy[oy + 1] : (v == 3 ? sz[oz + 1] : 1.0));
    return s * q[v * N + iz[oz + 1] * nxy + iy[oy + 1] * nx + ix[ox + 1]];
  };
  double Qc[5], Qb[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Qc[v] = at(v, 0, 0, 0);
    // the neighbour across the face (D and side are uniform: literal offsets)
    double qn;
    if (D == 0)
      qn = side ? at(v, 1, 0, 0) : at(v, -1, 0, 0);
    else if (D == 1)
      qn = side ? at(v, 0, 1, 0) : at(v, 0, -1, 0);
    else
      qn = side ? at(v, 0, 0, 1) : at(v, 0, 0, -1);
    Qb[v] = 0.5 * (Qc[v] + qn);
  }
  CharBasis B;
  char_basis(Qb, D, gamma, B);
  TC* base = out + coef_cell<TC>(idx);
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    double l[5];
    char_lrow(B, f, l);
    // d = L_f (Q_s - Q_c) over the 18 stencil cells, one conservative
    // variable per pass: the memory clobber keeps each pass's 18 loads from
    // being issued together with the others'.
    double acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      // the stencil indices are re-read by every pass, so that the 90
      // addresses of a field are not formed once and held in registers
      asm volatile("" : "+v"(ix[0]), "+v"(ix[1]), "+v"(ix[2]), "+v"(iy[0]), "+v"(iy[1]), "+v"(iy[2]),
                   "+v"(iz[0]), "+v"(iz[1]), "+v"(iz[2]));
#pragma unroll
      for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
          for (int ox = -1; ox <= 1; ++ox) {
            const int nz = (ox != 0) + (oy != 0) + (oz != 0);
            if (nz == 1 || nz == 2) acc[sidx(ox, oy, oz)] += l[v] * (at(v, ox, oy, oz) - Qc[v]);
          }
      asm volatile("" ::: "memory");
    }
    TC d[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) d[t] = TC(acc[t]);
    BoxRecon<TC> r;
    weno_box(d, P, r);
    TC* cv = base + f * 10 * kCB<TC>;
    cv[0] = TC(Qc[f]);  // the conservative mean of variable f
#pragma unroll
    for (int m = 0; m < 9; ++m) cv[(m + 1) * kCB<TC>] = r.c[m];
    // the next field's loads are not hoisted into this field's work
    asm volatile("" ::: "memory");
  }
}

// One lane per reconstruction-box cell, blockIdx.y = face 2 D + s.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_char_recon_box(const double* __restrict__ q, TC* faces, BoxGrid G,
                                                           WenoParams<TC> P, double gamma, size_t NR,
                                                           unsigned nblk) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nblk) return;
  const size_t idx = (size_t)b * kBlock + threadIdx.x;
  if (idx >= NR) return;
  const int fs = (int)blockIdx.y;
  char_recon_box_cell(q, faces + (size_t)fs * G.fs_stride, G, P, gamma, idx, fs >> 1, fs & 1);
}

}  // namespace hgks
