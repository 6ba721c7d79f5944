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

// LDS tile: kCX x kCY x kCZ reconstruction-box cells (one wave per x-row
// of 64, so that the coefficient stores of a wave are contiguous) and one
// layer around them.  The five variables of every tile cell are staged
// once, boundary images resolved (mirror images with the normal momentum
// reversed), and serve the six faces of every cell of the tile.
constexpr int kCX = 64, kCY = 2, kCZ = 2;
constexpr int kCHX = kCX + 2, kCHY = kCY + 2, kCHZ = kCZ + 2, kCHalo = kCHX * kCHY * kCHZ;

// Characteristic reconstruction of the tile cell at `base` (its index in
// the tile) for its face fs = 2 D + s, written into the face array `out`
// (coefficient layout) at reconstruction-box cell idx.
template <typename TC>
__device__ __forceinline__ void char_recon_tile_cell(const double (&T)[5][kCHalo], int base, TC* out,
                                                     const WenoParams<TC>& P, double gamma, size_t idx, int D,
                                                     int side) {
  auto at = [&](int v, int ox, int oy, int oz) -> double { return T[v][base + (oz * kCHY + oy) * kCHX + ox]; };
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
  TC* base_out = out + coef_cell<TC>(idx);
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    double l[5];
    char_lrow(B, f, l);
    // d = L_f (Q_s - Q_c) over the 18 stencil cells, one conservative
    // variable per pass: the memory fence keeps each pass's 18 loads from
    // being issued together with the others' (their values would all be
    // live at once).
    double acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
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
    TC* cv = base_out + f * 10 * kCB<TC>;
    cv[0] = TC(Qc[f]);  // the conservative mean of variable f
#pragma unroll
    for (int m = 0; m < 9; ++m) cv[(m + 1) * kCB<TC>] = r.c[m];
    asm volatile("" ::: "memory");
  }
}

// Tile b of the reconstruction box (tiles x-fastest, ntx x nty x ntz of
// them) by the whole workgroup: the tile is staged in T, then every lane
// reconstructs its cell for the six faces in turn.  Lanes of cells beyond
// the box only help to stage the tile.
template <typename TC>
__device__ __forceinline__ void char_recon_tile(const double* __restrict__ q, TC* faces, const BoxGrid& G,
                                                const WenoParams<TC>& P, double gamma, unsigned ntx, unsigned nty,
                                                unsigned b, double (&T)[5][kCHalo]) {
  static_assert(kCX * kCY * kCZ == kBlock, "one lane per tile cell");
  const int o[3] = {(int)(b % ntx) * kCX, (int)((b / ntx) % nty) * kCY, (int)(b / (ntx * nty)) * kCZ};
  const size_t nx = G.n[0], nxy = nx * G.n[1], N = nxy * G.n[2];
  for (int t = threadIdx.x; t < kCHalo; t += kBlock) {
    const int h[3] = {t % kCHX, (t / kCHX) % kCHY, t / (kCHX * kCHY)};
    int c[3];
    double sg[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // reconstruction-box coordinate, clamped to [-1, nr]: the reach of
      // the stencils of the box's own cells (tile overhang repeats the edge)
      const int r = min(max(o[d] + h[d] - 1, -1), G.nr[d]);
      c[d] = bc_index(G, d, r - G.g[d], sg[d]);
    }
    const size_t io = (size_t)c[2] * nxy + (size_t)c[1] * nx + c[0];
    T[0][t] = q[io];
    T[1][t] = sg[0] * q[N + io];
    T[2][t] = sg[1] * q[2 * N + io];
    T[3][t] = sg[2] * q[3 * N + io];
    T[4][t] = q[4 * N + io];
  }
  __syncthreads();
  const int l[3] = {(int)threadIdx.x % kCX, ((int)threadIdx.x / kCX) % kCY, (int)threadIdx.x / (kCX * kCY)};
  const int ri = o[0] + l[0], rj = o[1] + l[1], rk = o[2] + l[2];
  if (ri >= G.nr[0] || rj >= G.nr[1] || rk >= G.nr[2]) return;
  const size_t idx = ((size_t)rk * G.nr[1] + rj) * G.nr[0] + ri;
  const int base = ((l[2] + 1) * kCHY + (l[1] + 1)) * kCHX + (l[0] + 1);
#pragma unroll 1
  for (int fs = 0; fs < 6; ++fs)
    char_recon_tile_cell(T, base, faces + (size_t)fs * G.fs_stride, P, gamma, idx, fs >> 1, fs & 1);
}

// One workgroup per tile.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_char_recon_box(const double* __restrict__ q, TC* faces, BoxGrid G,
                                                           WenoParams<TC> P, double gamma, unsigned ntx,
                                                           unsigned nty, unsigned ntiles) {
  __shared__ double T[5][kCHalo];
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= ntiles) return;
  char_recon_tile(q, faces, G, P, gamma, ntx, nty, b, T);
}

}  // namespace hgks
