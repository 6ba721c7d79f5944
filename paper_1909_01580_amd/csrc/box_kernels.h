// Kernels of the HGKS stage on a uniform box grid (Pan & Xu, Sec. 2-4).
//
// Layout in HBM (structure of arrays, x fastest):
//   state     q[5][nz][ny][nx]                         double
//   coef      per reconstructed cell and variable: the cell mean and the
//             nine coefficients of the reconstructed quadratic in the
//             unit-cube coordinate xi, TC (double/float), in blocks of
//             64 / sizeof(TC) cells (coef_cell below); the cells are the
//             reconstruction box [NRz][NRy][NRx], NR = n + 2 on outflow axes
//             (one ghost layer), n on periodic.
//   mask      m[NRz][NRy][NRx]                           uint32, bit 4 f + g
//             set where Gauss point g of face f uses the first-order
//             fallback (Sec. 4 limiting procedure)
//   faces     F_d[10][fz][fy][fx] per direction d         TF
//             (F_p, dF_p/dt) of the face on the lower side of cell (i,j,k)
//             along d, summed over its 2x2 Gauss points with weight
//             Delta_a Delta_b / 4 (Eq. (11)); f_d = n_d (periodic) or
//             n_d + 1 (outflow), the other two extents n.
#pragma once

#include "common.h"
#include "char_basis.h"
#include "gks_flux.h"
#include "weno_box.h"

namespace hgks {

constexpr int kBlock = 256;
constexpr uint32_t kNeedsCheck = 0x80000000u;
constexpr double kGaussNode = 0.28867513459481288225457439025097873;  // 1/(2 sqrt 3)

struct BoxGrid {
  int n[3];
  int g[3];     // ghost layer of the reconstruction box
  int nr[3];    // reconstruction box
  int per[3];   // periodic axis
  int sym[3][2];  // symmetric (mirror) low / high end of a non-periodic axis; else outflow
  int nf[3][3]; // face grid per direction
  double inv_dx[3];
  double wface[3];  // Gauss weight 1/4 times the face area, faces normal to d
  double vol;
  // Reciprocals for index splitting (split_index): extents n[0], n[1];
  // nr[0], nr[1]; nf[d][0], nf[d][1].
  double inv_n[2], inv_nr[2], inv_nf[3][2];
  // Banded cell order of the flux blocks (face_cell): bands of `band`
  // rows along y; reciprocals of n0 band n2, n0 band and n0 (tail height).
  int band, band_full, band_tail;
  double inv_band[3];
  // Elements between the six per-face coefficient arrays of a cell
  // (reconstruction in characteristic variables: array 2 d + s holds the
  // quadratic for the cell's face normal to d on side s); 0 when one
  // reconstruction serves all faces.
  size_t fs_stride;
};

// floor(k / d) for k < 2^32 from inv = (1 + 2^-40) / d: the double product
// is at least k / d and exceeds it by less than the distance to the next
// integer, so truncation is exact and no integer divide is needed.
HGKS_FN double div_inv(int d) { return (1.0 + 0x1p-40) / (double)d; }

HGKS_FN void split_index(uint32_t k, int e0, int e1, double i0, double i1, int& c0, int& c1, int& c2) {
  const uint32_t q0 = (uint32_t)((double)k * i0);
  const uint32_t q1 = (uint32_t)((double)q0 * i1);
  c0 = (int)(k - q0 * (uint32_t)e0);
  c1 = (int)(q0 - q1 * (uint32_t)e1);
  c2 = (int)q1;
}

// Rows per band of the flux block order: the z-neighbour row of a cell is
// band * n0 cells earlier in that order, close enough to be found in L2.
constexpr int kFluxBand = 16;

// Fills the reciprocals of a grid whose extents are set; `band` rows per
// band of the flux block order (at most the grid's y extent).
inline void set_index_split(BoxGrid& G, int band = kFluxBand) {
  for (int a = 0; a < 2; ++a) {
    G.inv_n[a] = div_inv(G.n[a]);
    G.inv_nr[a] = div_inv(G.nr[a]);
    for (int d = 0; d < 3; ++d) G.inv_nf[d][a] = div_inv(G.nf[d][a]);
  }
  G.band = G.n[1] < band ? G.n[1] : band;
  G.band_full = G.n[1] / G.band;
  G.band_tail = G.n[1] - G.band_full * G.band;
  G.inv_band[0] = div_inv(G.n[0] * G.band * G.n[2]);
  G.inv_band[1] = div_inv(G.n[0] * G.band);
  G.inv_band[2] = div_inv(G.n[0] * (G.band_tail > 0 ? G.band_tail : 1));
}

// Flux blocks of 64 faces per direction d: one per 64 cells (the faces on
// the lower side of every cell) plus, on an outflow axis d, the faces of
// the upper boundary plane.
inline unsigned flux_main_blocks(const BoxGrid& G) {
  return (unsigned)(((size_t)G.n[0] * G.n[1] * G.n[2] + 63) / 64);
}
inline void flux_block_counts(const BoxGrid& G, unsigned (&nb)[3]) {
  for (int d = 0; d < 3; ++d) {
    nb[d] = flux_main_blocks(G);
    if (!G.per[d]) {
      const size_t nbnd = (size_t)G.n[0] * G.n[1] * G.n[2] / G.n[d];
      nb[d] += (unsigned)((nbnd + 63) / 64);
    }
  }
}

// Cell (i, j, k) at position p of the banded order: bands of `band` rows
// along y, then z, then y within the band, then x.  Consecutive flux blocks
// cover consecutive positions, so the lower y- and z-neighbours of a
// block's cells were read by blocks shortly before it.
HGKS_FN void banded_cell(const BoxGrid& G, uint32_t p, int (&c)[3]) {
  const uint32_t full = (uint32_t)G.n[0] * G.band * G.band_full * G.n[2];
  int jb, jj;
  if (p < full) {
    const uint32_t band = (uint32_t)((double)p * G.inv_band[0]);
    const uint32_t r = p - band * (uint32_t)(G.n[0] * G.band * G.n[2]);
    const uint32_t k = (uint32_t)((double)r * G.inv_band[1]);
    const uint32_t r2 = r - k * (uint32_t)(G.n[0] * G.band);
    const uint32_t j = (uint32_t)((double)r2 * G.inv_n[0]);
    c[0] = (int)(r2 - j * (uint32_t)G.n[0]);
    c[2] = (int)k;
    jb = (int)band * G.band;
    jj = (int)j;
  } else {
    const uint32_t r = p - full;
    const uint32_t k = (uint32_t)((double)r * G.inv_band[2]);
    const uint32_t r2 = r - k * (uint32_t)(G.n[0] * G.band_tail);
    const uint32_t j = (uint32_t)((double)r2 * G.inv_n[0]);
    c[0] = (int)(r2 - j * (uint32_t)G.n[0]);
    c[2] = (int)k;
    jb = G.band_full * G.band;
    jj = (int)j;
  }
  c[1] = jb + jj;
}

// Face of lane `slot` (0..63) of block lb of direction D: the cell on its
// upper side (which may be the outflow ghost beyond the last cell) and its
// index in the face grid.  Returns false for slots past the end (their
// face is the last one of the range, so that the four-lane sums stay
// well-defined; the result is not written).
HGKS_FN bool face_of_block(const BoxGrid& G, int D, unsigned lb, unsigned slot, int (&c)[3], size_t& f) {
  const unsigned nmain = (unsigned)(((size_t)G.n[0] * G.n[1] * G.n[2] + 63) / 64);
  const uint32_t N = (uint32_t)G.n[0] * G.n[1] * G.n[2];
  bool live;
  if (lb < nmain) {
    uint32_t p = lb * 64u + slot;
    live = p < N;
    if (!live) p = N - 1;
    banded_cell(G, p, c);
  } else {
    // Upper boundary plane of an outflow axis D: the other two axes in
    // increasing order, the first fastest.
    const int a0 = D == 0 ? 1 : 0, a1 = D == 2 ? 1 : 2;
    const uint32_t nbnd = (uint32_t)G.n[a0] * G.n[a1];
    uint32_t e = (lb - nmain) * 64u + slot;
    live = e < nbnd;
    if (!live) e = nbnd - 1;
    const uint32_t q = (uint32_t)((double)e * div_inv(G.n[a0]));
    const int u0 = (int)(e - q * (uint32_t)G.n[a0]), u1 = (int)q;
    // constant indices in each branch (no indexed private array)
    if (D == 0) {
      c[0] = G.n[0]; c[1] = u0; c[2] = u1;
    } else if (D == 1) {
      c[0] = u0; c[1] = G.n[1]; c[2] = u1;
    } else {
      c[0] = u0; c[1] = u1; c[2] = G.n[2];
    }
  }
  f = (size_t)c[0] + (size_t)G.nf[D][0] * ((size_t)c[1] + (size_t)G.nf[D][1] * c[2]);
  return live;
}

// Coefficient layout: blocks of kCB = 64 / sizeof(TC) consecutive
// reconstructed cells; a block holds the 50 values of its cells (variable
// v, coefficient k, row 10 v + k; k = 0 the cell mean) as 50 rows of kCB
// values.  All 50 values of a cell then lie within 3.2 KB of its first
// value, so one address serves all its loads (immediate offsets), and one
// row of a block is one 64-byte segment.
template <typename TC>
constexpr int kCB = 64 / (int)sizeof(TC);

template <typename TC>
HGKS_FN size_t coef_cell(size_t cell) {
  return (cell / kCB<TC>) * 50 * kCB<TC> + cell % kCB<TC>;
}

// Elements of the coefficient array of NR reconstructed cells.
constexpr size_t coef_elems(size_t NR, size_t elem_bytes) {
  const size_t cb = 64 / elem_bytes;
  return 50 * ((NR + cb - 1) / cb) * cb;
}

// Real index of cell i (within one layer of the grid) along axis ax after
// the boundary rule -- periodic wrap, zero-gradient clamp (outflow) or
// mirror (symmetric) -- and the sign (+1 or -1) of the momentum component
// along ax in that cell's value: -1 for a mirror image.
__device__ __forceinline__ int bc_index(const BoxGrid& G, int ax, int i, double& sign) {
  const int n = G.n[ax];
  sign = 1.0;
  if (G.per[ax]) return i < 0 ? i + n : (i >= n ? i - n : i);
  if (i < 0) {
    if (G.sym[ax][0]) {
      sign = -1.0;
      return -1 - i;
    }
    return 0;
  }
  if (i >= n) {
    if (G.sym[ax][1]) {
      sign = -1.0;
      return 2 * n - 1 - i;
    }
    return n - 1;
  }
  return i;
}

__device__ __forceinline__ int rec_index(const BoxGrid& G, int ax, int i) {
  // Reconstruction-box index of real cell i (i in [-1, n]).
  const int n = G.n[ax];
  if (G.per[ax]) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i + 1;
}

// ---------------------------------------------------------------- recon
// Reconstruction of reconstruction-box cell idx (< NR).  WIDE: the
// stencils of Remark 1 (the big stencil reaches two cells along the axes);
// COEF = false: the fallback mask only (the characteristic reconstruction
// stores its own coefficients).
template <typename TC, bool WIDE = false, bool COEF = true>
__device__ __forceinline__ void recon_box_cell(const double* __restrict__ q, TC* __restrict__ coef,
                                               uint32_t* __restrict__ mask, const BoxGrid& G,
                                               const WenoParams<TC>& P, TC margin, TC gm1, size_t NR, size_t idx) {
  int ri, rj, rk;
  split_index((uint32_t)idx, G.nr[0], G.nr[1], G.inv_nr[0], G.inv_nr[1], ri, rj, rk);
  const int i = ri - G.g[0], j = rj - G.g[1], k = rk - G.g[2];
  int ix[3], iy[3], iz[3];
  double sx[3], sy[3], sz[3];  // momentum signs of mirror images
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    ix[o] = bc_index(G, 0, i + o - 1, sx[o]);
    iy[o] = bc_index(G, 1, j + o - 1, sy[o]);
    iz[o] = bc_index(G, 2, k + o - 1, sz[o]);
  }
  // cells two steps away along each axis (wide stencil only)
  int fx[2] = {0, 0}, fy[2] = {0, 0}, fz[2] = {0, 0};
  double gx[2] = {1.0, 1.0}, gy[2] = {1.0, 1.0}, gz[2] = {1.0, 1.0};
  if constexpr (WIDE) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      fx[t] = bc_index(G, 0, i + 4 * t - 2, gx[t]);
      fy[t] = bc_index(G, 1, j + 4 * t - 2, gy[t]);
      fz[t] = bc_index(G, 2, k + 4 * t - 2, gz[t]);
    }
  }
  const size_t N = (size_t)G.n[0] * G.n[1] * G.n[2];
  // element offsets in 32 bits (fewer than 2^29 cells), byte offsets from
  // each variable's uniform base
  const unsigned nx = (unsigned)G.n[0], nxy = (unsigned)G.n[0] * (unsigned)G.n[1];
  TC qc[5], bnd[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double* qv = q + v * N;
    auto ld = [&](int z, int y, int x) {
      return *(const double*)((const char*)qv + ((unsigned)z * nxy + (unsigned)y * nx + (unsigned)x) * 8u);
    };
    // sign of variable v in the cell at offset o: the momentum component
    // along an axis flips in a mirror image across that axis
    auto sg = [&](int ox, int oy, int oz) -> double {
      return v == 1 ? sx[ox + 1] : (v == 2 ? sy[oy + 1] : (v == 3 ? sz[oz + 1] : 1.0));
    };
    const double c = sg(0, 0, 0) * ld(iz[1], iy[1], ix[1]);
    TC d[27];
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int nz = (ox != 0) + (oy != 0) + (oz != 0);
          if (nz == 0 || nz == 3) {
            d[sidx(ox, oy, oz)] = TC(0);
          } else {
            d[sidx(ox, oy, oz)] =
                TC(sg(ox, oy, oz) * ld(iz[oz + 1], iy[oy + 1], ix[ox + 1]) - c);
          }
        }
    BoxRecon<TC> r;
    if constexpr (WIDE) {
      // far cells: (-2x, +2x, -2y, +2y, -2z, +2z); a mirror flips the
      // momentum along its own axis
      TC f[6];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double s0 = v == 1 ? gx[t] : (v == 2 ? sy[1] : (v == 3 ? sz[1] : 1.0));
        const double s1 = v == 1 ? sx[1] : (v == 2 ? gy[t] : (v == 3 ? sz[1] : 1.0));
        const double s2 = v == 1 ? sx[1] : (v == 2 ? sy[1] : (v == 3 ? gz[t] : 1.0));
        f[t] = TC(s0 * ld(iz[1], iy[1], fx[t]) - c);
        f[2 + t] = TC(s1 * ld(iz[1], fy[t], ix[1]) - c);
        f[4 + t] = TC(s2 * ld(fz[t], iy[1], ix[1]) - c);
      }
      weno_box_wide(d, f, P, r);
    } else {
      weno_box(d, P, r);
    }
    if constexpr (COEF) {
      TC* cv = coef + coef_cell<TC>(idx) + v * 10 * kCB<TC>;
      cv[0] = TC(c);
#pragma unroll
      for (int m = 0; m < 9; ++m) cv[(m + 1) * kCB<TC>] = r.c[m];
    }
    qc[v] = TC(c);
    bnd[v] = r.bound;
    // The next variable's stencil loads wait for this variable's results
    // (an empty asm ties their indices to them), so the compiler does not
    // hoist all five stencils ahead and hold them in registers at once.
    asm volatile("" : "+v"(iz[0]), "+v"(iz[1]), "+v"(iz[2]) : "v"(r.c[0]), "v"(r.bound));
  }
  // Sufficient test that no polynomial can give rho <= 0 or p < 0 at a
  // Gauss point: bounds of every variable over all 25 polynomials and 24
  // points; the exact test runs only where this one fails.
  const TC rmin = qc[0] - bnd[0];
  bool safe = rmin > margin * qc[0];
  if (safe) {
    TC msq = TC(0);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
      const TC mm = d_abs(qc[1 + dd]) + bnd[1 + dd];
      msq += mm * mm;
    }
    const TC emin = qc[4] - bnd[4];
    safe = gm1 * (emin - TC(0.5) * msq * d_rcp(rmin)) > margin * gm1 * (d_abs(qc[4]) + bnd[4]);
  }
  mask[idx] = safe ? 0u : kNeedsCheck;
}

template <typename TC, bool WIDE = false, bool COEF = true>
__global__ void __launch_bounds__(kBlock) k_recon_box(const double* __restrict__ q, TC* __restrict__ coef,
                                                      uint32_t* __restrict__ mask, BoxGrid G,
                                                      WenoParams<TC> P, TC margin, TC gm1, size_t NR,
                                                      unsigned nblk) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nblk) return;
  const size_t idx = (size_t)b * kBlock + threadIdx.x;
  if (idx >= NR) return;
  recon_box_cell<TC, WIDE, COEF>(q, coef, mask, G, P, margin, gm1, NR, idx);
}

// Exact fallback test (Sec. 4): for every Gauss point of the cell, any of
// the 25 polynomials (9 with the stencils of Remark 1) with rho <= 0 or
// p < 0 marks the point.  poly_bits: the 24 point bits of polynomial m
// (m = 0 the big stencil's, then the sub-stencils') of a cell whose
// stencil values at(v, ox, oy, oz) (variable v of the cell at that offset,
// boundary images and mirror signs applied) the accessor gives.
template <typename TC, bool WIDE, typename AT>
__device__ __forceinline__ uint32_t poly_bits(const AT& at, TC gm1, int m) {
  TC qc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qc[v] = TC(at(v, 0, 0, 0));
  // Values at the 24 points of one polynomial per variable (coefficients in
  // registers, indices fixed after unrolling), then the test.
  auto test = [&](const TC (&cf)[5][9]) -> uint32_t {
    uint32_t bits = 0;
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const TC xs = (f & 1) ? TC(0.5) : TC(-0.5);
#pragma unroll
      for (int gp = 0; gp < 4; ++gp) {
      const int bit = 4 * f + gp;
      // the face axis d takes xs, axes d+1 and d+2 (cyclic) the Gauss nodes
      const TC pa = (gp >> 1) ? TC(kGaussNode) : TC(-kGaussNode);
      const TC pb = (gp & 1) ? TC(kGaussNode) : TC(-kGaussNode);
      const TC x0 = d == 0 ? xs : (d == 2 ? pa : pb);
      const TC x1 = d == 1 ? xs : (d == 0 ? pa : pb);
      const TC x2 = d == 2 ? xs : (d == 1 ? pa : pb);
      TC val[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        TC gx, gy, gz;
        quad_eval(qc[v], cf[v], x0, x1, x2, val[v], gx, gy, gz);
      }
      bool bad = !(val[0] > TC(0));
      if (!bad) {
        const TC p = gm1 * (val[4] - TC(0.5) * (val[1] * val[1] + val[2] * val[2] + val[3] * val[3]) / val[0]);
        bad = p < TC(0);
      }
      if (bad) bits |= 1u << bit;
      }
    }
    return bits;
  };
  if (m == 0) {
    // P_0 from the big stencil
    TC cf[5][9];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double c = at(v, 0, 0, 0);
      TC d[27];
#pragma unroll
      for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
          for (int ox = -1; ox <= 1; ++ox) {
            const int nz = (ox != 0) + (oy != 0) + (oz != 0);
            d[sidx(ox, oy, oz)] = (nz == 0 || nz == 3) ? TC(0) : TC(at(v, ox, oy, oz) - c);
          }
      if constexpr (WIDE) {
        const TC f[6] = {TC(at(v, -2, 0, 0) - c), TC(at(v, 2, 0, 0) - c), TC(at(v, 0, -2, 0) - c),
                         TC(at(v, 0, 2, 0) - c), TC(at(v, 0, 0, -2) - c), TC(at(v, 0, 0, 2) - c)};
        big_quadratic_wide(d, f, cf[v]);
      } else {
        big_quadratic(d, cf[v]);
      }
      // one variable's stencil in registers at a time
      asm volatile("" ::: "memory");
    }
    return test(cf);
  }
  {
    // linear sub-stencil polynomial m - 1
    const int ms = m - 1;
    TC cf[5][9];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double c = at(v, 0, 0, 0);
#pragma unroll
      for (int t = 3; t < 9; ++t) cf[v][t] = TC(0);
      TC b[3];
      if constexpr (WIDE) {
        const int sx = (ms & 1) ? -1 : 1, sy = (ms & 2) ? -1 : 1, sz = (ms & 4) ? -1 : 1;
        b[0] = TC(sx) * TC(at(v, sx, 0, 0) - c);
        b[1] = TC(sy) * TC(at(v, 0, sy, 0) - c);
        b[2] = TC(sz) * TC(at(v, 0, 0, sz) - c);
      } else {
        const int t = ms / 8, r = ms % 8;
        const int sa = (r & 1) ? -1 : 1, sb = (r & 2) ? -1 : 1, sc = (r & 4) ? -1 : 1;
        // axis triple (a, b; c) = (t, t+1; t+2) cyclic; offsets as (x, y, z)
        const int ea = t, eb = t == 2 ? 0 : t + 1, ec = t == 0 ? 2 : t - 1;
        const int oa[3] = {ea == 0 ? sa : 0, ea == 1 ? sa : 0, ea == 2 ? sa : 0};
        const int ob[3] = {eb == 0 ? sb : 0, eb == 1 ? sb : 0, eb == 2 ? sb : 0};
        const int oc[3] = {ec == 0 ? sc : 0, ec == 1 ? sc : 0, ec == 2 ? sc : 0};
        const TC da = TC(at(v, oa[0], oa[1], oa[2]) - c);
        const TC db = TC(at(v, ob[0], ob[1], ob[2]) - c);
        const TC dab = TC(at(v, oa[0] + ob[0], oa[1] + ob[1], oa[2] + ob[2]) - c);
        const TC dc = TC(at(v, oc[0], oc[1], oc[2]) - c);
        const TC ba = TC(sa) * (TC(2) * da - db + dab) * TC(1.0 / 3.0);
        const TC bb = TC(sb) * (TC(2) * db - da + dab) * TC(1.0 / 3.0);
        const TC bc = TC(sc) * dc;
        // slope along x, y, z by selects (the axis of each is uniform)
        b[0] = ea == 0 ? ba : (eb == 0 ? bb : bc);
        b[1] = ea == 1 ? ba : (eb == 1 ? bb : bc);
        b[2] = ea == 2 ? ba : (eb == 2 ? bb : bc);
      }
      cf[v][0] = b[0];
      cf[v][1] = b[1];
      cf[v][2] = b[2];
    }
    return test(cf);
  }
}

// poly_bits of reconstruction-box cell idx, its stencil read from the state.
template <typename TC, bool WIDE = false>
__device__ __forceinline__ uint32_t posit_poly_bits(const double* __restrict__ q, const BoxGrid& G, TC gm1, size_t idx,
                                                    int m) {
  int ri, rj, rk;
  split_index((uint32_t)idx, G.nr[0], G.nr[1], G.inv_nr[0], G.inv_nr[1], ri, rj, rk);
  const int i = ri - G.g[0], j = rj - G.g[1], k = rk - G.g[2];
  const size_t nx = G.n[0], nxy = (size_t)G.n[0] * G.n[1], N = nxy * G.n[2];
  auto at = [&](int v, int ox, int oy, int oz) -> double {
    double s[3];
    const int a = bc_index(G, 0, i + ox, s[0]), bb = bc_index(G, 1, j + oy, s[1]), c = bc_index(G, 2, k + oz, s[2]);
    const double val = q[v * N + c * nxy + bb * nx + a];
    return v == 1 ? s[0] * val : (v == 2 ? s[1] * val : (v == 3 ? s[2] * val : val));
  };
  return poly_bits<TC, WIDE>(at, gm1, m);
}

template <bool WIDE>
constexpr int kPosPolys = WIDE ? 9 : 25;

template <typename TC, bool WIDE = false>
__device__ __forceinline__ void posit_exact_box_cell(const double* __restrict__ q, uint32_t* __restrict__ mask,
                                                     const BoxGrid& G, TC gm1, size_t idx) {
  uint32_t bits = 0;
  for (int m = 0; m < kPosPolys<WIDE>; ++m) bits |= posit_poly_bits<TC, WIDE>(q, G, gm1, idx, m);
  mask[idx] = bits;
}

// The exact test runs on a list of the flagged cells: k_posit_compact
// appends them (one counter add per wave), then k_posit_group_box tests each
// listed cell.  counter[0] must be zero before k_posit_compact.
__global__ void __launch_bounds__(kBlock) k_posit_compact(const uint32_t* __restrict__ mask, size_t NR,
                                                          uint32_t* __restrict__ list, uint32_t* __restrict__ counter) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const bool flagged = idx < NR && (mask[idx] & kNeedsCheck);
  const uint64_t ballot = __ballot(flagged);
  if (ballot == 0) return;
  const int lane = (int)(threadIdx.x & 63u);
  const int leader = __ffsll((long long)ballot) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(ballot));
  base = __shfl(base, leader);
  if (flagged) {
    const uint64_t below = lane ? (ballot & ((~0ull) >> (64 - lane))) : 0ull;
    list[base + (uint32_t)__popcll(below)] = (uint32_t)idx;
  }
}

// Stencil points of the exact test: the 27 cells of the 3x3x3 block, then
// (Remark 1 only) the six cells two steps away along the axes.
template <bool WIDE>
constexpr int kPosPoints = WIDE ? 33 : 27;

HGKS_FN void pos_point(int t, int& ox, int& oy, int& oz) {
  if (t < 27) {
    ox = t % 3 - 1;
    oy = (t / 3) % 3 - 1;
    oz = t / 9 - 1;
  } else {
    const int a = (t - 27) >> 1, s = ((t - 27) & 1) ? 2 : -2;
    ox = a == 0 ? s : 0;
    oy = a == 1 ? s : 0;
    oz = a == 2 ? s : 0;
  }
}

HGKS_FN int pos_slot(int ox, int oy, int oz) {
  if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) return (oz + 1) * 9 + (oy + 1) * 3 + ox + 1;
  const int a = ox != 0 ? 0 : (oy != 0 ? 1 : 2);
  const int s = ox + oy + oz;
  return 27 + 2 * a + (s > 0 ? 1 : 0);
}

// The exact test on the list of flagged cells, one 32-lane group per cell:
// the group stages the cell's stencil (boundary images and mirror signs
// applied) in LDS once, then lane m tests polynomial m; the lanes' point
// bits are or-ed across the group and written as the cell's mask word,
// which also clears its "needs the test" bit.  The pass loop is uniform
// over the workgroup (its bound depends on the block only), so the
// barriers are reached by every lane.
constexpr int kPosGroups = kBlock / 32;

template <typename TC, bool WIDE = false>
__global__ void __launch_bounds__(kBlock) k_posit_group_box(const double* __restrict__ q,
                                                            uint32_t* __restrict__ mask, BoxGrid G, TC gm1,
                                                            const uint32_t* __restrict__ list,
                                                            const uint32_t* __restrict__ counter) {
  constexpr int NP = kPosPoints<WIDE>;
  __shared__ double st[kPosGroups][5][NP];
  const uint32_t count = counter[0];
  const int grp = (int)(threadIdx.x >> 5), lane = (int)(threadIdx.x & 31u);
  const size_t nx = G.n[0], nxy = (size_t)G.n[0] * G.n[1], N = nxy * G.n[2];
  for (uint32_t base = blockIdx.x * kPosGroups; base < count; base += gridDim.x * kPosGroups) {
    const uint32_t e = base + (uint32_t)grp;
    const bool live = e < count;
    const size_t idx = list[live ? e : base];
    int ri, rj, rk;
    split_index((uint32_t)idx, G.nr[0], G.nr[1], G.inv_nr[0], G.inv_nr[1], ri, rj, rk);
    const int i = ri - G.g[0], j = rj - G.g[1], k = rk - G.g[2];
    // NP may exceed the group's 32 lanes (33 points with Remark 1)
    for (int t = lane; t < NP; t += 32) {
      int ox, oy, oz;
      pos_point(t, ox, oy, oz);
      double s[3];
      const int a = bc_index(G, 0, i + ox, s[0]), b = bc_index(G, 1, j + oy, s[1]), c = bc_index(G, 2, k + oz, s[2]);
      const size_t o = (size_t)c * nxy + (size_t)b * nx + a;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double val = q[v * N + o];
        st[grp][v][t] = v == 1 ? s[0] * val : (v == 2 ? s[1] * val : (v == 3 ? s[2] * val : val));
      }
    }
    __syncthreads();
    uint32_t bits = 0;
    if (live && lane < kPosPolys<WIDE>) {
      auto at = [&](int v, int ox, int oy, int oz) -> double { return st[grp][v][pos_slot(ox, oy, oz)]; };
      bits = poly_bits<TC, WIDE>(at, gm1, lane);
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) bits |= __shfl_xor(bits, o);
    if (live && lane == 0) mask[idx] = bits;
    __syncthreads();
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p) { p[threadIdx.x] = 0u; }

// ---------------------------------------------------------------- flux
// Local frame of a face normal to axis D: local axes (D, A, B) with
// A = (D + 1) % 3 and B = (D + 2) % 3.  D is uniform over a workgroup, so
// the plane offsets below are scalar arithmetic and one copy of the flux
// code serves the three directions.
struct FaceAxes {
  int D, A, B;
};

HGKS_FN FaceAxes face_axes(int D) {
  return FaceAxes{D, D == 2 ? 0 : D + 1, D == 0 ? 2 : D - 1};
}

// Value and gradient of the five variables of reconstructed cell `cell` at
// the point with local coordinates (xD, xA, xB) of the unit cube, in the
// local frame of a face normal to axis D: W = (rho, M_D, M_A, M_B, E),
// dW[j] = derivative along local axis j.  The stored quadratic (x, y, z,
// xx, yy, zz, xy, yz, xz in global axes) is read with its coefficients
// permuted to the local axes: local linear and square terms of axis j come
// from global axis (D, A, B)[j], the local mixed terms (DA, AB, DB) from
// the global mixed terms 6 + D, 6 + A, 6 + B.  D is a template parameter
// so that every load has a constant offset from the cell's address.
template <int D, int CB, typename TC>
HGKS_FN void eval_rows_gp(const TC* cv, TC xD, TC xA, TC xB, bool fallback, const TC (&invd)[3], TC (&W)[5],
                          TC (&dW)[3][5]) {
  constexpr int A = (D + 1) % 3, B = (D + 2) % 3;
  constexpr int lv[5] = {0, 1 + D, 1 + A, 1 + B, 4};
  constexpr int cp[9] = {D, A, B, 3 + D, 3 + A, 3 + B, 6 + D, 6 + A, 6 + B};
#pragma unroll
  for (int kk = 0; kk < 5; ++kk) {
    const TC* ck = cv + lv[kk] * 10 * CB;
    TC c[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) c[m] = ck[(cp[m] + 1) * CB];
    TC val, g[3];
    quad_eval(ck[0], c, xD, xA, xB, val, g[0], g[1], g[2]);
    W[kk] = val;
#pragma unroll
    for (int j = 0; j < 3; ++j) dW[j][kk] = g[j] * invd[j];
  }
  if (fallback) {
    // First-order fallback of the Sec. 4 limiter: cell mean, zero gradient.
    // Rare, so a real branch (the empty asm keeps the compiler from turning
    // it into selects on every lane) that re-reads the means.
    asm volatile("");
#pragma unroll
    for (int kk = 0; kk < 5; ++kk) {
      W[kk] = cv[lv[kk] * 10 * CB];
#pragma unroll
      for (int j = 0; j < 3; ++j) dW[j][kk] = TC(0);
    }
  }
}

// The 50 values of a cell are rows 10 v + k, CB elements apart.
template <int D, typename TC>
HGKS_FN void eval_box_gp(const TC* __restrict__ coef, size_t cell, TC xD, TC xA, TC xB, bool fallback,
                         const TC (&invd)[3], TC (&W)[5], TC (&dW)[3][5]) {
  eval_rows_gp<D, kCB<TC>>(coef + coef_cell<TC>(cell), xD, xA, xB, fallback, invd, W, dW);
}

// eval_box_gp for a direction D that is uniform over the workgroup.
template <typename TC>
HGKS_FN void eval_box_gp_dir(int D, const TC* __restrict__ coef, size_t cell, TC xD, TC xA, TC xB,
                             bool fallback, const TC (&invd)[3], TC (&W)[5], TC (&dW)[3][5]) {
  if (D == 0)
    eval_box_gp<0>(coef, cell, xD, xA, xB, fallback, invd, W, dW);
  else if (D == 1)
    eval_box_gp<1>(coef, cell, xD, xA, xB, fallback, invd, W, dW);
  else
    eval_box_gp<2>(coef, cell, xD, xA, xB, fallback, invd, W, dW);
}

// Value and gradient (local axes D, A, B; per unit length) at the Gauss
// point of a cell reconstructed in characteristic variables: cv points at
// the cell in its face array, Qbar is the face's mean state.  The result is
// in the local variable order of eval_box_gp.
//
// From global memory (PRE) all 45 coefficients are requested before the
// eigenvectors are formed (the fence keeps the loads there), so that their
// latency overlaps it; from LDS each field's nine are read where they are
// used, which keeps the registers of the other 36 free.
template <int D, bool PRE = true, typename TC>
__device__ __forceinline__ void eval_char_gp(const TC* cv, const double (&Qbar)[5], double gamma, TC xD, TC xA,
                                             TC xB, bool fallback, const TC (&invd)[3], TC (&W)[5],
                                             TC (&dW)[3][5]) {
  constexpr int A = (D + 1) % 3, B = (D + 2) % 3, CB = kCB<TC>;
  constexpr int lv[5] = {0, 1 + D, 1 + A, 1 + B, 4};
  constexpr int cp[9] = {D, A, B, 3 + D, 3 + A, 3 + B, 6 + D, 6 + A, 6 + B};
  TC call[5][9];
  if constexpr (PRE) {
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
      for (int m = 0; m < 9; ++m) call[f][m] = cv[(f * 10 + cp[m] + 1) * CB];
    asm volatile("" ::: "memory");
  }
  CharBasis Bs;
  char_basis(Qbar, D, gamma, Bs);
  TC val[5], grad[5][3];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    val[v] = cv[v * 10 * CB];
    grad[v][0] = grad[v][1] = grad[v][2] = TC(0);
  }
  if (!fallback) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      TC c[9];
#pragma unroll
      for (int m = 0; m < 9; ++m) c[m] = PRE ? call[f][m] : cv[(f * 10 + cp[m] + 1) * CB];
      TC du, g[3];
      quad_eval(TC(0), c, xD, xA, xB, du, g[0], g[1], g[2]);
      double r[5];
      char_rcol(Bs, f, r);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const TC rv = TC(r[v]);
        val[v] += rv * du;
#pragma unroll
        for (int j = 0; j < 3; ++j) grad[v][j] += rv * g[j];
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < 5; ++kk) {
    W[kk] = val[lv[kk]];
#pragma unroll
    for (int j = 0; j < 3; ++j) dW[j][kk] = grad[lv[kk]][j] * invd[j];
  }
}

template <bool PRE = true, typename TC>
__device__ __forceinline__ void eval_char_gp_dir(int D, const TC* cv, const double (&Qbar)[5], double gamma, TC xD,
                                                 TC xA, TC xB, bool fallback, const TC (&invd)[3], TC (&W)[5],
                                                 TC (&dW)[3][5]) {
  if (D == 0)
    eval_char_gp<0, PRE>(cv, Qbar, gamma, xD, xA, xB, fallback, invd, W, dW);
  else if (D == 1)
    eval_char_gp<1, PRE>(cv, Qbar, gamma, xD, xA, xB, fallback, invd, W, dW);
  else
    eval_char_gp<2, PRE>(cv, Qbar, gamma, xD, xA, xB, fallback, invd, W, dW);
}

// LDS of the FP64 flux's right cells, in doubles: per group of 8 faces 50
// rows of 8 and one row of padding (it moves the second group's reads to
// other banks), two groups per wave.
constexpr int kStageGroup = 50 * 8 + 8;
constexpr int kStageWave = 2 * kStageGroup;

typedef const void __attribute__((address_space(1)))* GlobalPtr;
typedef void __attribute__((address_space(3)))* LdsPtr;

// Direct global-to-LDS copies of pieces K0..K1-1 of 256 bytes: piece k at
// immediate offset 256 k of both addresses (the offset is a constant of
// the instruction; the LDS address, in M0, stays the same for all).
template <int K0, int K1>
__device__ __forceinline__ void copy_pieces(GlobalPtr src, LdsPtr dst) {
  if constexpr (K0 < K1) {
    __builtin_amdgcn_global_load_lds(src, dst, 4, 256 * K0, 0);
    copy_pieces<K0 + 1, K1>(src, dst);
  }
}

// One lane = one Gauss point of one face normal to axis D; the four lanes of
// a face sum their weighted fluxes with quad-permute moves.  Lane l of the
// 256-lane block lb of direction D takes Gauss point l % 4 of face slot
// l / 4 (face_of_block).
// PR: the extended viscous model (viscosity law, Prandtl correction); FS:
// per-face coefficient arrays (characteristic reconstruction).
template <typename TC, bool PR = false, bool FS = false, bool DMA = false>
__device__ __forceinline__ void flux_box_face(const TC* __restrict__ coef, const uint32_t* __restrict__ mask,
                                              TC* __restrict__ face, const BoxGrid& G, const GasParams<TC>& gp,
                                              TC dt, TC idt, unsigned lb, int D, TC* stage = nullptr) {
  const FaceAxes ax = face_axes(D);
  const int gpi = (int)(threadIdx.x & 3);
  int cR[3];
  size_t f;
  const bool live = face_of_block(G, D, lb, threadIdx.x >> 2, cR, f);
  const int cL[3] = {cR[0] - (D == 0), cR[1] - (D == 1), cR[2] - (D == 2)};
  size_t iL = 0, iR = 0;
  {
    const size_t s1 = G.nr[0], s2 = (size_t)G.nr[0] * G.nr[1];
    iL = rec_index(G, 2, cL[2]) * s2 + rec_index(G, 1, cL[1]) * s1 + rec_index(G, 0, cL[0]);
    iR = rec_index(G, 2, cR[2]) * s2 + rec_index(G, 1, cR[1]) * s1 + rec_index(G, 0, cR[0]);
  }
  const TC xa = (gpi >> 1) ? TC(kGaussNode) : TC(-kGaussNode);
  const TC xb = (gpi & 1) ? TC(kGaussNode) : TC(-kGaussNode);
  const TC invd[3] = {TC(G.inv_dx[ax.D]), TC(G.inv_dx[ax.A]), TC(G.inv_dx[ax.B])};
  const bool fbL = (mask[iL] >> (4 * (2 * D + 1) + gpi)) & 1u;
  const bool fbR = (mask[iR] >> (4 * (2 * D) + gpi)) & 1u;

  // the left cell's quadratic for its high face, the right cell's for its
  // low face (the same array unless the faces have their own)
  const TC* coefL = FS ? coef + (size_t)(2 * D + 1) * G.fs_stride : coef;
  const TC* coefR = FS ? coef + (size_t)(2 * D) * G.fs_stride : coef;
  // the left side assigns the sums, the right side adds to them
  FluxAcc<TC> acc;
  acc_begin(acc);
  if constexpr (DMA) {
    // The right cells' 50 values go to LDS by direct loads issued before
    // the left side's terms: they arrive while those run and hold no
    // registers meanwhile.  Each wave copies the right cells of its own 16
    // faces, as two groups of 8 faces, into its own [50 rows][8 faces]
    // arrays and reads only those, after waiting for its own loads: no
    // workgroup barrier.  A row of 8 doubles is 64 bytes in LDS as in the
    // coefficient array, so one immediate offset steps the global and the
    // LDS address together and the 26 copies need no address arithmetic.
    static_assert(sizeof(TC) == 8 && kCB<TC> == 8, "rows of 8 doubles");
    const unsigned l = threadIdx.x & 63u;
    TC* rs = stage + (threadIdx.x >> 6) * kStageWave;
    // in piece k of group g lane l copies row 4 k + l / 16 of face slot
    // 8 g + (l / 2) % 8, 32-bit half l % 2: byte 4 l of the piece
    unsigned cell0 = __shfl((unsigned)iR, (int)(((l >> 1) & 7u) * 4u));
    unsigned cell1 = __shfl((unsigned)iR, (int)((8u + ((l >> 1) & 7u)) * 4u));
    // characteristic reconstruction: the face's mean state from the two
    // cells' conservative means gives R for both sides
    double Qbar[5];
    if constexpr (FS) {
#pragma unroll
      for (int v = 0; v < 5; ++v)
        Qbar[v] = 0.5 * ((double)coefL[coef_cell<TC>(iL) + v * 10 * kCB<TC>] +
                         (double)coefR[coef_cell<TC>(iR) + v * 10 * kCB<TC>]);
    }
    {
      TC W[5], dW[3][5];
      if constexpr (FS)
        eval_char_gp_dir(D, coefL + coef_cell<TC>(iL), Qbar, gp.gamma, TC(0.5), xa, xb, fbL, invd, W, dW);
      else
        eval_box_gp_dir(D, coefL, iL, TC(0.5), xa, xb, fbL, invd, W, dW);
      // The copies are issued once the left cell's values have arrived: the
      // memory counter is waited on in issue order, so copies issued
      // earlier would hold up the left side's first use of its loads.
      asm volatile("" : "+v"(cell0), "+v"(cell1) : "v"(W[0]), "v"(dW[2][4]));
      const unsigned lane = (l >> 4) * 64 + (l & 1u) * 4;
      const GlobalPtr s0 = (GlobalPtr)((const char*)(coefR + coef_cell<TC>(cell0)) + lane);
      const GlobalPtr s1 = (GlobalPtr)((const char*)(coefR + coef_cell<TC>(cell1)) + lane);
      const LdsPtr d0 = (LdsPtr)rs;
      const LdsPtr d1 = (LdsPtr)(rs + kStageGroup);
      // rows 0-47: twelve pieces of four rows per group
      copy_pieces<0, 12>(s0, d0);
      copy_pieces<0, 12>(s1, d1);
      // rows 48 and 49: the lanes of the next piece's first two rows
      if (l < 32u) {
        copy_pieces<12, 13>(s0, d0);
        copy_pieces<12, 13>(s1, d1);
      }
      side_terms<+1, PR, kAssignFirst<TC>>(W, dW, gp, acc);
    }
    // the right side's LDS reads wait for the left side's results and for
    // this wave's copies
    size_t slot = threadIdx.x >> 2 & 15u;
    after_left_side(slot, acc);
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("" ::: "memory");
    {
      TC W[5], dW[3][5];
      const TC* cv = rs + (slot >> 3) * kStageGroup + (slot & 7u);
      if constexpr (FS)
        eval_char_gp_dir<false>(D, cv, Qbar, gp.gamma, TC(-0.5), xa, xb, fbR, invd, W, dW);
      else if (D == 0)
        eval_rows_gp<0, 8>(cv, TC(-0.5), xa, xb, fbR, invd, W, dW);
      else if (D == 1)
        eval_rows_gp<1, 8>(cv, TC(-0.5), xa, xb, fbR, invd, W, dW);
      else
        eval_rows_gp<2, 8>(cv, TC(-0.5), xa, xb, fbR, invd, W, dW);
      side_terms<-1, PR>(W, dW, gp, acc);
    }
  } else if constexpr (FS) {
    double Qbar[5];
#pragma unroll
    for (int v = 0; v < 5; ++v)
      Qbar[v] = 0.5 * ((double)coefL[coef_cell<TC>(iL) + v * 10 * kCB<TC>] +
                       (double)coefR[coef_cell<TC>(iR) + v * 10 * kCB<TC>]);
    // Both sides' Gauss-point states are formed before any side terms,
    // while the flux accumulators are not yet live: there are registers for
    // each side's 45 coefficient loads to be in flight together.
    TC WL[5], dWL[3][5], WR[5], dWR[3][5];
    eval_char_gp_dir(D, coefL + coef_cell<TC>(iL), Qbar, gp.gamma, TC(0.5), xa, xb, fbL, invd, WL, dWL);
    eval_char_gp_dir(D, coefR + coef_cell<TC>(iR), Qbar, gp.gamma, TC(-0.5), xa, xb, fbR, invd, WR, dWR);
    side_terms<+1, PR, kAssignFirst<TC>>(WL, dWL, gp, acc);
    side_terms<-1, PR>(WR, dWR, gp, acc);
  } else {
    {
      TC W[5], dW[3][5];
      eval_box_gp_dir(D, coefL, iL, TC(0.5), xa, xb, fbL, invd, W, dW);
      side_terms<+1, PR, kAssignFirst<TC>>(W, dW, gp, acc);
    }
    after_left_side(iR, acc);
    {
      TC W[5], dW[3][5];
      eval_box_gp_dir(D, coefR, iR, TC(-0.5), xa, xb, fbR, invd, W, dW);
      side_terms<-1, PR>(W, dW, gp, acc);
    }
  }
  TC F[5], dF[5];
  finish_flux<PR>(acc, gp, dt, idt, F, dF);
  // Face weight of Eq. (11): Gauss weight 1/4 times the area element.
  const TC w = TC(G.wface[D]);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    F[i] *= w;
    dF[i] *= w;
    F[i] = quad_xor_add<2>(quad_xor_add<1>(F[i]));
    dF[i] = quad_xor_add<2>(quad_xor_add<1>(dF[i]));
  }
  if (live && gpi == 0) {
    const size_t NF = (size_t)G.nf[D][0] * G.nf[D][1] * G.nf[D][2];
    const int gv[5] = {0, 1 + ax.D, 1 + ax.A, 1 + ax.B, 4};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      face[(size_t)gv[i] * NF + f] = F[i];
      face[(size_t)(5 + gv[i]) * NF + f] = dF[i];
    }
  }
}

// Direction and block within that direction of logical flux block b, for
// nb[d] blocks of 64 faces per direction.  The three directions are
// interleaved (b % 3) while all have blocks left, so that the x-, y- and
// z-faces of the same cells run at nearly the same time on the same XCD
// and share its L2 for the cells' coefficients; the remaining blocks of
// the longer directions follow in order.
HGKS_FN void flux_block(unsigned b, const unsigned (&nb)[3], int& D, unsigned& lb) {
  const unsigned m = min(nb[0], min(nb[1], nb[2]));
  if (b < 3 * m) {
    D = (int)(b % 3);
    lb = b / 3;
    return;
  }
  b -= 3 * m;
  D = 0;
  while (D < 2 && b >= nb[D] - m) {
    b -= nb[D] - m;
    ++D;
  }
  lb = m + b;
}

// All faces of the three directions in one launch (see flux_block).
template <typename TC, bool PR = false, bool FS = false>
__global__ void __launch_bounds__(kBlock) HGKS_FLUX_OCCUPANCY k_flux_box(
    const TC* __restrict__ coef, const uint32_t* __restrict__ mask, TC* __restrict__ fx, TC* __restrict__ fy,
    TC* __restrict__ fz, BoxGrid G, GasParams<TC> gp, TC dt, TC idt, unsigned nb0, unsigned nb1, unsigned nb2) {
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nb0 + nb1 + nb2) return;
  const unsigned nb[3] = {nb0, nb1, nb2};
  int D;
  unsigned lb;
  flux_block(b, nb, D, lb);
  TC* face = D == 0 ? fx : (D == 1 ? fy : fz);
  if constexpr (sizeof(TC) == 8) {
    __shared__ double stage[kBlock / 64 * kStageWave];
    flux_box_face<TC, PR, FS, true>(coef, mask, face, G, gp, dt, idt, lb, D, stage);
  } else {
    flux_box_face<TC, PR, FS>(coef, mask, face, G, gp, dt, idt, lb, D);
  }
}

// ---------------------------------------------------------------- update
// mode 0: one-stage update q = q + dt L + dt^2/2 dL
// mode 1: first stage: qs = q + dt/2 L + dt^2/8 dL, acc = q + dt L + dt^2/6 dL
// mode 2: second stage: q = acc + dt^2/3 dL(q*)
template <typename TF>
__device__ __forceinline__ void update_box_cell(double* __restrict__ q, double* __restrict__ qs,
                                                double* __restrict__ acc, const TF* __restrict__ fx,
                                                const TF* __restrict__ fy, const TF* __restrict__ fz,
                                                const BoxGrid& G, double dt, int mode, size_t N, size_t idx) {
  int c[3];
  split_index((uint32_t)idx, G.n[0], G.n[1], G.inv_n[0], G.inv_n[1], c[0], c[1], c[2]);
  const TF* fs[3] = {fx, fy, fz};
  double R[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) R[k] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int* nf = G.nf[d];
    const size_t NF = (size_t)nf[0] * nf[1] * nf[2];
    int hi[3] = {c[0], c[1], c[2]};
    hi[d] += 1;
    if (G.per[d] && hi[d] == G.n[d]) hi[d] = 0;
    // byte offsets in 32 bits from each array's uniform base (every array
    // has fewer than 2^29 elements)
    const unsigned lo_b = (unsigned)(((unsigned)c[2] * nf[1] + c[1]) * nf[0] + c[0]) * (unsigned)sizeof(TF);
    const unsigned hi_b = (unsigned)(((unsigned)hi[2] * nf[1] + hi[1]) * nf[0] + hi[0]) * (unsigned)sizeof(TF);
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const char* base = (const char*)(fs[d] + k * NF);
      R[k] -= (double)*(const TF*)(base + hi_b) - (double)*(const TF*)(base + lo_b);
    }
  }
  const double iv = 1.0 / G.vol;
  const unsigned ob = (unsigned)idx * 8u;
  auto at = [&](double* a, int v) -> double& { return *(double*)((char*)(a + (size_t)v * N) + ob); };
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double L = R[v] * iv, dL = R[5 + v] * iv;
    if (mode == 0) {
      at(q, v) = at(q, v) + dt * L + 0.5 * dt * dt * dL;
    } else if (mode == 1) {
      const double q0 = at(q, v);
      at(qs, v) = q0 + 0.5 * dt * L + 0.125 * dt * dt * dL;
      at(acc, v) = q0 + dt * L + dt * dt / 6.0 * dL;
    } else {
      at(q, v) = at(acc, v) + dt * dt / 3.0 * dL;
    }
  }
}

template <typename TF>
__global__ void __launch_bounds__(kBlock) k_update_box(double* __restrict__ q, double* __restrict__ qs,
                                                       double* __restrict__ acc, const TF* __restrict__ fx,
                                                       const TF* __restrict__ fy, const TF* __restrict__ fz,
                                                       BoxGrid G, double dt, int mode, size_t N) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  update_box_cell(q, qs, acc, fx, fy, fz, G, dt, mode, N, idx);
}

// ---------------------------------------------------------------- reductions
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* sh, Op op) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

struct MinOp {
  __device__ double operator()(double a, double b) const { return a < b ? a : b; }
};
struct SumOp {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
};

// Time-step bound h / (|U| + c) per cell, minimum per block.
__global__ void __launch_bounds__(kBlock) k_dt_box(const double* __restrict__ q, BoxGrid G, double gamma,
                                                   double* __restrict__ part, size_t N) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double v = 1e300;
  if (idx < N) {
    const double rho = q[idx];
    const double u = q[N + idx] / rho, w1 = q[2 * N + idx] / rho, w2 = q[3 * N + idx] / rho;
    const double p = (gamma - 1.0) * (q[4 * N + idx] - 0.5 * rho * (u * u + w1 * w1 + w2 * w2));
    const double c = sqrt(gamma * p / rho);
    double h = 1.0 / G.inv_dx[0];
    h = fmin(h, 1.0 / G.inv_dx[1]);
    h = fmin(h, 1.0 / G.inv_dx[2]);
    v = h / (sqrt(u * u + w1 * w1 + w2 * w2) + c);
    if (!(v > 0.0)) v = -1.0;  // non-physical state: reported as a negative bound
  }
  const double r = block_reduce(v, sh, MinOp());
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_min_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double v = 1e300;
  for (int i = threadIdx.x; i < n; i += kBlock) v = fmin(v, part[i]);
  const double r = block_reduce(v, sh, MinOp());
  if (threadIdx.x == 0) out[0] = r;
}

// sum |Omega| Q_v: fixed-order block sums, then a fixed-order final sum.
__global__ void __launch_bounds__(kBlock) k_totals_box(const double* __restrict__ q, double vol,
                                                       double* __restrict__ part, size_t N, int nblk) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  for (int v = 0; v < 5; ++v) {
    const double x = idx < N ? q[(size_t)v * N + idx] * vol : 0.0;
    const double r = block_reduce(x, sh, SumOp());
    if (threadIdx.x == 0) part[(size_t)v * nblk + blockIdx.x] = r;
    __syncthreads();
  }
}

// Kinetic energy of the cell averages, sum |Omega_i| |M_i|^2 / (2 rho_i)
// (the integrand of the volume-averaged kinetic energy of Sec. 4, Taylor-
// Green vortex, taken on the cell averages), and the volume sum |Omega_i|,
// per block in a fixed order.  geo = null: every cell has volume vol; else
// the hexahedral geometry record, whose first row is the cell volume.
__global__ void __launch_bounds__(kBlock) k_kinetic(const double* __restrict__ q, const double* __restrict__ geo,
                                                    double vol, double* __restrict__ part, size_t N, int nblk) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double e = 0.0, v = 0.0;
  if (idx < N) {
    const double V = geo ? geo[idx] : vol;
    const double m2 = q[N + idx] * q[N + idx] + q[2 * N + idx] * q[2 * N + idx] + q[3 * N + idx] * q[3 * N + idx];
    e = V * 0.5 * m2 / q[idx];
    v = V;
  }
  const double r1 = block_reduce(e, sh, SumOp());
  if (threadIdx.x == 0) part[blockIdx.x] = r1;
  __syncthreads();
  const double r2 = block_reduce(v, sh, SumOp());
  if (threadIdx.x == 0) part[(size_t)nblk + blockIdx.x] = r2;
}

__global__ void __launch_bounds__(kBlock) k_sum_final(const double* __restrict__ part, int n, int nvec,
                                                      double* __restrict__ out) {
  __shared__ double sh[kBlock];
  for (int v = 0; v < nvec; ++v) {
    double x = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) x += part[(size_t)v * n + i];
    const double r = block_reduce(x, sh, SumOp());
    if (threadIdx.x == 0) out[v] = r;
    __syncthreads();
  }
}

// Counts of non-physical cells and of fallback Gauss points of real cells.
__global__ void __launch_bounds__(kBlock) k_check_box(const double* __restrict__ q, const uint32_t* __restrict__ mask,
                                                      BoxGrid G, double gamma, double* __restrict__ part,
                                                      size_t N, int nblk) {
  __shared__ double sh[kBlock];
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double bad = 0.0, fb = 0.0;
  if (idx < N) {
    const double rho = q[idx];
    const double e = q[4 * N + idx];
    const double m2 = q[N + idx] * q[N + idx] + q[2 * N + idx] * q[2 * N + idx] + q[3 * N + idx] * q[3 * N + idx];
    const double p = (gamma - 1.0) * (e - 0.5 * m2 / rho);
    bad = (rho > 0.0 && p > 0.0) ? 0.0 : 1.0;
    const int c0 = (int)(idx % G.n[0]), c1 = (int)((idx / G.n[0]) % G.n[1]);
    const int c2 = (int)(idx / ((size_t)G.n[0] * G.n[1]));
    const size_t r = ((size_t)(c2 + G.g[2]) * G.nr[1] + (c1 + G.g[1])) * G.nr[0] + (c0 + G.g[0]);
    fb = (double)__popc(mask[r] & 0x00FFFFFFu);
  }
  double r1 = block_reduce(bad, sh, SumOp());
  if (threadIdx.x == 0) part[blockIdx.x] = r1;
  __syncthreads();
  double r2 = block_reduce(fb, sh, SumOp());
  if (threadIdx.x == 0) part[(size_t)nblk + blockIdx.x] = r2;
}

// ---------------------------------------------------------------- debug
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_debug_gp_box(const TC* __restrict__ coef, const uint32_t* __restrict__ mask,
                                                         BoxGrid G, size_t NR, size_t N, double gamma,
                                                         double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  const int c0 = (int)(idx % G.n[0]), c1 = (int)((idx / G.n[0]) % G.n[1]);
  const int c2 = (int)(idx / ((size_t)G.n[0] * G.n[1]));
  const size_t r = ((size_t)(c2 + G.g[2]) * G.nr[1] + (c1 + G.g[1])) * G.nr[0] + (c0 + G.g[0]);
  const uint32_t mk = mask[r];
  for (int bit = 0; bit < 24; ++bit) {
    const int f = bit >> 2, gp = bit & 3, d = f >> 1;
    TC xi[3];
    xi[d] = (f & 1) ? TC(0.5) : TC(-0.5);
    xi[(d + 1) % 3] = (gp >> 1) ? TC(kGaussNode) : TC(-kGaussNode);
    xi[(d + 2) % 3] = (gp & 1) ? TC(kGaussNode) : TC(-kGaussNode);
    const bool fb = (mk >> bit) & 1u;
    if (G.fs_stride) {
      // characteristic reconstruction: R from the mean of the two cells
      // sharing face f, the fields' deviations projected back
      const TC* cv = coef + (size_t)f * G.fs_stride + coef_cell<TC>(r);
      int cc[3] = {c0, c1, c2};
      cc[d] += (f & 1) ? 1 : -1;
      const size_t rn = ((size_t)rec_index(G, 2, cc[2]) * G.nr[1] + rec_index(G, 1, cc[1])) * G.nr[0] +
                        rec_index(G, 0, cc[0]);
      const TC* cn = coef + (size_t)f * G.fs_stride + coef_cell<TC>(rn);
      double Qbar[5];
      for (int v = 0; v < 5; ++v) Qbar[v] = 0.5 * ((double)cv[v * 10 * kCB<TC>] + (double)cn[v * 10 * kCB<TC>]);
      CharBasis Bs;
      char_basis(Qbar, d, gamma, Bs);
      double val[5], g[5][3];
      for (int v = 0; v < 5; ++v) {
        val[v] = (double)cv[v * 10 * kCB<TC>];
        g[v][0] = g[v][1] = g[v][2] = 0.0;
      }
      if (!fb) {
        for (int fld = 0; fld < 5; ++fld) {
          const TC* ck = cv + fld * 10 * kCB<TC>;
          TC c[9];
          for (int m = 0; m < 9; ++m) c[m] = ck[(m + 1) * kCB<TC>];
          TC du, gu[3];
          quad_eval(TC(0), c, xi[0], xi[1], xi[2], du, gu[0], gu[1], gu[2]);
          double rc[5];
          char_rcol(Bs, fld, rc);
          for (int v = 0; v < 5; ++v) {
            const TC rv = TC(rc[v]);
            val[v] += (double)(rv * du);
            for (int j = 0; j < 3; ++j) g[v][j] += (double)(rv * gu[j]);
          }
        }
      }
      for (int v = 0; v < 5; ++v) {
        double* o = out + ((idx * 24 + bit) * 5 + v) * 4;
        o[0] = val[v];
        for (int j = 0; j < 3; ++j) o[1 + j] = g[v][j] * G.inv_dx[j];
      }
      continue;
    }
    for (int v = 0; v < 5; ++v) {
      const TC* cv = coef + (size_t)f * G.fs_stride + coef_cell<TC>(r) + v * 10 * kCB<TC>;
      TC c[9];
      for (int m = 0; m < 9; ++m) c[m] = cv[(m + 1) * kCB<TC>];
      TC val, g[3];
      quad_eval(cv[0], c, xi[0], xi[1], xi[2], val, g[0], g[1], g[2]);
      if (fb) {
        val = cv[0];
        g[0] = g[1] = g[2] = TC(0);
      }
      double* o = out + ((idx * 24 + bit) * 5 + v) * 4;
      o[0] = (double)val;
      o[1] = (double)g[0] * G.inv_dx[0];
      o[2] = (double)g[1] * G.inv_dx[1];
      o[3] = (double)g[2] * G.inv_dx[2];
    }
  }
}

// Fallback mask words of the real cells, [nz][ny][nx]: bit 4 f + g set where
// Gauss point g of face f took the first-order fallback (the "needs the
// exact test" bit is clear after a stage).  rec = 1: box grid (masks over
// the reconstruction box); rec = 0: one mask per cell (hexahedral grids).
__global__ void __launch_bounds__(kBlock) k_debug_mask(const uint32_t* __restrict__ mask, BoxGrid G, int rec,
                                                       size_t N, uint32_t* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  size_t r = idx;
  if (rec) {
    const int c0 = (int)(idx % G.n[0]), c1 = (int)((idx / G.n[0]) % G.n[1]);
    const int c2 = (int)(idx / ((size_t)G.n[0] * G.n[1]));
    r = ((size_t)(c2 + G.g[2]) * G.nr[1] + (c1 + G.g[1])) * G.nr[0] + (c0 + G.g[0]);
  }
  out[idx] = mask[r] & 0x00FFFFFFu;
}

template <typename TF>
__global__ void __launch_bounds__(kBlock) k_debug_face_box(const TF* __restrict__ face, BoxGrid G, int d, size_t N,
                                                           double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= N) return;
  const int c0 = (int)(idx % G.n[0]), c1 = (int)((idx / G.n[0]) % G.n[1]);
  const int c2 = (int)(idx / ((size_t)G.n[0] * G.n[1]));
  const int* nf = G.nf[d];
  const size_t NF = (size_t)nf[0] * nf[1] * nf[2];
  const size_t fi = ((size_t)c2 * nf[1] + c1) * nf[0] + c0;
  for (int k = 0; k < 10; ++k) out[((size_t)d * N + idx) * 10 + k] = (double)face[(size_t)k * NF + fi];
}

}  // namespace hgks
