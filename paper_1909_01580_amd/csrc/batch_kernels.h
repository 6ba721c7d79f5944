// Batched stage: many independent periodic box grids of uneven sizes
// advanced together, one persistent launch per phase (reconstruction,
// fallback test, face flux, update) and per-grid time steps read from
// device memory, so that whole steps can be captured in a HIP graph.
//
// Work is cut into tiles of 256 items (cells, or 64 faces x 4 Gauss
// points); every grid owns a contiguous range of tiles.  A cell tile is
// either 256 consecutive cells (x fastest) or a tx x ty x tz box of cells
// (tx ty tz = 256), the tile shape the autotuner chooses; a flux tile is 64
// consecutive faces of one direction in the banded cell order, whose band
// height is tunable too.  A persistent
// launch of P workgroups (P a multiple of 8) gives each of the eight XCDs
// one contiguous eighth of the tile range, walked by its P/8 workgroups
// with stride P/8, so that neighbouring tiles of a grid share an L2.
#pragma once

#include "box_kernels.h"
#include "char_box.h"

namespace hgks {

template <typename TC>
struct BatchGrid {
  BoxGrid G;
  WenoParams<TC> P;
  GasParams<TC> gp;
  size_t N, NF[3];
  size_t q_off;        // doubles: start of the grid's [5][N] state
  size_t coef_off;     // TC: start of the grid's coefficients (coef_cell layout)
  size_t mask_off;     // uint32: start of the grid's [N] masks
  size_t face_off[3];  // TC: start of the grid's [10][NF_d] face sums
  unsigned t_cell;     // first cell tile
  unsigned t_flux;     // first flux tile
  unsigned nt_cell;    // cell tiles
  unsigned nt_flux[3]; // flux tiles per direction
  int ct[3];           // cell tile shape; ct[0] = 0: 256 consecutive cells
  int nct[3];          // cell tiles per axis (box tiles)
  unsigned t_char;     // characteristic variables: first tile of k_batch_char_recon
  unsigned nt_char;    // its tiles (kCX x kCY x kCZ cells each)
  unsigned ncx, ncy;   // its tiles along x and y
};

// Cell of lane `lane` in cell tile lt (counted from the grid's first):
// false for lanes past the grid's extent.
template <typename TC>
__device__ __forceinline__ bool batch_cell(const BatchGrid<TC>& b, unsigned lt, unsigned lane, size_t& idx) {
  if (b.ct[0] == 0) {
    idx = (size_t)lt * kBlock + lane;
    return idx < b.N;
  }
  const unsigned bx = lt % (unsigned)b.nct[0], r = lt / (unsigned)b.nct[0];
  const unsigned by = r % (unsigned)b.nct[1], bz = r / (unsigned)b.nct[1];
  const int i = (int)(bx * b.ct[0] + lane % b.ct[0]);
  const int j = (int)(by * b.ct[1] + (lane / b.ct[0]) % b.ct[1]);
  const int k = (int)(bz * b.ct[2] + lane / (b.ct[0] * b.ct[1]));
  if (i >= b.G.n[0] || j >= b.G.n[1] || k >= b.G.n[2]) return false;
  idx = ((size_t)k * b.G.n[1] + j) * b.G.n[0] + i;
  return true;
}

// Grid owning tile t (binary search over the first-tile table).
template <typename TC, bool FLUX>
__device__ __forceinline__ int batch_grid_of(const BatchGrid<TC>* __restrict__ B, int ng, unsigned t) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const unsigned first = FLUX ? B[mid].t_flux : B[mid].t_cell;
    if (first <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Grid owning tile t of the characteristic reconstruction.
template <typename TC>
__device__ __forceinline__ int batch_grid_of_char(const BatchGrid<TC>* __restrict__ B, int ng, unsigned t) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (B[mid].t_char <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Persistent tile walk: XCD x = blockIdx % 8 takes tiles
// [x * chunk, (x + 1) * chunk), its workgroups striding by P / 8.
struct TileWalk {
  unsigned t, end, stride;
  __device__ __forceinline__ TileWalk(unsigned ntiles) {
    const unsigned P = gridDim.x, per = P >> 3;
    const unsigned x = blockIdx.x & 7u, w = blockIdx.x >> 3;
    const unsigned chunk = (ntiles + 7u) >> 3;
    t = x * chunk + w;
    end = min(ntiles, (x + 1) * chunk);
    stride = per;
  }
};

// Tiles of this workgroup: LOOP = false, a launch of one workgroup per tile
// (rounded up to a multiple of 8, logical tile = xcd_block of the block
// id, the same order as the walk); LOOP = true, the persistent walk.  The
// loop-free form keeps the compiler from holding loop-invariant values in
// registers across the whole walk, which costs the flux kernel spills.
template <bool LOOP, typename F>
__device__ __forceinline__ void for_tiles(unsigned ntiles, F&& body) {
  if constexpr (LOOP) {
    for (TileWalk w(ntiles); w.t < w.end; w.t += w.stride) body(w.t);
  } else {
    const unsigned t = xcd_block(blockIdx.x, gridDim.x);
    if (t < ntiles) body(t);
  }
}

// WIDE: the stencils of Remark 1 for every grid of the batch (the flux and
// update do not depend on the stencil family).  COEF = false: the fallback
// mask only (characteristic variables).
template <typename TC, bool LOOP, bool WIDE = false, bool COEF = true>
__global__ void __launch_bounds__(kBlock) k_batch_recon(const BatchGrid<TC>* __restrict__ B, int ng, unsigned ntiles,
                                                        const double* __restrict__ q, TC* __restrict__ coef,
                                                        uint32_t* __restrict__ mask, TC margin, TC gm1) {
  for_tiles<LOOP>(ntiles, [&](unsigned t) {
    const int g = batch_grid_of<TC, false>(B, ng, t);
    size_t idx;
    if (batch_cell(B[g], t - B[g].t_cell, threadIdx.x, idx))
      recon_box_cell<TC, WIDE, COEF>(q + B[g].q_off, coef + B[g].coef_off, mask + B[g].mask_off, B[g].G, B[g].P, margin,
                               gm1, B[g].N, idx);
  });
}

template <typename TC, bool LOOP, bool WIDE = false>
__global__ void __launch_bounds__(kBlock) k_batch_posit(const BatchGrid<TC>* __restrict__ B, int ng, unsigned ntiles,
                                                        const double* __restrict__ q, uint32_t* __restrict__ mask,
                                                        TC gm1) {
  for_tiles<LOOP>(ntiles, [&](unsigned t) {
    const int g = batch_grid_of<TC, false>(B, ng, t);
    size_t idx;
    if (batch_cell(B[g], t - B[g].t_cell, threadIdx.x, idx) && mask[B[g].mask_off + idx] == kNeedsCheck)
      posit_exact_box_cell<TC, WIDE>(q + B[g].q_off, mask + B[g].mask_off, B[g].G, gm1, idx);
  });
}

// Reconstruction in characteristic variables (Sec. 4) for every grid of the
// batch: one workgroup per tile of each grid (the tile is staged in LDS
// behind a workgroup barrier), the six per-face arrays of a grid following
// its component-wise coefficient array.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_batch_char_recon(const BatchGrid<TC>* __restrict__ B, int ng,
                                                             unsigned ntiles, const double* __restrict__ q,
                                                             TC* __restrict__ coef, double gamma) {
  __shared__ double T[5][kCHalo];
  const unsigned t = xcd_block(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;
  const BatchGrid<TC>& b = B[batch_grid_of_char(B, ng, t)];
  char_recon_tile(q + b.q_off, coef + b.coef_off + b.G.fs_stride, b.G, b.P, gamma, b.ncx, b.ncy, t - b.t_char, T);
}

// PR: the extended viscous model (viscosity law, Prandtl correction), per
// grid through its gas parameters (trivial for grids that use neither).
// FP64 stages the right cells in LDS as the single-grid flux does; in the
// persistent form a wave's staged values are consumed before its next
// tile's copies are issued.  FS: the per-face arrays of the
// characteristic reconstruction.
template <typename TC, bool LOOP, bool PR = false, bool FS = false>
__global__ void __launch_bounds__(kBlock) HGKS_FLUX_OCCUPANCY
    k_batch_flux(const BatchGrid<TC>* __restrict__ B, int ng, unsigned ntiles, const TC* __restrict__ coef,
                 const uint32_t* __restrict__ mask, TC* __restrict__ face, const double* __restrict__ dt) {
  constexpr bool kStage = sizeof(TC) == 8;
  __shared__ TC stage[kStage ? kBlock / 64 * kStageWave : 1];
  for_tiles<LOOP>(ntiles, [&](unsigned t) {
    const int g = batch_grid_of<TC, true>(B, ng, t);
    const BatchGrid<TC>& b = B[g];
    if (!(dt[g] > 0.0)) return;  // a grid without a time step is not advanced
    unsigned lt;
    const TC dtg = TC(dt[g]);
    const TC idtg = TC(1.0 / dt[g]);
    const TC* cf = coef + b.coef_off + (FS ? b.G.fs_stride : 0);
    const uint32_t* mk = mask + b.mask_off;
    const unsigned nb[3] = {b.nt_flux[0], b.nt_flux[1], b.nt_flux[2]};
    int D;
    flux_block(t - b.t_flux, nb, D, lt);
    flux_box_face<TC, PR, FS, kStage>(cf, mk, face + b.face_off[D], b.G, b.gp, dtg, idtg, lt, D, stage);
  });
}

template <typename TC, bool LOOP>
__global__ void __launch_bounds__(kBlock) k_batch_update(const BatchGrid<TC>* __restrict__ B, int ng, unsigned ntiles,
                                                         double* __restrict__ q, double* __restrict__ qs,
                                                         double* __restrict__ acc, const TC* __restrict__ face,
                                                         const double* __restrict__ dt, int mode) {
  for_tiles<LOOP>(ntiles, [&](unsigned t) {
    const int g = batch_grid_of<TC, false>(B, ng, t);
    const BatchGrid<TC>& b = B[g];
    size_t idx;
    if (batch_cell(b, t - b.t_cell, threadIdx.x, idx) && dt[g] > 0.0)
      update_box_cell(q + b.q_off, qs + b.q_off, acc + b.q_off, face + b.face_off[0], face + b.face_off[1],
                      face + b.face_off[2], b.G, dt[g], mode, b.N, idx);
  });
}

// Per-tile minimum of h / (|U| + c), then per-grid dt = cfl * minimum.
template <typename TC, bool LOOP>
__global__ void __launch_bounds__(kBlock) k_batch_dt_part(const BatchGrid<TC>* __restrict__ B, int ng,
                                                          unsigned ntiles, const double* __restrict__ q, double gamma,
                                                          double* __restrict__ part) {
  __shared__ double sh[kBlock];
  for_tiles<LOOP>(ntiles, [&](unsigned t) {
    const int g = batch_grid_of<TC, false>(B, ng, t);
    const BatchGrid<TC>& b = B[g];
    size_t idx;
    double v = 1e300;
    if (batch_cell(b, t - b.t_cell, threadIdx.x, idx)) {
      const double* qg = q + b.q_off;
      const size_t N = b.N;
      const double rho = qg[idx];
      const double u = qg[N + idx] / rho, v1 = qg[2 * N + idx] / rho, v2 = qg[3 * N + idx] / rho;
      const double p = (gamma - 1.0) * (qg[4 * N + idx] - 0.5 * rho * (u * u + v1 * v1 + v2 * v2));
      const double c = sqrt(gamma * p / rho);
      const double h = fmin(fmin(1.0 / b.G.inv_dx[0], 1.0 / b.G.inv_dx[1]), 1.0 / b.G.inv_dx[2]);
      v = h / (sqrt(u * u + v1 * v1 + v2 * v2) + c);
      if (!(v > 0.0)) v = -1.0;
    }
    const double r = block_reduce(v, sh, MinOp());
    if (threadIdx.x == 0) part[t] = r;
    __syncthreads();
  });
}

// A grid with a non-physical cell (density or pressure not positive, or
// NaN: the per-cell bound is then -1) gets dt = 0, which the flux and update
// kernels take as "do not advance", and sets bit 0 of *status.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_batch_dt_final(const BatchGrid<TC>* __restrict__ B,
                                                           const double* __restrict__ part, double cfl,
                                                           double* __restrict__ dt, uint32_t* __restrict__ status) {
  __shared__ double sh[kBlock];
  const int g = blockIdx.x;
  double v = 1e300;
  for (unsigned t = threadIdx.x; t < B[g].nt_cell; t += kBlock) v = fmin(v, part[B[g].t_cell + t]);
  const double r = block_reduce(v, sh, MinOp());
  if (threadIdx.x == 0) {
    const bool ok = r > 0.0;
    dt[g] = ok ? cfl * r : 0.0;
    if (!ok) atomicOr(status, 1u);
  }
}

// sum |Omega| Q_v per grid, fixed order.
template <typename TC>
__global__ void __launch_bounds__(kBlock) k_batch_totals(const BatchGrid<TC>* __restrict__ B,
                                                         const double* __restrict__ q, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  const int g = blockIdx.x;
  const BatchGrid<TC>& b = B[g];
  for (int v = 0; v < 5; ++v) {
    double s = 0.0;
    for (size_t i = threadIdx.x; i < b.N; i += kBlock) s += q[b.q_off + v * b.N + i];
    const double r = block_reduce(s, sh, SumOp());
    if (threadIdx.x == 0) out[g * 5 + v] = r * b.G.vol;
    __syncthreads();
  }
}

}  // namespace hgks
