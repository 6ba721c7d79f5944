// Reconstruction in characteristic variables on hexahedral grids (Pan & Xu,
// Sec. 4: the option stated after the limiting procedure), static or moving.
//
// For face fs = 2 D + s of a cell (s = 0 the face on the cell's low side
// along index axis D, s = 1 the high one) the stencil data are projected to
// U = L Q, L = R^-1, R the right eigenvectors of the Euler Jacobian along
// the frame of Sec. 3 at the face's centre (n along X_a x X_b, the shear
// fields along X_b x n and X_b), taken at the mean of the two cell averages
// that share the face.  The least squares of Sec. 2 are linear, so the 25
// polynomials of U are L times those of Q; indicators and nonlinear weights
// belong to each characteristic field.  As on box grids, each cell gets six
// reconstructions stored as six coefficient arrays (array fs): row 10 v the
// conservative cell mean of variable v, rows 10 f + 1 .. 10 f + 9 the nine
// coefficients of characteristic field f in the cell's scaled basis.  The
// face flux forms R from the two cells' means and the same frame and
// projects back at its Gauss points: value Q_c + R dU(x), gradient
// R grad U(x).  The positivity fallback stays on the conservative
// polynomials (the mask of the component-wise reconstruction).
#pragma once

#include "char_basis.h"
#include "hex_kernels.h"

namespace hgks {

// Eigenvectors of face fs of tile cell `base` (cell (i, j, k)): the mean of
// the cell's and its neighbour's averages across the face, the frame at the
// face centre.
__device__ __forceinline__ void char_face_basis(const HexGrid& H, const HexTile& T, int base, int i, int j, int k,
                                                int fs, double gamma, CharFrame& B) {
  const int D = fs >> 1, side = fs & 1;
  const int step = D == 0 ? 1 : (D == 1 ? kHX : kHX * kHY);
  const int nbr = base + (side ? step : -step);
  double Qb[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Qb[v] = 0.5 * (T.q[v][base] + T.q[v][nbr]);
  int c[3] = {i, j, k};
  c[D] += side;
  double n[3], t1[3], t2[3];
  face_centre_frame(H, D, c[0], c[1], c[2], n, t1, t2);
  char_frame(Qb, n, t1, t2, gamma, B);
}

// One workgroup per kTX x kTY x kTZ tile (the LDS tile of the component-wise
// reconstruction); every lane reconstructs its cell for the six faces.  The
// big-stencil fit runs once per cell in the conservative variables and is
// projected for every face (stored in the face arrays, read back for the
// face's indicators and combination); the 24 sub-stencil fits run in each
// face's pass, projected as they come.
template <typename TS>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
    k_char_recon_hex(HexGrid H, const double* __restrict__ geo, const double* __restrict__ q, TS* __restrict__ faces,
                     size_t fs_stride, WenoParams<double> P, double gamma, size_t N, unsigned ntx, unsigned nty,
                     unsigned ntiles) {
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
  const int base = ((lz + 1) * kHY + (ly + 1)) * kHX + (lx + 1);
  const NbrTile nb{T, base};
  HexCell Ci;
  load_cell(geo, N, idx, Ci);
  double qc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qc[v] = T.q[v][base];
  constexpr int CB = kCB<TS>;
  {
    double a[5][9];
    big_fit<false>(nb, nb, Ci, qc, a);
#pragma unroll 1
    for (int fs = 0; fs < 6; ++fs) {
      CharFrame B;
      char_face_basis(H, T, base, i, j, k, fs, gamma, B);
      TS* out = faces + (size_t)fs * fs_stride + coef_cell<TS>(idx);
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double l[5];
        char_lrow(B, f, l);
#pragma unroll
        for (int e = 0; e < 9; ++e)
          out[(10 * f + 1 + e) * CB] =
              TS(l[0] * a[0][e] + l[1] * a[1][e] + l[2] * a[2][e] + l[3] * a[3][e] + l[4] * a[4][e]);
      }
    }
  }
  // The stored projections are read back by the lane that wrote them.
  asm volatile("" ::: "memory");
#pragma unroll 1
  for (int fs = 0; fs < 6; ++fs) {
    double L[5][5];
    {
      CharFrame B;
      char_face_basis(H, T, base, i, j, k, fs, gamma, B);
#pragma unroll
      for (int f = 0; f < 5; ++f) char_lrow(B, f, L[f]);
    }
    TS* out = faces + (size_t)fs * fs_stride + coef_cell<TS>(idx);
    double beta0[5], r0[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      double c[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) c[e] = (double)out[(10 * f + 1 + e) * CB];
      beta0[f] = hex_beta0(c, Ci);
      r0[f] = d_rcp(beta0[f] + P.eps);
    }
    // weights affine in tau, as in the component-wise reconstruction
    double tsum[5], rsum[5], db[5][3];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      tsum[f] = rsum[f] = 0.0;
      db[f][0] = db[f][1] = db[f][2] = 0.0;
    }
    each_sub_fit(nb, Ci, qc, [&](const double (&bq)[5][3]) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double bu[3];
#pragma unroll
        for (int e = 0; e < 3; ++e)
          bu[e] = L[f][0] * bq[0][e] + L[f][1] * bq[1][e] + L[f][2] * bq[2][e] + L[f][3] * bq[3][e] +
                  L[f][4] * bq[4][e];
        const double bm = bu[0] * bu[0] + bu[1] * bu[1] + bu[2] * bu[2];
        tsum[f] += fabs(beta0[f] - bm);
        const double rm = d_rcp(bm + P.eps);
        rsum[f] += rm;
        const double dr = rm - r0[f];
#pragma unroll
        for (int e = 0; e < 3; ++e) db[f][e] += dr * bu[e];
      }
    });
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const double tau = tsum[f] * (1.0 / 24.0);
      const double w0r = 1.0 + tau * r0[f];
      const double iS = d_rcp(P.gamma0 * w0r + P.Gamma * (24.0 + tau * rsum[f]));
      const double w0g = w0r * iS;  // wbar_0 / gamma_0
      TS* cv = out + 10 * f * CB;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        const double au = (double)cv[(1 + e) * CB];
        cv[(1 + e) * CB] = TS(e < 3 ? w0g * au + iS * P.Gamma * tau * db[f][e] : w0g * au);
      }
      cv[0] = TS(qc[f]);  // the conservative mean of variable f
    }
  }
}

}  // namespace hgks
