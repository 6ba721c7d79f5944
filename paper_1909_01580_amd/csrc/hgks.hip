// Host side of the HGKS library: context, workspace carving, validation and
// the launch sequence of one time stage (Pan & Xu, Sec. 3, two-stage
// fourth-order scheme).  The C ABI is declared in include/hgks.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hgks.h"
#include "box_kernels.h"
#include "hex_kernels.h"
#include "batch_kernels.h"
#include "char_box.h"
#include "char_hex.h"

using namespace hgks;

namespace {

thread_local std::string g_err;

hgks_status fail(hgks_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
unsigned pad8(unsigned nb) { return (nb + 7u) & ~7u; }

struct Layout {
  size_t q, qs, acc, back, coef, mask, plist, face[3], vface[3], red, geo, verts, vnext, vol, vacc, total;
};

struct Dims {
  int n[3], g[3], nr[3], per[3], sym[3][2], nf[3][3];
  size_t N, NR, NF[3];
  size_t nred;  // doubles of reduction scratch
};

// Boundary at the high end of axis d (bc_hi may say "the same as the low end").
int bc_high(const hgks_config* c, int d) { return c->bc_hi[d] == HGKS_BC_SAME ? c->bc[d] : c->bc_hi[d]; }

bool valid_bc(int b) { return b == HGKS_BC_PERIODIC || b == HGKS_BC_OUTFLOW || b == HGKS_BC_SYMMETRIC; }

bool valid_config(const hgks_config* c) {
  if (!c) return false;
  if (c->nx < 2 || c->ny < 2 || c->nz < 2) return false;
  for (int d = 0; d < 3; ++d) {
    if (!valid_bc(c->bc[d]) || !valid_bc(bc_high(c, d))) return false;
    if ((c->bc[d] == HGKS_BC_PERIODIC) != (bc_high(c, d) == HGKS_BC_PERIODIC)) return false;
  }
  if (!(c->gamma > 1.0 && c->gamma < 5.0 / 3.0)) return false;
  if (!(c->mu >= 0.0) || !(c->weno_Gamma > 0.0 && c->weno_Gamma < 1.0 / 24.0)) return false;
  if (!(c->weno_eps > 0.0) || !(c->tau_eps >= 0.0) || !(c->tau_C >= 0.0)) return false;
  if (c->precision != HGKS_FP64 && c->precision != HGKS_MIXED) return false;
  if (c->moving != 0 && c->moving != 1) return false;
  if (c->characteristic != 0 && c->characteristic != 1) return false;
  if (!(c->mu_T0 > 0.0) || !std::isfinite(c->mu_exponent) || !(c->prandtl > 0.0) || !std::isfinite(c->prandtl))
    return false;
  // the stencils of Remark 1: component-wise reconstruction (box and
  // hexahedral grids); a mirror two cells past the ghost layer needs three
  // cells on that axis
  if (c->stencil != 0 && c->stencil != 1) return false;
  if (c->stencil && (c->characteristic || !(c->weno_Gamma < 1.0 / 24.0))) return false;
  if (c->stencil) {
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int d = 0; d < 3; ++d)
      if ((c->bc[d] == HGKS_BC_SYMMETRIC || bc_high(c, d) == HGKS_BC_SYMMETRIC) && n[d] < 3) return false;
  }
  if (c->moving)
    for (int d = 0; d < 3; ++d)
      if (c->bc[d] != HGKS_BC_PERIODIC) return false;
  // Cell and face indices are split in 32-bit arithmetic, and kernels
  // address their arrays with 32-bit byte offsets from uniform bases: fewer
  // than 2^29 elements per array (a grid that large would need some 400 GB
  // of workspace in FP64 anyway).
  if (((uint64_t)c->nx + 2) * ((uint64_t)c->ny + 2) * ((uint64_t)c->nz + 2) >= (1ull << 29)) return false;
  return true;
}

Dims make_dims(const hgks_config* c) {
  Dims D;
  const int n[3] = {c->nx, c->ny, c->nz};
  D.N = 1;
  D.NR = 1;
  for (int d = 0; d < 3; ++d) {
    D.n[d] = n[d];
    D.per[d] = c->bc[d] == HGKS_BC_PERIODIC;
    D.sym[d][0] = c->bc[d] == HGKS_BC_SYMMETRIC;
    D.sym[d][1] = bc_high(c, d) == HGKS_BC_SYMMETRIC;
    D.g[d] = D.per[d] ? 0 : 1;
    D.nr[d] = n[d] + 2 * D.g[d];
    D.N *= (size_t)n[d];
    D.NR *= (size_t)D.nr[d];
  }
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) D.nf[d][e] = n[e];
    if (!D.per[d]) D.nf[d][d] += 1;
    D.NF[d] = (size_t)D.nf[d][0] * D.nf[d][1] * D.nf[d][2];
  }
  D.nred = 8 * (size_t)blocks_for(D.N) + 64;
  return D;
}

Layout make_layout(const hgks_config* c, const Dims& D) {
  Layout L;
  const size_t tc = c->precision == HGKS_MIXED ? sizeof(float) : sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.q = take(5 * D.N * sizeof(double));
  L.qs = take(5 * D.N * sizeof(double));
  L.acc = take(5 * D.N * sizeof(double));
  // copy of the state for hgks_step_checked (static grids only)
  L.back = c->moving ? 0 : take(5 * D.N * sizeof(double));
  // one coefficient array, plus six per-face arrays in characteristic mode
  L.coef = take(coef_elems(D.NR, tc) * tc * (c->characteristic ? 7 : 1));
  L.mask = take(D.NR * sizeof(uint32_t));
  // list of the cells the exact positivity test examines, and its counter
  L.plist = c->moving ? 0 : take((D.NR + 64) * sizeof(uint32_t));
  for (int d = 0; d < 3; ++d) L.face[d] = take(10 * D.NF[d] * tc);
  // volume rates R_V, dR_V of the moving faces, double in every mode
  for (int d = 0; d < 3; ++d) L.vface[d] = c->moving ? take(2 * D.NF[d] * sizeof(double)) : 0;
  L.red = take(D.nred * sizeof(double));
  if (c->moving) {
    L.geo = take((size_t)kHexGeo * D.N * sizeof(double));
    L.verts = take(3 * D.N * sizeof(double));
    L.vnext = take(3 * D.N * sizeof(double));
    L.vol = take(D.N * sizeof(double));
    L.vacc = take(2 * D.N * sizeof(double));
  } else {
    L.geo = L.verts = L.vnext = L.vol = L.vacc = 0;
  }
  L.total = off;
  return L;
}

}  // namespace

struct hgks_ctx_s {
  hgks_config cfg;
  hipStream_t stream;
  Dims D;
  Layout L;
  BoxGrid G;
  HexGrid H;
  char* ws;
  bool grid_set = false, state_set = false, next_set = false;
  hgks_status sticky = HGKS_OK;
  double period[3];
  // Phase timing (hgks_profile_begin / hgks_profile_end).
  static constexpr int kProfCap = 512;
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev[HGKS_NPHASES];
  int prof_used[HGKS_NPHASES] = {0, 0, 0, 0, 0};
  bool prof_open[HGKS_NPHASES] = {false, false, false, false, false};

  double* q() { return (double*)(ws + L.q); }
  double* qs() { return (double*)(ws + L.qs); }
  double* acc() { return (double*)(ws + L.acc); }
  double* back() { return (double*)(ws + L.back); }
  void* coef() { return ws + L.coef; }
  uint32_t* mask() { return (uint32_t*)(ws + L.mask); }
  uint32_t* plist() { return (uint32_t*)(ws + L.plist); }
  void* face(int d) { return ws + L.face[d]; }
  double* vface(int d) { return (double*)(ws + L.vface[d]); }
  double* red() { return (double*)(ws + L.red); }
  double* geo() { return (double*)(ws + L.geo); }
  double* verts() { return (double*)(ws + L.verts); }
  double* vnext() { return (double*)(ws + L.vnext); }
  double* vol() { return (double*)(ws + L.vol); }
  double* vacc() { return (double*)(ws + L.vacc); }
  bool mixed() const { return cfg.precision == HGKS_MIXED; }
};

namespace {

hgks_status check_hip(hgks_ctx c, hipError_t e, const char* what) {
  if (e == hipSuccess) return HGKS_OK;
  c->sticky = HGKS_EDEVICE;
  return fail(HGKS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

hgks_status launched(hgks_ctx c, const char* what) { return check_hip(c, hipGetLastError(), what); }

// Records the start or end event of one timed launch of a phase.
void prof_mark(hgks_ctx c, int phase, bool start) {
  if (!c->prof_on) return;
  int& k = c->prof_used[phase];
  if (start) {
    if (k >= hgks_ctx_s::kProfCap) return;
    hipEventRecord(c->prof_ev[phase][2 * k], c->stream);
    c->prof_open[phase] = true;
  } else if (c->prof_open[phase]) {
    hipEventRecord(c->prof_ev[phase][2 * k + 1], c->stream);
    c->prof_open[phase] = false;
    ++k;
  }
}

hgks_status usable(hgks_ctx c) {
  if (!c) return fail(HGKS_EINVAL, "null context");
  if (c->sticky != HGKS_OK) return fail(c->sticky, "context has a previous device error");
  return HGKS_OK;
}

template <typename T>
WenoParams<T> weno_params(const hgks_config& cfg, const double dx[3]) {
  WenoParams<T> P;
  // 24 sub-stencils (Sec. 2) or 8 (Remark 1)
  P.gamma0 = T(1.0 - (cfg.stencil ? 8.0 : 24.0) * cfg.weno_Gamma);
  P.Gamma = T(cfg.weno_Gamma);
  P.eps = T(cfg.weno_eps);
  const double h = std::cbrt(dx[0] * dx[1] * dx[2]);
  double s[3];
  for (int d = 0; d < 3; ++d) s[d] = (h / dx[d]) * (h / dx[d]);
  for (int d = 0; d < 3; ++d) {
    P.kl[d] = T(s[d]);
    P.kq[d] = T(s[d] / 3.0 + 4.0 * s[d] * s[d]);
  }
  const int pd[3] = {0, 1, 0}, pe[3] = {1, 2, 2};
  for (int k = 0; k < 3; ++k) P.km[k] = T(s[pd[k]] * s[pe[k]] + (s[pd[k]] + s[pe[k]]) / 12.0);
  return P;
}

template <typename T>
GasParams<T> gas_params(const hgks_config& cfg) {
  GasParams<T> g;
  const double K = (5.0 - 3.0 * cfg.gamma) / (cfg.gamma - 1.0);
  g.gm1 = T(cfg.gamma - 1.0);
  g.K = T(K);
  g.K3 = T(K + 3.0);
  g.inv_K3 = T(1.0 / (K + 3.0));
  g.two_gm1 = T(2.0 / (cfg.gamma - 1.0));
  g.K2 = T(K + 2.0);
  g.mu = T(cfg.mu);
  g.tau_eps = T(cfg.tau_eps);
  g.tau_C = T(cfg.tau_C);
  g.viscous = cfg.mu > 0.0;
  g.mu_exp = T(cfg.mu_exponent);
  g.mu_iT0 = T(1.0 / cfg.mu_T0);
  g.pr_fix = T(1.0 / cfg.prandtl - 1.0);
  g.gamma = cfg.gamma;
  return g;
}

// Coefficients the face flux reads: the cell quadratics, or in characteristic
// mode the six per-face arrays that follow them.
template <typename TC>
TC* face_coef(hgks_ctx c) {
  TC* coef = (TC*)c->coef();
  return c->cfg.characteristic ? coef + c->G.fs_stride : coef;
}

// Reconstruction (with the fallback mask) and face fluxes of the state qin.
template <typename TC>
hgks_status box_stage(hgks_ctx c, const double* qin, double dt) {
  const Dims& D = c->D;
  const double dx[3] = {1.0 / c->G.inv_dx[0], 1.0 / c->G.inv_dx[1], 1.0 / c->G.inv_dx[2]};
  const WenoParams<TC> P = weno_params<TC>(c->cfg, dx);
  const GasParams<TC> gp = gas_params<TC>(c->cfg);
  const TC margin = sizeof(TC) == 8 ? TC(1e-10) : TC(1e-5);
  TC* coef = (TC*)c->coef();
  {
    const unsigned nb = blocks_for(D.NR);
    prof_mark(c, HGKS_PHASE_RECON, true);
    if (c->cfg.stencil)
      hipLaunchKernelGGL((k_recon_box<TC, true>), dim3(pad8(nb)), dim3(kBlock), 0, c->stream, qin, coef, c->mask(),
                         c->G, P, margin, TC(c->cfg.gamma - 1.0), D.NR, nb);
    else if (c->cfg.characteristic)  // the fallback mask only
      hipLaunchKernelGGL((k_recon_box<TC, false, false>), dim3(pad8(nb)), dim3(kBlock), 0, c->stream, qin, coef,
                         c->mask(), c->G, P, margin, TC(c->cfg.gamma - 1.0), D.NR, nb);
    else
      hipLaunchKernelGGL((k_recon_box<TC, false>), dim3(pad8(nb)), dim3(kBlock), 0, c->stream, qin, coef, c->mask(),
                         c->G, P, margin, TC(c->cfg.gamma - 1.0), D.NR, nb);
    prof_mark(c, HGKS_PHASE_RECON, false);
    if (hgks_status s = launched(c, "recon")) return s;
    prof_mark(c, HGKS_PHASE_FALLBACK, true);
    // flagged cells to a list, then one 32-lane group per listed cell on a
    // fixed grid of 8 workgroups per compute unit
    uint32_t* counter = c->plist() + D.NR;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c->stream, counter);
    hipLaunchKernelGGL(k_posit_compact, dim3(nb), dim3(kBlock), 0, c->stream, c->mask(), D.NR, c->plist(), counter);
    const unsigned pg = 2048;
    if (c->cfg.stencil)
      hipLaunchKernelGGL((k_posit_group_box<TC, true>), dim3(pg), dim3(kBlock), 0, c->stream, qin, c->mask(), c->G,
                         TC(c->cfg.gamma - 1.0), c->plist(), counter);
    else
      hipLaunchKernelGGL((k_posit_group_box<TC, false>), dim3(pg), dim3(kBlock), 0, c->stream, qin, c->mask(), c->G,
                         TC(c->cfg.gamma - 1.0), c->plist(), counter);
    prof_mark(c, HGKS_PHASE_FALLBACK, false);
    if (hgks_status s = launched(c, "positivity")) return s;
    if (c->cfg.characteristic) {
      prof_mark(c, HGKS_PHASE_RECON, true);
      const unsigned ntx = (unsigned)((c->G.nr[0] + kCX - 1) / kCX), nty = (unsigned)((c->G.nr[1] + kCY - 1) / kCY);
      const unsigned ntiles = ntx * nty * (unsigned)((c->G.nr[2] + kCZ - 1) / kCZ);
      hipLaunchKernelGGL((k_char_recon_box<TC>), dim3(pad8(ntiles)), dim3(kBlock), 0, c->stream, qin,
                         face_coef<TC>(c), c->G, P, c->cfg.gamma, ntx, nty, ntiles);
      prof_mark(c, HGKS_PHASE_RECON, false);
      if (hgks_status s = launched(c, "characteristic recon")) return s;
    }
  }
  unsigned nb[3];
  flux_block_counts(c->G, nb);
  prof_mark(c, HGKS_PHASE_FLUX, true);
  const dim3 grid(pad8(nb[0] + nb[1] + nb[2]));
  const TC* fc = face_coef<TC>(c);
  TC* f[3] = {(TC*)c->face(0), (TC*)c->face(1), (TC*)c->face(2)};
  // compile-time variants: the extended viscous model and per-face arrays
  const bool ext = c->cfg.prandtl != 1.0 || c->cfg.mu_exponent != 0.0, fs = c->cfg.characteristic != 0;
#define HGKS_FLUX_LAUNCH(E, F)                                                                                   \
  hipLaunchKernelGGL((k_flux_box<TC, E, F>), grid, dim3(kBlock), 0, c->stream, fc, c->mask(), f[0], f[1], f[2], \
                     c->G, gp, TC(dt), TC(1.0 / dt), nb[0], nb[1], nb[2])
  if (ext && fs)
    HGKS_FLUX_LAUNCH(true, true);
  else if (ext)
    HGKS_FLUX_LAUNCH(true, false);
  else if (fs)
    HGKS_FLUX_LAUNCH(false, true);
  else
    HGKS_FLUX_LAUNCH(false, false);
#undef HGKS_FLUX_LAUNCH
  prof_mark(c, HGKS_PHASE_FLUX, false);
  return launched(c, "flux");
}

template <typename TF>
hgks_status box_update(hgks_ctx c, double dt, int mode) {
  prof_mark(c, HGKS_PHASE_UPDATE, true);
  hipLaunchKernelGGL((k_update_box<TF>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, c->q(), c->qs(),
                     c->acc(), (const TF*)c->face(0), (const TF*)c->face(1), (const TF*)c->face(2), c->G, dt, mode,
                     c->D.N);
  prof_mark(c, HGKS_PHASE_UPDATE, false);
  return launched(c, "update");
}

template <typename T>
hgks_status box_step(hgks_ctx c, double dt, int n_stages) {
  if (hgks_status s = box_stage<T>(c, c->q(), dt)) return s;
  if (n_stages == 1) return box_update<T>(c, dt, 0);
  if (hgks_status s = box_update<T>(c, dt, 1)) return s;
  if (hgks_status s = box_stage<T>(c, c->qs(), dt)) return s;
  return box_update<T>(c, dt, 2);
}

// ------------------------------------------------------------ hexahedral grids
HexGrid hex_grid(hgks_ctx c, double dt, double alpha, bool moving) {
  HexGrid H = c->H;
  H.x0 = c->verts();
  H.x1 = (moving && c->next_set) ? c->vnext() : nullptr;
  H.alpha = alpha;
  H.inv_dt = dt > 0.0 ? 1.0 / dt : 0.0;
  return H;
}

hgks_status hex_geometry(hgks_ctx c, const HexGrid& H) {
  hipLaunchKernelGGL(k_geometry_hex, dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, H, c->geo(), c->D.N);
  return launched(c, "geometry");
}

// Stage geometry, reconstruction (double; coefficients stored in TC), the
// fallback mask and the face fluxes of the state qin at t_n + alpha dt.
template <typename TC>
hgks_status hex_stage(hgks_ctx c, const double* qin, double dt, double alpha) {
  const HexGrid H = hex_grid(c, dt, alpha, true);
  const size_t N = c->D.N;
  if (hgks_status s = hex_geometry(c, H)) return s;
  const double dx[3] = {1.0, 1.0, 1.0};
  const WenoParams<double> P = weno_params<double>(c->cfg, dx);
  const GasParams<TC> gp = gas_params<TC>(c->cfg);
  prof_mark(c, HGKS_PHASE_RECON, true);
  const unsigned ntx = (unsigned)((c->D.n[0] + kTX - 1) / kTX), nty = (unsigned)((c->D.n[1] + kTY - 1) / kTY);
  const unsigned ntiles = ntx * nty * (unsigned)((c->D.n[2] + kTZ - 1) / kTZ);
  if (c->cfg.stencil)
    hipLaunchKernelGGL((k_recon_hex<TC, true>), dim3(pad8(ntiles)), dim3(kBlock), 0, c->stream, H, c->geo(), qin,
                       (TC*)c->coef(), c->mask(), P, c->cfg.gamma - 1.0, N, ntx, nty, ntiles);
  else
    hipLaunchKernelGGL((k_recon_hex<TC>), dim3(pad8(ntiles)), dim3(kBlock), 0, c->stream, H, c->geo(), qin,
                       (TC*)c->coef(), c->mask(), P, c->cfg.gamma - 1.0, N, ntx, nty, ntiles);
  prof_mark(c, HGKS_PHASE_RECON, false);
  if (hgks_status s = launched(c, "recon")) return s;
  prof_mark(c, HGKS_PHASE_FALLBACK, true);
  if (c->cfg.stencil)
    hipLaunchKernelGGL((k_posit_exact_hex<true>), dim3(blocks_for(N)), dim3(kBlock), 0, c->stream, H, c->geo(), qin,
                       c->mask(), c->cfg.gamma - 1.0, N);
  else
    hipLaunchKernelGGL((k_posit_exact_hex<false>), dim3(blocks_for(N)), dim3(kBlock), 0, c->stream, H, c->geo(), qin,
                       c->mask(), c->cfg.gamma - 1.0, N);
  prof_mark(c, HGKS_PHASE_FALLBACK, false);
  if (hgks_status s = launched(c, "positivity")) return s;
  const bool fs = c->cfg.characteristic != 0;
  if (fs) {
    // six per-face reconstructions in characteristic variables; the
    // component-wise one above supplies the fallback mask
    prof_mark(c, HGKS_PHASE_RECON, true);
    hipLaunchKernelGGL((k_char_recon_hex<TC>), dim3(pad8(ntiles)), dim3(kBlock), 0, c->stream, H, c->geo(), qin,
                       (TC*)c->coef() + c->G.fs_stride, c->G.fs_stride, P, c->cfg.gamma, N, ntx, nty, ntiles);
    prof_mark(c, HGKS_PHASE_RECON, false);
    if (hgks_status s = launched(c, "characteristic recon")) return s;
  }
  const unsigned nb = blocks_for(4 * N);
  prof_mark(c, HGKS_PHASE_FLUX, true);
  // the extended viscous model and the per-face arrays are compile-time
  // variants
  const bool ext = c->cfg.prandtl != 1.0 || c->cfg.mu_exponent != 0.0;
  const TC* fc = (const TC*)c->coef() + (fs ? c->G.fs_stride : 0);
#define HGKS_HEX_FLUX(E, F)                                                                                      \
  hipLaunchKernelGGL((k_flux_hex<TC, E, F>), dim3(pad8(3 * nb)), dim3(kBlock), 0, c->stream, H, fc, c->geo(),    \
                     c->mask(), (TC*)c->face(0), (TC*)c->face(1), (TC*)c->face(2), c->vface(0), c->vface(1),     \
                     c->vface(2), gp, TC(dt), TC(1.0 / dt), N, nb)
  if (ext && fs)
    HGKS_HEX_FLUX(true, true);
  else if (ext)
    HGKS_HEX_FLUX(true, false);
  else if (fs)
    HGKS_HEX_FLUX(false, true);
  else
    HGKS_HEX_FLUX(false, false);
#undef HGKS_HEX_FLUX
  prof_mark(c, HGKS_PHASE_FLUX, false);
  return launched(c, "flux");
}

template <typename TF>
hgks_status hex_update(hgks_ctx c, double dt, int mode) {
  const HexGrid H = hex_grid(c, dt, 0.0, true);
  prof_mark(c, HGKS_PHASE_UPDATE, true);
  hipLaunchKernelGGL((k_update_hex<TF>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, H, c->q(), c->qs(),
                     c->acc(), c->vacc(), c->geo(), (const TF*)c->face(0), (const TF*)c->face(1),
                     (const TF*)c->face(2), c->vface(0), c->vface(1), c->vface(2), dt, mode, c->D.N);
  prof_mark(c, HGKS_PHASE_UPDATE, false);
  return launched(c, "update");
}

template <typename T>
hgks_status hex_step(hgks_ctx c, double dt, int n_stages) {
  if (hgks_status s = hex_stage<T>(c, c->q(), dt, 0.0)) return s;
  if (n_stages == 1) {
    if (hgks_status s = hex_update<T>(c, dt, 0)) return s;
  } else {
    if (hgks_status s = hex_update<T>(c, dt, 1)) return s;
    if (hgks_status s = hex_stage<T>(c, c->qs(), dt, 0.5)) return s;
    if (hgks_status s = hex_update<T>(c, dt, 2)) return s;
  }
  if (c->next_set) {
    // The vertices at t_{n+1} become the current ones.
    const size_t t = c->L.verts;
    c->L.verts = c->L.vnext;
    c->L.vnext = t;
    c->next_set = false;
  }
  return HGKS_OK;
}

hgks_status hex_dt(hgks_ctx c, double* part, unsigned nb) {
  const HexGrid H = hex_grid(c, 0.0, 0.0, false);
  hipLaunchKernelGGL(k_dt_hex, dim3(nb), dim3(kBlock), 0, c->stream, H, c->q(), c->cfg.gamma, part, c->D.N);
  return launched(c, "dt");
}

hgks_status hex_totals(hgks_ctx c, double* part, unsigned nb) {
  const HexGrid H = hex_grid(c, 0.0, 0.0, false);
  if (hgks_status s = hex_geometry(c, H)) return s;
  hipLaunchKernelGGL(k_totals_hex, dim3(nb), dim3(kBlock), 0, c->stream, c->q(), c->geo(), part, c->D.N, (int)nb);
  return launched(c, "totals");
}

hgks_status hex_debug_gp(hgks_ctx c, double dt, double* out) {
  hgks_status s = c->mixed() ? hex_stage<float>(c, c->q(), dt, 0.0) : hex_stage<double>(c, c->q(), dt, 0.0);
  if (s) return s;
  const HexGrid H = hex_grid(c, dt, 0.0, true);
  const size_t fs = c->cfg.characteristic ? c->G.fs_stride : 0;
  if (c->mixed())
    hipLaunchKernelGGL((k_debug_gp_hex<float>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, H,
                       (const float*)c->coef() + fs, c->geo(), c->mask(), c->D.N, c->cfg.gamma, fs, out);
  else
    hipLaunchKernelGGL((k_debug_gp_hex<double>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, H,
                       (const double*)c->coef() + fs, c->geo(), c->mask(), c->D.N, c->cfg.gamma, fs, out);
  return launched(c, "debug gp");
}

hgks_status hex_debug_face(hgks_ctx c, double dt, double* out) {
  hgks_status s = c->mixed() ? hex_stage<float>(c, c->q(), dt, 0.0) : hex_stage<double>(c, c->q(), dt, 0.0);
  if (s) return s;
  for (int d = 0; d < 3; ++d) {
    if (c->mixed())
      hipLaunchKernelGGL((k_debug_face_hex<float>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                         (const float*)c->face(d), d, c->D.N, out);
    else
      hipLaunchKernelGGL((k_debug_face_hex<double>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                         (const double*)c->face(d), d, c->D.N, out);
  }
  return launched(c, "debug face");
}

// Context fields from a valid configuration and a workspace base (no
// device work, no device allocation).
void init_ctx(hgks_ctx c, const hgks_config* cfg, char* ws) {
  c->cfg = *cfg;
  c->stream = (hipStream_t)cfg->stream;
  c->D = make_dims(cfg);
  c->L = make_layout(cfg, c->D);
  c->ws = ws;
  std::memset(&c->G, 0, sizeof c->G);
  for (int d = 0; d < 3; ++d) {
    c->G.n[d] = c->D.n[d];
    c->G.g[d] = c->D.g[d];
    c->G.nr[d] = c->D.nr[d];
    c->G.per[d] = c->D.per[d];
    c->G.sym[d][0] = c->D.sym[d][0];
    c->G.sym[d][1] = c->D.sym[d][1];
    for (int e = 0; e < 3; ++e) c->G.nf[d][e] = c->D.nf[d][e];
  }
  set_index_split(c->G);
  if (cfg->characteristic) c->G.fs_stride = coef_elems(c->D.NR, c->mixed() ? sizeof(float) : sizeof(double));
  std::memset(&c->H, 0, sizeof c->H);
}

// Uniform box geometry; all three axes are checked before anything is set,
// so a refused call leaves the grid as it was.
hgks_status set_box(hgks_ctx c, const double origin[3], const double length[3]) {
  if (!origin || !length) return fail(HGKS_EINVAL, "null origin or length");
  for (int d = 0; d < 3; ++d)
    if (!(length[d] > 0.0) || !std::isfinite(length[d]) || !std::isfinite(origin[d]))
      return fail(HGKS_EINVAL, "bad box");
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    const double h = length[d] / c->D.n[d];
    c->G.inv_dx[d] = 1.0 / h;
    vol *= h;
  }
  for (int d = 0; d < 3; ++d) c->G.wface[d] = 0.25 * vol * c->G.inv_dx[d];
  c->G.vol = vol;
  c->grid_set = true;
  return HGKS_OK;
}

hgks_status sync_copy(hgks_ctx c, void* dst, const void* src, size_t bytes) {
  if (hgks_status s = check_hip(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream), "copy"))
    return s;
  return check_hip(c, hipStreamSynchronize(c->stream), "synchronise");
}

}  // namespace

extern "C" {

hgks_status hgks_default_config(hgks_config* cfg, int32_t nx, int32_t ny, int32_t nz) {
  if (!cfg) return fail(HGKS_EINVAL, "null config");
  std::memset(cfg, 0, sizeof *cfg);
  cfg->nx = nx;
  cfg->ny = ny;
  cfg->nz = nz;
  cfg->gamma = 1.4;
  cfg->mu = 0.0;
  cfg->weno_Gamma = 0.0025;
  cfg->weno_eps = 1e-8;
  cfg->tau_eps = 0.01;
  cfg->tau_C = 1.0;
  cfg->precision = HGKS_FP64;
  for (int d = 0; d < 3; ++d) cfg->bc_hi[d] = HGKS_BC_SAME;
  cfg->mu_T0 = 1.0;
  cfg->mu_exponent = 0.0;
  cfg->prandtl = 1.0;
  return HGKS_OK;
}

hgks_status hgks_workspace_size(const hgks_config* cfg, size_t* bytes) {
  if (!valid_config(cfg) || !bytes) return fail(HGKS_EINVAL, "invalid configuration");
  const Dims D = make_dims(cfg);
  *bytes = make_layout(cfg, D).total;
  return HGKS_OK;
}

hgks_status hgks_create(const hgks_config* cfg, void* workspace_dev, size_t bytes, hgks_ctx* out) {
  if (!out) return fail(HGKS_EINVAL, "null output");
  *out = nullptr;
  if (!valid_config(cfg)) return fail(HGKS_EINVAL, "invalid configuration");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255u)) return fail(HGKS_EINVAL, "workspace must be 256-byte aligned");
  hgks_ctx c = new (std::nothrow) hgks_ctx_s;
  if (!c) return fail(HGKS_ENOMEM, "host allocation failed");
  init_ctx(c, cfg, (char*)workspace_dev);
  if (bytes < c->L.total) {
    const size_t need = c->L.total;
    delete c;
    return fail(HGKS_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
  }
  *out = c;
  return HGKS_OK;
}

hgks_status hgks_destroy(hgks_ctx ctx) {
  if (ctx)
    for (int p = 0; p < HGKS_NPHASES; ++p)
      for (auto& e : ctx->prof_ev[p]) hipEventDestroy(e);
  delete ctx;
  return HGKS_OK;
}

hgks_status hgks_set_uniform_grid(hgks_ctx c, const double origin[3], const double length[3]) {
  if (hgks_status s = usable(c)) return s;
  if (c->cfg.moving) return fail(HGKS_EINVAL, "context expects vertices (moving = 1)");
  return set_box(c, origin, length);
}

hgks_status hgks_set_vertices(hgks_ctx c, const double* xyz_dev, const double period[3]) {
  if (hgks_status s = usable(c)) return s;
  if (!c->cfg.moving) return fail(HGKS_EINVAL, "context expects a uniform grid (moving = 0)");
  if (!xyz_dev || !period) return fail(HGKS_EINVAL, "null vertices or period");
  for (int d = 0; d < 3; ++d)
    if (!(period[d] > 0.0)) return fail(HGKS_EINVAL, "bad period");
  if (hgks_status s = check_hip(c, hipMemcpyAsync(c->verts(), xyz_dev, 3 * c->D.N * sizeof(double),
                                                  hipMemcpyDeviceToDevice, c->stream),
                                "copy vertices"))
    return s;
  for (int d = 0; d < 3; ++d) c->period[d] = period[d];
  hex_setup(c->H, c->D.n, period);
  c->H.box.fs_stride = c->G.fs_stride;  // per-face arrays (characteristic variables)
  c->grid_set = true;
  c->next_set = false;
  return HGKS_OK;
}

hgks_status hgks_set_next_vertices(hgks_ctx c, const double* xyz_dev) {
  if (hgks_status s = usable(c)) return s;
  if (!c->cfg.moving || !c->grid_set) return fail(HGKS_ESTATE, "set_vertices first");
  if (!xyz_dev) return fail(HGKS_EINVAL, "null vertices");
  if (hgks_status s = check_hip(c, hipMemcpyAsync(c->vnext(), xyz_dev, 3 * c->D.N * sizeof(double),
                                                  hipMemcpyDeviceToDevice, c->stream),
                                "copy next vertices"))
    return s;
  c->next_set = true;
  return HGKS_OK;
}

hgks_status hgks_set_state(hgks_ctx c, const double* q_dev) {
  if (hgks_status s = usable(c)) return s;
  if (!q_dev) return fail(HGKS_EINVAL, "null state");
  if (hgks_status s = check_hip(c, hipMemcpyAsync(c->q(), q_dev, 5 * c->D.N * sizeof(double),
                                                  hipMemcpyDeviceToDevice, c->stream),
                                "copy state"))
    return s;
  c->state_set = true;
  return HGKS_OK;
}

hgks_status hgks_get_state(hgks_ctx c, double* q_dev_out) {
  if (hgks_status s = usable(c)) return s;
  if (!c->state_set) return fail(HGKS_ESTATE, "no state");
  if (!q_dev_out) return fail(HGKS_EINVAL, "null output");
  return check_hip(c, hipMemcpyAsync(q_dev_out, c->q(), 5 * c->D.N * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream),
                   "copy state out");
}

static hgks_status ready(hgks_ctx c) {
  if (hgks_status s = usable(c)) return s;
  if (!c->grid_set) return fail(HGKS_ESTATE, "grid not set");
  if (!c->state_set) return fail(HGKS_ESTATE, "state not set");
  return HGKS_OK;
}

hgks_status hgks_step(hgks_ctx c, double dt, int32_t n_stages) {
  if (hgks_status s = ready(c)) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HGKS_EINVAL, "dt must be positive");
  if (n_stages != 1 && n_stages != 2) return fail(HGKS_EINVAL, "n_stages must be 1 or 2");
  hgks_status s;
  if (c->cfg.moving)
    s = c->mixed() ? hex_step<float>(c, dt, n_stages) : hex_step<double>(c, dt, n_stages);
  else
    s = c->mixed() ? box_step<float>(c, dt, n_stages) : box_step<double>(c, dt, n_stages);
  return s;
}

hgks_status hgks_step_checked(hgks_ctx c, double dt, int32_t n_stages, int32_t max_halvings, double* dt_taken) {
  if (hgks_status s = ready(c)) return s;
  if (c->cfg.moving) return fail(HGKS_EUNSUPPORTED, "step_checked needs a static grid");
  if (!dt_taken || max_halvings < 0 || max_halvings > 60) return fail(HGKS_EINVAL, "bad max_halvings or output");
  *dt_taken = 0.0;
  const size_t bytes = 5 * c->D.N * sizeof(double);
  if (hgks_status s = check_hip(c, hipMemcpyAsync(c->back(), c->q(), bytes, hipMemcpyDeviceToDevice, c->stream),
                                "save state"))
    return s;
  for (int k = 0;; ++k) {
    if (hgks_status s = hgks_step(c, dt, n_stages)) return s;
    int64_t bad = 0, fb = 0;
    if (hgks_status s = hgks_check(c, &bad, &fb)) return s;
    if (bad == 0) {
      *dt_taken = dt;
      return HGKS_OK;
    }
    if (hgks_status s = check_hip(c, hipMemcpyAsync(c->q(), c->back(), bytes, hipMemcpyDeviceToDevice, c->stream),
                                  "restore state"))
      return s;
    if (k == max_halvings) {
      if (hgks_status s = check_hip(c, hipStreamSynchronize(c->stream), "restore state")) return s;
      return fail(HGKS_ENONPHYS, "non-physical state after %d halvings of the step", k);
    }
    dt *= 0.5;
  }
}

hgks_status hgks_max_dt(hgks_ctx c, double cfl, double* dt_host) {
  if (hgks_status s = ready(c)) return s;
  if (!(cfl > 0.0) || !std::isfinite(cfl) || !dt_host) return fail(HGKS_EINVAL, "bad cfl or output");
  const unsigned nb = blocks_for(c->D.N);
  double* part = c->red();
  prof_mark(c, HGKS_PHASE_REDUCE, true);
  if (c->cfg.moving) {
    if (hgks_status s = hex_dt(c, part, nb)) return s;
  } else {
    hipLaunchKernelGGL(k_dt_box, dim3(nb), dim3(kBlock), 0, c->stream, c->q(), c->G, c->cfg.gamma, part, c->D.N);
  }
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, c->stream, part, (int)nb, part + c->D.nred - 8);
  prof_mark(c, HGKS_PHASE_REDUCE, false);
  if (hgks_status s = launched(c, "max_dt")) return s;
  double m = 0.0;
  if (hgks_status s = sync_copy(c, &m, part + c->D.nred - 8, sizeof(double))) return s;
  if (!(m > 0.0)) return fail(HGKS_ENONPHYS, "non-physical state in max_dt");
  *dt_host = cfl * m;
  return HGKS_OK;
}

hgks_status hgks_totals(hgks_ctx c, double out[5]) {
  if (hgks_status s = ready(c)) return s;
  if (!out) return fail(HGKS_EINVAL, "null output");
  const unsigned nb = blocks_for(c->D.N);
  double* part = c->red();
  if (c->cfg.moving) {
    if (hgks_status s = hex_totals(c, part, nb)) return s;
  } else {
    hipLaunchKernelGGL(k_totals_box, dim3(nb), dim3(kBlock), 0, c->stream, c->q(), c->G.vol, part, c->D.N, (int)nb);
  }
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, c->stream, part, (int)nb, 5, part + c->D.nred - 8);
  if (hgks_status s = launched(c, "totals")) return s;
  return sync_copy(c, out, part + c->D.nred - 8, 5 * sizeof(double));
}

hgks_status hgks_check(hgks_ctx c, int64_t* nonphys, int64_t* fallback) {
  if (hgks_status s = ready(c)) return s;
  if (!nonphys || !fallback) return fail(HGKS_EINVAL, "null output");
  const unsigned nb = blocks_for(c->D.N);
  double* part = c->red();
  hipLaunchKernelGGL(k_check_box, dim3(nb), dim3(kBlock), 0, c->stream, c->q(), c->mask(), c->G, c->cfg.gamma, part,
                     c->D.N, (int)nb);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, c->stream, part, (int)nb, 2, part + c->D.nred - 8);
  if (hgks_status s = launched(c, "check")) return s;
  double r[2];
  if (hgks_status s = sync_copy(c, r, part + c->D.nred - 8, 2 * sizeof(double))) return s;
  *nonphys = (int64_t)r[0];
  *fallback = (int64_t)r[1];
  return HGKS_OK;
}

hgks_status hgks_kinetic_energy(hgks_ctx c, double rho0, double* ek_host) {
  if (hgks_status s = ready(c)) return s;
  if (!ek_host || !(rho0 > 0.0) || !std::isfinite(rho0)) return fail(HGKS_EINVAL, "bad rho0 or output");
  const unsigned nb = blocks_for(c->D.N);
  double* part = c->red();
  const double* geo = nullptr;
  if (c->cfg.moving) {
    // the geometry record of the current vertices
    if (hgks_status s = hex_geometry(c, hex_grid(c, 0.0, 0.0, false))) return s;
    geo = c->geo();
  }
  hipLaunchKernelGGL(k_kinetic, dim3(nb), dim3(kBlock), 0, c->stream, c->q(), geo, c->G.vol, part, c->D.N, (int)nb);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, c->stream, part, (int)nb, 2, part + c->D.nred - 8);
  if (hgks_status s = launched(c, "kinetic energy")) return s;
  double r[2];
  if (hgks_status s = sync_copy(c, r, part + c->D.nred - 8, 2 * sizeof(double))) return s;
  *ek_host = r[0] / (rho0 * r[1]);
  return HGKS_OK;
}

hgks_status hgks_debug_fallback_mask(hgks_ctx c, double dt, uint32_t* mask_dev_out) {
  if (hgks_status s = ready(c)) return s;
  if (!mask_dev_out || !(dt > 0.0) || !std::isfinite(dt)) return fail(HGKS_EINVAL, "bad arguments");
  hgks_status s;
  if (c->cfg.moving)
    s = c->mixed() ? hex_stage<float>(c, c->q(), dt, 0.0) : hex_stage<double>(c, c->q(), dt, 0.0);
  else
    s = c->mixed() ? box_stage<float>(c, c->q(), dt) : box_stage<double>(c, c->q(), dt);
  if (s) return s;
  hipLaunchKernelGGL(k_debug_mask, dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream, c->mask(), c->G,
                     c->cfg.moving ? 0 : 1, c->D.N, mask_dev_out);
  return launched(c, "debug mask");
}

hgks_status hgks_debug_gp_states(hgks_ctx c, double dt, double* out) {
  if (hgks_status s = ready(c)) return s;
  if (!out || !(dt > 0.0)) return fail(HGKS_EINVAL, "bad arguments");
  if (c->cfg.moving) return hex_debug_gp(c, dt, out);
  hgks_status s = c->mixed() ? box_stage<float>(c, c->q(), dt) : box_stage<double>(c, c->q(), dt);
  if (s) return s;
  if (c->mixed())
    hipLaunchKernelGGL((k_debug_gp_box<float>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                       (const float*)face_coef<float>(c), c->mask(), c->G, c->D.NR, c->D.N, c->cfg.gamma, out);
  else
    hipLaunchKernelGGL((k_debug_gp_box<double>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                       (const double*)face_coef<double>(c), c->mask(), c->G, c->D.NR, c->D.N, c->cfg.gamma, out);
  return launched(c, "debug gp");
}

hgks_status hgks_debug_face_flux(hgks_ctx c, double dt, double* out) {
  if (hgks_status s = ready(c)) return s;
  if (!out || !(dt > 0.0)) return fail(HGKS_EINVAL, "bad arguments");
  if (c->cfg.moving) return hex_debug_face(c, dt, out);
  hgks_status s = c->mixed() ? box_stage<float>(c, c->q(), dt) : box_stage<double>(c, c->q(), dt);
  if (s) return s;
  for (int d = 0; d < 3; ++d) {
    if (c->mixed())
      hipLaunchKernelGGL((k_debug_face_box<float>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                         (const float*)c->face(d), c->G, d, c->D.N, out);
    else
      hipLaunchKernelGGL((k_debug_face_box<double>), dim3(blocks_for(c->D.N)), dim3(kBlock), 0, c->stream,
                         (const double*)c->face(d), c->G, d, c->D.N, out);
  }
  return launched(c, "debug face");
}

hgks_status hgks_sync(hgks_ctx c) {
  if (hgks_status s = usable(c)) return s;
  return check_hip(c, hipStreamSynchronize(c->stream), "synchronise");
}

hgks_status hgks_profile_begin(hgks_ctx c) {
  if (hgks_status s = usable(c)) return s;
  if (c->prof_on) return fail(HGKS_ESTATE, "profiling already on");
  for (int p = 0; p < HGKS_NPHASES; ++p) {
    if (c->prof_ev[p].empty()) {
      c->prof_ev[p].resize(2 * hgks_ctx_s::kProfCap);
      for (auto& e : c->prof_ev[p])
        if (hgks_status s = check_hip(c, hipEventCreate(&e), "event create")) return s;
    }
    c->prof_used[p] = 0;
    c->prof_open[p] = false;
  }
  c->prof_on = true;
  return HGKS_OK;
}

hgks_status hgks_profile_end(hgks_ctx c, double ms[5], int64_t launches[5]) {
  if (hgks_status s = usable(c)) return s;
  if (!c->prof_on) return fail(HGKS_ESTATE, "profiling is off");
  if (!ms || !launches) return fail(HGKS_EINVAL, "null output");
  c->prof_on = false;
  if (hgks_status s = check_hip(c, hipStreamSynchronize(c->stream), "synchronise")) return s;
  for (int p = 0; p < HGKS_NPHASES; ++p) {
    double tot = 0.0;
    for (int k = 0; k < c->prof_used[p]; ++k) {
      float t = 0.f;
      if (hgks_status s = check_hip(c, hipEventElapsedTime(&t, c->prof_ev[p][2 * k], c->prof_ev[p][2 * k + 1]),
                                    "event time"))
        return s;
      tot += t;
    }
    ms[p] = tot;
    launches[p] = c->prof_used[p];
  }
  return HGKS_OK;
}

const char* hgks_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------------ allocation-free step
// hgks_step_noalloc keeps its whole workspace (intermediate state, stage
// accumulator, reconstruction coefficients, fallback masks and list, face
// sums, reduction scratch) in this file-scope device array; every device the
// library runs on holds its own copy until the process ends.  Host code uses
// the array only through the per-device address hipGetSymbolAddress gives.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of the current device's scratch array, looked up once per
// device (with that device current) on the first call there.
hgks_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(HGKS_EDEVICE, "no usable current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(HGKS_EDEVICE, "scratch address: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HGKS_OK;
}

}  // namespace

extern "C" {

size_t hgks_noalloc_capacity(void) { return kScratchBytes; }

hgks_status hgks_step_noalloc(const hgks_config* cfg, const double origin[3], const double length[3], double* q_dev,
                              double dt, int32_t n_stages) {
  if (!valid_config(cfg)) return fail(HGKS_EINVAL, "invalid configuration");
  if (cfg->moving) return fail(HGKS_EUNSUPPORTED, "the allocation-free step takes box grids (moving = 0)");
  if (!q_dev) return fail(HGKS_EINVAL, "null state");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HGKS_EINVAL, "dt must be positive");
  if (n_stages != 1 && n_stages != 2) return fail(HGKS_EINVAL, "n_stages must be 1 or 2");
  const size_t need = make_layout(cfg, make_dims(cfg)).total;
  if (need > kScratchBytes)
    return fail(HGKS_EINVAL, "grid needs %zu bytes of scratch; the allocation-free step holds at most %zu", need,
                kScratchBytes);
  void* base = nullptr;
  if (hgks_status s = scratch_address(&base)) return s;
  hgks_ctx_s ctx;
  hgks_ctx c = &ctx;
  init_ctx(c, cfg, (char*)base);
  if (hgks_status s = set_box(c, origin, length)) return s;
  const size_t bytes = 5 * c->D.N * sizeof(double);
  if (hgks_status s = check_hip(c, hipMemcpyAsync(c->q(), q_dev, bytes, hipMemcpyDeviceToDevice, c->stream),
                                "copy state in"))
    return s;
  c->state_set = true;
  if (hgks_status s = c->mixed() ? box_step<float>(c, dt, n_stages) : box_step<double>(c, dt, n_stages)) return s;
  return check_hip(c, hipMemcpyAsync(q_dev, c->q(), bytes, hipMemcpyDeviceToDevice, c->stream), "copy state out");
}

}  // extern "C"

// ================================================================ batches
struct hgks_batch_s {
  hgks_config base;
  std::vector<hgks_config> cfgs;
  int ng = 0;
  hipStream_t stream;
  char* ws = nullptr;
  size_t desc = 0, q = 0, qs = 0, acc = 0, coef = 0, mask = 0, face = 0, part = 0, dt = 0, tot = 0, status = 0,
         total = 0;
  size_t tc = 8;
  unsigned tiles_cell = 0, tiles_flux = 0;
  int ct[3] = {0, 0, 0};   // cell tile shape (0: 256 consecutive cells)
  int band = kFluxBand;    // rows per band of the flux block order
  bool ext = false;  // some grid uses the viscosity law or the Prandtl correction
  bool wide = false;  // every grid reconstructs with the stencils of Remark 1
  bool chr = false;   // every grid reconstructs in characteristic variables
  unsigned tiles_char = 0;  // tiles of the characteristic reconstruction
  std::vector<BatchGrid<double>> gd;  // host copies of the descriptors
  std::vector<BatchGrid<float>> gf;
  std::vector<bool> grid_set, state_set;
  int wg[HGKS_NPHASES] = {0, 0, 0, 0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hgks_status sticky = HGKS_OK;
  bool mixed() const { return base.precision == HGKS_MIXED; }
};

namespace {

hgks_status bcheck(hgks_batch b, hipError_t e, const char* what) {
  if (e == hipSuccess) return HGKS_OK;
  b->sticky = HGKS_EDEVICE;
  return fail(HGKS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

hgks_status busable(hgks_batch b) {
  if (!b) return fail(HGKS_EINVAL, "null batch");
  if (b->sticky != HGKS_OK) return fail(b->sticky, "batch has a previous device error");
  return HGKS_OK;
}

bool batch_compatible(const hgks_config& a, const hgks_config& c) {
  if (!valid_config(&c) || c.moving) return false;
  for (int d = 0; d < 3; ++d)
    if (c.bc[d] != HGKS_BC_PERIODIC) return false;
  return c.gamma == a.gamma && c.weno_Gamma == a.weno_Gamma && c.weno_eps == a.weno_eps &&
         c.tau_eps == a.tau_eps && c.tau_C == a.tau_C && c.precision == a.precision && c.stencil == a.stencil &&
         c.characteristic == a.characteristic;
}

// Offsets of every arena and the per-grid descriptors (without the grid
// spacing, set later).
// Cell tiles of a grid of extents n for tile shape ct (ct[0] = 0: 256
// consecutive cells); nct receives the tiles per axis of a box shape.
unsigned cell_tiles(const int n[3], const int ct[3], int nct[3]) {
  if (ct[0] == 0) {
    nct[0] = nct[1] = nct[2] = 0;
    return blocks_for((size_t)n[0] * n[1] * n[2]);
  }
  for (int d = 0; d < 3; ++d) nct[d] = (n[d] + ct[d] - 1) / ct[d];
  return (unsigned)nct[0] * nct[1] * nct[2];
}

// A valid cell tile shape: 0 x 0 x 0 (consecutive cells) or powers of two
// with tx ty tz = 256.
bool valid_tile(const int ct[3]) {
  if (ct[0] == 0 && ct[1] == 0 && ct[2] == 0) return true;
  for (int d = 0; d < 3; ++d)
    if (ct[d] < 1 || ct[d] > kBlock || (ct[d] & (ct[d] - 1))) return false;
  return ct[0] * ct[1] * ct[2] == kBlock;
}

// Largest cell-tile count of a grid over every valid shape (the size of the
// per-tile reduction scratch).
unsigned max_cell_tiles(const int n[3]) {
  int ct[3] = {0, 0, 0}, nct[3];
  unsigned m = cell_tiles(n, ct, nct);
  for (int a = 1; a <= kBlock; a *= 2)
    for (int c = 1; a * c <= kBlock; c *= 2) {
      const int sh[3] = {a, c, kBlock / (a * c)};
      m = std::max(m, cell_tiles(n, sh, nct));
    }
  return m;
}

// Cell and flux tiles of every grid for the batch's tile shape and flux
// band height (descriptors on the host; the caller uploads them).
template <typename TC>
void batch_tiles(std::vector<BatchGrid<TC>>& G, const int ct[3], int band, unsigned& tiles_cell,
                 unsigned& tiles_flux, unsigned& tiles_char) {
  unsigned tc = 0, tf = 0, th = 0;
  for (auto& g : G) {
    // tiles of the characteristic reconstruction (fixed shape)
    g.ncx = (unsigned)((g.G.n[0] + kCX - 1) / kCX);
    g.ncy = (unsigned)((g.G.n[1] + kCY - 1) / kCY);
    g.t_char = th;
    g.nt_char = g.ncx * g.ncy * (unsigned)((g.G.n[2] + kCZ - 1) / kCZ);
    th += g.nt_char;
    set_index_split(g.G, band);
    for (int d = 0; d < 3; ++d) g.ct[d] = ct[d];
    g.t_cell = tc;
    g.nt_cell = cell_tiles(g.G.n, ct, g.nct);
    tc += g.nt_cell;
    g.t_flux = tf;
    unsigned nb[3];
    flux_block_counts(g.G, nb);
    for (int d = 0; d < 3; ++d) {
      g.nt_flux[d] = nb[d];
      tf += nb[d];
    }
  }
  tiles_cell = tc;
  tiles_flux = tf;
  tiles_char = th;
}

template <typename TC>
size_t batch_layout(const hgks_config* cfgs, int n, hgks_batch b, std::vector<BatchGrid<TC>>& G) {
  G.assign(n, BatchGrid<TC>());
  size_t N = 0, F = 0, C = 0, tmax = 0;
  for (int i = 0; i < n; ++i) {
    const Dims D = make_dims(&cfgs[i]);
    BatchGrid<TC>& g = G[i];
    std::memset(&g, 0, sizeof g);
    for (int d = 0; d < 3; ++d) {
      g.G.n[d] = D.n[d];
      g.G.g[d] = 0;
      g.G.nr[d] = D.n[d];
      g.G.per[d] = 1;
      for (int e = 0; e < 3; ++e) g.G.nf[d][e] = D.nf[d][e];
    }
    g.N = D.N;
    g.q_off = 5 * N;
    g.coef_off = C;
    g.mask_off = N;
    for (int d = 0; d < 3; ++d) {
      g.NF[d] = D.NF[d];
      g.face_off[d] = F;
      F += 10 * D.NF[d];
    }
    tmax += max_cell_tiles(D.n);
    N += D.N;
    // characteristic variables: the component-wise array (fallback mask
    // polynomials are not stored, but the layout is kept) and six per-face
    // arrays after it
    g.G.fs_stride = cfgs[i].characteristic ? coef_elems(D.N, sizeof(TC)) : 0;
    C += coef_elems(D.N, sizeof(TC)) * (cfgs[i].characteristic ? 7 : 1);
    g.gp = gas_params<TC>(cfgs[i]);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  {
    const int lin[3] = {0, 0, 0};
    unsigned tc, tf, th;
    batch_tiles(G, b ? b->ct : lin, b ? b->band : kFluxBand, tc, tf, th);
    if (b) {
      b->tiles_cell = tc;
      b->tiles_flux = tf;
      b->tiles_char = th;
    }
  }
  const size_t desc = take(n * sizeof(BatchGrid<TC>));
  const size_t q = take(5 * N * 8), qs = take(5 * N * 8), acc = take(5 * N * 8);
  const size_t coef = take(C * sizeof(TC)), mask = take(N * 4), face = take(F * sizeof(TC));
  const size_t part = take(tmax * 8), dt = take(n * 8), tot = take(5 * n * 8), status = take(4);
  if (b) {
    b->desc = desc; b->q = q; b->qs = qs; b->acc = acc; b->coef = coef; b->mask = mask; b->face = face;
    b->part = part; b->dt = dt; b->tot = tot; b->status = status; b->total = off;
  }
  return off;
}

template <typename TC>
std::vector<BatchGrid<TC>>& batch_desc(hgks_batch b);
template <>
std::vector<BatchGrid<double>>& batch_desc<double>(hgks_batch b) { return b->gd; }
template <>
std::vector<BatchGrid<float>>& batch_desc<float>(hgks_batch b) { return b->gf; }

template <typename TC>
hgks_status batch_upload(hgks_batch b) {
  auto& G = batch_desc<TC>(b);
  if (hgks_status s = bcheck(b, hipMemcpyAsync(b->ws + b->desc, G.data(), G.size() * sizeof(BatchGrid<TC>),
                                               hipMemcpyHostToDevice, b->stream),
                             "upload descriptors"))
    return s;
  return bcheck(b, hipStreamSynchronize(b->stream), "upload descriptors");
}

unsigned batch_wg(hgks_batch b, int phase, unsigned tiles) {
  const int w = b->wg[phase];
  if (w <= 0) return pad8(tiles);
  return (unsigned)w;
}

// Persistent tile walk (a workgroup count was set) or one workgroup per tile.
bool batch_loop(hgks_batch b, int phase) { return b->wg[phase] > 0; }

// The same with a third template argument W (the stencil family).
#define HGKS_BATCH_LAUNCH_W(kernel, TC, W, loop, grid, ...)                                              \
  do {                                                                                                 \
    if (loop)                                                                                          \
      hipLaunchKernelGGL((kernel<TC, true, W>), dim3(grid), dim3(kBlock), 0, __VA_ARGS__);            \
    else                                                                                               \
      hipLaunchKernelGGL((kernel<TC, false, W>), dim3(grid), dim3(kBlock), 0, __VA_ARGS__);           \
  } while (0)

#define HGKS_BATCH_LAUNCH(kernel, TC, loop, grid, ...)                                                   \
  do {                                                                                                 \
    if (loop)                                                                                          \
      hipLaunchKernelGGL((kernel<TC, true>), dim3(grid), dim3(kBlock), 0, __VA_ARGS__);               \
    else                                                                                               \
      hipLaunchKernelGGL((kernel<TC, false>), dim3(grid), dim3(kBlock), 0, __VA_ARGS__);              \
  } while (0)

template <typename TC>
hgks_status batch_dt(hgks_batch b, double cfl, double* dt_dev) {
  const BatchGrid<TC>* D = (const BatchGrid<TC>*)(b->ws + b->desc);
  double* part = (double*)(b->ws + b->part);
  HGKS_BATCH_LAUNCH(k_batch_dt_part, TC, batch_loop(b, HGKS_PHASE_REDUCE),
                    batch_wg(b, HGKS_PHASE_REDUCE, b->tiles_cell), b->stream, D, b->ng, b->tiles_cell,
                    (const double*)(b->ws + b->q), b->base.gamma, part);
  hipLaunchKernelGGL((k_batch_dt_final<TC>), dim3(b->ng), dim3(kBlock), 0, b->stream, D, part, cfl, dt_dev,
                     (uint32_t*)(b->ws + b->status));
  return bcheck(b, hipGetLastError(), "batch dt");
}

template <typename TC>
hgks_status batch_stage(hgks_batch b, const double* qin, const double* dt_dev) {
  const BatchGrid<TC>* D = (const BatchGrid<TC>*)(b->ws + b->desc);
  TC* coef = (TC*)(b->ws + b->coef);
  uint32_t* mask = (uint32_t*)(b->ws + b->mask);
  const TC margin = sizeof(TC) == 8 ? TC(1e-10) : TC(1e-5);
  const TC gm1 = TC(b->base.gamma - 1.0);
  const bool rl = batch_loop(b, HGKS_PHASE_RECON), pl = batch_loop(b, HGKS_PHASE_FALLBACK);
  const unsigned rg = batch_wg(b, HGKS_PHASE_RECON, b->tiles_cell), pg = batch_wg(b, HGKS_PHASE_FALLBACK, b->tiles_cell);
  if (b->chr) {
    // the component-wise pass for the fallback mask only, then the six
    // per-face reconstructions in characteristic variables
    if (rl)
      hipLaunchKernelGGL((k_batch_recon<TC, true, false, false>), dim3(rg), dim3(kBlock), 0, b->stream, D, b->ng,
                         b->tiles_cell, qin, coef, mask, margin, gm1);
    else
      hipLaunchKernelGGL((k_batch_recon<TC, false, false, false>), dim3(rg), dim3(kBlock), 0, b->stream, D, b->ng,
                         b->tiles_cell, qin, coef, mask, margin, gm1);
    HGKS_BATCH_LAUNCH_W(k_batch_posit, TC, false, pl, pg, b->stream, D, b->ng, b->tiles_cell, qin, mask, gm1);
    hipLaunchKernelGGL((k_batch_char_recon<TC>), dim3(pad8(b->tiles_char)), dim3(kBlock), 0, b->stream, D, b->ng,
                       b->tiles_char, qin, coef, b->base.gamma);
  } else if (b->wide) {
    HGKS_BATCH_LAUNCH_W(k_batch_recon, TC, true, rl, rg, b->stream, D, b->ng, b->tiles_cell, qin, coef, mask, margin,
                        gm1);
    HGKS_BATCH_LAUNCH_W(k_batch_posit, TC, true, pl, pg, b->stream, D, b->ng, b->tiles_cell, qin, mask, gm1);
  } else {
    HGKS_BATCH_LAUNCH_W(k_batch_recon, TC, false, rl, rg, b->stream, D, b->ng, b->tiles_cell, qin, coef, mask, margin,
                        gm1);
    HGKS_BATCH_LAUNCH_W(k_batch_posit, TC, false, pl, pg, b->stream, D, b->ng, b->tiles_cell, qin, mask, gm1);
  }
  {
    const bool loop = batch_loop(b, HGKS_PHASE_FLUX);
    const dim3 grid(batch_wg(b, HGKS_PHASE_FLUX, b->tiles_flux));
    // characteristic variables: one workgroup per tile only (the per-face
    // instantiations are not built in the persistent form)
    auto flux = b->chr ? (b->ext ? k_batch_flux<TC, false, true, true> : k_batch_flux<TC, false, false, true>)
                : loop ? (b->ext ? k_batch_flux<TC, true, true> : k_batch_flux<TC, true, false>)
                       : (b->ext ? k_batch_flux<TC, false, true> : k_batch_flux<TC, false, false>);
    const dim3 fgrid = b->chr ? dim3(pad8(b->tiles_flux)) : grid;
    hipLaunchKernelGGL(flux, fgrid, dim3(kBlock), 0, b->stream, D, b->ng, b->tiles_flux, (const TC*)coef,
                       (const uint32_t*)mask, (TC*)(b->ws + b->face), dt_dev);
  }
  return bcheck(b, hipGetLastError(), "batch stage");
}

template <typename TC>
hgks_status batch_update(hgks_batch b, const double* dt_dev, int mode) {
  const BatchGrid<TC>* D = (const BatchGrid<TC>*)(b->ws + b->desc);
  HGKS_BATCH_LAUNCH(k_batch_update, TC, batch_loop(b, HGKS_PHASE_UPDATE),
                    batch_wg(b, HGKS_PHASE_UPDATE, b->tiles_cell), b->stream, D, b->ng, b->tiles_cell,
                    (double*)(b->ws + b->q), (double*)(b->ws + b->qs), (double*)(b->ws + b->acc),
                    (const TC*)(b->ws + b->face), dt_dev, mode);
  return bcheck(b, hipGetLastError(), "batch update");
}

template <typename TC>
hgks_status batch_step(hgks_batch b, const double* dt_dev, int n_stages) {
  if (hgks_status s = batch_stage<TC>(b, (const double*)(b->ws + b->q), dt_dev)) return s;
  if (n_stages == 1) return batch_update<TC>(b, dt_dev, 0);
  if (hgks_status s = batch_update<TC>(b, dt_dev, 1)) return s;
  if (hgks_status s = batch_stage<TC>(b, (const double*)(b->ws + b->qs), dt_dev)) return s;
  return batch_update<TC>(b, dt_dev, 2);
}

hgks_status batch_ready(hgks_batch b) {
  if (hgks_status s = busable(b)) return s;
  for (int i = 0; i < b->ng; ++i) {
    if (!b->grid_set[i]) return fail(HGKS_ESTATE, "grid %d has no box", i);
    if (!b->state_set[i]) return fail(HGKS_ESTATE, "grid %d has no state", i);
  }
  return HGKS_OK;
}

// Reads and clears the device status word the time-step reduction sets for
// a grid with a non-physical cell; synchronises the stream.
hgks_status batch_status(hgks_batch b) {
  uint32_t* st = (uint32_t*)(b->ws + b->status);
  uint32_t h = 0;
  if (hgks_status s = bcheck(b, hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, b->stream), "copy status"))
    return s;
  if (hgks_status s = bcheck(b, hipStreamSynchronize(b->stream), "synchronise")) return s;
  if (h == 0) return HGKS_OK;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, b->stream, st);
  if (hgks_status s = bcheck(b, hipGetLastError(), "clear status")) return s;
  if (hgks_status s = bcheck(b, hipStreamSynchronize(b->stream), "synchronise")) return s;
  return fail(HGKS_ENONPHYS, "a time-step reduction found a non-physical cell (its grid got dt = 0 and was not "
                             "advanced)");
}

}  // namespace

extern "C" {

hgks_status hgks_batch_workspace_size(const hgks_config* cfgs, int32_t n, size_t* bytes) {
  if (!cfgs || n < 1 || !bytes) return fail(HGKS_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i)
    if (!batch_compatible(cfgs[0], cfgs[i])) return fail(HGKS_EINVAL, "grid %d: incompatible configuration", i);
  if (cfgs[0].precision == HGKS_MIXED) {
    std::vector<BatchGrid<float>> G;
    *bytes = batch_layout<float>(cfgs, n, nullptr, G);
  } else {
    std::vector<BatchGrid<double>> G;
    *bytes = batch_layout<double>(cfgs, n, nullptr, G);
  }
  return HGKS_OK;
}

hgks_status hgks_batch_create(const hgks_config* cfgs, int32_t n, void* ws, size_t bytes, hgks_batch* out) {
  if (!out) return fail(HGKS_EINVAL, "null output");
  *out = nullptr;
  size_t need = 0;
  if (hgks_status s = hgks_batch_workspace_size(cfgs, n, &need)) return s;
  if (!ws || ((uintptr_t)ws & 255u)) return fail(HGKS_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need) return fail(HGKS_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
  hgks_batch b = new (std::nothrow) hgks_batch_s;
  if (!b) return fail(HGKS_ENOMEM, "host allocation failed");
  b->base = cfgs[0];
  b->cfgs.assign(cfgs, cfgs + n);
  b->ng = n;
  b->stream = (hipStream_t)cfgs[0].stream;
  b->ws = (char*)ws;
  b->tc = b->mixed() ? 4 : 8;
  if (b->mixed())
    batch_layout<float>(cfgs, n, b, b->gf);
  else
    batch_layout<double>(cfgs, n, b, b->gd);
  for (int i = 0; i < n; ++i) b->ext = b->ext || cfgs[i].prandtl != 1.0 || cfgs[i].mu_exponent != 0.0;
  b->wide = cfgs[0].stencil == 1;
  b->chr = cfgs[0].characteristic == 1;
  b->grid_set.assign(n, false);
  b->state_set.assign(n, false);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, b->stream, (uint32_t*)(b->ws + b->status));
  if (hipGetLastError() != hipSuccess) {
    delete b;
    return fail(HGKS_EDEVICE, "clear status");
  }
  *out = b;
  return HGKS_OK;
}

hgks_status hgks_batch_destroy(hgks_batch b) {
  if (b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
  }
  delete b;
  return HGKS_OK;
}

hgks_status hgks_batch_set_uniform_grid(hgks_batch b, int32_t i, const double origin[3], const double length[3]) {
  if (hgks_status s = busable(b)) return s;
  if (i < 0 || i >= b->ng || !origin || !length) return fail(HGKS_EINVAL, "bad grid index or box");
  const int n[3] = {b->cfgs[i].nx, b->cfgs[i].ny, b->cfgs[i].nz};
  double dx[3], vol = 1.0, inv[3];
  for (int d = 0; d < 3; ++d) {
    if (!(length[d] > 0.0) || !std::isfinite(length[d])) return fail(HGKS_EINVAL, "bad box");
    dx[d] = length[d] / n[d];
    inv[d] = 1.0 / dx[d];
    vol *= dx[d];
  }
  auto set = [&](auto& G) {
    using TC = std::decay_t<decltype(G[0].P.eps)>;
    for (int d = 0; d < 3; ++d) {
      G[i].G.inv_dx[d] = inv[d];
      G[i].G.wface[d] = 0.25 * vol * inv[d];
    }
    G[i].G.vol = vol;
    G[i].P = weno_params<TC>(b->cfgs[i], dx);
  };
  hgks_status s;
  if (b->mixed()) {
    set(b->gf);
    s = batch_upload<float>(b);
  } else {
    set(b->gd);
    s = batch_upload<double>(b);
  }
  if (s) return s;
  b->grid_set[i] = true;
  return HGKS_OK;
}

static size_t batch_qoff(hgks_batch b, int i) { return b->mixed() ? b->gf[i].q_off : b->gd[i].q_off; }
static size_t batch_N(hgks_batch b, int i) { return b->mixed() ? b->gf[i].N : b->gd[i].N; }

hgks_status hgks_batch_set_state(hgks_batch b, int32_t i, const double* q_dev) {
  if (hgks_status s = busable(b)) return s;
  if (i < 0 || i >= b->ng || !q_dev) return fail(HGKS_EINVAL, "bad grid index or state");
  double* dst = (double*)(b->ws + b->q) + batch_qoff(b, i);
  if (hgks_status s = bcheck(b, hipMemcpyAsync(dst, q_dev, 5 * batch_N(b, i) * 8, hipMemcpyDeviceToDevice, b->stream),
                             "copy state"))
    return s;
  b->state_set[i] = true;
  return HGKS_OK;
}

hgks_status hgks_batch_get_state(hgks_batch b, int32_t i, double* q_dev_out) {
  if (hgks_status s = busable(b)) return s;
  if (i < 0 || i >= b->ng || !q_dev_out) return fail(HGKS_EINVAL, "bad grid index or output");
  if (!b->state_set[i]) return fail(HGKS_ESTATE, "grid %d has no state", i);
  const double* src = (const double*)(b->ws + b->q) + batch_qoff(b, i);
  return bcheck(b, hipMemcpyAsync(q_dev_out, src, 5 * batch_N(b, i) * 8, hipMemcpyDeviceToDevice, b->stream),
                "copy state out");
}

hgks_status hgks_batch_max_dt(hgks_batch b, double cfl, double* dt_dev) {
  if (hgks_status s = batch_ready(b)) return s;
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(HGKS_EINVAL, "bad cfl");
  double* out = dt_dev ? dt_dev : (double*)(b->ws + b->dt);
  return b->mixed() ? batch_dt<float>(b, cfl, out) : batch_dt<double>(b, cfl, out);
}

hgks_status hgks_batch_step(hgks_batch b, const double* dt_dev, int32_t n_stages) {
  if (hgks_status s = batch_ready(b)) return s;
  if (!dt_dev || (n_stages != 1 && n_stages != 2)) return fail(HGKS_EINVAL, "bad dt array or n_stages");
  return b->mixed() ? batch_step<float>(b, dt_dev, n_stages) : batch_step<double>(b, dt_dev, n_stages);
}

hgks_status hgks_batch_set_launch(hgks_batch b, int32_t phase, int32_t workgroups) {
  if (hgks_status s = busable(b)) return s;
  if (phase < 0 || phase >= HGKS_NPHASES) return fail(HGKS_EINVAL, "bad phase");
  if (workgroups != 0 && (workgroups < 8 || workgroups > 65536 || (workgroups & 7)))
    return fail(HGKS_EINVAL, "workgroups must be 0 or a multiple of 8 in [8, 65536]");
  b->wg[phase] = workgroups;
  return HGKS_OK;
}

hgks_status hgks_batch_set_tiles(hgks_batch b, int32_t tile_x, int32_t tile_y, int32_t tile_z, int32_t flux_band) {
  if (hgks_status s = busable(b)) return s;
  const int ct[3] = {tile_x, tile_y, tile_z};
  if (!valid_tile(ct)) return fail(HGKS_EINVAL, "cell tile must be 0 x 0 x 0 or powers of two with product 256");
  if (flux_band < 1 || flux_band > 256) return fail(HGKS_EINVAL, "flux band must be in [1, 256]");
  for (int d = 0; d < 3; ++d) b->ct[d] = ct[d];
  b->band = flux_band;
  hgks_status s;
  if (b->mixed()) {
    batch_tiles(b->gf, b->ct, b->band, b->tiles_cell, b->tiles_flux, b->tiles_char);
    s = batch_upload<float>(b);
  } else {
    batch_tiles(b->gd, b->ct, b->band, b->tiles_cell, b->tiles_flux, b->tiles_char);
    s = batch_upload<double>(b);
  }
  if (s) return s;
  // a captured graph holds the old launch shapes
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  return HGKS_OK;
}

hgks_status hgks_batch_capture(hgks_batch b, double cfl, int32_t n_steps, int32_t n_stages) {
  if (hgks_status s = batch_ready(b)) return s;
  if (!(cfl > 0.0) || !std::isfinite(cfl) || n_steps < 1 || (n_stages != 1 && n_stages != 2))
    return fail(HGKS_EINVAL, "bad arguments");
  if (b->stream == nullptr) return fail(HGKS_EINVAL, "capture needs a non-default stream");
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  if (hgks_status s = bcheck(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture"))
    return s;
  double* dt = (double*)(b->ws + b->dt);
  hgks_status st = HGKS_OK;
  for (int k = 0; k < n_steps && st == HGKS_OK; ++k) {
    st = b->mixed() ? batch_dt<float>(b, cfl, dt) : batch_dt<double>(b, cfl, dt);
    if (st == HGKS_OK) st = b->mixed() ? batch_step<float>(b, dt, n_stages) : batch_step<double>(b, dt, n_stages);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != HGKS_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (hgks_status s = bcheck(b, e, "end capture")) return s;
  b->graph = g;
  return bcheck(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "instantiate graph");
}

hgks_status hgks_batch_replay(hgks_batch b) {
  if (hgks_status s = batch_ready(b)) return s;
  if (!b->exec) return fail(HGKS_ESTATE, "no captured graph");
  return bcheck(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
}

hgks_status hgks_batch_dt(hgks_batch b, double* dt_host) {
  if (hgks_status s = busable(b)) return s;
  if (!dt_host) return fail(HGKS_EINVAL, "null output");
  if (hgks_status s = bcheck(b, hipMemcpyAsync(dt_host, b->ws + b->dt, b->ng * 8, hipMemcpyDeviceToHost, b->stream),
                             "copy dt"))
    return s;
  return batch_status(b);
}

hgks_status hgks_batch_totals(hgks_batch b, double* out_host) {
  if (hgks_status s = batch_ready(b)) return s;
  if (!out_host) return fail(HGKS_EINVAL, "null output");
  double* tot = (double*)(b->ws + b->tot);
  if (b->mixed())
    hipLaunchKernelGGL((k_batch_totals<float>), dim3(b->ng), dim3(kBlock), 0, b->stream,
                       (const BatchGrid<float>*)(b->ws + b->desc), (const double*)(b->ws + b->q), tot);
  else
    hipLaunchKernelGGL((k_batch_totals<double>), dim3(b->ng), dim3(kBlock), 0, b->stream,
                       (const BatchGrid<double>*)(b->ws + b->desc), (const double*)(b->ws + b->q), tot);
  if (hgks_status s = bcheck(b, hipGetLastError(), "totals")) return s;
  if (hgks_status s = bcheck(b, hipMemcpyAsync(out_host, tot, 5 * b->ng * 8, hipMemcpyDeviceToHost, b->stream),
                             "copy totals"))
    return s;
  return bcheck(b, hipStreamSynchronize(b->stream), "synchronise");
}

hgks_status hgks_batch_sync(hgks_batch b) {
  if (hgks_status s = busable(b)) return s;
  return batch_status(b);
}

}  // extern "C"
