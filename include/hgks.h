/*
 * hgks.h - C ABI of the MI355X (gfx950) HGKS time-stage library.
 *
 * The library advances cell averages of the five conservative variables
 * (rho, rho U, rho V, rho W, rho E) of the compressible Euler / Navier-Stokes
 * equations on a structured hexahedral grid with the high-order gas-kinetic
 * scheme of Pan & Xu, "High-order gas-kinetic scheme with three-dimensional
 * WENO reconstruction for the Euler and Navier-Stokes solutions"
 * (arXiv:1909.01580):
 *   - third-order WENO-AO reconstruction in every cell (Sec. 2, Eqs. (1)-(5));
 *   - the BGK gas-kinetic flux at the 2x2 Gauss points of every face
 *     (Sec. 3, Eqs. (7)-(16)), with the collision time of Sec. 4;
 *   - the two-stage fourth-order update (Sec. 3, after Eq. (9)), with the
 *     grid velocity on moving meshes (Sec. 3, Remark 2).
 *
 * Conventions for every entry point:
 *   - Plain C types only; every call returns an hgks_status; no call throws.
 *   - Pointers named *_dev are device pointers (HIP device memory of the
 *     current device); pointers named *_host are host pointers.
 *   - The caller owns every buffer it passes, including the workspace.  The
 *     library never frees caller memory and allocates no device memory.
 *   - Device work is enqueued on the stream given in the configuration
 *     (NULL = the default stream) and is asynchronous, except for calls
 *     with *_host outputs, which synchronise that stream before returning.
 *   - State arrays are structure-of-arrays [5][nz][ny][nx] of double, x
 *     fastest, in every precision mode.
 *   - The first HIP error seen by a context is sticky: later calls on that
 *     context return HGKS_EDEVICE.  hgks_last_error() returns a message for
 *     the last failing call of the calling thread.
 */
#ifndef HGKS_H
#define HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hgks_ctx_s* hgks_ctx;
typedef struct hgks_batch_s* hgks_batch;

typedef enum {
  HGKS_OK = 0,
  HGKS_EINVAL = 1,        /* bad argument, size or configuration            */
  HGKS_ENOMEM = 2,        /* workspace smaller than hgks_workspace_size     */
  HGKS_EDEVICE = 3,       /* a HIP call failed (sticky per context)         */
  HGKS_ESTATE = 4,        /* call order: e.g. step before set_state         */
  HGKS_ENONPHYS = 5,      /* rho <= 0 or p <= 0 found by a check            */
  HGKS_EUNSUPPORTED = 6   /* valid request the library does not provide     */
} hgks_status;

/* Boundary conditions of Sec. 4.  OUTFLOW is the non-reflecting condition:
 * zero-gradient ghost cells (each ghost a copy of the nearest interior cell,
 * axis by axis).  SYMMETRIC is the symmetric condition of the octant
 * problems: ghost cell g outside the boundary face is the mirror image of
 * interior cell g inside, with the momentum component normal to that face
 * reversed.  A periodic axis is periodic at both ends.  SAME is only for
 * bc_hi: the high end takes the low end's condition. */
typedef enum {
  HGKS_BC_SAME = -1,
  HGKS_BC_PERIODIC = 0,
  HGKS_BC_OUTFLOW = 1,
  HGKS_BC_SYMMETRIC = 2
} hgks_bc;

typedef enum {
  HGKS_FP64 = 0,  /* every step of the stage in double                        */
  HGKS_MIXED = 1  /* reconstruction and gas-kinetic flux in float, and the
                     face sums (F_p, dF_p) stored in float; in double: the
                     stencil differences, the stage accumulation of the state,
                     the hexahedral geometry and least-squares reconstruction
                     (its quadratics then stored in float), the moving-mesh
                     volume and its rates, and all totals                     */
} hgks_prec;

typedef struct {
  int32_t nx, ny, nz;     /* cells per axis, each >= 2, with
                             (nx+2)(ny+2)(nz+2) < 2^29                        */
  int32_t bc[3];          /* hgks_bc per axis (x, y, z): the low end, and the
                             high end too unless bc_hi says otherwise         */
  double gamma;           /* ratio of specific heats, 1 < gamma < 5/3 (1.4)   */
  double mu;              /* dynamic viscosity; 0 selects the inviscid
                             collision time (Sec. 4)                          */
  double weno_Gamma;      /* linear weight of each sub-stencil, 0 < G < 1/24
                             (Sec. 2 suggests 0.0025)                         */
  double weno_eps;        /* epsilon of the nonlinear weights, Eq. (3)       */
  double tau_eps, tau_C;  /* collision time tau = tau_eps dt + tau_C
                             |p_l - p_r|/(p_l + p_r) dt (inviscid) or
                             mu/p + tau_C |...| dt (viscous), Sec. 4; the
                             paper uses 0.01 and 1                            */
  int32_t precision;      /* hgks_prec                                        */
  int32_t moving;         /* 1: hexahedral vertex grid given by
                             hgks_set_vertices (all axes periodic); 0: uniform
                             box grid from hgks_set_uniform_grid              */
  void* stream;           /* hipStream_t, NULL for the default stream         */
  int32_t bc_hi[3];       /* hgks_bc at the high end of each axis, or
                             HGKS_BC_SAME (the default): as bc[d]             */
  int32_t characteristic; /* 1: reconstruct in characteristic variables (Sec.
                             4): per face, Euler eigenvectors along the face
                             frame at the face centre (the normal and the two
                             tangential axes) at the mean of the two cell
                             averages; box and hexahedral grids and batches
                             (one choice for every grid of a batch).  0: the
                             conservative variables component-wise (default) */
  double mu_T0;           /* viscosity law mu (T / mu_T0)^mu_exponent with T =
                             p / rho of the interface equilibrium state, as in
                             the isotropic-turbulence test of Sec. 4 (0.76);  */
  double mu_exponent;     /* exponent 0 (default): constant mu; mu_T0 > 0     */
  double prandtl;         /* Prandtl number of the viscous flux: 1 (default)
                             is the BGK flux as it stands; otherwise (1/Pr - 1)
                             times the heat flux relative to the interface
                             velocity is added to the energy flux (Sec. 4
                             gives Pr = 0.71).  Both on box and hexahedral
                             grids and in batches (per grid)                  */
  int32_t stencil;        /* 0 (default): the big stencil S and 24
                             sub-stencils of Sec. 2; 1: the alternative of
                             Remark 1 (S plus the cells two steps away along
                             the axes, 8 octant sub-stencils, linear weights
                             1 - 8 Gamma and Gamma).  Box and hexahedral
                             grids and batches (one family for every grid of
                             a batch), component-wise reconstruction; a
                             symmetric end needs at least 3 cells on its
                             axis                                            */
} hgks_config;

/* Fills *cfg with the paper's defaults (gamma 1.4, Gamma 0.0025, eps 1e-8,
 * tau_eps 0.01, tau_C 1, FP64, periodic, inviscid; bc_hi = HGKS_BC_SAME;
 * component-wise reconstruction; constant mu, Prandtl number 1)
 * for an nx x ny x nz grid. */
hgks_status hgks_default_config(hgks_config* cfg, int32_t nx, int32_t ny, int32_t nz);

/* Device bytes of the workspace a context with this configuration needs. */
hgks_status hgks_workspace_size(const hgks_config* cfg, size_t* bytes);

/* Creates a context bound to the caller's workspace (device memory of at
 * least hgks_workspace_size bytes, 256-byte aligned).  The configuration
 * is copied.  HGKS_ENOMEM if bytes is too small. */
hgks_status hgks_create(const hgks_config* cfg, void* workspace_dev, size_t bytes,
                        hgks_ctx* out);
hgks_status hgks_destroy(hgks_ctx ctx);

/* Uniform box grid: cell (i,j,k) = origin + [i,i+1]x[j,j+1]x[k,k+1] * h with
 * h = length / n per axis.  Only for contexts with moving = 0.
 * HGKS_EINVAL for a non-positive or non-finite length or a non-finite
 * origin on any axis; a refused call leaves the grid as it was. */
hgks_status hgks_set_uniform_grid(hgks_ctx ctx, const double origin_host[3],
                                  const double length_host[3]);

/* Hexahedral grid (Sec. 2, trilinear cells; Sec. 3, bilinear faces): vertex
 * positions [3][nz][ny][nx] (one vertex per cell and axis; all axes
 * periodic, vertex n along an axis is vertex 0 shifted by the period).
 * The vertices are copied into the workspace.  Only for moving = 1. */
hgks_status hgks_set_vertices(hgks_ctx ctx, const double* xyz_dev, const double period_host[3]);

/* Vertex positions at t_{n+1} for the next hgks_step (moving meshes,
 * Sec. 3 Remark 2): the grid velocity is (next - current)/dt over the step,
 * the stage geometry is at t_n and t_n + dt/2, and after the step the next
 * vertices become the current ones.  Without a call the grid is static. */
hgks_status hgks_set_next_vertices(hgks_ctx ctx, const double* xyz_dev);

/* Copies cell averages [5][nz][ny][nx] (device) into / out of the context. */
hgks_status hgks_set_state(hgks_ctx ctx, const double* q_dev);
hgks_status hgks_get_state(hgks_ctx ctx, double* q_dev_out);

/* dt = cfl * min over cells of h_cell / (|U| + c), h_cell the smallest
 * distance between centres of opposite faces (the paper fixes only
 * CFL = 0.35, Sec. 4).  Synchronises the stream.  HGKS_EINVAL unless
 * 0 < cfl < infinity; HGKS_ESTATE before the grid and the state are set. */
hgks_status hgks_max_dt(hgks_ctx ctx, double cfl, double* dt_host);

/* One time step of size dt: n_stages = 2 is the two-stage fourth-order
 * scheme of Sec. 3; n_stages = 1 the one-stage update Q + dt L + dt^2/2 dL.
 * Asynchronous: it never waits for the device, so it cannot see the state it
 * produces and never returns HGKS_ENONPHYS.  A non-physical result is
 * reported by the next hgks_max_dt (HGKS_ENONPHYS; every CFL-driven loop
 * calls it before each step), by hgks_check, and by hgks_step_checked,
 * which rejects such a step. */
hgks_status hgks_step(hgks_ctx ctx, double dt, int32_t n_stages);

/* hgks_step with step rejection, for static grids: the step is taken with
 * dt / 2^k for the smallest k <= max_halvings (0..60) after which every
 * cell has positive density and pressure; *dt_taken_host receives that
 * step.  The paper prints only the CFL number, and a small one (0.01) for
 * the singular start of its Sedov problem (Sec. 4); at that CFL the
 * two-stage step can still leave a negative pressure next to the energy
 * cell, which a shorter step removes.  When dt / 2^max_halvings also
 * fails the state is left as it was, *dt_taken_host = 0 and the call
 * returns HGKS_ENONPHYS.  Keeps a copy of the state in the workspace;
 * synchronises the stream once per attempt.  HGKS_EUNSUPPORTED on a
 * moving mesh. */
hgks_status hgks_step_checked(hgks_ctx ctx, double dt, int32_t n_stages, int32_t max_halvings,
                              double* dt_taken_host);

/* out[v] = sum over cells of |Omega| Q_v (deterministic order, double).
 * Synchronises the stream. */
hgks_status hgks_totals(hgks_ctx ctx, double out_host[5]);

/* Number of cells whose density or pressure is not positive, and the
 * number of (cell, Gauss point) pairs where the last stage used the
 * first-order fallback of Sec. 4.  Synchronises the stream. */
hgks_status hgks_check(hgks_ctx ctx, int64_t* nonphysical_host, int64_t* fallback_host);

/* Volume-averaged kinetic energy of the Taylor-Green test (Sec. 4),
 * E_k = (1 / (rho0 |Omega|)) int rho |U|^2 / 2, taken on the cell averages:
 * *ek_host = sum_i |Omega_i| |M_i|^2 / (2 rho_i) / (rho0 sum_i |Omega_i|),
 * both sums in a fixed order (deterministic), in double.  Its dissipation
 * rate -dE_k/dt is the difference of two calls over the time between them.
 * HGKS_EINVAL unless 0 < rho0 < infinity.  Synchronises the stream. */
hgks_status hgks_kinetic_energy(hgks_ctx ctx, double rho0, double* ek_host);

/* Parity hooks.  Both run one stage-1 reconstruction (and flux) of the
 * current state with time step dt, without changing the state.
 * gp states: [nz][ny][nx][24][5][4] = (value, d/dx, d/dy, d/dz) of each
 *   variable at Gauss point 4*face + g, faces (-x,+x,-y,+y,-z,+z), g =
 *   2*[a>0] + [b>0] in the face's cyclic parameters, after the fallback.
 * face flux: [3][nz][ny][nx][2][5] = (F_p, dF_p/dt) summed over the lower
 *   face of each cell along x, y, z (Eq. (11) with its time derivative). */
hgks_status hgks_debug_gp_states(hgks_ctx ctx, double dt, double* dev_out);
hgks_status hgks_debug_face_flux(hgks_ctx ctx, double dt, double* dev_out);

/* Parity hook of the limiter (Sec. 4): runs one stage-1 reconstruction of
 * the current state like the hooks above and writes, per cell
 * ([nz][ny][nx], uint32, device), the fallback word: bit 4*face + g set
 * where Gauss point g of that face (numbered as in hgks_debug_gp_states)
 * takes the cell mean and zero gradient; bits 24-31 are zero. */
hgks_status hgks_debug_fallback_mask(hgks_ctx ctx, double dt, uint32_t* mask_dev_out);

/* Kernel timing by phase.  Between hgks_profile_begin and hgks_profile_end
 * the context records a pair of HIP events on its stream around every
 * launch of a phase (at most 512 launches per phase are timed; later ones
 * run untimed).  hgks_profile_end synchronises the stream and returns, per
 * phase, the summed kernel time in milliseconds and the number of timed
 * launches.  Phases: reconstruction, exact fallback test, face flux (one
 * launch covers the faces of all three directions), stage update,
 * reductions (time step, totals, checks). */
typedef enum {
  HGKS_PHASE_RECON = 0,
  HGKS_PHASE_FALLBACK = 1,
  HGKS_PHASE_FLUX = 2,
  HGKS_PHASE_UPDATE = 3,
  HGKS_PHASE_REDUCE = 4,
  HGKS_NPHASES = 5
} hgks_phase;

hgks_status hgks_profile_begin(hgks_ctx ctx);
hgks_status hgks_profile_end(hgks_ctx ctx, double ms_host[5], int64_t launches_host[5]);

/* Waits for the context's stream. */
hgks_status hgks_sync(hgks_ctx ctx);

/* ---------------------------------------------------------------- batches
 * Many independent periodic box grids of uneven sizes advanced together
 * by the same stage as hgks_step: one persistent launch per phase covers
 * every grid, each grid with its own time step read from device memory, so
 * whole steps can be captured in a HIP graph and replayed.
 *
 * cfgs[i] describes grid i (sizes, mu, and the viscosity law and Prandtl
 * number, mu_T0, mu_exponent, prandtl); every grid must be a uniform box
 * (moving = 0) with all axes periodic, and gamma, weno_Gamma, weno_eps,
 * tau_eps, tau_C, precision, the stencil family (stencil: Sec. 2 or
 * Remark 1) and the reconstruction variables (characteristic) must equal
 * those of cfgs[0]; otherwise HGKS_EINVAL and nothing is created.  In
 * characteristic variables the flux phase always runs one workgroup per
 * tile (a flux workgroup count set by hgks_batch_set_launch is not used)
 * and the coefficient arena is seven times as large.  The stream
 * of cfgs[0] is used; it must not be the legacy default stream when
 * hgks_batch_capture is used.  Grid i's state is [5][nz_i][ny_i][nx_i]. */
hgks_status hgks_batch_workspace_size(const hgks_config* cfgs, int32_t n, size_t* bytes);
hgks_status hgks_batch_create(const hgks_config* cfgs, int32_t n, void* workspace_dev, size_t bytes,
                              hgks_batch* out);
hgks_status hgks_batch_destroy(hgks_batch b);
hgks_status hgks_batch_set_uniform_grid(hgks_batch b, int32_t i, const double origin_host[3],
                                        const double length_host[3]);
/* HGKS_EINVAL for an index outside [0, n), a non-positive or non-finite
 * length, or a null pointer; HGKS_ESTATE for get_state before set_state.
 * A refused call changes nothing. */
hgks_status hgks_batch_set_state(hgks_batch b, int32_t i, const double* q_dev);
hgks_status hgks_batch_get_state(hgks_batch b, int32_t i, double* q_dev_out);
/* dt_dev[i] = cfl * min over grid i of h / (|U| + c), as hgks_max_dt;
 * asynchronous, dt_dev is a device array of n doubles (NULL: the batch's
 * own array).  A grid with a cell whose density or pressure is not
 * positive (or not a number) gets dt_dev[i] = 0 and sets the batch's
 * device status word, which the next hgks_batch_dt or hgks_batch_sync
 * reports (HGKS_ENONPHYS) and clears. */
hgks_status hgks_batch_max_dt(hgks_batch b, double cfl, double* dt_dev);
/* One step of every grid i with time step dt_dev[i] (device array);
 * asynchronous.  A grid whose dt_dev[i] is not positive is not advanced
 * (its state is left as it was). */
hgks_status hgks_batch_step(hgks_batch b, const double* dt_dev, int32_t n_stages);
/* Workgroups of the persistent launch of a phase (hgks_phase; a multiple
 * of 8 between 8 and 65536; 0 restores one workgroup per tile). */
hgks_status hgks_batch_set_launch(hgks_batch b, int32_t phase, int32_t workgroups);
/* Tile shapes of the batch (the autotuner's second dimension beside the
 * workgroup counts).  Cell tiles (reconstruction, fallback test, update,
 * time-step reduction): tile_x = tile_y = tile_z = 0 for 256 consecutive
 * cells (x fastest, the default), else a tile_x x tile_y x tile_z box of
 * cells, powers of two with product 256.  Flux tiles are 64 faces of one
 * direction in the banded cell order; flux_band is its band height in rows
 * along y (1..256, default 16; capped at each grid's y extent).  Results do
 * not depend on either.  A captured graph is discarded (capture again). */
hgks_status hgks_batch_set_tiles(hgks_batch b, int32_t tile_x, int32_t tile_y, int32_t tile_z, int32_t flux_band);
/* Captures n_steps steps, each preceded by the per-grid time-step
 * reduction into the batch's own dt array, into a HIP graph (replacing a
 * previous one); hgks_batch_replay launches it.  Nothing runs at capture. */
hgks_status hgks_batch_capture(hgks_batch b, double cfl, int32_t n_steps, int32_t n_stages);
hgks_status hgks_batch_replay(hgks_batch b);
/* The batch's own dt array (last reduction of a replayed graph or of
 * hgks_batch_max_dt with dt_dev = NULL); synchronises.  Returns
 * HGKS_ENONPHYS (after filling dt_host) when a reduction since the last
 * report found a non-physical grid: its dt is 0 and it was not advanced. */
hgks_status hgks_batch_dt(hgks_batch b, double* dt_host);
/* out_host[5 i + v] = sum over grid i of |Omega| Q_v; synchronises. */
hgks_status hgks_batch_totals(hgks_batch b, double* out_host);
/* Waits for the batch's stream; HGKS_ENONPHYS as hgks_batch_dt. */
hgks_status hgks_batch_sync(hgks_batch b);

/* ------------------------------------------------- allocation-free step
 * For callers that cannot allocate device memory or hand the library a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): one step of hgks_step on a box grid (moving = 0)
 * without a context.  cfg, origin and length are as for hgks_create and
 * hgks_set_uniform_grid; q_dev ([5][nz][ny][nx] double, device) is read and
 * overwritten with the state after the step, on cfg->stream,
 * asynchronously.  Every intermediate array lives in one static device
 * array of hgks_noalloc_capacity() bytes (64 MiB) per device, held until
 * the process ends; the call allocates nothing.  HGKS_EINVAL when the grid
 * needs more (hgks_workspace_size(cfg) > the capacity; about 87,000 cells in
 * FP64), HGKS_EUNSUPPORTED for moving = 1.  Calls on one device share the
 * array: calls that overlap (other streams or threads) race and must not be
 * issued. */
hgks_status hgks_step_noalloc(const hgks_config* cfg, const double origin_host[3], const double length_host[3],
                              double* q_dev, double dt, int32_t n_stages);
size_t hgks_noalloc_capacity(void);

/* Message of the last failing call on this thread ("" if none). */
const char* hgks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HGKS_H */
