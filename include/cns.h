/*
 * cns.h -- C-ABI of the MI355X (gfx950) library for the right-hand side of the
 * 3-D compressible Navier-Stokes equations on a triply periodic Cartesian grid
 * and its classical RK4 time integration.
 *
 * Method (arXiv 2211.16718): Sec. 2.1 defines the equations -- conserved state
 * u = [rho, rho u, rho v, rho w, e], convective fluxes f, g, h, the equation of
 * state e = p/(gamma-1) + rho |v|^2 / 2, the viscous fluxes with stress tau_ij
 * and heat flux q_i, T = gamma p / rho, Pr = 0.72.  Sec. 2.2 defines the
 * discretisation -- conservative finite differences, the Roe flux with Harten's
 * entropy fix and |A| = X |Lambda| X^-1 at the Roe average, component-wise
 * WENO5 (Jiang-Shu weights, epsilon = 1e-6) of f^{L,R} and u^{L,R}, 4th-order
 * central differences for the viscous terms, and RK4 in time.
 *
 * Conventions shared by every call:
 *  - Return value: CNS_OK (0) or a negative CNS_E* code; cns_last_error() gives a
 *    thread-local message for the last failure on the calling thread.  No C++
 *    exception crosses this interface.
 *  - Memory: every array argument named *_dev or typed as a state is DEVICE
 *    memory owned by the caller (allocated through PyTorch or hipMalloc).  The
 *    library never allocates device memory; the scratch it needs is the caller's
 *    workspace (cns_workspace_bytes / cns_set_workspace).  A plan owns host-side
 *    state only.
 *  - State layout: structure-of-arrays u[v][k][j][i], v = 0..4 the conserved
 *    variable, i (x) fastest, contiguous, 256-byte aligned.  The element type is
 *    double for CNS_FP64 plans and float for CNS_MIXED plans.
 *  - Streams: `stream` is a hipStream_t passed as void*.  Calls enqueue on the
 *    plan's stream and return without synchronising, except where a call
 *    returns host values (stated per call).
 *  - Periodic grid: x_i = i * lx / nx, i = 0..nx-1, likewise y and z; nx, ny, nz >= 8 and at
 *    most 536870911 points per box (8 nx ny nz < 2^32).
 *  - Physics: gamma > 1, mu_eff >= 0, Prandtl > 0 when mu_eff > 0, weno_eps in
 *    [1e-30, 1e30], harten_delta >= 0; otherwise CNS_EINVAL.
 */
#ifndef CNS_H
#define CNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CNS_OK 0
#define CNS_EINVAL (-1)        /* null/misaligned pointer, bad size, bad parameter */
#define CNS_EHIP (-2)          /* a HIP runtime error (message from hipGetErrorString) */
#define CNS_ENONFINITE (-3)    /* a non-finite value was produced or found */
#define CNS_ENONPHYSICAL (-4)  /* rho <= 0 or p <= 0 found */
#define CNS_EWORKSPACE (-5)    /* workspace missing or too small */
#define CNS_EUNSUPPORTED (-6)  /* operation not available for this plan */

/* diagnostics record: K = <|m|^2/(2 rho)>, Omega = <|curl v|^2>/2 (4th-order central
 * derivatives), <rho>, <rho u>, <rho v>, <rho w>, <e> (grid means),
 * max over points and directions of |v_d| + c, count of bad points
 * (non-finite, rho <= 0 or p <= 0). */
#define CNS_NDIAG 9

typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;
} cns_grid;

typedef struct {
    double gamma;        /* ratio of specific heats, > 1 */
    double prandtl;      /* Prandtl number, > 0 when mu_eff > 0 */
    double mu_eff;       /* mu * M_inf / Re_inf (Sec. 2.1 scaling); 0 = Euler (viscous terms skipped) */
    double weno_eps;     /* epsilon of the WENO weights, in [1e-30, 1e30] (paper: 1e-6) */
    double harten_delta; /* Harten threshold delta >= 0; 0 = plain |lambda| */
    int32_t weno_weights; /* CNS_WENO_JS (Sec. 2.2: Jiang-Shu), CNS_WENO_Z (Borges et al. 2008,
                             exponent 2) or CNS_WENO_M (mapped, Henrick et al. 2005): the two
                             improved nonlinear weights the paper cites (Sec. 1) */
} cns_physics;

enum { CNS_WENO_JS = 0, CNS_WENO_Z = 1, CNS_WENO_M = 2 };

enum { CNS_FP64 = 0, CNS_MIXED = 1 };

typedef struct cns_plan cns_plan;

/* Create a plan for one periodic box.  precision: CNS_FP64 (state and arithmetic in
 * double) or CNS_MIXED (state, stage states and WENO/flux arithmetic in float; WENO
 * smoothness-indicator sums and the RK4 accumulator in double; the float weights are
 * scaled so that no jump overflows them).  stream: hipStream_t or NULL for the default
 * stream.  *out receives the plan. */
int cns_plan_create(cns_plan **out, const cns_grid *grid, const cns_physics *phys, int32_t precision,
                    void *stream);
int cns_plan_destroy(cns_plan *plan);

/* Bytes of device workspace the plan needs (for every call below). */
size_t cns_workspace_bytes(const cns_plan *plan);
/* Bind caller-owned device workspace (>= cns_workspace_bytes, 256-byte aligned). */
int cns_set_workspace(cns_plan *plan, void *ws_dev, size_t bytes);

/* Launch tuning: segment length (points per thread along the sweep) for each
 * direction's sweep kernel, and threads per block.  0 keeps the current value.
 * Results do not depend on these values (bitwise). */
int cns_set_tiles(cns_plan *plan, int32_t seg_x, int32_t seg_y, int32_t seg_z, int32_t block);

/* x-direction sweep kernel: 0 = periodic rows staged in LDS, one thread per interface
 * (default: whole rows, several per block, when nx <= 256; longer rows walked in chunks of
 * 256 interfaces by one block each), 1 = the marching kernel used for y and z.  Results
 * agree to round-off. */
int cns_set_x_kernel(cns_plan *plan, int32_t kind);

/* Sec. 2.1 equation of state: u = [rho, rho v, p/(gamma-1) + rho|v|^2/2] from device
 * primitives rho[N3], vel[3][N3], p[N3] (double).  u in plan precision. */
int cns_init_state(const cns_plan *plan, const double *rho_dev, const double *vel_dev, const double *p_dev,
                   void *u_dev);

/* Sec. 2.2: full right-hand side rhs = du/dt of the semi-discrete equations. */
int cns_rhs(const cns_plan *plan, const void *u_dev, void *rhs_dev);

/* Sec. 2.2: the convective term along one direction, out = -(F_{j+1/2} - F_{j-1/2})/dx_dir,
 * dir 0 = x, 1 = y, 2 = z (Roe + Harten + WENO5 interface fluxes). */
int cns_rhs_dir(const cns_plan *plan, const void *u_dev, int32_t dir, void *out_dev);

/* Sec. 2.1/2.2: the viscous and heat-flux terms, out = sum_d D_d G^v_d. */
int cns_viscous(const cns_plan *plan, const void *u_dev, void *out_dev);

/* nsteps classical RK4 steps of size dt, in place on u.  diag_dev (may be NULL)
 * receives [nsteps][CNS_NDIAG] diagnostics of the state after each step.
 * Bad points are reported in the diagnostics (the call does not synchronise). */
int cns_rk4(cns_plan *plan, void *u_dev, double dt, int32_t nsteps, double *diag_dev);

/* Time integrators.  CNS_RK4: the classical four-stage scheme.  CNS_TVDRK3: the
 * three-stage third-order TVD scheme of Shu and Osher, the integrator of the
 * paper's production runs (Sec. 2.2 names both; Sec. 5 times TVD-RK3 steps). */
#define CNS_RK4 0
#define CNS_TVDRK3 1
/* nsteps TVD-RK3 steps of size dt, in place on u:
 *   U1 = u + dt R(u);  U2 = 3/4 u + 1/4 (U1 + dt R(U1));  u <- 1/3 u + 2/3 (U2 + dt R(U2)).
 * Arguments, diagnostics and errors as cns_rk4.  In the mixed form each convex
 * combination is formed in FP64 from the FP32 states and rounded once. */
int cns_tvdrk3(cns_plan *plan, void *u_dev, double dt, int32_t nsteps, double *diag_dev);

/* Kinetic-energy spectrum (Sec. 2.3 and Sec. 5 characterise the turbulence by E(k) and the
 * Taylor microscale).  With v = m/rho, v_hat(k) = (1/N) sum_x v(x) exp(-i k.x) (N points) and the
 * physical wavenumber k_d = 2 pi n_d / L_d:
 *   E_dev[s]      = sum over modes with round(|k|) = s of |v_hat|^2 / 2,  s = 0..nshell-1;
 *   moments_dev[0] = sum_s E[s] (= <|v|^2>/2), moments_dev[1] = sum over modes of |k|^2 |v_hat|^2 / 2,
 *   moments_dev[2] = the Taylor microscale sqrt(5 moments[0] / moments[1]) of isotropic
 *   turbulence (+inf for a uniform velocity).
 * moments_dev holds three doubles.  FP64 for either precision.
 * Uses the plan's stage buffers as scratch (ordered with other calls on the plan's
 * stream).  nshell must equal cns_spectrum_shells(plan) (round(|k|max) + 1), else
 * CNS_EINVAL; grids with a dimension above 2047, more than 4096 shells, or more than one
 * shell per 1.2 grid points (24 bytes of scratch per shell) give CNS_EUNSUPPORTED.  Shell
 * sums use LDS atomics, so their last bits may differ between runs. */
int cns_spectrum_shells(const cns_plan *plan);
int cns_spectrum(const cns_plan *plan, const void *u_dev, double *E_dev, int32_t nshell, double *moments_dev);

/* The CFL wave speed of Sec. 2.2's explicit time step: out_dev[0] = max over grid points
 * and directions d of |v_d| + c, c = sqrt(gamma p / rho) (FP64, one device double; the
 * same value as slot 7 of the diagnostics).  NaN when a point is non-finite or has
 * rho <= 0 or p <= 0.  Uses the plan's diagnostics scratch (ordered on its stream). */
int cns_max_wave_speed(const cns_plan *plan, const void *u_dev, double *out_dev);

/* Diagnostics of u into device memory out_dev[CNS_NDIAG]. */
int cns_diagnostics(const cns_plan *plan, const void *u_dev, double *out_dev);
/* For callers that cannot allocate (code under hipGraph capture, tight serving loops,
 * harnesses that forbid allocation): the diagnostics record of cns_diagnostics for a box
 * described by grid, phys and precision, with no plan and no workspace.  Its scratch (the
 * device table of the box and at most 1024 per-block partial sums, whatever the grid
 * size) lives in a static device array of 128 KiB that every GPU the library runs on holds
 * until the process ends; the call allocates nothing and copies nothing from the host (the
 * table is written by a kernel), so it can be captured.  The current device must be the
 * stream's device.  Every partial sum is written before it is read, so nothing needs
 * clearing between calls.  Calls that overlap on one GPU (other streams or threads) share
 * the array and race; order them.  Results equal cns_diagnostics bitwise.  Errors as
 * cns_plan_create for the arguments, CNS_EUNSUPPORTED if the scratch need exceeded the
 * array. */
int cns_diagnostics_static(const cns_grid *grid, const cns_physics *phys, int32_t precision, const void *u_dev,
                           double *out_dev, void *stream);
/* Same, copied to host memory out_host[CNS_NDIAG]; synchronises the plan's stream.
 * Returns CNS_ENONFINITE / CNS_ENONPHYSICAL when bad points are present (the record
 * is still written). */
int cns_diagnostics_host(const cns_plan *plan, const void *u_dev, double *out_host);

/* Per-kernel timing of cns_rk4 with HIP events recorded on the plan's stream around
 * every launch (an event wait after each step).  Kernel kinds, in order:
 * viscous primitives (formed inside the viscous-flux kernel: no launches, kept so the
 * indices stay stable), viscous fluxes, x sweep, y sweep, z sweep with the fused RK4
 * stage update, diagnostics.  enable != 0 clears the totals and turns timing on. */
#define CNS_NKERNEL 6
int cns_profile_enable(cns_plan *plan, int32_t enable);
/* Summed milliseconds and launch counts per kernel kind since the last enable
 * (host arrays of CNS_NKERNEL entries). */
int cns_profile_read(const cns_plan *plan, double *ms_host, int64_t *count_host);

/* hipGraph replay of cns_rk4 / cns_tvdrk3: the launches of all nsteps are captured once
 * per (integrator, nsteps, diagnostics on or off) and replayed; the state pointer, dt and
 * the diagnostics pointer of each call reach the replay through a device record in the
 * workspace, written by a kernel enqueued before every replay (so calls with new
 * buffers or step sizes replay the same graph).  enable = 0 launches eagerly.  Needs a
 * plan created on a non-default stream (else CNS_EUNSUPPORTED).  Replays are bitwise
 * identical to eager launches. */
int cns_set_graph(cns_plan *plan, int32_t enable);
/* Number of graph captures made by the plan so far (>= 0), or a negative error code. */
int64_t cns_plan_graph_captures(const cns_plan *plan);

/* ---- ensembles: independent periodic boxes of uneven sizes advanced together ----
 * Every kernel launch covers all boxes (virtual blocks mapped to boxes by prefix
 * sums), so one RK4 step of the whole ensemble is 18 launches (viscous fluxes and three
 * sweeps per stage, two for the diagnostics), optionally replayed
 * from a captured hipGraph.  A box advanced in an ensemble gives bitwise the result
 * of its own single-box plan (same kernels, same arithmetic).  Extension beyond the
 * paper, which advances one domain. */
typedef struct cns_ensemble cns_ensemble;
/* grids[nbox], phys[nbox], dt[nbox]: host arrays.  u_packed: device buffer holding
 * every box's state [5][N3_i] at element offset offsets[i] (host array; each box
 * 256-byte aligned, no overlap), element type by precision.  The ensemble keeps
 * u_packed, which must outlive it. */
int cns_ensemble_create(cns_ensemble **out, int32_t nbox, const cns_grid *grids, const cns_physics *phys,
                        const double *dt, int32_t precision, void *u_packed, const int64_t *offsets, void *stream);
int cns_ensemble_destroy(cns_ensemble *ens);
size_t cns_ensemble_workspace_bytes(const cns_ensemble *ens);
int cns_ensemble_set_workspace(cns_ensemble *ens, void *ws_dev, size_t bytes);
/* segment lengths of box `box` (-1: every box) and the block size; 0 keeps a value. */
int cns_ensemble_set_tiles(cns_ensemble *ens, int32_t box, int32_t seg_x, int32_t seg_y, int32_t seg_z,
                           int32_t block);
int cns_ensemble_get_tiles(const cns_ensemble *ens, int32_t box, int32_t *seg3_host, int32_t *block_host);
/* Choose launch shapes by timing them on the device, keeping the fastest: per box size,
 * the segment length of the y/z marching sweeps and the rows per block of the x rows
 * kernel (the default power of two and every count with the same points per thread that
 * keeps 90 % of a block's threads busy); for the batch, the threads per block of the marching sweeps and the launched
 * grids (one block per virtual block, or persistent grids of one or two rounds of the
 * blocks the chip holds at once, for the sweeps and for the tiled viscous-flux and
 * diagnostics kernels).  Only scratch buffers are written while timing.  cache_path (may
 * be NULL): a JSON file read first (known choices are not re-timed) and rewritten with
 * new ones.  Synchronises the ensemble's stream.  Launch shapes never change results. */
int cns_ensemble_autotune(cns_ensemble *ens, const char *cache_path);
/* The launch shapes of box `box`: rows per block of its x rows kernel (0: the marching
 * x sweep), and the launched blocks of the marching sweeps and of the tiled kernels of the
 * whole ensemble (0: one block per virtual block). */
int cns_ensemble_get_launch(const cns_ensemble *ens, int32_t box, int32_t *rows_host, int64_t *sweep_grid_host,
                            int64_t *tile_grid_host);
/* Set launch shapes by hand: rows per block of the x rows kernel of box `box` (-1: every
 * box; 0: the default; a count that does not fit gives CNS_EINVAL), and the launched blocks
 * of the marching sweeps and of the tiled kernels (0: one per virtual block; any positive
 * count: a persistent launch whose blocks loop over the virtual blocks).  Results do not
 * depend on the launched blocks (bitwise), nor on the rows as long as the points per
 * thread of the x rows kernel (rows * nx / 256, rounded up, the largest over the boxes)
 * stay the same; another count of points per thread runs another instantiation of the
 * kernel, whose results agree to round-off. */
int cns_ensemble_set_launch(cns_ensemble *ens, int32_t box, int32_t rows, int64_t sweep_grid, int64_t tile_grid);
/* nsteps steps (RK4 unless cns_ensemble_set_integrator chose TVD-RK3) of every box with its own dt; diag_dev (may be NULL) receives
 * [nbox][nsteps][CNS_NDIAG].  use_graph != 0 captures the whole run once and
 * replays it (non-default stream required). */
int cns_ensemble_run(cns_ensemble *ens, int32_t nsteps, double *diag_dev, int32_t use_graph);
/* Number of graph captures made by the ensemble so far (>= 0; a capture is reused while
 * nsteps, the integrator and whether diagnostics are written stay the same), or a
 * negative error code. */
int64_t cns_ensemble_graph_captures(const cns_ensemble *ens);
/* Integrator of cns_ensemble_run: CNS_RK4 (default) or CNS_TVDRK3 (else CNS_EINVAL). */
int cns_ensemble_set_integrator(cns_ensemble *ens, int32_t scheme);
int cns_ensemble_profile_enable(cns_ensemble *ens, int32_t enable);
int cns_ensemble_profile_read(const cns_ensemble *ens, double *ms_host, int64_t *count_host);

/* ---- adjoint (FP64 plans, any of the WENO weights; CNS_EUNSUPPORTED for mixed) ----
 * Reverse-mode derivatives of the discrete operator of Sec. 2.2, hand-written:
 * vector-Jacobian products of the WENO5 reconstructions (Jiang-Shu, Z or mapped
 * weights), the Roe flux with Harten's fix, the Euler fluxes and the central viscous
 * terms.  Extension beyond the paper.
 * adj_ws: caller-owned device scratch of cns_adjoint_workspace_bytes bytes. */
size_t cns_adjoint_workspace_bytes(const cns_plan *plan, int32_t nsteps, int32_t ckpt_every);
/* ubar = (dR/du)^T rbar at u (all [5][N3] device arrays, FP64; ubar must not alias u
 * or rbar).  The product needs no scratch: adj_ws and bytes are not read (NULL and 0
 * are fine). */
int cns_rhs_vjp(const cns_plan *plan, const void *u_dev, const void *rbar_dev, void *ubar_dev, void *adj_ws,
                size_t bytes);
/* J = K(u^N) after nsteps RK4 steps of size dt from u0 (K = <|m|^2/(2 rho)>), and
 * u0_bar = dJ/du0.  Checkpoints every ckpt_every steps; the reverse sweep takes one
 * segment at a time, recomputed from its checkpoint (the last one is kept during the
 * forward pass) with the start and stage states of each of its steps kept.  J_dev
 * (may be NULL): one device double. */
int cns_adjoint_rk4(cns_plan *plan, const void *u0_dev, double dt, int32_t nsteps, int32_t ckpt_every,
                    void *adj_ws, size_t bytes, double *J_dev, void *u0_bar_dev);
/* The same for nsteps steps of the three-stage TVD Runge-Kutta scheme (Shu-Osher form,
 * as cns_tvdrk3), the integrator of the paper's production runs; the same workspace
 * (cns_adjoint_workspace_bytes covers either integrator). */
int cns_adjoint_tvdrk3(cns_plan *plan, const void *u0_dev, double dt, int32_t nsteps, int32_t ckpt_every,
                       void *adj_ws, size_t bytes, double *J_dev, void *u0_bar_dev);
/* The same gradient in two calls, for callers that want J before deciding on the
 * gradient (an autograd forward and backward): cns_adjoint_forward runs the nsteps
 * steps of `scheme` (CNS_RK4 or CNS_TVDRK3) from u0 with a checkpoint every ckpt_every
 * steps, keeps the last segment's start and stage states, writes J = K(u^N) to J_dev
 * (may be NULL) and leaves all of it in adj_ws; cns_adjoint_reverse then runs the reverse
 * sweep from that workspace and writes u0_bar = dJ/du0.  The reverse call needs the same
 * plan, scheme, dt, nsteps, ckpt_every and an untouched workspace (any other adjoint call
 * on it in between invalidates it).  The pair computes exactly what cns_adjoint_rk4 /
 * cns_adjoint_tvdrk3 compute. */
int cns_adjoint_forward(cns_plan *plan, int32_t scheme, const void *u0_dev, double dt, int32_t nsteps,
                        int32_t ckpt_every, void *adj_ws, size_t bytes, double *J_dev);
int cns_adjoint_reverse(cns_plan *plan, int32_t scheme, double dt, int32_t nsteps, int32_t ckpt_every, void *adj_ws,
                        size_t bytes, void *u0_bar_dev);
/* Transpose of the initial-state map at fixed rho and p:
 * vbar_i = rho (mbar_i + ebar v_i); rho[N3], vel[3][N3], ubar[5][N3] -> vbar[3][N3]. */
int cns_ic_vjp(const cns_plan *plan, const double *rho_dev, const double *vel_dev, const double *ubar_dev,
               double *vbar_dev);

/* ---- measurement helper ----
 * A plain streaming copy of `bytes` (a multiple of 16) from src_dev to dst_dev (16-byte
 * aligned, not overlapping) on `stream`: 16-byte non-temporal loads and stores, a grid of
 * 2048 blocks of 256 threads.  It is the bandwidth reference the benchmark reports kernel
 * rates against, and the known-size dispatch that calibrates hardware byte counters. */
int cns_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, void *stream);

/* Thread-local message of the last error on this thread ("" if none). */
const char *cns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
