/*
 * erf.h -- C-ABI of liberf.so, an MI355X (gfx950) implementation of one RK3
 * large time step of ERF's compressible dynamical core (Lattanzi et al.,
 * "ERF: Energy Research and Forecasting Model", arXiv 2412.04395).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: Arakawa C-grid (Sec. 3.4), nx x ny x nz cells, x fastest.  Lateral
 * boundaries are periodic; the bottom and the top are free-slip rigid lids.
 * Vertical spacing may vary per level (Sec. 3.4, stretched grids).
 *
 * Field layout in device memory (row-major, x fastest, no halo):
 *   rho, rhotheta         [nz][ny][nx]    cell centres
 *   rhou                  [nz][ny][nx]    x-face i lies between cells i-1 and i
 *   rhov                  [nz][ny][nx]    y-face j lies between cells j-1 and j
 *   rhow                  [nz+1][ny][nx]  z-face k lies below cell k; faces 0
 *                                         and nz carry rho w = 0
 *   rhoq                  [n_scalars][nz][ny][nx]
 * Element type: double for ERF_FP64.  For ERF_FP32_MIXED every field is float
 * and rho / rhotheta hold the perturbations rho - rho0(z) and
 * rho*theta - rho0(z)*theta0(z) about the hydrostatic base state.
 *
 * Ownership: the caller owns every state, tendency and flux buffer (device
 * memory, for instance torch tensors); the library never frees them.  The
 * context owns its workspace, allocated once in erf_create.
 *
 * Streams: every call that takes a context enqueues its work on the HIP stream
 * given to erf_create and returns without waiting, except erf_init_base_state
 * and erf_diagnostics, which write host memory and wait for their own work.
 *
 * Errors: every call returns an erf_status.  Argument and shape errors are
 * detected before anything is launched and leave the context usable.  A HIP
 * error is sticky: the context then refuses further work (ERF_E_HIP) until it
 * is destroyed.  erf_last_error returns a description of the latest failure.
 * No call aborts or exits the process.
 */
#ifndef ERF_H
#define ERF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ERF_OK = 0,
    ERF_E_ARG = -1,         /* null pointer or parameter out of range        */
    ERF_E_SHAPE = -2,       /* grid sizes not supported                     */
    ERF_E_HIP = -3,         /* a HIP runtime call failed (sticky)           */
    ERF_E_NONFINITE = -4,   /* diagnostics found NaN or Inf                 */
    ERF_E_UNSUPPORTED = -5, /* option combination not provided              */
    ERF_E_NOMEM = -6,       /* device allocation failed                     */
    ERF_E_STATE = -7        /* call out of order (no base state yet)        */
} erf_status;

typedef enum { ERF_FP64 = 0, ERF_FP32_MIXED = 1 } erf_precision;
/* ERF_SGS_MLP: the learned closure of erf_mlp.h in place of the Smagorinsky
 * stresses; needs erf_mlp_set_weights before the first right-hand side, and
 * nu_m = alpha_m = 0, n_scalars = 0. */
/* ERF_SGS_DEARDORFF: the 1.5-order TKE closure of Deardorff (1980) with the
 * coefficients of Moeng (1984) (Sec. 2.3): rhoq component 0 is rho e (TKE e
 * [m^2/s^2]), the only scalar (n_scalars = 1, dry, alpha_m = 0).  Length
 * l = Delta = (dx dy dz)^(1/3), or 0.76 sqrt(e)/N where smaller in stable air
 * (N^2 = g/theta0 dtheta/dz); K_m = 0.1 l sqrt(e) gives mu_t = rho K_m, the
 * heat diffusivity is rho (1 + 2 l/Delta) K_m; rho e gains rho (K_m 2 S:S -
 * K_h N^2 - (0.19 + 0.51 l/Delta) e^(3/2)/l) + div(2 rho K_m grad e), which
 * erf_slow_rhs computes and erf_scalar_advance adds (times dts), clipping
 * rho e at zero. */
typedef enum { ERF_SGS_NONE = 0, ERF_SGS_SMAGORINSKY = 1, ERF_SGS_MLP = 2, ERF_SGS_DEARDORFF = 3 } erf_sgs_model;
typedef enum { ERF_SCALAR_INTERP = 0, ERF_SCALAR_WENO5 = 1 } erf_scalar_scheme;

typedef struct {
    int32_t nx, ny, nz;  /* cells; nx, ny >= 1, 2 <= nz <= 256                   */
    double dx, dy;       /* horizontal spacing [m]                              */
    const double *dz;    /* host array of nz cell thicknesses [m], copied       */
} erf_grid;

typedef struct {
    double dt;               /* large time step [s]                               */
    int32_t n_substeps;      /* acoustic substeps per step, even (Sec. 3.3)       */
    double beta_s;           /* off-centring of the vertical implicit terms
                                (App. C; the paper uses 0.1)                      */
    double beta_d;           /* divergence damping: horizontal pressure gradient
                                uses Theta'' + beta_d (Theta'' - Theta''_prev)
                                (Sec. 3.1)                                        */
    int32_t adv_order_h;     /* 2..6, interpolants of Sec. 3.6, horizontal        */
    int32_t adv_order_v;     /* 2..6, vertical                                    */
    int32_t scalar_scheme;   /* erf_scalar_scheme for the passive scalars         */
    int32_t n_scalars;       /* 0..8 advected scalars rho*q                       */
    int32_t sgs;             /* erf_sgs_model                                     */
    double Cs, Pr_t;         /* Smagorinsky constant, turbulent Prandtl number    */
    double nu_m, alpha_m;    /* constant kinematic viscosity and diffusivity      */
    double f_cor, Ug, Vg;    /* f-plane Coriolis parameter, geostrophic wind      */
    double surf_heat_flux;   /* prescribed kinematic surface heat flux [K m/s]    */
    double grav;             /* magnitude of gravity [m/s^2]                      */
    int32_t precision;       /* erf_precision                                     */
    int32_t moist;           /* 1: rhoq components 0, 1, 2 are rho q_v, rho q_c,
                                rho q_r and enter the dynamics (Sec. 2.1): the
                                equation of state with water vapour, the factor
                                1/(1 + q_v + q_c) on the pressure gradient and
                                the buoyancy, buoyancy from the total density,
                                and the acoustic coefficients of App. C with
                                the moist Exner function.  No phase change.
                                Needs n_scalars >= 3; 0: dry, the scalars are
                                passive                                          */
    int32_t microphysics;    /* 1: Kessler warm rain (erf_kessler) over dt after
                                every erf_rk3_step, the rain reaching the ground
                                accumulated by the context; needs moist.  0: none */
    int32_t anelastic;       /* 1: the anelastic equation set (Sec. 2.2): density
                                fixed at rho0(z), the constraint div(rho0 u) = 0,
                                buoyancy g rho0 (theta - theta0) / theta0 and a
                                perturbation pressure that only the projections
                                set; stepped by erf_ssprk2_step (Sec. 3.2).
                                Needs ERF_FP64, a dry context, no learned
                                closure, and nx, ny powers of two <= 2048
                                (ERF_E_SHAPE otherwise); n_substeps is then
                                ignored.  0: compressible                        */
    double most_z0;          /* bottom boundary: 0 a free-slip wall; > 0 (and
                                < dz_0/2) the roughness length [m] of a
                                Monin-Obukhov surface layer (Sec. 3.8): per
                                column u* from the lowest cell's centre wind U
                                (at least 0.1 m/s) by the log law with the
                                Businger-Dyer psi_m, von Karman 0.4, Obukhov
                                length from surf_heat_flux (z1/L clamped to
                                [-5, 1]), twenty fixed-point steps; the surface
                                stresses -rho u*^2 (u, v)/U act on the bottom
                                faces (means of the two columns at each face) */
} erf_params;

/* Device pointers to one state (or tendency, or flux) set; unused members may
 * be NULL where a call says so. */
typedef struct {
    void *rho, *rhotheta, *rhou, *rhov, *rhow, *rhoq;
} erf_state;

typedef struct {
    double mass;          /* sum rho dV [kg]                                   */
    double theta_mass;    /* sum rho theta dV                                   */
    double energy;        /* sum (rho |u|^2/2 + rho c_v T + rho g z) dV [J]      */
    double max_w;         /* max |w| over interior z-faces [m/s]               */
    int64_t nonfinite;    /* number of NaN / Inf values in the state           */
    double scalar_mass[8];/* sum rho q dV per scalar                           */
} erf_diag;

typedef struct erf_ctx erf_ctx;

/* Fields of a state, for erf_layout. */
typedef enum {
    ERF_FIELD_RHO = 0,
    ERF_FIELD_RHOTHETA = 1,
    ERF_FIELD_RHOU = 2,
    ERF_FIELD_RHOV = 3,
    ERF_FIELD_RHOW = 4,
    ERF_FIELD_RHOQ = 5
} erf_field;

/* Memory layout of one state field (the C-grid of Sec. 3.4 as stored). */
typedef struct {
    int32_t nx, ny, nz;      /* extent in x, y and levels (nz + 1 for rhow)        */
    int32_t components;      /* n_scalars for rhoq (may be 0), else 1              */
    int64_t stride_y;        /* elements between rows (x stride is 1)              */
    int64_t stride_z;        /* elements between levels                            */
    int64_t stride_c;        /* elements between rhoq components                   */
    int64_t count;           /* elements in the field                              */
    int64_t bytes;           /* count * elem_bytes                                 */
    int32_t elem_bytes;      /* 8 (ERF_FP64) or 4 (ERF_FP32_MIXED)                 */
    int32_t perturbation;    /* 1: stored as the departure from the base state     */
} erf_field_layout;

/* Result of erf_autotune. */
typedef struct {
    int32_t levels_per_wave; /* acoustic substep: levels per wavefront (8 or 16)   */
    int32_t tile_rows;       /* acoustic substep: 64 columns as 1, 2 or 4 rows     */
    double ms_per_step;      /* measured RK3 step time of the choice [ms]          */
    int32_t from_cache;      /* 1: read from the cache file, nothing was timed     */
} erf_tuning;

/* Hydrostatic base state on the host, no GPU involved (Sec. 2, Sec. 3.8):
 * dp0/dz = -rho0 g discretised between level centres with the trapezoidal
 * density, p0 = EOS(rho0 theta0) (Sec. 2.1), solved level by level with
 * Newton-Raphson from p(0) = p_surface.  qv0 [nz] (may be NULL: dry) is the
 * base-state water vapour mixing ratio: rho0 is then the dry density, the
 * column weighs rho0 (1 + qv0) and p0 is the moist equation of state of
 * rho0 theta0 and qv0; qv0 = 0 gives the dry state bit for bit.  Outputs are
 * host arrays of nz values; pi0 (Exner function) may be NULL.  ERF_E_ARG for a
 * non-positive theta0 or dz, or a negative qv0. */
erf_status erf_base_state_host(int32_t nz, const double *dz, const double *theta0, const double *qv0,
                               double p_surface, double grav, double *rho0, double *p0,
                               double *pi0);

/* Layout of state field `field` (erf_field) for a grid and parameter set, as
 * every call of this library reads and writes it (see the conventions above):
 * the caller sizes its buffers from it.  Host only; ERF_E_ARG for an unknown
 * field or NULL pointers, ERF_E_SHAPE / ERF_E_ARG for a grid or parameter set
 * that erf_create would refuse on its sizes, precision or scalar count. */
erf_status erf_layout(const erf_grid *grid, const erf_params *params, int32_t field, erf_field_layout *out);

/* Create a context for one grid and one parameter set.  hip_stream is a
 * hipStream_t (NULL: the default stream).  The grid's dz array is copied.
 * Allocates the whole workspace; returns ERF_E_NOMEM if it does not fit. */
erf_status erf_create(const erf_grid *grid, const erf_params *params, void *hip_stream,
                      erf_ctx **out);
void erf_destroy(erf_ctx *ctx);
const char *erf_last_error(const erf_ctx *ctx);

/* Device bytes of the context's workspace. */
int64_t erf_workspace_bytes(const erf_ctx *ctx);

/* Build the hydrostatic base state (as erf_base_state_host) from theta0 [nz]
 * and qv0 [nz] (host; qv0 may be NULL: dry) and upload it.  Must precede the
 * calls below.  A moist context (erf_params.moist) uses qv0 in the pressure
 * perturbation and the buoyancy; a dry one refuses a non-NULL qv0 (ERF_E_ARG).
 * Optional host outputs rho0, p0, pi0 [nz] may be NULL.  Synchronous. */
erf_status erf_init_base_state(erf_ctx *ctx, const double *theta0, const double *qv0, double p_surface,
                               double *rho0, double *p0, double *pi0);

/* Terrain-following coordinates (Sec. 3.4, App. A, App. B, App. C).  h: host
 * array [ny][nx] of terrain heights [m] at the nodes, node (i, j) being the
 * low-x, low-y corner of cell (i, j), periodic; beta: the smoothing exponent
 * of z = zeta + (1 - zeta / z_t)^beta h (1: basic terrain following, 3:
 * Sullivan; 1 <= beta <= 8), zeta the flat grid's level and z_t its top.  The
 * geometry is copied to the device.  From then on erf_slow_rhs,
 * erf_acoustic_substeps, erf_rk3_step and erf_diagnostics take the metric
 * terms: horizontal fluxes weighted by h_zeta, rho Omega = rho w - h_xi rho u -
 * h_eta rho v through the z-faces (App. A; the momenta averaged from the four
 * faces around each z-face and h_xi, h_eta there by fourth-order differences,
 * App. B), divergences divided by h_zeta, and the horizontal pressure gradient
 * p_xi - h_xi (p_zeta / h_zeta) (App. B; one-sided vertical differences in the
 * lowest and highest cells); the substeps likewise with Omega'' (App. C).
 * A surface heat flux (surf_heat_flux, per unit horizontal area) enters the
 * lowest cell over its physical height.
 * Passive scalars move with the stage-averaged fluxes, whose vertical part
 * erf_acoustic_substeps returns as rho Omega (the mean of the substeps'
 * beta-weighted Omega''), with h_zeta-weighted horizontal fluxes.
 * Needs a dry, inviscid (sgs none, nu_m = alpha_m = 0) ERF_FP64 compressible
 * context without surface layer, not an ensemble member
 * (ERF_E_UNSUPPORTED otherwise; erf_mlp_features and erf_box_filter then
 * refuse the context too); ERF_E_ARG for non-finite heights or a
 * terrain so high that a cell would have no positive height.  Invalidates the
 * base state: erf_init_base_state_columns must follow (erf_init_base_state is
 * refused).  Synchronous; allocates the terrain arrays on the first call. */
erf_status erf_set_terrain(erf_ctx *ctx, const double *h, double beta);
/* The physical height Hc [n] of every cell (the mean of its four vertical
 * edges) and the height zc [n] of its centre (the mean of its eight nodes),
 * host arrays in cell order; either may be NULL.  ERF_E_STATE without terrain. */
erf_status erf_terrain_heights(const erf_ctx *ctx, double *Hc, double *zc);
/* Hydrostatic base state of every column of a terrain context (as
 * erf_init_base_state, along the column's physical cell heights) from theta0
 * [nz][ny][nx] at the cell centres and the pressure p_surf [ny][nx] at each
 * column's ground (host arrays); optional host outputs rho0, p0, pi0 [n].
 * ERF_E_STATE without terrain; synchronous. */
erf_status erf_init_base_state_columns(erf_ctx *ctx, const double *theta0, const double *p_surf, double *rho0,
                                       double *p0, double *pi0);

/* Slow right-hand side f(S) of eqs. (con), (mom), (theta) (Sec. 2.1): flux-form
 * advection with the interpolants of Sec. 3.6, the perturbation pressure
 * gradient, buoyancy -(rho - rho0) g on z-faces, the stress tensor of
 * eq. (stresstensor) with constant or Smagorinsky viscosity (Sec. 2.3),
 * f-plane Coriolis with geostrophic forcing and the surface heat flux
 * (Sec. 3.7-3.8).  Moist contexts: the pressure gradient and the buoyancy
 * -g (rho (1 + q_v + q_c + q_r) - rho0 (1 + qv0)) are divided by the face
 * mean of 1 + q_v + q_c, and p' follows the moist equation of state; S->rhoq
 * must then be given.  Anelastic contexts: p' is the context's perturbation
 * pressure (erf_anelastic_pressure) and the buoyancy g rho0 (theta - theta0) /
 * theta0 on the face (mean of its two cells); R->rho is then -div(rho0 u).
 * S and R use the state layout; R->rhoq is ignored and
 * may be NULL.  R->rhow is zero on faces 0 and nz. */
erf_status erf_slow_rhs(erf_ctx *ctx, const erf_state *S, erf_state *R);

/* One RK stage of semi-implicit acoustic substepping (Sec. 3.1, App. C).
 * Starting from S'' = S_n - S_t, takes n_sub substeps of length dtau with the
 * linearisation frozen at S_t and the slow tendencies R_t, and writes the stage
 * end S_t + S'' to S_out (rho, rhotheta, rhou, rhov, rhow; rhoq untouched) and
 * the stage-averaged normal momenta used for scalar transport to
 * flux_avg->rhou / rhov / rhow (may be NULL).  S_out may alias S_n.  Moist
 * contexts freeze the mixing ratios of S_t->rhoq (required) with the rest of
 * the linearisation: the pressure-gradient coefficient gamma R_d pi^t becomes
 * gamma R_d pi^t (1 + R_v/R_d q_v)/(1 + q_v + q_c), the exact dp/dTheta over
 * the momentum equation's moisture factor, with pi^t the moist Exner
 * function, and the buoyancy coefficient carries the base state's total
 * density and rho_d / rho_m. */
erf_status erf_acoustic_substeps(erf_ctx *ctx, const erf_state *S_n, const erf_state *S_t,
                                 const erf_state *R_t, int32_t n_sub, double dtau,
                                 erf_state *S_out, erf_state *flux_avg);

/* Scalar update after substepping (Sec. 3.1): (rho q)^new = (rho q)^n
 * - dts div(F q^t), q^t = (rho q)^t / rho^t, with F the stage-averaged momenta
 * (flux_avg) and the interpolant or WENO5 of Sec. 3.6 upwinded by the sign of
 * F.  rhoq_out [n_scalars][nz][ny][nx] may alias S_n->rhoq.  Deardorff
 * contexts add dts times the source of rho e that the latest erf_slow_rhs
 * computed (from its S: S_t in the RK3 driver) and clip rho e at zero. */
erf_status erf_scalar_advance(erf_ctx *ctx, const erf_state *S_n, const erf_state *S_t,
                              const erf_state *flux_avg, double dts, void *rhoq_out);

/* One full RK3 step (Sec. 3.1): stages of dt/3, dt/2 and dt with 1, n_s/2 and
 * n_s substeps of length dt/3, dt/n_s and dt/n_s (Sec. 3.3), each stage being
 * erf_slow_rhs, erf_acoustic_substeps and erf_scalar_advance.  S holds S^n on
 * entry and S^{n+1} on return (in place). */
erf_status erf_rk3_step(erf_ctx *ctx, erf_state *S);

/* Kessler warm-rain microphysics (Sec. 2.4: the scheme of Kessler 1969 in the
 * form of Klemp & Wilhelmson 1978) over dt on a moist context's state S
 * (rhoq components rho q_v, rho q_c, rho q_r and rho theta for the latent
 * heat, in place), process-split after a dynamics step: sedimentation of
 * rain (flux form, sub-stepped), autoconversion, accretion, evaporation of
 * rain and the saturation adjustment of cloud water, at the pressure of the
 * step's start.  The rain reaching the ground [kg/m^2] is added to precip
 * (device double[ny][nx]; NULL: the context's own accumulator).  Saturation
 * pressure of Bolton (1980) (the paper's polynomial fit is not printed).
 * ERF_E_UNSUPPORTED for a dry context. */
erf_status erf_kessler(erf_ctx *ctx, erf_state *S, double dt, double *precip);
/* Copy the context's accumulated precipitation [kg/m^2] to host_out (host
 * double[ny][nx]); reset = 1 then sets it to zero.  Synchronous. */
erf_status erf_precipitation(erf_ctx *ctx, double *host_out, int32_t reset);

/* Anelastic contexts (erf_params.anelastic).
 *
 * erf_project: the projection of Sec. 3.2.  Solves dt div grad psi =
 * div(rho u) for the face momenta of S (the C-grid divergence, periodic in x
 * and y, no flux through the lids) by discrete Fourier transforms in x and y
 * and a tridiagonal solve per horizontal wavenumber in z, the horizontally
 * uniform part of psi being zero in the lowest cell; then rho u -= dt grad psi
 * on every face (S->rhou, rhov, rhow in place; only those three are used) and
 * adds psi to the context's perturbation pressure.  ERF_E_UNSUPPORTED on a
 * compressible context.
 *
 * erf_ssprk2_step: one step of dt (Sec. 3.2): S* = S^n + dt f(S^n) with the
 * lagged perturbation pressure, projected; S^{n+1} = S^n + dt (f(S^n) +
 * f(S*)) / 2, projected; each projection adds its psi to the pressure.
 * Scalars take the same two stages with the current momenta as fluxes and
 * q = rho q / rho (erf_scalar_advance).  S->rho must hold rho0 of each level
 * and is not changed; S holds S^n on entry and S^{n+1} on return (in place).
 * Uses the workspace of the RK3 driver.  ERF_E_UNSUPPORTED on a compressible
 * context, which steps with erf_rk3_step (which an anelastic context refuses,
 * as it refuses erf_acoustic_substeps and erf_autotune).
 *
 * erf_anelastic_pressure: copies the context's perturbation pressure p'
 * (device double[nz][ny][nx], zero when the context is created) to p
 * (set = 0) or from p (set = 1), device to device on the context's stream. */
erf_status erf_project(erf_ctx *ctx, erf_state *S, double dt);
erf_status erf_ssprk2_step(erf_ctx *ctx, erf_state *S);
erf_status erf_anelastic_pressure(erf_ctx *ctx, void *p, int32_t set);

/* FP64 global sums of the mass and energy budgets (Sec. 4.1.2) and a count of
 * non-finite values.  Synchronous.  Returns ERF_E_NONFINITE (with *out filled)
 * if any state value is NaN or Inf. */
erf_status erf_diagnostics(erf_ctx *ctx, const erf_state *S, erf_diag *out);

/* Choose the launch shape of the acoustic substep kernel (App. C: the
 * vertically implicit solve over whole columns) for this context by timing:
 * levels per wavefront 8 (nz <= 128) or 16, and the 64 columns of a workgroup
 * as 1, 2 or 4 rows.  Every candidate runs one untimed and then `trials` timed
 * erf_rk3_step calls on S, which therefore advances; the fastest is kept for
 * the context's later calls.  Results do not depend on the row shape; the
 * level count changes the rounding of the chunked tridiagonal sweeps only.
 * cache_path (may be NULL): a text file of earlier choices, one line per grid
 * size and precision; a matching line is applied without timing
 * (out->from_cache = 1), otherwise the choice is appended to it (ERF_E_ARG if
 * the file cannot be written; the choice is applied all the same).
 * Synchronous.  out may be NULL. */
erf_status erf_autotune(erf_ctx *ctx, erf_state *S, int32_t trials, const char *cache_path, erf_tuning *out);

/* Kernel timing for measurement.  While enabled, every launch of the named
 * kernel is bracketed by two HIP events recorded on the context's stream; up to
 * max_launches launches are timed, later ones run untimed.  Kernel names:
 * "prep", "mut", "stress", "rhs", "stage_init", "coef", "substep", "finalize",
 * "mixing_ratio", "scalar", "mlp" (closure network), "mlp_div" (its stress
 * divergence), "kessler" (microphysics), and of the anelastic step
 * "ssp_update", "div_fftx", "ffty" (both directions), "poisson_z", "ifftx",
 * "project", the surface layer "most" and the TKE diffusion "tke".  erf_timing_begin allocates the events
 * (ERF_E_NOMEM on failure) and returns ERF_E_ARG for an unknown name. */
erf_status erf_timing_begin(erf_ctx *ctx, const char *kernel, int32_t max_launches);
/* Waits for the stream, returns the summed event time [ms] of the timed
 * launches and their number, frees the events and stops timing. */
erf_status erf_timing_end(erf_ctx *ctx, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* ERF_H */
