/*
 * erf_oracle.h -- plain FP64 CPU oracle of ERF's compressible RK3 step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * library; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * library.  Every routine is a direct, slow transcription of the equations of
 * Lattanzi et al., "ERF: Energy Research and Forecasting Model" (arXiv
 * 2412.04395); each function names the passage it follows.
 *
 * Layout (all arrays host, double, x fastest):
 *   cell-centred  f[(k*ny + j)*nx + i],            k < nz
 *   x-faces       U[(k*ny + j)*nx + i]  face i sits between cells i-1 and i
 *   y-faces       V[(k*ny + j)*nx + i]  face j sits between cells j-1 and j
 *   z-faces       W[(k*ny + j)*nx + i],            k <= nz, face k below cell k
 * Lateral boundaries are periodic; bottom and top are free-slip rigid lids
 * (W = 0 on faces 0 and nz).
 */
#ifndef ERF_ORACLE_H
#define ERF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy;
    const double *dz; /* nz cell thicknesses */
    /* terrain-following coordinates (App. A, App. B); NULL: flat.  Terrain
     * heights h[ny][nx] at the nodes, node (i, j) being the low-x, low-y corner
     * of cell (i, j) (periodic); node heights z = zeta + (1 - zeta/z_t)^beta h
     * with zeta the flat grid's level and z_t its top.  With terrain the base
     * state (orc_base) holds one value per cell, and the slow right-hand side,
     * the substeps, the scalars and the diagnostics take the metric terms;
     * dry, inviscid (sgs 0, no constant viscosity, no surface layer),
     * compressible only; a surface heat flux enters the lowest cell per unit
     * horizontal area. */
    const double *terrain;
    double terrain_beta; /* 1: basic terrain following; 3: Sullivan */
} orc_grid;

typedef struct {
    double dt;
    int32_t n_substeps;     /* per full step; even                            */
    double beta_s;          /* off-centring (App. C), 0.1 in the paper          */
    double beta_d;          /* forward-prediction weight of divergence damping */
    int32_t adv_order_h;    /* 2..6, Sec. 3.6                                   */
    int32_t adv_order_v;    /* 2..6                                            */
    int32_t scalar_scheme;  /* 0: same interpolants as momentum; 1: WENO5-JS   */
    int32_t n_scalars;
    int32_t sgs;            /* 0 none, 1 Smagorinsky, 2 learned closure (MLP),
                               3 Deardorff 1.5-order TKE (scalar 0 is rho e)    */
    double Cs, Pr_t;
    double nu_m, alpha_m;   /* constant kinematic viscosity / diffusivity       */
    double f_cor, Ug, Vg;   /* f-plane Coriolis and geostrophic wind           */
    double surf_heat_flux;  /* kinematic, K m/s                                 */
    double grav;            /* magnitude of gravity                             */
    /* learned closure (sgs == 2): parameters, norm stats, BF16 emulation */
    const double *mlp_params, *mlp_norm;
    int32_t mlp_bf16;
    /* moist dynamics: the first three scalars are rho q_v, rho q_c, rho q_r;
     * they enter the EOS, the pressure-gradient and buoyancy terms and the
     * acoustic coefficients (Sec. 2.1, App. C); needs n_scalars >= 3 */
    int32_t moist;
    /* anelastic equation set (Sec. 2.2): rho stays at rho0, the pressure
     * gradient uses the lagged perturbation pressure p_anel [nz][ny][nx]
     * instead of the equation of state, and the buoyancy is
     * g rho0 (theta - theta0) / theta0; dry only */
    int32_t anelastic;
    const double *p_anel;
    /* bottom boundary: 0 a free-slip wall; > 0 the roughness length z0 [m] of
     * a Monin-Obukhov surface layer (Sec. 3.8) giving the surface stress from
     * the lowest level's wind, with the surface heat flux surf_heat_flux */
    double most_z0;
} orc_params;

typedef struct {
    const double *rho0, *theta0, *p0, *pi0; /* nz each (with terrain: nz*ny*nx) */
    const double *qv0;                      /* nz, base-state vapour; NULL: dry */
} orc_base;

typedef struct {
    double *rho, *rt, *ru, *rv, *rw, *rq; /* rq: n_scalars consecutive fields */
} orc_state;

/* physical constants used by the oracle (gas constant, heat capacity, P00) */
double orc_const(int which); /* 0 R_d, 1 c_p, 2 c_v, 3 gamma, 4 P00, 5 R_v */

/* Hydrostatic base state by Newton iteration, Sec. 2 and Sec. 3.8. */
int orc_base_state(int32_t nz, const double *dz, const double *theta0, double p_surface,
                   double grav, double *rho0, double *p0, double *pi0);
/* The same with a base-state water vapour mixing ratio qv0[nz] (NULL: dry):
 * the moist EOS and the weight of the vapour, dp0/dz = -g rho0 (1 + qv0). */
int orc_base_state_moist(int32_t nz, const double *dz, const double *theta0, const double *qv0,
                         double p_surface, double grav, double *rho0, double *p0, double *pi0);

/* Terrain geometry (App. A, App. B): the physical height Hc[n] of every cell
 * (its four vertical edges averaged) and the height zc[n] of its centre (its
 * eight nodes averaged); either may be NULL.  Flat grids give dz and the flat
 * centre heights. */
int orc_terrain_heights(const orc_grid *g, double *Hc, double *zc);
/* Hydrostatic base state of every column (dry) from theta0[n] at the cell
 * centres and the pressure p_surf[ny][nx] at each column's ground, with the
 * column's physical cell heights; rho0, p0, pi0 [n].  On a flat grid every
 * column equals orc_base_state's. */
int orc_base_state_columns(const orc_grid *g, const double *theta0, const double *p_surf, double grav,
                           double *rho0, double *p0, double *pi0);

/* Equation of state, Sec. 2.1: p = P00 (R_d Theta / P00)^gamma. */
double orc_eos_p(double Theta);
/* p' = p(Theta) - p(Theta0) evaluated without cancellation. */
double orc_eos_pprime(double Theta, double Theta0, double p0);
/* Moist EOS, Sec. 2.1: p = P00 (R_d Theta (1 + R_v/R_d q_v) / P00)^gamma. */
double orc_eos_p_moist(double Theta, double qv);
/* p' = p(Theta, q_v) - p0 with p0 = p(Theta0, q_v0), without cancellation. */
double orc_eos_pprime_moist(double Theta, double qv, double Theta0, double qv0, double p0);

/* Face interpolant q_{m-1/2} of Sec. 3.6; q = {q_{m-3},...,q_{m+2}}. */
double orc_interp(int32_t order, const double *q6, double sgn);
/* WENO5-JS face value q_{m-1/2}; q = {q_{m-3},...,q_{m+2}}, eps is the
 * regulariser of the smoothness weights. */
double orc_weno5(const double *q6, double sgn, double eps);

/* Thomas algorithm for a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = r[i], n >= 1. */
int orc_thomas(int32_t n, const double *a, const double *b, const double *c,
               const double *r, double *x);

/* Slow right-hand side f(S) of eqs. (con), (mom), (theta) (Sec. 2.1, 2.3,
 * 3.6, 3.7, 3.8).  R->rq is not touched, except with the Deardorff closure
 * (sgs 3): R->rq (component 0) then receives the source of rho e, everything
 * but its advection (shear and buoyancy production, dissipation, diffusion). */
int orc_slow_rhs(const orc_grid *g, const orc_params *P, const orc_base *B,
                 const orc_state *S, orc_state *R);

/* One RK stage of semi-implicit acoustic substepping, App. C and Sec. 3.1.
 * Starts from S'' = S_n - S_t, takes n_sub substeps of size dtau, writes the
 * stage-end state S_t + S'' into Sout (rho, rt, ru, rv, rw) and the
 * stage-averaged normal momenta into Fu, Fv, Fw. */
int orc_acoustic_substeps(const orc_grid *g, const orc_params *P, const orc_base *B,
                          const orc_state *Sn, const orc_state *St, const orc_state *Rt,
                          int32_t n_sub, double dtau, orc_state *Sout,
                          double *Fu, double *Fv, double *Fw);

/* Scalar update with time-averaged fluxes (Sec. 3.1):
 * (rho q)^new = (rho q)^n - dts div(F q^t).  With the Deardorff closure,
 * component 0 (rho e) also gains dts src (src: the slow right-hand side's
 * R->rq at S^t; may be NULL otherwise) and is clipped at zero. */
int orc_scalar_advance(const orc_grid *g, const orc_params *P, const orc_state *Sn,
                       const orc_state *St, const double *Fu, const double *Fv,
                       const double *Fw, double dts, const double *src, double *rq_out);

/* One full RK3 step with substeps (Sec. 3.1, 3.3), in place. */
int orc_rk3_step(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S);

/* FP64 diagnostics: out[0] mass, out[1] sum Theta dV, out[2] total energy,
 * out[3] max |w|, out[4] number of non-finite values, out[5..5+nq) scalar
 * masses. */
int orc_diagnostics(const orc_grid *g, const orc_params *P, const orc_base *B,
                    const orc_state *S, double *out);

/* ---------------- learned SGS closure (MLP 10 -> 64 -> 64 -> 64 -> 9) ---------------- */
/* Parameters, flat: W1[10][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
 * W4[64][9], b4[9] (row = input feature, column = output unit); 9609 values.
 * Norm stats: mean_x[10], std_x[10], mean_y[9], std_y[9]. */
int orc_mlp_nparams(void);
/* Forward pass on standardised inputs x[n][10] -> standardised outputs y[n][9].
 * bf16 = 1 rounds every matrix operand to bfloat16 (through float, round to
 * nearest even) and accumulates in double, as the GPU's BF16 products do. */
int orc_mlp_forward(const double *params, const double *x, int64_t n, double *y, int bf16);
/* Mean-squared error over n samples x 9 outputs and its gradient (9609). */
int orc_mlp_loss_grad(const double *params, const double *x, const double *t, int64_t n, int bf16,
                      double *loss, double *grad);
/* Error scale of the gradient: for every parameter, the sum of the magnitudes
 * of the terms whose sum is its gradient (the backpropagation with absolute
 * values), gabs[9609]. */
int orc_mlp_grad_abs(const double *params, const double *x, const double *t, int64_t n, int bf16,
                     double *gabs);
/* Per sample of the BF16-mode forward pass on x[n][10] and per hidden unit of
 * the three hidden layers (margin[n][192]): the distance of the unit's value
 * to a bfloat16 rounding boundary (or to zero) relative to the sum of the
 * magnitudes of its terms.  With flip_layer/flip_unit (nullable) each sample
 * may round one hidden unit to the bfloat16 neighbour on the other side of its
 * value; y[n][9] (nullable) receives the outputs of that pass. */
int orc_mlp_unit_margins(const double *params, const double *x, int64_t n, double *margin,
                         const int32_t *flip_layer, const int32_t *flip_unit, double *y);
/* One Adam step (beta1, beta2, eps), step counts from 1. */
int orc_adam(double *params, const double *grad, double *m, double *v, int64_t np, int64_t step,
             double lr, double beta1, double beta2, double eps);
/* Round to bfloat16 through float (round to nearest even). */
double orc_bf16(double x);

/* The 10 closure inputs at every cell centre: du/dx, du/dy, du/dz, dv/dx,
 * dv/dy, dv/dz, dw/dx, dw/dy, dw/dz, dtheta/dz; feat[n][10] (cell order). */
int orc_sgs_features(const orc_grid *g, const orc_state *S, double *feat);
/* Box filter by an integer factor r (nx, ny, nz divisible by r) onto the
 * coarse grid (dz summed over blocks): rho and rho*theta as block means, face
 * momenta as means over the r x r fine faces on each coarse face (conservative
 * restriction), and the SGS targets from cell-centre velocities and theta,
 * tau_ij = <u_i u_j> - <u_i><u_j> (11,22,33,12,13,23) and
 * q_j = <u_j theta> - <u_j><theta> (1,2,3), targets[nc][9].  With Cs > 0 the
 * block mean of the fine grid's own Smagorinsky stress and heat flux (built at
 * centres from the closure inputs, Prandtl number Pr_t) is added. */
int orc_box_filter(const orc_grid *g, const orc_state *S, int32_t r, double Cs, double Pr_t,
                   orc_state *coarse, double *targets);

/* Slow right-hand side with the learned closure in place of the Smagorinsky
 * stresses: the MLP gives kinematic tau_ij and q_j at cell centres; stresses
 * rho tau act on the staggered points by 4-cell (2-cell) averages; a cell falls
 * back to Smagorinsky when its output is not finite or its backscatter exceeds
 * twice the Smagorinsky dissipation.  norm = mean_x, std_x, mean_y, std_y.
 * P->sgs must be 2.  fallback_out (nullable) receives the number of fallback
 * cells. */
int orc_slow_rhs_mlp(const orc_grid *g, const orc_params *P, const orc_base *B, const orc_state *S,
                     const double *params, const double *norm, int bf16, orc_state *R, int64_t *fallback_out);

/* Kessler warm-rain microphysics (Sec. 2.4; the scheme of Kessler 1969 in the
 * form of Klemp & Wilhelmson 1978) over dt, after a dynamics step: rain
 * sedimentation, autoconversion, accretion, rain evaporation and the
 * saturation adjustment of cloud water, on scalars 0, 1, 2 = rho q_v, rho q_c,
 * rho q_r and rho theta (latent heat), in place.  precip [ny][nx] (may be
 * NULL) accumulates the rain mass reaching the ground [kg/m^2]. */
int orc_kessler(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S, double dt,
                double *precip);
/* Monin-Obukhov surface layer (Sec. 3.8): the friction velocity u_star for wind
 * speed U at height z1 over roughness z0 with kinematic surface heat flux Qs
 * and potential temperature th1 (Businger-Dyer stability functions). */
double orc_most_ustar(double U, double z1, double z0, double Qs, double th1, double grav);

/* saturation vapour pressure [Pa] over water and mixing ratio at (T, p) */
double orc_esat(double T);
double orc_qvsat(double T, double p);
/* the condensed amount of the saturation adjustment at fixed pressure */
double orc_sat_adjust(double T, double p, double qv, double qc);

/* ---------------- anelastic mode (Sec. 2.2, Sec. 3.2) ---------------- */
/* Discrete divergence of face momenta at the cell centres: the left side of
 * the constraint div(rho0 u) = 0, eq. (anelastic).  rw is zero on the lids. */
int orc_divergence(const orc_grid *g, const double *ru, const double *rv, const double *rw, double *D);
/* Poisson problem of the projection: L phi = D with L = D(G(.)) the C-grid
 * divergence of the face gradient (periodic in x and y, no flux through the
 * lids).  Solved by discrete Fourier transforms in x and y and a tridiagonal
 * solve per horizontal wavenumber in z.  The constant null space is fixed by
 * giving the horizontally uniform part of phi the value 0 in the lowest cell.
 * D must have zero volume-weighted sum (the divergence of lid-bounded face
 * fields has it). */
int orc_poisson(const orc_grid *g, const double *D, double *phi);
/* Projection (Sec. 3.2): solves L phi = div(rho u) with phi = dt psi,
 * subtracts grad phi from the face momenta (in place) and adds psi = phi / dt
 * to the perturbation pressure pp [nz][ny][nx] (NULL: not kept). */
int orc_project(const orc_grid *g, double *ru, double *rv, double *rw, double dt, double *pp);
/* One SSP-RK2 step of the anelastic equations with projections after each
 * stage (Sec. 3.2), in place; pp is the lagged perturbation pressure
 * [nz][ny][nx], updated in place.  S->rho must hold rho0 of each level. */
int orc_ssprk2_step(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S, double *pp);

#ifdef __cplusplus
}
#endif
#endif
