/*
 * erf_oracle.c -- plain FP64 CPU oracle of one RK3 step of ERF's compressible
 * dynamical core (Lattanzi et al., arXiv 2412.04395).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code
 * with the HIP library.  Written for obviousness, not speed: every operator is
 * a loop over the points it defines, neighbours are fetched through wrap /
 * reflection helpers, and temporaries are allocated per call.  Compiled with
 * -ffp-contract=off so that every product and sum is rounded as written.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include "erf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- constants.  Only P00 and gamma = c_p/(c_p - R_d) are printed in the
 * paper (Sec. 2.1); R_d and c_p take the usual dry-air values (reading). ---- */
static const double R_D = 287.0;
static const double C_P = 1004.5;
static const double P_00 = 1.0e5;
#define C_V (C_P - R_D)
#define GAM (C_P / (C_P - R_D))
/* gas constant of water vapour, the usual value (reading) */
static const double R_V = 461.6;
#define EPS_V (R_V / R_D)

double orc_const(int which)
{
    switch (which) {
    case 0: return R_D;
    case 1: return C_P;
    case 2: return C_V;
    case 3: return GAM;
    case 4: return P_00;
    case 5: return R_V;
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* indexing helpers                                                          */
/* ------------------------------------------------------------------------ */
static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* even reflection of a cell index about the bottom and top lids:
 * k = -1 -> 0, -2 -> 1, nz -> nz-1, ... (reading: ghost cells by reflection) */
static int refl_c(int k, int nz)
{
    int p = 2 * nz;
    int r = ((k % p) + p) % p;
    return r >= nz ? p - 1 - r : r;
}

#define CIDX(g, i, j, k) (((size_t)(k) * (size_t)(g)->ny + (size_t)(j)) * (size_t)(g)->nx + (size_t)(i))

/* centre (or horizontal-face) quantity: periodic in x and y, even in z */
static double cget(const orc_grid *g, const double *f, int i, int j, int k)
{
    return f[CIDX(g, wrap(i, g->nx), wrap(j, g->ny), refl_c(k, g->nz))];
}

/* z-face quantity: periodic in x and y, odd reflection about the lids */
static double wget(const orc_grid *g, const double *w, int i, int j, int k)
{
    int nz = g->nz, p = 2 * nz;
    int r = ((k % p) + p) % p;
    i = wrap(i, g->nx);
    j = wrap(j, g->ny);
    if (r <= nz) return w[CIDX(g, i, j, r)];
    return -w[CIDX(g, i, j, p - r)];
}

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* ------------------------------------------------------------------------ */
/* terrain-following coordinates (App. A, App. B)                             */
/* ------------------------------------------------------------------------ */
/* Node heights z = zeta + s(zeta) h(x, y) with s = (1 - zeta/z_t)^beta (the
 * canonical form of Sec. 3.4).  Readings: the flat grid's levels are
 * zeta_k = dz_0 + ... + dz_{k-1} and z_t = zeta_nz; a cell's physical height
 * is the mean of its four vertical edges, Hc = dz_k + (s_{k+1} - s_k) hbar
 * with hbar the mean of its four corner heights, and the Jacobian
 * h_zeta = Hc / dz_k; heights are kept as displacements from the flat grid so
 * that flat terrain gives dz, 1 and 0 exactly. */
typedef struct {
    int on;
    double *s;  /* nz + 1 node levels */
    double *hb; /* ny * nx, corner mean of h per column */
    double *Hc; /* nz * ny * nx */
} ter_t;

static double node_h(const orc_grid *g, int i, int j)
{
    return g->terrain[(size_t)wrap(j, g->ny) * g->nx + wrap(i, g->nx)];
}

static ter_t ter_build(const orc_grid *g)
{
    ter_t T = {0, NULL, NULL, NULL};
    if (!g->terrain) return T;
    int nx = g->nx, ny = g->ny, nz = g->nz;
    T.on = 1;
    T.s = dalloc((size_t)nz + 1);
    T.hb = dalloc((size_t)nx * ny);
    T.Hc = dalloc((size_t)nx * ny * nz);
    double zt = 0.0;
    for (int k = 0; k < nz; ++k) zt += g->dz[k];
    double zeta = 0.0;
    for (int k = 0; k <= nz; ++k) {
        T.s[k] = (k == nz) ? 0.0 : pow(1.0 - zeta / zt, g->terrain_beta);
        if (k < nz) zeta += g->dz[k];
    }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            T.hb[(size_t)j * nx + i] = 0.25 * ((node_h(g, i, j) + node_h(g, i + 1, j)) +
                                               (node_h(g, i, j + 1) + node_h(g, i + 1, j + 1)));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                T.Hc[CIDX(g, i, j, k)] = g->dz[k] + (T.s[k + 1] - T.s[k]) * T.hb[(size_t)j * nx + i];
    return T;
}

static void ter_free(ter_t *T)
{
    free(T->s); free(T->hb); free(T->Hc);
}

static double t_hb(const orc_grid *g, const ter_t *T, int i, int j)
{
    return T->hb[(size_t)wrap(j, g->ny) * g->nx + wrap(i, g->nx)];
}
/* physical cell height and Jacobian h_zeta at a cell (periodic in x, y) */
static double t_Hc(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    return T->on ? T->Hc[CIDX(g, wrap(i, g->nx), wrap(j, g->ny), k)] : g->dz[k];
}
static double t_J(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    return T->on ? t_Hc(g, T, i, j, k) / g->dz[k] : 1.0;
}
/* h_zeta on the x-face i (between cells i-1 and i) and on the y-face j */
static double t_JU(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    return T->on ? 0.5 * (t_J(g, T, i - 1, j, k) + t_J(g, T, i, j, k)) : 1.0;
}
static double t_JV(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    return T->on ? 0.5 * (t_J(g, T, i, j - 1, k) + t_J(g, T, i, j, k)) : 1.0;
}
/* h_xi on the x-face i at level k: the difference of the two cells' centre
 * heights over dx (App. B, second order); h_eta on the y-face j likewise */
static double t_hxU(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    if (!T->on) return 0.0;
    return 0.5 * (T->s[k] + T->s[k + 1]) * (t_hb(g, T, i, j) - t_hb(g, T, i - 1, j)) / g->dx;
}
static double t_heV(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    if (!T->on) return 0.0;
    return 0.5 * (T->s[k] + T->s[k + 1]) * (t_hb(g, T, i, j) - t_hb(g, T, i, j - 1)) / g->dy;
}
/* h_xi and h_eta on the z-face (i, j, k): the fourth-order centred difference
 * of the face-centre heights (the mean of the face's four nodes) (App. B) */
static double t_hxW(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    if (!T->on) return 0.0;
    return T->s[k] * ((t_hb(g, T, i - 2, j) - t_hb(g, T, i + 2, j)) + 8.0 * (t_hb(g, T, i + 1, j) - t_hb(g, T, i - 1, j))) /
           (12.0 * g->dx);
}
static double t_heW(const orc_grid *g, const ter_t *T, int i, int j, int k)
{
    if (!T->on) return 0.0;
    return T->s[k] * ((t_hb(g, T, i, j - 2) - t_hb(g, T, i, j + 2)) + 8.0 * (t_hb(g, T, i, j + 1) - t_hb(g, T, i, j - 1))) /
           (12.0 * g->dy);
}
/* rho Omega on the z-face (i, j, k), the momentum normal to the face (App. A):
 * rho w - h_xi (rho u) - h_eta (rho v), the horizontal momenta averaged from the
 * four x-faces (y-faces) around the face (App. B); the lid faces keep rho w */
static double t_M(const orc_grid *g, const ter_t *T, const double *ru, const double *rv, int i, int j, int k)
{
    if (!T->on || k == 0 || k == g->nz) return 0.0;
    double su = (cget(g, ru, i, j, k) + cget(g, ru, i + 1, j, k)) + (cget(g, ru, i, j, k - 1) + cget(g, ru, i + 1, j, k - 1));
    double sv = (cget(g, rv, i, j, k) + cget(g, rv, i, j + 1, k)) + (cget(g, rv, i, j, k - 1) + cget(g, rv, i, j + 1, k - 1));
    return 0.25 * t_hxW(g, T, i, j, k) * su + 0.25 * t_heW(g, T, i, j, k) * sv;
}
static double t_rOm(const orc_grid *g, const ter_t *T, const double *ru, const double *rv, const double *rw,
                    int i, int j, int k)
{
    double W = rw[CIDX(g, wrap(i, g->nx), wrap(j, g->ny), k)];
    if (!T->on || k == 0 || k == g->nz) return W;
    return W - t_M(g, T, ru, rv, i, j, k);
}
/* (f_zeta / h_zeta) at a cell: the centred difference of f over the physical
 * distance of the centres above and below (App. B); one-sided in the lowest
 * and highest cells (reading), zero in a single-level column */
static double t_fz(const orc_grid *g, const ter_t *T, const double *f, int i, int j, int k)
{
    int nz = g->nz;
    if (nz < 2) return 0.0;
    int kl = k > 0 ? k - 1 : 0, ku = k < nz - 1 ? k + 1 : nz - 1;
    double dzc = 0.5 * t_Hc(g, T, i, j, kl) + 0.5 * t_Hc(g, T, i, j, ku);
    for (int m = kl + 1; m < ku; ++m) dzc += t_Hc(g, T, i, j, m);
    return (cget(g, f, i, j, ku) - cget(g, f, i, j, kl)) / dzc;
}

int orc_terrain_heights(const orc_grid *g, double *Hc, double *zc)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (nx < 1 || ny < 1 || nz < 1 || !g->dz) return -1;
    ter_t T = ter_build(g);
    double zeta = 0.0;
    for (int k = 0; k < nz; ++k) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                if (Hc) Hc[c] = t_Hc(g, &T, i, j, k);
                if (zc) zc[c] = (zeta + 0.5 * g->dz[k]) + (T.on ? 0.5 * (T.s[k] + T.s[k + 1]) * t_hb(g, &T, i, j) : 0.0);
            }
        zeta += g->dz[k];
    }
    ter_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* equation of state, Sec. 2.1                                               */
/* ------------------------------------------------------------------------ */
double orc_eos_p(double Theta) { return P_00 * pow(R_D * Theta / P_00, GAM); }

/* p' = p(Theta) - p0 with p0 = p(Theta0).  Since p/p0 = (Theta/Theta0)^gamma,
 * p' = p0 ((1 + Theta'/Theta0)^gamma - 1), evaluated with log1p/expm1 so that a
 * small perturbation is not lost to cancellation against 1e5 Pa. */
double orc_eos_pprime(double Theta, double Theta0, double p0)
{
    return p0 * expm1(GAM * log1p((Theta - Theta0) / Theta0));
}

/* Exner function pi = (p/P00)^(R_d/c_p) = (R_d Theta / P00)^(gamma - 1). */
static double exner(double Theta) { return pow(R_D * Theta / P_00, GAM - 1.0); }

/* Moist EOS of Sec. 2.1: water vapour enters through the factor
 * 1 + (R_v/R_d) q_v on rho_d theta_d, so every dry formula applies to
 * Theta (1 + R_v/R_d q_v).  With q_v = 0 the factor is exactly 1. */
double orc_eos_p_moist(double Theta, double qv) { return orc_eos_p(Theta * (1.0 + EPS_V * qv)); }

/* p' = p(Theta, q_v) - p(Theta0, q_v0).  With X = Theta (1 + eps q_v) and
 * X0 = Theta0 (1 + eps q_v0), p/p0 = (X/X0)^gamma and
 * X - X0 = (Theta - Theta0)(1 + eps q_v) + eps Theta0 (q_v - q_v0), an exact
 * rewriting that keeps the small differences apart from the large values. */
double orc_eos_pprime_moist(double Theta, double qv, double Theta0, double qv0, double p0)
{
    double x = ((Theta - Theta0) * (1.0 + EPS_V * qv) + EPS_V * Theta0 * (qv - qv0)) / (Theta0 * (1.0 + EPS_V * qv0));
    return p0 * expm1(GAM * log1p(x));
}

/* ------------------------------------------------------------------------ */
/* base state: dp0/dz = -rho0 g and p0 = EOS(rho0 theta0) (Sec. 2, Sec. 3.8) */
/* ------------------------------------------------------------------------ */
/* reading: between level centres the hydrostatic relation is discretised with
 * the trapezoidal density, p_k - p_{k-1} = -g dzf_k (rho_k + rho_{k-1})/2, and
 * the lowest centre sits dz_0/2 above the surface where p = p_surface.  Each
 * level is one scalar Newton-Raphson root find for rho_k. */
int orc_base_state(int32_t nz, const double *dz, const double *theta0, double p_surface,
                   double grav, double *rho0, double *p0, double *pi0)
{
    return orc_base_state_moist(nz, dz, theta0, NULL, p_surface, grav, rho0, p0, pi0);
}

/* reading (moist, Sec. 2 and Sec. 3.8): rho0 is the dry density; the column
 * weighs rho0 (1 + q_v0) and the pressure is the moist EOS of rho0 theta0 and
 * q_v0.  With q_v0 = 0 (or NULL) every factor is exactly 1 and the dry state
 * is reproduced bit for bit. */
int orc_base_state_moist(int32_t nz, const double *dz, const double *theta0, const double *qv0,
                         double p_surface, double grav, double *rho0, double *p0, double *pi0)
{
    if (nz < 1 || !dz || !theta0 || !rho0 || !p0) return -1;
    double p_below = p_surface, rho_below = 0.0, q_below = 0.0;
    for (int k = 0; k < nz; ++k) {
        double q = qv0 ? qv0[k] : 0.0;
        if (!(q >= 0.0)) return -1;
        double h = (k == 0) ? 0.5 * dz[0] : 0.5 * (dz[k - 1] + dz[k]);
        double rho = (k == 0) ? p_surface / (R_D * theta0[0] * (1.0 + EPS_V * q)) : rho_below;
        for (int it = 0; it < 30; ++it) {
            double p = orc_eos_p_moist(rho * theta0[k], q);
            double f, df;
            if (k == 0) {
                f = p - p_below + grav * h * (rho * (1.0 + q));
                df = GAM * p / rho + grav * h * (1.0 + q);
            } else {
                f = p - p_below + grav * h * 0.5 * (rho * (1.0 + q) + rho_below * (1.0 + q_below));
                df = GAM * p / rho + grav * h * 0.5 * (1.0 + q);
            }
            double d = f / df;
            rho = rho - d;
            if (fabs(d) <= 1e-15 * rho) break;
        }
        rho0[k] = rho;
        p0[k] = orc_eos_p_moist(rho * theta0[k], q);
        if (pi0) pi0[k] = pow(p0[k] / P_00, R_D / C_P);
        p_below = p0[k];
        rho_below = rho;
        q_below = q;
    }
    return 0;
}

/* reading (terrain, App. A): the base state is hydrostatic in every column,
 * along the column's physical cell heights, from the pressure at its ground */
int orc_base_state_columns(const orc_grid *g, const double *theta0, const double *p_surf, double grav,
                           double *rho0, double *p0, double *pi0)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (nx < 1 || ny < 1 || nz < 1 || !theta0 || !p_surf || !rho0 || !p0 || !pi0) return -1;
    ter_t T = ter_build(g);
    double *dzc = dalloc(nz), *th = dalloc(nz), *r = dalloc(nz), *p = dalloc(nz), *pi = dalloc(nz);
    int rc = 0;
    for (int j = 0; j < ny && rc == 0; ++j)
        for (int i = 0; i < nx && rc == 0; ++i) {
            for (int k = 0; k < nz; ++k) {
                dzc[k] = t_Hc(g, &T, i, j, k);
                th[k] = theta0[CIDX(g, i, j, k)];
            }
            rc = orc_base_state_moist(nz, dzc, th, NULL, p_surf[(size_t)j * nx + i], grav, r, p, pi);
            for (int k = 0; k < nz; ++k) {
                size_t c = CIDX(g, i, j, k);
                rho0[c] = r[k];
                p0[c] = p[k];
                pi0[c] = pi[k];
            }
        }
    free(dzc); free(th); free(r); free(p); free(pi);
    ter_free(&T);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* interpolants of Sec. 3.6                                                  */
/* ------------------------------------------------------------------------ */
/* q6 = {q_{m-3}, q_{m-2}, q_{m-1}, q_m, q_{m+1}, q_{m+2}}; returns q_{m-1/2}.
 * sgn is the sign of the normal momentum at the face (reading of sign(u_m)). */
double orc_interp(int32_t order, const double *q6, double s)
{
    double qm3 = q6[0], qm2 = q6[1], qm1 = q6[2], q0 = q6[3], qp1 = q6[4], qp2 = q6[5];
    double c4 = 7.0 / 12.0 * (q0 + qm1) - 1.0 / 12.0 * (qp1 + qm2);
    double c6 = 37.0 / 60.0 * (q0 + qm1) - 2.0 / 15.0 * (qp1 + qm2) + 1.0 / 60.0 * (qp2 + qm3);
    switch (order) {
    case 2: return 0.5 * (q0 + qm1);
    case 3: return c4 + s / 12.0 * ((qp1 - qm2) - 3.0 * (q0 - qm1));
    case 4: return c4;
    case 5: return c6 - s / 60.0 * ((qp2 - qm3) - 5.0 * (qp1 - qm2) + 10.0 * (q0 - qm1));
    case 6: return c6;
    default: return NAN;
    }
}

/* WENO5-JS (Jiang & Shu 1996, cited in Sec. 3.6): linear weights 0.1/0.6/0.3,
 * smoothness indicators of the three 3-point candidate stencils, power 2.
 * For positive flow the stencil is q_{m-3}..q_{m+1} (upwind cell m-1); for
 * negative flow it is mirrored. */
double orc_weno5(const double *q6, double s, double eps)
{
    double v0, v1, v2, v3, v4; /* v2 is the upwind cell */
    if (s >= 0.0) {
        v0 = q6[0]; v1 = q6[1]; v2 = q6[2]; v3 = q6[3]; v4 = q6[4];
    } else {
        v0 = q6[5]; v1 = q6[4]; v2 = q6[3]; v3 = q6[2]; v4 = q6[1];
    }
    double p0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) / 6.0;
    double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) / 6.0;
    double p2 = (2.0 * v2 + 5.0 * v3 - v4) / 6.0;
    double b0 = 13.0 / 12.0 * (v0 - 2.0 * v1 + v2) * (v0 - 2.0 * v1 + v2)
              + 0.25 * (v0 - 4.0 * v1 + 3.0 * v2) * (v0 - 4.0 * v1 + 3.0 * v2);
    double b1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - v3) * (v1 - v3);
    double b2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (3.0 * v2 - 4.0 * v3 + v4) * (3.0 * v2 - 4.0 * v3 + v4);
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

static const double WENO_EPS = 1.0e-6; /* reading: the usual JS regulariser */

/* ------------------------------------------------------------------------ */
/* Thomas algorithm (no pivoting)                                            */
/* ------------------------------------------------------------------------ */
int orc_thomas(int32_t n, const double *a, const double *b, const double *c,
               const double *r, double *x)
{
    if (n < 1) return 0;
    double cp[n], dp[n];
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* primitive variables                                                       */
/* ------------------------------------------------------------------------ */
/* reading: velocities are momenta divided by the arithmetic mean of the two
 * densities on either side of the face (index space). */
static void primitives(const orc_grid *g, const orc_state *S, double *th, double *u, double *v,
                       double *w)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                th[c] = S->rt[c] / S->rho[c];
                u[c] = S->ru[c] / (0.5 * (cget(g, S->rho, i - 1, j, k) + S->rho[c]));
                v[c] = S->rv[c] / (0.5 * (cget(g, S->rho, i, j - 1, k) + S->rho[c]));
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                if (k == 0 || k == nz)
                    w[c] = 0.0;
                else
                    w[c] = S->rw[c] / (0.5 * (S->rho[CIDX(g, i, j, k - 1)] + S->rho[CIDX(g, i, j, k)]));
            }
}

/* face value q_{m-1/2} along x of a centre-located (or y-face / z-face-in-x)
 * field f, m = i, evaluated with the given order and upwind sign */
static double ix(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = cget(g, f, i - 3 + o, j, k);
    return orc_interp(order, q, s);
}
static double iy(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = cget(g, f, i, j - 3 + o, k);
    return orc_interp(order, q, s);
}
/* along z for centre-located / horizontal-face fields (even ghosts) */
static double izc(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = cget(g, f, i, j, k - 3 + o);
    return orc_interp(order, q, s);
}
/* along z for z-face fields (odd ghosts) */
static double izw(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = wget(g, f, i, j, k - 3 + o);
    return orc_interp(order, q, s);
}
/* a z-face field read at a given face along x (periodic, no vertical ghost) */
static double ixw(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = wget(g, f, i - 3 + o, j, k);
    return orc_interp(order, q, s);
}
static double iyw(const orc_grid *g, const double *f, int i, int j, int k, int order, double s)
{
    double q[6];
    for (int o = 0; o < 6; ++o) q[o] = wget(g, f, i, j - 3 + o, k);
    return orc_interp(order, q, s);
}

/* ------------------------------------------------------------------------ */
/* Monin-Obukhov surface layer (Sec. 3.8)                                    */
/* ------------------------------------------------------------------------ */
/* reading: von Karman constant 0.4; Businger-Dyer stability function for
 * momentum, psi_m = 2 ln((1+x)/2) + ln((1+x^2)/2) - 2 atan(x) + pi/2 with
 * x = (1 - 16 zeta)^(1/4) for zeta < 0 and psi_m = -5 zeta for zeta >= 0;
 * zeta = z1/L with L = -u_star^3 theta_1 / (kappa g Qs), clamped to [-5, 1]; u_star
 * from the log law U = (u_star / kappa)(ln(z1/z0) - psi_m(zeta)) by twenty fixed-point
 * steps from the neutral value. */
static const double KARMAN = 0.4;
static double psi_m(double zeta)
{
    if (zeta >= 0.0) return -5.0 * zeta;
    double x = pow(1.0 - 16.0 * zeta, 0.25);
    return 2.0 * log(0.5 * (1.0 + x)) + log(0.5 * (1.0 + x * x)) - 2.0 * atan(x) + 2.0 * atan(1.0);
}

double orc_most_ustar(double U, double z1, double z0, double Qs, double th1, double grav)
{
    double lnz = log(z1 / z0);
    double ust = KARMAN * U / lnz;
    for (int it = 0; it < 20; ++it) {
        double zeta = 0.0;
        if (Qs != 0.0) {
            zeta = -z1 * KARMAN * grav * Qs / (ust * ust * ust * th1);
            if (zeta < -5.0) zeta = -5.0;
            if (zeta > 1.0) zeta = 1.0;
        }
        ust = KARMAN * U / (lnz - psi_m(zeta));
    }
    return ust;
}

/* ------------------------------------------------------------------------ */
/* stress tensor and heat flux, eq. (stresstensor), Sec. 2.3                 */
/* ------------------------------------------------------------------------ */
/* reading: tau = -2 mu (S - D), mu = rho nu_m + rho (Cs Delta)^2 |S| with
 * Delta = (dx dy dz)^(1/3) and |S| = sqrt(2 S:S).  Diagonal strain at cell
 * centres, off-diagonal strain on cell edges, mu averaged from the four cells
 * around an edge.  Heat diffusivity rho alpha_m + mu_t / Pr_t.  Free-slip lids:
 * S13 = S23 = 0 on the bottom and top faces. */
static void add_diffusion(const orc_grid *g, const orc_params *P, const orc_base *B, const orc_state *S,
                          const double *th, const double *u, const double *v, const double *w,
                          orc_state *R)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    double dx = g->dx, dy = g->dy;
    const double *dz = g->dz;
    double *s11 = dalloc(n), *s22 = dalloc(n), *s33 = dalloc(n);
    double *s12 = dalloc(n), *s13 = dalloc(nw), *s23 = dalloc(nw);
    double *mu = dalloc(n), *kh = dalloc(n);
    /* Deardorff closure: e (clipped at zero), rho K_m and the local part of the
     * source of rho e */
    double *ee = dalloc(n), *rkm = dalloc(n), *esrc = dalloc(n);

    /* strain rates */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                s11[c] = (cget(g, u, i + 1, j, k) - u[c]) / dx;
                s22[c] = (cget(g, v, i, j + 1, k) - v[c]) / dy;
                s33[c] = (w[CIDX(g, i, j, k + 1)] - w[c]) / dz[k];
                /* S12 on the edge of x-face i and y-face j */
                s12[c] = 0.5 * ((u[c] - cget(g, u, i, j - 1, k)) / dy + (v[c] - cget(g, v, i - 1, j, k)) / dx);
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                if (k == 0 || k == nz) {
                    s13[c] = 0.0;
                    s23[c] = 0.0;
                } else {
                    double dzf = 0.5 * (dz[k - 1] + dz[k]);
                    s13[c] = 0.5 * ((u[c] - u[CIDX(g, i, j, k - 1)]) / dzf + (w[c] - wget(g, w, i - 1, j, k)) / dx);
                    s23[c] = 0.5 * ((v[c] - v[CIDX(g, i, j, k - 1)]) / dzf + (w[c] - wget(g, w, i, j - 1, k)) / dy);
                }
            }
    /* viscosity and diffusivity at centres */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double mut = 0.0;
                if (P->sgs == 1) {
                    double a12 = 0.25 * (s12[c] + cget(g, s12, i + 1, j, k) + cget(g, s12, i, j + 1, k) + cget(g, s12, i + 1, j + 1, k));
                    double a13 = 0.25 * (s13[c] + wget(g, s13, i + 1, j, k) + s13[CIDX(g, i, j, k + 1)] + wget(g, s13, i + 1, j, k + 1));
                    double a23 = 0.25 * (s23[c] + wget(g, s23, i, j + 1, k) + s23[CIDX(g, i, j, k + 1)] + wget(g, s23, i, j + 1, k + 1));
                    double ss = 2.0 * (s11[c] * s11[c] + s22[c] * s22[c] + s33[c] * s33[c])
                              + 4.0 * (a12 * a12 + a13 * a13 + a23 * a23);
                    double delta = cbrt(dx * dy * dz[k]);
                    double cd = P->Cs * delta;
                    mut = S->rho[c] * cd * cd * sqrt(ss);
                }
                double khs = P->sgs == 1 ? mut / P->Pr_t : 0.0;
                if (P->sgs == 3) {
                    /* Deardorff (1980) 1.5-order closure, the coefficients of
                     * Moeng (1984) (Sec. 2.3 and the LES cases of Sec. 4):
                     * length l = Delta, or 0.76 sqrt(e)/N where that is
                     * smaller in stable air; K_m = 0.1 l sqrt(e);
                     * K_h = (1 + 2 l/Delta) K_m; production K_m 2 S:S
                     * - K_h N^2; dissipation C_eps e^(3/2)/l with
                     * C_eps = 0.19 + 0.51 l/Delta.  N^2 = g/theta0 dtheta/dz,
                     * dtheta/dz the mean of the two face differences (zero
                     * through the lids). */
                    double a12 = 0.25 * (s12[c] + cget(g, s12, i + 1, j, k) + cget(g, s12, i, j + 1, k) + cget(g, s12, i + 1, j + 1, k));
                    double a13 = 0.25 * (s13[c] + wget(g, s13, i + 1, j, k) + s13[CIDX(g, i, j, k + 1)] + wget(g, s13, i + 1, j, k + 1));
                    double a23 = 0.25 * (s23[c] + wget(g, s23, i, j + 1, k) + s23[CIDX(g, i, j, k + 1)] + wget(g, s23, i, j + 1, k + 1));
                    double ss = 2.0 * (s11[c] * s11[c] + s22[c] * s22[c] + s33[c] * s33[c])
                              + 4.0 * (a12 * a12 + a13 * a13 + a23 * a23);
                    double e = S->rq[c] / S->rho[c];
                    if (e < 0.0) e = 0.0;
                    double up = k < nz - 1 ? (th[CIDX(g, i, j, k + 1)] - th[c]) / (0.5 * (dz[k] + dz[k + 1])) : 0.0;
                    double dn = k > 0 ? (th[c] - th[CIDX(g, i, j, k - 1)]) / (0.5 * (dz[k - 1] + dz[k])) : 0.0;
                    double N2 = P->grav / B->theta0[k] * 0.5 * (up + dn);
                    double delta = cbrt(dx * dy * dz[k]);
                    double l = delta, eps;
                    int limited = N2 > 0.0 && 0.76 * sqrt(e) / sqrt(N2) < delta;
                    if (limited) l = 0.76 * sqrt(e) / sqrt(N2);
                    double Km = 0.1 * l * sqrt(e), Kh = (1.0 + 2.0 * l / delta) * Km;
                    double ceps = 0.19 + 0.51 * l / delta;
                    /* e^(3/2)/l, written as e N/0.76 where l is the stable length */
                    eps = limited ? ceps * e * sqrt(N2) / 0.76 : ceps * e * sqrt(e) / delta;
                    mut = S->rho[c] * Km;
                    khs = S->rho[c] * Kh;
                    ee[c] = e;
                    rkm[c] = mut;
                    esrc[c] = S->rho[c] * (Km * ss - Kh * N2 - eps);
                }
                mu[c] = S->rho[c] * P->nu_m + mut;
                kh[c] = S->rho[c] * P->alpha_m + khs;
            }
    if (P->sgs == 3) {
        /* source of rho e: the local terms plus the diffusion div(2 rho K_m
         * grad e), face coefficients the mean of the two cells, no flux
         * through the lids */
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = CIDX(g, i, j, k);
                    double fx0 = -(cget(g, rkm, i - 1, j, k) + rkm[c]) * (ee[c] - cget(g, ee, i - 1, j, k)) / dx;
                    double fx1 = -(rkm[c] + cget(g, rkm, i + 1, j, k)) * (cget(g, ee, i + 1, j, k) - ee[c]) / dx;
                    double fy0 = -(cget(g, rkm, i, j - 1, k) + rkm[c]) * (ee[c] - cget(g, ee, i, j - 1, k)) / dy;
                    double fy1 = -(rkm[c] + cget(g, rkm, i, j + 1, k)) * (cget(g, ee, i, j + 1, k) - ee[c]) / dy;
                    double fz0 = 0.0, fz1 = 0.0;
                    if (k > 0)
                        fz0 = -(rkm[CIDX(g, i, j, k - 1)] + rkm[c]) * (ee[c] - ee[CIDX(g, i, j, k - 1)]) / (0.5 * (dz[k - 1] + dz[k]));
                    if (k < nz - 1)
                        fz1 = -(rkm[c] + rkm[CIDX(g, i, j, k + 1)]) * (ee[CIDX(g, i, j, k + 1)] - ee[c]) / (0.5 * (dz[k] + dz[k + 1]));
                    R->rq[c] = esrc[c] - ((fx1 - fx0) / dx + (fy1 - fy0) / dy + (fz1 - fz0) / dz[k]);
                }
    }

    /* stress components: tau_ii at centres, tau_12 at xy-edges, tau_13/23 at z-face edges */
    double *t11 = dalloc(n), *t22 = dalloc(n), *t33 = dalloc(n), *t12 = dalloc(n);
    double *t13 = dalloc(nw), *t23 = dalloc(nw);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double d = (s11[c] + s22[c] + s33[c]) / 3.0;
                t11[c] = -2.0 * mu[c] * (s11[c] - d);
                t22[c] = -2.0 * mu[c] * (s22[c] - d);
                t33[c] = -2.0 * mu[c] * (s33[c] - d);
                double me = 0.25 * (cget(g, mu, i - 1, j - 1, k) + cget(g, mu, i, j - 1, k) + cget(g, mu, i - 1, j, k) + mu[c]);
                t12[c] = -2.0 * me * s12[c];
            }
    if (P->most_z0 > 0.0) {
        /* surface stresses of the Monin-Obukhov layer on the bottom faces:
         * per column -rho u_star^2 (u, v)/U from the lowest cell's centre wind
         * (reading: U at least 0.1 m/s), on each face edge the mean of the two
         * columns beside it */
        double *c13 = dalloc((size_t)nx * ny), *c23 = dalloc((size_t)nx * ny);
        double z1 = 0.5 * dz[0];
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, 0);
                double u1 = 0.5 * (u[c] + cget(g, u, i + 1, j, 0));
                double v1 = 0.5 * (v[c] + cget(g, v, i, j + 1, 0));
                double U = sqrt(u1 * u1 + v1 * v1);
                if (U < 0.1) U = 0.1;
                double ust = orc_most_ustar(U, z1, P->most_z0, P->surf_heat_flux, th[c], P->grav);
                c13[c] = -S->rho[c] * ust * ust * u1 / U;
                c23[c] = -S->rho[c] * ust * ust * v1 / U;
            }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, 0);
                t13[c] = 0.5 * (cget(g, c13, i - 1, j, 0) + c13[c]);
                t23[c] = 0.5 * (cget(g, c23, i, j - 1, 0) + c23[c]);
            }
        free(c13);
        free(c23);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double mxz = 0.25 * (cget(g, mu, i - 1, j, k - 1) + cget(g, mu, i, j, k - 1) + cget(g, mu, i - 1, j, k) + cget(g, mu, i, j, k));
                double myz = 0.25 * (cget(g, mu, i, j - 1, k - 1) + cget(g, mu, i, j, k - 1) + cget(g, mu, i, j - 1, k) + cget(g, mu, i, j, k));
                t13[c] = -2.0 * mxz * s13[c];
                t23[c] = -2.0 * myz * s23[c];
            }

    /* R += -div(tau) on each momentum face; R_Theta += div(K grad theta) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                R->ru[c] -= (t11[c] - cget(g, t11, i - 1, j, k)) / dx
                          + (cget(g, t12, i, j + 1, k) - t12[c]) / dy
                          + (t13[CIDX(g, i, j, k + 1)] - t13[c]) / dz[k];
                R->rv[c] -= (cget(g, t12, i + 1, j, k) - t12[c]) / dx
                          + (t22[c] - cget(g, t22, i, j - 1, k)) / dy
                          + (t23[CIDX(g, i, j, k + 1)] - t23[c]) / dz[k];
                /* heat: upward/rightward diffusive flux H = -K dtheta/dn */
                double hx0 = -0.5 * (cget(g, kh, i - 1, j, k) + kh[c]) * (th[c] - cget(g, th, i - 1, j, k)) / dx;
                double hx1 = -0.5 * (kh[c] + cget(g, kh, i + 1, j, k)) * (cget(g, th, i + 1, j, k) - th[c]) / dx;
                double hy0 = -0.5 * (cget(g, kh, i, j - 1, k) + kh[c]) * (th[c] - cget(g, th, i, j - 1, k)) / dy;
                double hy1 = -0.5 * (kh[c] + cget(g, kh, i, j + 1, k)) * (cget(g, th, i, j + 1, k) - th[c]) / dy;
                double hz0 = 0.0, hz1 = 0.0;
                if (k > 0)
                    hz0 = -0.5 * (kh[CIDX(g, i, j, k - 1)] + kh[c]) * (th[c] - th[CIDX(g, i, j, k - 1)]) / (0.5 * (dz[k - 1] + dz[k]));
                if (k < nz - 1)
                    hz1 = -0.5 * (kh[c] + kh[CIDX(g, i, j, k + 1)]) * (th[CIDX(g, i, j, k + 1)] - th[c]) / (0.5 * (dz[k] + dz[k + 1]));
                R->rt[c] -= (hx1 - hx0) / dx + (hy1 - hy0) / dy + (hz1 - hz0) / dz[k];
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double dzf = 0.5 * (dz[k - 1] + dz[k]);
                R->rw[c] -= (wget(g, t13, i + 1, j, k) - t13[c]) / dx
                          + (wget(g, t23, i, j + 1, k) - t23[c]) / dy
                          + (t33[c] - t33[CIDX(g, i, j, k - 1)]) / dzf;
            }
    free(s11); free(s22); free(s33); free(s12); free(s13); free(s23);
    free(mu); free(kh); free(t11); free(t22); free(t33); free(t12); free(t13); free(t23);
    free(ee); free(rkm); free(esrc);
}

/* ------------------------------------------------------------------------ */
/* slow right-hand side                                                      */
/* ------------------------------------------------------------------------ */
int orc_slow_rhs_mlp(const orc_grid *g, const orc_params *P, const orc_base *B, const orc_state *S,
                     const double *params, const double *norm, int bf16, orc_state *R, int64_t *fallback_out);

int orc_slow_rhs(const orc_grid *g, const orc_params *P, const orc_base *B,
                 const orc_state *S, orc_state *R)
{
    if (P->anelastic && (P->moist || P->sgs == 2 || P->sgs == 3 || !P->p_anel)) return -1;
    if (g->terrain && (P->moist || P->anelastic || P->sgs != 0 || P->nu_m != 0.0 || P->alpha_m != 0.0 ||
                       P->most_z0 > 0.0))
        return -1;
    /* the Deardorff closure carries rho e as scalar 0 and nothing else */
    if (P->sgs == 3 && (P->n_scalars != 1 || P->moist || !S->rq || !R->rq)) return -1;
    if (P->most_z0 < 0.0 || (P->most_z0 > 0.0 && !(P->most_z0 < 0.5 * g->dz[0]))) return -1;
    if (P->sgs == 2) {
        if (!P->mlp_params || !P->mlp_norm) return -1;
        return orc_slow_rhs_mlp(g, P, B, S, P->mlp_params, P->mlp_norm, P->mlp_bf16, R, NULL);
    }
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (nx < 1 || ny < 1 || nz < 1) return -2;
    int oh = P->adv_order_h, ov = P->adv_order_v;
    if (oh < 2 || oh > 6 || ov < 2 || ov > 6) return -1;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    double dx = g->dx, dy = g->dy, gr = P->grav;
    const double *dz = g->dz;
    int moist = P->moist != 0;
    if (moist && (P->n_scalars < 3 || !S->rq)) return -1;
    double *th = dalloc(n), *u = dalloc(n), *v = dalloc(n), *w = dalloc(nw), *pp = dalloc(n);
    /* moist: 1 + q_v + q_c (divides the pressure gradient and the buoyancy,
     * eq. (mom)) and the departure of the total density rho_d (1 + q_v + q_c
     * + q_r) from the base state's rho0 (1 + q_v0) (the buoyancy) */
    double *qf = moist ? dalloc(n) : NULL, *bm = moist ? dalloc(n) : NULL;
    primitives(g, S, th, u, v, w);
    ter_t T = ter_build(g);
    for (int k = 0; k < nz; ++k) {
        double qv0 = B->qv0 ? B->qv0[k] : 0.0;
        for (size_t c = (size_t)k * nx * ny; c < (size_t)(k + 1) * nx * ny; ++c) {
            size_t kb = T.on ? c : (size_t)k; /* base state per cell with terrain */
            double T0 = B->rho0[kb] * B->theta0[kb];
            if (moist) {
                double rqv = S->rq[c], rqc = S->rq[n + c], rqr = S->rq[2 * n + c];
                double qv = rqv / S->rho[c], qc = rqc / S->rho[c];
                pp[c] = orc_eos_pprime_moist(S->rt[c], qv, T0, qv0, B->p0[k]);
                qf[c] = 1.0 + qv + qc;
                bm[c] = (S->rho[c] - B->rho0[k]) + (rqv + rqc + rqr) - B->rho0[k] * qv0;
            } else if (P->anelastic) {
                /* anelastic: the pressure perturbation is the one the
                 * projections left, not a function of the state (Sec. 2.2) */
                pp[c] = P->p_anel[c];
            } else {
                pp[c] = orc_eos_pprime(S->rt[c], T0, B->p0[kb]);
            }
        }
    }

    /* --- continuity and potential temperature, eqs. (con), (theta) --- */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                /* terrain (App. A): h_zeta-weighted horizontal fluxes, rho Omega
                 * on the z-faces, the divergence divided by the cell's h_zeta */
                double U0 = t_JU(g, &T, i, j, k) * S->ru[c], U1 = t_JU(g, &T, i + 1, j, k) * cget(g, S->ru, i + 1, j, k);
                double V0 = t_JV(g, &T, i, j, k) * S->rv[c], V1 = t_JV(g, &T, i, j + 1, k) * cget(g, S->rv, i, j + 1, k);
                double W0 = t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k), W1 = t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k + 1);
                double Jc = t_J(g, &T, i, j, k);
                R->rho[c] = -((U1 - U0) / dx + (V1 - V0) / dy + (W1 - W0) / dz[k]) / Jc;
                double fx0 = U0 * ix(g, th, i, j, k, oh, sgn(U0));
                double fx1 = U1 * ix(g, th, i + 1, j, k, oh, sgn(U1));
                double fy0 = V0 * iy(g, th, i, j, k, oh, sgn(V0));
                double fy1 = V1 * iy(g, th, i, j + 1, k, oh, sgn(V1));
                double fz0 = (k == 0) ? 0.0 : W0 * izc(g, th, i, j, k, ov, sgn(W0));
                double fz1 = (k == nz - 1) ? 0.0 : W1 * izc(g, th, i, j, k + 1, ov, sgn(W1));
                R->rt[c] = -((fx1 - fx0) / dx + (fy1 - fy0) / dy + (fz1 - fz0) / dz[k]) / Jc;
            }

    /* --- x-momentum on x-faces, eq. (mom) --- */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                /* xx-flux at the centres right (i) and left (i-1) of the face */
                /* terrain: the mass fluxes carry h_zeta (rho Omega vertically)
                 * and the divergence is divided by h_zeta of the x-face */
                double a_r = 0.5 * (t_JU(g, &T, i, j, k) * S->ru[c] + t_JU(g, &T, i + 1, j, k) * cget(g, S->ru, i + 1, j, k));
                double a_l = 0.5 * (t_JU(g, &T, i - 1, j, k) * cget(g, S->ru, i - 1, j, k) + t_JU(g, &T, i, j, k) * S->ru[c]);
                double fxx_r = a_r * ix(g, u, i + 1, j, k, oh, sgn(a_r));
                double fxx_l = a_l * ix(g, u, i, j, k, oh, sgn(a_l));
                /* xy-flux on the edges at y-faces j and j+1 */
                double b_0 = 0.5 * (t_JV(g, &T, i - 1, j, k) * cget(g, S->rv, i - 1, j, k) + t_JV(g, &T, i, j, k) * S->rv[c]);
                double b_1 = 0.5 * (t_JV(g, &T, i - 1, j + 1, k) * cget(g, S->rv, i - 1, j + 1, k) +
                                    t_JV(g, &T, i, j + 1, k) * cget(g, S->rv, i, j + 1, k));
                double fxy0 = b_0 * iy(g, u, i, j, k, oh, sgn(b_0));
                double fxy1 = b_1 * iy(g, u, i, j + 1, k, oh, sgn(b_1));
                /* xz-flux on the edges at z-faces k and k+1 */
                double e_0 = (k == 0) ? 0.0 : 0.5 * (t_rOm(g, &T, S->ru, S->rv, S->rw, i - 1, j, k) + t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k));
                double e_1 = (k == nz - 1) ? 0.0 : 0.5 * (t_rOm(g, &T, S->ru, S->rv, S->rw, i - 1, j, k + 1) + t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k + 1));
                double fxz0 = (k == 0) ? 0.0 : e_0 * izc(g, u, i, j, k, ov, sgn(e_0));
                double fxz1 = (k == nz - 1) ? 0.0 : e_1 * izc(g, u, i, j, k + 1, ov, sgn(e_1));
                double adv = ((fxx_r - fxx_l) / dx + (fxy1 - fxy0) / dy + (fxz1 - fxz0) / dz[k]) / t_JU(g, &T, i, j, k);
                double pgf = (pp[c] - cget(g, pp, i - 1, j, k)) / dx;
                /* terrain: p_x = p_xi - h_xi (p_zeta / h_zeta), the last factor
                 * the mean of the two cells' vertical differences (App. B) */
                if (T.on) pgf -= 0.5 * t_hxU(g, &T, i, j, k) * (t_fz(g, &T, pp, i, j, k) + t_fz(g, &T, pp, i - 1, j, k));
                /* reading (moist): 1 + q_v + q_c on the face is the mean of its two cells */
                if (moist) pgf = pgf / (0.5 * (cget(g, qf, i - 1, j, k) + qf[c]));
                double rho_f = 0.5 * (cget(g, S->rho, i - 1, j, k) + S->rho[c]);
                /* reading: f-plane Coriolis with geostrophic forcing, the
                 * v-momentum averaged from the four surrounding y-faces */
                double vbar = 0.25 * (cget(g, S->rv, i - 1, j, k) + S->rv[c] + cget(g, S->rv, i - 1, j + 1, k) + cget(g, S->rv, i, j + 1, k));
                double cor = P->f_cor * (vbar - rho_f * P->Vg);
                R->ru[c] = -adv - pgf + cor;
            }

    /* --- y-momentum on y-faces --- */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double b_r = 0.5 * (t_JV(g, &T, i, j, k) * S->rv[c] + t_JV(g, &T, i, j + 1, k) * cget(g, S->rv, i, j + 1, k));
                double b_l = 0.5 * (t_JV(g, &T, i, j - 1, k) * cget(g, S->rv, i, j - 1, k) + t_JV(g, &T, i, j, k) * S->rv[c]);
                double fyy_r = b_r * iy(g, v, i, j + 1, k, oh, sgn(b_r));
                double fyy_l = b_l * iy(g, v, i, j, k, oh, sgn(b_l));
                double a_0 = 0.5 * (t_JU(g, &T, i, j - 1, k) * cget(g, S->ru, i, j - 1, k) + t_JU(g, &T, i, j, k) * S->ru[c]);
                double a_1 = 0.5 * (t_JU(g, &T, i + 1, j - 1, k) * cget(g, S->ru, i + 1, j - 1, k) +
                                    t_JU(g, &T, i + 1, j, k) * cget(g, S->ru, i + 1, j, k));
                double fyx0 = a_0 * ix(g, v, i, j, k, oh, sgn(a_0));
                double fyx1 = a_1 * ix(g, v, i + 1, j, k, oh, sgn(a_1));
                double e_0 = (k == 0) ? 0.0 : 0.5 * (t_rOm(g, &T, S->ru, S->rv, S->rw, i, j - 1, k) + t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k));
                double e_1 = (k == nz - 1) ? 0.0 : 0.5 * (t_rOm(g, &T, S->ru, S->rv, S->rw, i, j - 1, k + 1) + t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k + 1));
                double fyz0 = (k == 0) ? 0.0 : e_0 * izc(g, v, i, j, k, ov, sgn(e_0));
                double fyz1 = (k == nz - 1) ? 0.0 : e_1 * izc(g, v, i, j, k + 1, ov, sgn(e_1));
                double adv = ((fyx1 - fyx0) / dx + (fyy_r - fyy_l) / dy + (fyz1 - fyz0) / dz[k]) / t_JV(g, &T, i, j, k);
                double pgf = (pp[c] - cget(g, pp, i, j - 1, k)) / dy;
                if (T.on) pgf -= 0.5 * t_heV(g, &T, i, j, k) * (t_fz(g, &T, pp, i, j, k) + t_fz(g, &T, pp, i, j - 1, k));
                if (moist) pgf = pgf / (0.5 * (cget(g, qf, i, j - 1, k) + qf[c]));
                double rho_f = 0.5 * (cget(g, S->rho, i, j - 1, k) + S->rho[c]);
                double ubar = 0.25 * (cget(g, S->ru, i, j - 1, k) + cget(g, S->ru, i + 1, j - 1, k) + S->ru[c] + cget(g, S->ru, i + 1, j, k));
                double cor = -P->f_cor * (ubar - rho_f * P->Ug);
                R->rv[c] = -adv - pgf + cor;
            }

    /* --- z-momentum on interior z-faces; buoyancy B = -(rho - rho0) g --- */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            R->rw[CIDX(g, i, j, 0)] = 0.0;
            R->rw[CIDX(g, i, j, nz)] = 0.0;
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k), cm = CIDX(g, i, j, k - 1);
                size_t kb = T.on ? c : (size_t)k, kbm = T.on ? cm : (size_t)(k - 1);
                double dzf = 0.5 * (dz[k - 1] + dz[k]);
                /* terrain: the physical distance of the two centres and h_zeta
                 * of the z-face */
                double dzp = T.on ? 0.5 * (t_Hc(g, &T, i, j, k - 1) + t_Hc(g, &T, i, j, k)) : dzf;
                double JW = T.on ? dzp / dzf : 1.0;
                /* zx-flux on the edges at x-faces i and i+1 */
                double a_0 = 0.5 * (t_JU(g, &T, i, j, k - 1) * S->ru[cm] + t_JU(g, &T, i, j, k) * S->ru[c]);
                double a_1 = 0.5 * (t_JU(g, &T, i + 1, j, k - 1) * cget(g, S->ru, i + 1, j, k - 1) +
                                    t_JU(g, &T, i + 1, j, k) * cget(g, S->ru, i + 1, j, k));
                double fzx0 = a_0 * ixw(g, w, i, j, k, oh, sgn(a_0));
                double fzx1 = a_1 * ixw(g, w, i + 1, j, k, oh, sgn(a_1));
                double b_0 = 0.5 * (t_JV(g, &T, i, j, k - 1) * S->rv[cm] + t_JV(g, &T, i, j, k) * S->rv[c]);
                double b_1 = 0.5 * (t_JV(g, &T, i, j + 1, k - 1) * cget(g, S->rv, i, j + 1, k - 1) +
                                    t_JV(g, &T, i, j + 1, k) * cget(g, S->rv, i, j + 1, k));
                double fzy0 = b_0 * iyw(g, w, i, j, k, oh, sgn(b_0));
                double fzy1 = b_1 * iyw(g, w, i, j + 1, k, oh, sgn(b_1));
                /* zz-flux at the centres above (k) and below (k-1) the face */
                double Om = t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k);
                double e_u = 0.5 * (Om + t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k + 1));
                double e_d = 0.5 * (t_rOm(g, &T, S->ru, S->rv, S->rw, i, j, k - 1) + Om);
                double fzz_u = e_u * izw(g, w, i, j, k + 1, ov, sgn(e_u));
                double fzz_d = e_d * izw(g, w, i, j, k, ov, sgn(e_d));
                double adv = ((fzx1 - fzx0) / dx + (fzy1 - fzy0) / dy + (fzz_u - fzz_d) / dzf) / JW;
                double pgf = (pp[c] - pp[cm]) / dzp;
                /* reading of the garbled sign: heavier-than-base air sinks */
                if (moist) {
                    /* reading (moist): B = -g (rho_m - rho_m0) with the total
                     * densities, and -grad p' + B divided by 1 + q_v + q_c */
                    double buoy = -gr * 0.5 * (bm[c] + bm[cm]);
                    double qfm = 0.5 * (qf[cm] + qf[c]);
                    R->rw[c] = -adv - pgf / qfm + buoy / qfm;
                } else if (P->anelastic) {
                    /* anelastic buoyancy g rho0 (theta - theta0) / theta0
                     * (Sec. 2.2), the mean of the two cells on the face */
                    double b_up = B->rho0[k] * (th[c] - B->theta0[k]) / B->theta0[k];
                    double b_dn = B->rho0[k - 1] * (th[cm] - B->theta0[k - 1]) / B->theta0[k - 1];
                    R->rw[c] = -adv - pgf + gr * 0.5 * (b_up + b_dn);
                } else {
                    double buoy = -gr * 0.5 * ((S->rho[c] - B->rho0[kb]) + (S->rho[cm] - B->rho0[kbm]));
                    R->rw[c] = -adv - pgf + buoy;
                }
            }

    if (P->sgs == 1 || P->sgs == 3 || P->nu_m != 0.0 || P->alpha_m != 0.0 || P->most_z0 > 0.0)
        add_diffusion(g, P, B, S, th, u, v, w, R);

    /* prescribed kinematic surface heat flux enters the lowest cell (Sec. 3.8) */
    if (P->surf_heat_flux != 0.0)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, 0);
                /* terrain: the flux per unit horizontal area over the lowest
                 * cell's physical height (reading) */
                R->rt[c] += S->rho[c] * P->surf_heat_flux / t_Hc(g, &T, i, j, 0);
            }

    free(th); free(u); free(v); free(w); free(pp); free(qf); free(bm);
    ter_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* acoustic substepping, App. C                                              */
/* ------------------------------------------------------------------------ */
/* Readings: coefficients are frozen at the stage state S^t (Sec. 3.1); face
 * values of theta^t and pi^t are two-point means; in the buoyancy correction
 * of the W'' equation rho-bar and pi-bar are the base state on the face; the
 * horizontal pressure gradient uses Theta'' predicted forward by
 * beta_d (Theta'' - Theta''_previous substep) (divergence damping, Sec. 3.1),
 * with no prediction on a stage's first substep. */
int orc_acoustic_substeps(const orc_grid *g, const orc_params *P, const orc_base *B,
                          const orc_state *Sn, const orc_state *St, const orc_state *Rt,
                          int32_t n_sub, double dtau, orc_state *Sout,
                          double *Fu, double *Fv, double *Fw)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (n_sub < 1) return -1;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    double dx = g->dx, dy = g->dy, gr = P->grav;
    double b1 = 0.5 * (1.0 - P->beta_s), b2 = 0.5 * (1.0 + P->beta_s), bd = P->beta_d;

    int moist = P->moist != 0;
    if (moist && (P->n_scalars < 3 || !St->rq)) return -1;
    if (g->terrain && (moist || P->anelastic)) return -1;
    ter_t T = ter_build(g);
    double *tht = dalloc(n), *pit = dalloc(n), *pim = dalloc(n), *rdm = dalloc(n);
    /* terrain: the predicted Theta'' of the horizontal pressure gradient */
    double *tt = T.on ? dalloc(n) : NULL;
    double *U2 = dalloc(n), *V2 = dalloc(n), *W2 = dalloc(nw), *T2 = dalloc(n), *R2 = dalloc(n);
    double *T2p = dalloc(n), *Un = dalloc(n), *Vn = dalloc(n), *Wn = dalloc(nw), *Tn = dalloc(n), *Rn = dalloc(n);
    double *sU = dalloc(n), *sV = dalloc(n), *sW = dalloc(nw);

    /* reading (moist, App. C with the moist EOS of Sec. 2.1): pi^t is the
     * Exner function of the moist stage state; the pressure-gradient
     * coefficient gamma R_d pi^t becomes the exact dp/dTheta divided by
     * 1 + q_v + q_c, i.e. gamma R_d pi^t (1 + R_v/R_d q_v^t)/(1 + q_v^t + q_c^t)
     * (pim); rho_d/rho_m = 1/(1 + q_v + q_c + q_r) multiplies the buoyancy
     * correction.  Dry: pim = pi^t and rho_d/rho_m = 1 exactly. */
    for (size_t c = 0; c < n; ++c) {
        tht[c] = St->rt[c] / St->rho[c];
        if (moist) {
            double qv = St->rq[c] / St->rho[c], qc = St->rq[n + c] / St->rho[c], qr = St->rq[2 * n + c] / St->rho[c];
            double fv = 1.0 + EPS_V * qv;
            pit[c] = exner(St->rt[c] * fv);
            pim[c] = pit[c] * (fv / (1.0 + qv + qc));
            rdm[c] = 1.0 / (1.0 + qv + qc + qr);
        } else {
            pit[c] = exner(St->rt[c]);
            pim[c] = pit[c];
            rdm[c] = 1.0;
        }
        U2[c] = Sn->ru[c] - St->ru[c];
        V2[c] = Sn->rv[c] - St->rv[c];
        T2[c] = Sn->rt[c] - St->rt[c];
        R2[c] = Sn->rho[c] - St->rho[c];
        T2p[c] = T2[c];
    }
    for (size_t c = 0; c < nw; ++c) W2[c] = Sn->rw[c] - St->rw[c];

    for (int s = 0; s < n_sub; ++s) {
        if (T.on)
            for (size_t c = 0; c < n; ++c) tt[c] = T2[c] + bd * (T2[c] - T2p[c]);
        /* 1. horizontal momenta, explicit forward step with the predicted Theta'' */
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = CIDX(g, i, j, k);
                    double tt_c = T2[c] + bd * (T2[c] - T2p[c]);
                    double tt_w = cget(g, T2, i - 1, j, k) + bd * (cget(g, T2, i - 1, j, k) - cget(g, T2p, i - 1, j, k));
                    double tt_s = cget(g, T2, i, j - 1, k) + bd * (cget(g, T2, i, j - 1, k) - cget(g, T2p, i, j - 1, k));
                    double pfx = 0.5 * (cget(g, pim, i - 1, j, k) + pim[c]);
                    double pfy = 0.5 * (cget(g, pim, i, j - 1, k) + pim[c]);
                    if (T.on) {
                        /* App. C: d/dxi - (h_xi / h_zeta) d/dzeta of the predicted
                         * Theta'', discretised as the pressure gradient (App. B) */
                        double cx = 0.5 * t_hxU(g, &T, i, j, k) * (t_fz(g, &T, tt, i, j, k) + t_fz(g, &T, tt, i - 1, j, k));
                        double cy = 0.5 * t_heV(g, &T, i, j, k) * (t_fz(g, &T, tt, i, j, k) + t_fz(g, &T, tt, i, j - 1, k));
                        Un[c] = U2[c] + dtau * (-GAM * R_D * pfx * (tt_c - tt_w) / dx + GAM * R_D * pfx * cx + Rt->ru[c]);
                        Vn[c] = V2[c] + dtau * (-GAM * R_D * pfy * (tt_c - tt_s) / dy + GAM * R_D * pfy * cy + Rt->rv[c]);
                    } else {
                        Un[c] = U2[c] + dtau * (-GAM * R_D * pfx * (tt_c - tt_w) / dx + Rt->ru[c]);
                        Vn[c] = V2[c] + dtau * (-GAM * R_D * pfy * (tt_c - tt_s) / dy + Rt->rv[c]);
                    }
                }
        /* 2. per column: explicit parts of Theta'', rho''; implicit W'' */
#pragma omp parallel for collapse(2) schedule(static)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double th_hat[nz], rh_hat[nz], ta[nz + 1], tb[nz + 1], tc[nz + 1], tr[nz + 1], tx[nz + 1];
                /* terrain: physical cell heights of the column; the metric part
                 * h_xi U'' + h_eta V'' of Omega'' on its z-faces before (Mo) and
                 * after (Mn) this substep's horizontal step (App. C) */
                double Hc[nz], Mo[nz + 1], Mn[nz + 1];
                for (int k = 0; k < nz; ++k) Hc[k] = t_Hc(g, &T, i, j, k);
                for (int k = 0; k <= nz; ++k) {
                    Mo[k] = t_M(g, &T, U2, V2, i, j, k);
                    Mn[k] = t_M(g, &T, Un, Vn, i, j, k);
                }
                /* face theta^t in this column (lids carry W = 0, value unused) */
#define THZ(kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : 0.5 * (tht[CIDX(g, i, j, (kk) - 1)] + tht[CIDX(g, i, j, (kk))]))
                for (int k = 0; k < nz; ++k) {
                    size_t c = CIDX(g, i, j, k);
                    double thx0 = 0.5 * (cget(g, tht, i - 1, j, k) + tht[c]);
                    double thx1 = 0.5 * (tht[c] + cget(g, tht, i + 1, j, k));
                    double thy0 = 0.5 * (cget(g, tht, i, j - 1, k) + tht[c]);
                    double thy1 = 0.5 * (tht[c] + cget(g, tht, i, j + 1, k));
                    /* terrain: h_zeta-weighted horizontal fluxes and Omega'' on the
                     * z-faces, divided by h_zeta (by the physical height) */
                    double Ue = t_JU(g, &T, i + 1, j, k) * cget(g, Un, i + 1, j, k), Uw = t_JU(g, &T, i, j, k) * Un[c];
                    double Vn_ = t_JV(g, &T, i, j + 1, k) * cget(g, Vn, i, j + 1, k), Vs = t_JV(g, &T, i, j, k) * Vn[c];
                    double Wt = W2[CIDX(g, i, j, k + 1)] - Mo[k + 1], Wb = W2[c] - Mo[k];
                    double Jc = t_J(g, &T, i, j, k);
                    double hdiv_t = (Ue * thx1 - Uw * thx0) / dx + (Vn_ * thy1 - Vs * thy0) / dy;
                    double hdiv_r = (Ue - Uw) / dx + (Vn_ - Vs) / dy;
                    th_hat[k] = T2[c] + dtau * (-hdiv_t / Jc - b1 * (Wt * THZ(k + 1) - Wb * THZ(k)) / Hc[k] + Rt->rt[c]);
                    rh_hat[k] = R2[c] + dtau * (-hdiv_r / Jc - b1 * (Wt - Wb) / Hc[k] + Rt->rho[c]);
                    if (T.on) {
                        /* the known part -h_xi U''_new - h_eta V''_new of Omega''_new */
                        th_hat[k] += dtau * b2 * (Mn[k + 1] * THZ(k + 1) - Mn[k] * THZ(k)) / Hc[k];
                        rh_hat[k] += dtau * b2 * (Mn[k + 1] - Mn[k]) / Hc[k];
                    }
                }
                /* Tridiagonal system for W at faces 1..nz-1, obtained by
                 * substituting Theta''_new = th_hat - dtau b2 dz(W theta_f)/dz and
                 * rho''_new = rh_hat - dtau b2 dz(W)/dz into the W'' equation.  Its
                 * rows are (k - 1) in ta/tb/tc/tr. */
                int m = nz - 1;
                double D = dtau * dtau * b2 * b2;
                for (int k = 1; k < nz; ++k) {
                    size_t c = CIDX(g, i, j, k), cm = CIDX(g, i, j, k - 1);
                    size_t kb = T.on ? c : (size_t)k, kbm = T.on ? cm : (size_t)(k - 1);
                    /* terrain: the column's physical heights in place of dz */
                    double dzf = 0.5 * (Hc[k - 1] + Hc[k]);
                    double pif = 0.5 * (pit[cm] + pit[c]);
                    double A = GAM * R_D * (0.5 * (pim[cm] + pim[c]));
                    /* rho-bar: the base state's total density on the face */
                    double qb0 = B->qv0 ? B->qv0[k - 1] : 0.0, qb1 = B->qv0 ? B->qv0[k] : 0.0;
                    double Cc = gr * 0.5 * (B->rho0[kbm] * (1.0 + qb0) + B->rho0[kb] * (1.0 + qb1)) * (R_D / C_V)
                              * (pif / (0.5 * (B->pi0[kbm] + B->pi0[kb])))
                              / (0.5 * (St->rt[cm] + St->rt[c]))
                              * (0.5 * (rdm[cm] + rdm[c]));
                    double idzm = 1.0 / Hc[k - 1], idz = 1.0 / Hc[k];
                    double tfm = THZ(k - 1), tf = THZ(k), tfp = THZ(k + 1);
                    ta[k - 1] = -D * (A * tfm * idzm / dzf + 0.5 * Cc * tfm * idzm - 0.5 * gr * idzm);
                    tc[k - 1] = -D * (A * tfp * idz / dzf - 0.5 * Cc * tfp * idz + 0.5 * gr * idz);
                    tb[k - 1] = 1.0 + D * (A * tf * (idz + idzm) / dzf + 0.5 * Cc * tf * (idzm - idz) - 0.5 * gr * (idzm - idz));
                    double tbk = b1 * T2[c] + b2 * th_hat[k], tbm = b1 * T2[cm] + b2 * th_hat[k - 1];
                    double rbk = b1 * R2[c] + b2 * rh_hat[k], rbm = b1 * R2[cm] + b2 * rh_hat[k - 1];
                    tr[k - 1] = W2[c] + dtau * (-A * (tbk - tbm) / dzf + 0.5 * Cc * (tbk + tbm) - 0.5 * gr * (rbk + rbm) + Rt->rw[c]);
                }
                if (m > 0) {
                    ta[0] = 0.0;
                    tc[m - 1] = 0.0;
                    orc_thomas(m, ta, tb, tc, tr, tx);
                }
                Wn[CIDX(g, i, j, 0)] = 0.0;
                Wn[CIDX(g, i, j, nz)] = 0.0;
                for (int k = 1; k < nz; ++k) Wn[CIDX(g, i, j, k)] = tx[k - 1];
                for (int k = 0; k < nz; ++k) {
                    size_t c = CIDX(g, i, j, k);
                    double Wt = Wn[CIDX(g, i, j, k + 1)], Wb = Wn[c];
                    Tn[c] = th_hat[k] - dtau * b2 * (Wt * THZ(k + 1) - Wb * THZ(k)) / Hc[k];
                    Rn[c] = rh_hat[k] - dtau * b2 * (Wt - Wb) / Hc[k];
                }
                /* terrain: the vertical flux of the scalars is Omega'', weighted
                 * as in the Theta'' and rho'' updates (W'' - M, old and new) */
                for (int k = 0; k <= nz; ++k) {
                    size_t c = CIDX(g, i, j, k);
                    sW[c] += b1 * (W2[c] - Mo[k]) + b2 * (Wn[c] - Mn[k]);
                }
#undef THZ
            }
        /* 3. time sums of the horizontal momenta; advance the substep state */
        for (size_t c = 0; c < n; ++c) {
            sU[c] += Un[c];
            sV[c] += Vn[c];
            T2p[c] = T2[c];
            T2[c] = Tn[c];
            R2[c] = Rn[c];
            U2[c] = Un[c];
            V2[c] = Vn[c];
        }
        for (size_t c = 0; c < nw; ++c) W2[c] = Wn[c];
    }

    /* stage end: S = S^t + S'' (App. C); stage-averaged momenta (Sec. 3.1) */
    for (size_t c = 0; c < n; ++c) {
        Sout->rho[c] = St->rho[c] + R2[c];
        Sout->rt[c] = St->rt[c] + T2[c];
        Sout->ru[c] = St->ru[c] + U2[c];
        Sout->rv[c] = St->rv[c] + V2[c];
        if (Fu) Fu[c] = St->ru[c] + sU[c] / n_sub;
        if (Fv) Fv[c] = St->rv[c] + sV[c] / n_sub;
    }
    for (size_t c = 0; c < nw; ++c) {
        Sout->rw[c] = St->rw[c] + W2[c];
        if (Fw) {
            /* terrain: the stage-averaged rho Omega, Omega of S^t plus the
             * average of the substeps' Omega'' */
            int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
            Fw[c] = t_rOm(g, &T, St->ru, St->rv, St->rw, i, j, k) + sW[c] / n_sub;
        }
    }

    free(tht); free(pit); free(pim); free(rdm); free(U2); free(V2); free(W2); free(T2); free(R2); free(T2p);
    free(Un); free(Vn); free(Wn); free(Tn); free(Rn); free(sU); free(sV); free(sW); free(tt);
    ter_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* scalar advance with stage-averaged fluxes (Sec. 3.1)                     */
/* ------------------------------------------------------------------------ */
int orc_scalar_advance(const orc_grid *g, const orc_params *P, const orc_state *Sn,
                       const orc_state *St, const double *Fu, const double *Fv,
                       const double *Fw, double dts, const double *src, double *rq_out)
{
    int nx = g->nx, ny = g->ny, nz = g->nz, nq = P->n_scalars;
    if (nq <= 0) return 0;
    /* scalar diffusion is provided for the Deardorff closure's rho e only */
    if ((P->sgs != 0 && P->sgs != 3) || P->alpha_m != 0.0) return -5;
    if (P->sgs == 3 && (nq != 1 || !src)) return -5;
    size_t n = (size_t)nx * ny * nz;
    int oh = P->adv_order_h, ov = P->adv_order_v;
    if (g->terrain && (P->moist || P->sgs != 0)) return -5;
    ter_t T = ter_build(g);
    double *q = dalloc(n);
    for (int s = 0; s < nq; ++s) {
        const double *rqn = Sn->rq + (size_t)s * n, *rqt = St->rq + (size_t)s * n;
        double *out = rq_out + (size_t)s * n;
        for (size_t c = 0; c < n; ++c) q[c] = rqt[c] / St->rho[c];
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = CIDX(g, i, j, k);
                    double f[6]; /* x0, x1, y0, y1, z0, z1 */
                    double adv[6] = {Fu[c], cget(g, Fu, i + 1, j, k), Fv[c], cget(g, Fv, i, j + 1, k),
                                     Fw[c], Fw[CIDX(g, i, j, k + 1)]};
                    double qq[6];
                    for (int side = 0; side < 2; ++side) {
                        for (int o = 0; o < 6; ++o) qq[o] = cget(g, q, i + side - 3 + o, j, k);
                        double fa = adv[side];
                        f[side] = fa * (P->scalar_scheme == 1 ? orc_weno5(qq, sgn(fa), WENO_EPS) : orc_interp(oh, qq, sgn(fa)));
                        for (int o = 0; o < 6; ++o) qq[o] = cget(g, q, i, j + side - 3 + o, k);
                        fa = adv[2 + side];
                        f[2 + side] = fa * (P->scalar_scheme == 1 ? orc_weno5(qq, sgn(fa), WENO_EPS) : orc_interp(oh, qq, sgn(fa)));
                        int kf = k + side;
                        if (kf == 0 || kf == nz) {
                            f[4 + side] = 0.0;
                        } else {
                            for (int o = 0; o < 6; ++o) qq[o] = cget(g, q, i, j, kf - 3 + o);
                            fa = adv[4 + side];
                            f[4 + side] = fa * (P->scalar_scheme == 1 ? orc_weno5(qq, sgn(fa), WENO_EPS) : orc_interp(ov, qq, sgn(fa)));
                        }
                    }
                    /* terrain: the horizontal fluxes carry h_zeta of their face,
                     * Fw is rho Omega, and the divergence is divided by the
                     * cell's h_zeta (App. A) */
                    double div;
                    if (T.on)
                        div = ((t_JU(g, &T, i + 1, j, k) * f[1] - t_JU(g, &T, i, j, k) * f[0]) / g->dx +
                               (t_JV(g, &T, i, j + 1, k) * f[3] - t_JV(g, &T, i, j, k) * f[2]) / g->dy +
                               (f[5] - f[4]) / g->dz[k]) / t_J(g, &T, i, j, k);
                    else
                        div = (f[1] - f[0]) / g->dx + (f[3] - f[2]) / g->dy + (f[5] - f[4]) / g->dz[k];
                    out[c] = rqn[c] - dts * div;
                    if (P->sgs == 3 && s == 0) {
                        /* rho e: its source at S^t; negative values are cut to zero */
                        out[c] = out[c] + dts * src[c];
                        if (out[c] < 0.0) out[c] = 0.0;
                    }
                }
    }
    free(q);
    ter_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* RK3 step with acoustic substeps (Sec. 3.1, Sec. 3.3)                      */
/* ------------------------------------------------------------------------ */
/* Stage s advances from S^n with the right-hand side at the latest stage
 * state: dt/3 with one substep, dt/2 with n_s/2 substeps, dt with n_s
 * substeps, the substep length being dt/n_s in the last two stages. */
int orc_rk3_step(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S)
{
    int nx = g->nx, ny = g->ny, nz = g->nz, nq = P->n_scalars;
    int ns = P->n_substeps;
    if (ns < 2 || ns % 2 != 0) return -1;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1), nqn = (size_t)(nq > 0 ? nq : 0) * n;
    orc_state Sn, St, Rt, Snew;
    double *bufs[4][6];
    size_t sz[6] = {n, n, n, n, nw, nqn};
    for (int b = 0; b < 4; ++b)
        for (int f = 0; f < 6; ++f) bufs[b][f] = dalloc(sz[f]);
#define BIND(st, b) st.rho = bufs[b][0], st.rt = bufs[b][1], st.ru = bufs[b][2], st.rv = bufs[b][3], st.rw = bufs[b][4], st.rq = bufs[b][5]
    BIND(Sn, 0);
    BIND(St, 1);
    BIND(Rt, 2);
    BIND(Snew, 3);
#undef BIND
    double *Fu = dalloc(n), *Fv = dalloc(n), *Fw = dalloc(nw);
    memcpy(Sn.rho, S->rho, n * 8); memcpy(Sn.rt, S->rt, n * 8); memcpy(Sn.ru, S->ru, n * 8);
    memcpy(Sn.rv, S->rv, n * 8); memcpy(Sn.rw, S->rw, nw * 8);
    if (nqn) memcpy(Sn.rq, S->rq, nqn * 8);
    memcpy(St.rho, S->rho, n * 8); memcpy(St.rt, S->rt, n * 8); memcpy(St.ru, S->ru, n * 8);
    memcpy(St.rv, S->rv, n * 8); memcpy(St.rw, S->rw, nw * 8);
    if (nqn) memcpy(St.rq, S->rq, nqn * 8);

    int rc = 0;
    for (int stage = 0; stage < 3 && rc == 0; ++stage) {
        double dts = stage == 0 ? P->dt / 3.0 : (stage == 1 ? P->dt / 2.0 : P->dt);
        int nsub = stage == 0 ? 1 : (stage == 1 ? ns / 2 : ns);
        double dtau = stage == 0 ? P->dt / 3.0 : P->dt / ns;
        rc = orc_slow_rhs(g, P, B, &St, &Rt);
        if (rc) break;
        rc = orc_acoustic_substeps(g, P, B, &Sn, &St, &Rt, nsub, dtau, &Snew, Fu, Fv, Fw);
        if (rc) break;
        if (nq > 0) rc = orc_scalar_advance(g, P, &Sn, &St, Fu, Fv, Fw, dts, P->sgs == 3 ? Rt.rq : NULL, Snew.rq);
        /* the new stage state */
        orc_state tmp = St;
        St = Snew;
        Snew = tmp;
    }
    if (rc == 0) {
        memcpy(S->rho, St.rho, n * 8); memcpy(S->rt, St.rt, n * 8); memcpy(S->ru, St.ru, n * 8);
        memcpy(S->rv, St.rv, n * 8); memcpy(S->rw, St.rw, nw * 8);
        if (nqn) memcpy(S->rq, St.rq, nqn * 8);
    }
    for (int b = 0; b < 4; ++b)
        for (int f = 0; f < 6; ++f) free(bufs[b][f]);
    free(Fu); free(Fv); free(Fw);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* diagnostics (mass and energy budgets, Sec. 4.1.2)                          */
/* ------------------------------------------------------------------------ */
/* Kahan-compensated sums in the plain cell order. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double x)
{
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

int orc_diagnostics(const orc_grid *g, const orc_params *P, const orc_base *B,
                    const orc_state *S, double *out)
{
    (void)B;
    int nx = g->nx, ny = g->ny, nz = g->nz, nq = P->n_scalars;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    ksum mass = {0, 0}, theta = {0, 0}, energy = {0, 0};
    /* terrain: cell volumes dx dy Hc and the centres' physical heights */
    ter_t Tr = ter_build(g);
    ksum *qm = (ksum *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(ksum));
    double wmax = 0.0, nonfinite = 0.0;
    double z = 0.0;
    for (int k = 0; k < nz; ++k) {
        double zc0 = z + 0.5 * g->dz[k];
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double vol = g->dx * g->dy * t_Hc(g, &Tr, i, j, k);
                double zc = Tr.on ? zc0 + 0.5 * (Tr.s[k] + Tr.s[k + 1]) * t_hb(g, &Tr, i, j) : zc0;
                double r = S->rho[c], T = S->rt[c];
                kadd(&mass, r * vol);
                kadd(&theta, T * vol);
                double uc = 0.5 * (S->ru[c] / (0.5 * (cget(g, S->rho, i - 1, j, k) + r))
                                 + cget(g, S->ru, i + 1, j, k) / (0.5 * (r + cget(g, S->rho, i + 1, j, k))));
                double vc = 0.5 * (S->rv[c] / (0.5 * (cget(g, S->rho, i, j - 1, k) + r))
                                 + cget(g, S->rv, i, j + 1, k) / (0.5 * (r + cget(g, S->rho, i, j + 1, k))));
                double wb = (k == 0) ? 0.0 : S->rw[c] / (0.5 * (S->rho[CIDX(g, i, j, k - 1)] + r));
                double wt = (k == nz - 1) ? 0.0 : S->rw[CIDX(g, i, j, k + 1)] / (0.5 * (r + S->rho[CIDX(g, i, j, k + 1)]));
                double wc = 0.5 * (wb + wt);
                double temp = (T / r) * exner(T);
                kadd(&energy, (0.5 * r * (uc * uc + vc * vc + wc * wc) + r * C_V * temp + r * P->grav * zc) * vol);
                for (int s = 0; s < nq; ++s) kadd(&qm[s], S->rq[(size_t)s * n + c] * vol);
                nonfinite += (double)!isfinite(r) + (double)!isfinite(T) + (double)!isfinite(S->ru[c]) +
                             (double)!isfinite(S->rv[c]);
            }
        z += g->dz[k];
    }
    for (size_t c = 0; c < nw; ++c) {
        if (!isfinite(S->rw[c])) nonfinite += 1.0;
    }
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double wv = fabs(S->rw[CIDX(g, i, j, k)] / (0.5 * (S->rho[CIDX(g, i, j, k - 1)] + S->rho[CIDX(g, i, j, k)])));
                if (wv > wmax) wmax = wv;
            }
    out[0] = mass.s;
    out[1] = theta.s;
    out[2] = energy.s;
    out[3] = wmax;
    out[4] = nonfinite;
    for (int s = 0; s < nq; ++s) out[5 + s] = qm[s].s;
    free(qm);
    ter_free(&Tr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* learned SGS closure: MLP 10 -> 64 -> 64 -> 64 -> 9, ReLU hidden layers     */
/* ------------------------------------------------------------------------ */
/* Not part of the paper's method: the paper names surrogate models only as
 * future work (Sec. 6).  This is the reference for the closure that replaces
 * the Smagorinsky stresses. */
enum { MI = 10, MH = 64, MO = 9 };
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MI * MH)
#define OFF_W2 (OFF_B1 + MH)
#define OFF_B2 (OFF_W2 + MH * MH)
#define OFF_W3 (OFF_B2 + MH)
#define OFF_B3 (OFF_W3 + MH * MH)
#define OFF_W4 (OFF_B3 + MH)
#define OFF_B4 (OFF_W4 + MH * MO)
#define N_PARAMS (OFF_B4 + MO)

int orc_mlp_nparams(void) { return N_PARAMS; }

/* bfloat16 = the upper 16 bits of a float, rounded to nearest even */
double orc_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double rb(double x, int bf16) { return bf16 ? orc_bf16(x) : x; }

/* one dense layer: out[j] = b[j] + sum_i in[i] W[i][j] (operands rounded) */
static void dense(const double *in, int nin, const double *W, const double *b, int nout, int bf16,
                  double *out)
{
    for (int j = 0; j < nout; ++j) {
        double acc = 0.0;
        for (int i = 0; i < nin; ++i) acc += rb(in[i], bf16) * rb(W[i * nout + j], bf16);
        out[j] = b[j] + acc;
    }
}

static void relu(double *h, int n)
{
    for (int j = 0; j < n; ++j)
        if (!(h[j] > 0.0)) h[j] = 0.0;
}

int orc_mlp_forward(const double *p, const double *x, int64_t n, double *y, int bf16)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double h1[MH], h2[MH], h3[MH];
        dense(x + s * MI, MI, p + OFF_W1, p + OFF_B1, MH, bf16, h1);
        relu(h1, MH);
        dense(h1, MH, p + OFF_W2, p + OFF_B2, MH, bf16, h2);
        relu(h2, MH);
        dense(h2, MH, p + OFF_W3, p + OFF_B3, MH, bf16, h3);
        relu(h3, MH);
        dense(h3, MH, p + OFF_W4, p + OFF_B4, MO, bf16, y + s * MO);
    }
    return 0;
}

/* Loss L = mean over samples and outputs of (y - t)^2; backpropagation through
 * the four layers (ReLU derivative 0 at 0). */
int orc_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t n, int bf16,
                      double *loss, double *grad)
{
    memset(grad, 0, sizeof(double) * N_PARAMS);
    double L = 0.0;
    const double scale = 2.0 / ((double)n * MO);
    for (int64_t s = 0; s < n; ++s) {
        const double *xs = x + s * MI;
        double h1[MH], h2[MH], h3[MH], y[MO], dy[MO], d3[MH], d2[MH], d1[MH];
        dense(xs, MI, p + OFF_W1, p + OFF_B1, MH, bf16, h1);
        relu(h1, MH);
        dense(h1, MH, p + OFF_W2, p + OFF_B2, MH, bf16, h2);
        relu(h2, MH);
        dense(h2, MH, p + OFF_W3, p + OFF_B3, MH, bf16, h3);
        relu(h3, MH);
        dense(h3, MH, p + OFF_W4, p + OFF_B4, MO, bf16, y);
        for (int j = 0; j < MO; ++j) {
            double e = y[j] - t[s * MO + j];
            L += e * e;
            dy[j] = scale * e;
        }
        /* layer 4 */
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MO; ++j) grad[OFF_W4 + i * MO + j] += rb(h3[i], bf16) * rb(dy[j], bf16);
        for (int j = 0; j < MO; ++j) grad[OFF_B4 + j] += dy[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MO; ++j) acc += rb(dy[j], bf16) * rb(p[OFF_W4 + i * MO + j], bf16);
            d3[i] = h3[i] > 0.0 ? acc : 0.0;
        }
        /* layer 3 */
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MH; ++j) grad[OFF_W3 + i * MH + j] += rb(h2[i], bf16) * rb(d3[j], bf16);
        for (int j = 0; j < MH; ++j) grad[OFF_B3 + j] += d3[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MH; ++j) acc += rb(d3[j], bf16) * rb(p[OFF_W3 + i * MH + j], bf16);
            d2[i] = h2[i] > 0.0 ? acc : 0.0;
        }
        /* layer 2 */
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MH; ++j) grad[OFF_W2 + i * MH + j] += rb(h1[i], bf16) * rb(d2[j], bf16);
        for (int j = 0; j < MH; ++j) grad[OFF_B2 + j] += d2[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MH; ++j) acc += rb(d2[j], bf16) * rb(p[OFF_W2 + i * MH + j], bf16);
            d1[i] = h1[i] > 0.0 ? acc : 0.0;
        }
        /* layer 1 */
        for (int i = 0; i < MI; ++i)
            for (int j = 0; j < MH; ++j) grad[OFF_W1 + i * MH + j] += rb(xs[i], bf16) * rb(d1[j], bf16);
        for (int j = 0; j < MH; ++j) grad[OFF_B1 + j] += d1[j];
    }
    if (loss) *loss = L / ((double)n * MO);
    return 0;
}

/* Error scale of the gradient: the same backpropagation with every product
 * replaced by the product of absolute values (and no ReLU sign cancellation
 * in the deltas), i.e. for each parameter the sum of the magnitudes of all the
 * terms whose sum is its gradient.  A sum of m terms computed in a precision
 * with unit roundoff u differs from the exact sum by at most about m u times
 * this scale, and a changed rounding of one operand (a BF16 boundary flip)
 * changes it by at most 2^-8 of it. */
int orc_mlp_grad_abs(const double *p, const double *x, const double *t, int64_t n, int bf16, double *gabs)
{
    memset(gabs, 0, sizeof(double) * N_PARAMS);
    const double scale = 2.0 / ((double)n * MO);
    for (int64_t s = 0; s < n; ++s) {
        const double *xs = x + s * MI;
        double h1[MH], h2[MH], h3[MH], y[MO], dy[MO], d3[MH], d2[MH], d1[MH];
        dense(xs, MI, p + OFF_W1, p + OFF_B1, MH, bf16, h1);
        relu(h1, MH);
        dense(h1, MH, p + OFF_W2, p + OFF_B2, MH, bf16, h2);
        relu(h2, MH);
        dense(h2, MH, p + OFF_W3, p + OFF_B3, MH, bf16, h3);
        relu(h3, MH);
        dense(h3, MH, p + OFF_W4, p + OFF_B4, MO, bf16, y);
        for (int j = 0; j < MO; ++j) dy[j] = fabs(scale * (y[j] - t[s * MO + j]));
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MO; ++j) gabs[OFF_W4 + i * MO + j] += fabs(rb(h3[i], bf16)) * fabs(rb(dy[j], bf16));
        for (int j = 0; j < MO; ++j) gabs[OFF_B4 + j] += dy[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MO; ++j) acc += fabs(rb(dy[j], bf16)) * fabs(rb(p[OFF_W4 + i * MO + j], bf16));
            d3[i] = h3[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MH; ++j) gabs[OFF_W3 + i * MH + j] += fabs(rb(h2[i], bf16)) * rb(d3[j], bf16);
        for (int j = 0; j < MH; ++j) gabs[OFF_B3 + j] += d3[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MH; ++j) acc += rb(d3[j], bf16) * fabs(rb(p[OFF_W3 + i * MH + j], bf16));
            d2[i] = h2[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < MH; ++i)
            for (int j = 0; j < MH; ++j) gabs[OFF_W2 + i * MH + j] += fabs(rb(h1[i], bf16)) * rb(d2[j], bf16);
        for (int j = 0; j < MH; ++j) gabs[OFF_B2 + j] += d2[j];
        for (int i = 0; i < MH; ++i) {
            double acc = 0.0;
            for (int j = 0; j < MH; ++j) acc += rb(d2[j], bf16) * fabs(rb(p[OFF_W2 + i * MH + j], bf16));
            d1[i] = h1[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < MI; ++i)
            for (int j = 0; j < MH; ++j) gabs[OFF_W1 + i * MH + j] += fabs(rb(xs[i], bf16)) * rb(d1[j], bf16);
        for (int j = 0; j < MH; ++j) gabs[OFF_B1 + j] += d1[j];
    }
    return 0;
}

/* Distance of v > 0 to the nearest point where its bfloat16 rounding changes:
 * v lies between the bfloat16 values lo <= v < hi; it rounds to lo or hi with
 * the boundary at their midpoint, and to the value below lo past the midpoint
 * of that value and lo. */
static double bf16_boundary_distance(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return INFINITY;
    uint32_t lo = u & 0xffff0000u, hi = lo + 0x10000u;
    float flo, fhi;
    memcpy(&flo, &lo, 4);
    memcpy(&fhi, &hi, 4);
    double up = 0.5 * ((double)flo + (double)fhi) - v;
    double down = INFINITY;
    if (lo >= 0x10000u) {
        uint32_t pv = lo - 0x10000u;
        float fpv;
        memcpy(&fpv, &pv, 4);
        down = v - 0.5 * ((double)fpv + (double)flo);
    }
    return fabs(up) < fabs(down) ? fabs(up) : fabs(down);
}

/* For each sample of a BF16-mode forward pass and each hidden unit of the
 * three hidden layers (margin[n][192], layer-major): the distance of the
 * unit's exact pre-activation to the nearest point where its bfloat16 rounding
 * changes (or, for a value at or below zero, to zero, where ReLU switches),
 * divided by the sum of the magnitudes of its terms (|bias| + sum |x W|).
 * Where this is below the relative accumulation error of another evaluation
 * (at most about 64 * 2^-24 in FP32), that evaluation may round the unit to
 * the neighbouring bfloat16 value; where it is above, both round it the same
 * way.  A unit without terms reports infinity.  If flip_layer is not NULL,
 * sample s rounds unit flip_unit[s] of hidden layer flip_layer[s] (0..2; -1:
 * none) to the bfloat16 neighbour on the other side of its value instead of
 * the nearest, and writes its outputs to y[n][9] (y may be NULL otherwise). */
int orc_mlp_unit_margins(const double *p, const double *x, int64_t n, double *margin,
                         const int32_t *flip_layer, const int32_t *flip_unit, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double in[MH], out[MH];
        int nin = MI;
        for (int i = 0; i < MI; ++i) in[i] = x[s * MI + i];
        const int offw[3] = {OFF_W1, OFF_W2, OFF_W3}, offb[3] = {OFF_B1, OFF_B2, OFF_B3};
        for (int layer = 0; layer < 3; ++layer) {
            for (int j = 0; j < MH; ++j) {
                double acc = 0.0, mag = fabs(p[offb[layer] + j]);
                for (int i = 0; i < nin; ++i) {
                    double term = rb(in[i], 1) * rb(p[offw[layer] + i * MH + j], 1);
                    acc += term;
                    mag += fabs(term);
                }
                double v = p[offb[layer] + j] + acc;
                if (margin) {
                    /* positive: the nearest bfloat16 boundary (always closer
                     * than zero); otherwise the distance to zero */
                    double dist = v > 0.0 ? bf16_boundary_distance(v) : -v;
                    margin[s * 3 * MH + layer * MH + j] = mag > 0.0 ? dist / mag : INFINITY;
                }
                out[j] = v > 0.0 ? v : 0.0;
                if (flip_layer && flip_layer[s] == layer && flip_unit[s] == j && out[j] > 0.0) {
                    /* the next layer rounds its inputs: hand it the neighbour
                     * on the other side instead (exactly representable, so its
                     * own rounding leaves it unchanged) */
                    float f = (float)out[j];
                    uint32_t u;
                    memcpy(&u, &f, 4);
                    uint32_t lo = u & 0xffff0000u, hi = lo + 0x10000u;
                    double near = rb(out[j], 1);
                    float fl, fh;
                    memcpy(&fl, &lo, 4);
                    memcpy(&fh, &hi, 4);
                    out[j] = (near == (double)fl) ? (double)fh : (double)fl;
                }
            }
            for (int j = 0; j < MH; ++j) in[j] = out[j];
            nin = MH;
        }
        if (y) dense(in, MH, p + OFF_W4, p + OFF_B4, MO, 1, y + s * MO);
    }
    return 0;
}

/* Adam (Kingma & Ba 2015) with bias correction */
int orc_adam(double *p, const double *g, double *m, double *v, int64_t np, int64_t step, double lr,
             double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* closure inputs at cell centres                                            */
/* ------------------------------------------------------------------------ */
/* Diagonal gradients from the two faces of the cell; off-diagonal ones as the
 * mean of the four edge differences around the centre (free-slip lids: du/dz,
 * dv/dz, dw/dx, dw/dy vanish on the lid edges); dtheta/dz as the mean of the
 * two face differences (zero through the lids). */
int orc_sgs_features(const orc_grid *g, const orc_state *S, double *feat)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    double *th = dalloc(n), *u = dalloc(n), *v = dalloc(n), *w = dalloc(nw);
    primitives(g, S, th, u, v, w);
    const double dx = g->dx, dy = g->dy;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                double *f = feat + c * MI;
                /* edge differences */
#define DUDY(ii, jj) ((cget(g, u, ii, jj, k) - cget(g, u, ii, (jj) - 1, k)) / dy)
#define DVDX(ii, jj) ((cget(g, v, ii, jj, k) - cget(g, v, (ii) - 1, jj, k)) / dx)
#define DUDZ(ii, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : (cget(g, u, ii, j, kk) - cget(g, u, ii, j, (kk) - 1)) / (0.5 * (g->dz[(kk) - 1] + g->dz[kk])))
#define DVDZ(jj, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : (cget(g, v, i, jj, kk) - cget(g, v, i, jj, (kk) - 1)) / (0.5 * (g->dz[(kk) - 1] + g->dz[kk])))
#define DWDX(ii, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : (wget(g, w, ii, j, kk) - wget(g, w, (ii) - 1, j, kk)) / dx)
#define DWDY(jj, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : (wget(g, w, i, jj, kk) - wget(g, w, i, (jj) - 1, kk)) / dy)
                f[0] = (cget(g, u, i + 1, j, k) - u[c]) / dx;
                f[1] = 0.25 * (DUDY(i, j) + DUDY(i + 1, j) + DUDY(i, j + 1) + DUDY(i + 1, j + 1));
                f[2] = 0.25 * (DUDZ(i, k) + DUDZ(i + 1, k) + DUDZ(i, k + 1) + DUDZ(i + 1, k + 1));
                f[3] = 0.25 * (DVDX(i, j) + DVDX(i + 1, j) + DVDX(i, j + 1) + DVDX(i + 1, j + 1));
                f[4] = (cget(g, v, i, j + 1, k) - v[c]) / dy;
                f[5] = 0.25 * (DVDZ(j, k) + DVDZ(j + 1, k) + DVDZ(j, k + 1) + DVDZ(j + 1, k + 1));
                f[6] = 0.25 * (DWDX(i, k) + DWDX(i + 1, k) + DWDX(i, k + 1) + DWDX(i + 1, k + 1));
                f[7] = 0.25 * (DWDY(j, k) + DWDY(j + 1, k) + DWDY(j, k + 1) + DWDY(j + 1, k + 1));
                f[8] = (w[CIDX(g, i, j, k + 1)] - w[c]) / g->dz[k];
                double gb = (k == 0) ? 0.0 : (th[c] - th[CIDX(g, i, j, k - 1)]) / (0.5 * (g->dz[k - 1] + g->dz[k]));
                double gt = (k == nz - 1) ? 0.0 : (th[CIDX(g, i, j, k + 1)] - th[c]) / (0.5 * (g->dz[k] + g->dz[k + 1]));
                f[9] = 0.5 * (gb + gt);
#undef DUDY
#undef DVDX
#undef DUDZ
#undef DVDZ
#undef DWDX
#undef DWDY
            }
    free(th); free(u); free(v); free(w);
    return 0;
}

/* Smagorinsky stress and heat flux at a cell centre from its closure inputs
 * f[10] and the centred horizontal theta gradients (Sec. 2.3): kinematic
 * tau_ij = -2 nu_t (S_ij - delta_ij tr S / 3), q_j = -(nu_t / Pr_t) dtheta/dx_j;
 * returns nu_t |S|^2, the dissipation -tau:S of the deviatoric part. */
static double centre_smagorinsky(const double *f, double dthx, double dthy, double Cs, double Pr_t,
                                 double delta, double *t)
{
    double s11 = f[0], s22 = f[4], s33 = f[8];
    double s12 = 0.5 * (f[1] + f[3]), s13 = 0.5 * (f[2] + f[6]), s23 = 0.5 * (f[5] + f[7]);
    double ss = 2.0 * (s11 * s11 + s22 * s22 + s33 * s33) + 4.0 * (s12 * s12 + s13 * s13 + s23 * s23);
    double cd = Cs * delta;
    double nut = cd * cd * sqrt(ss);
    if (t) {
        double dd = (s11 + s22 + s33) / 3.0;
        t[0] = -2.0 * nut * (s11 - dd);
        t[1] = -2.0 * nut * (s22 - dd);
        t[2] = -2.0 * nut * (s33 - dd);
        t[3] = -2.0 * nut * s12;
        t[4] = -2.0 * nut * s13;
        t[5] = -2.0 * nut * s23;
        t[6] = -(nut / Pr_t) * dthx;
        t[7] = -(nut / Pr_t) * dthy;
        t[8] = -(nut / Pr_t) * f[9];
    }
    return nut * ss;
}

/* ------------------------------------------------------------------------ */
/* box filter and SGS targets                                                */
/* ------------------------------------------------------------------------ */
int orc_box_filter(const orc_grid *g, const orc_state *S, int32_t r, double Cs, double Pr_t, orc_state *C,
                   double *targets)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (r < 1 || nx % r || ny % r || nz % r) return -2;
    int cx = nx / r, cy = ny / r, cz = nz / r;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    double *th = dalloc(n), *u = dalloc(n), *v = dalloc(n), *w = dalloc(nw);
    primitives(g, S, th, u, v, w);
    double *fsgs = NULL;
    if (Cs > 0.0) {
        double *feat = dalloc(n * MI);
        fsgs = dalloc(n * MO);
        orc_sgs_features(g, S, feat);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = CIDX(g, i, j, k);
                    double dthx = 0.5 * (cget(g, th, i + 1, j, k) - cget(g, th, i - 1, j, k)) / g->dx;
                    double dthy = 0.5 * (cget(g, th, i, j + 1, k) - cget(g, th, i, j - 1, k)) / g->dy;
                    centre_smagorinsky(feat + c * MI, dthx, dthy, Cs, Pr_t, cbrt(g->dx * g->dy * g->dz[k]),
                                       fsgs + c * MO);
                }
        free(feat);
    }
    orc_grid cg = {cx, cy, cz, g->dx * r, g->dy * r, NULL};
    double r3 = (double)r * r * r, r2 = (double)r * r;
#pragma omp parallel for collapse(2) schedule(static)
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                size_t cc = CIDX(&cg, I, J, K);
                double mr = 0, mt = 0, su[3] = {0, 0, 0}, sth = 0, suu[6] = {0, 0, 0, 0, 0, 0}, sut[3] = {0, 0, 0};
                double ssg[MO] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                for (int kk = 0; kk < r; ++kk)
                    for (int jj = 0; jj < r; ++jj)
                        for (int ii = 0; ii < r; ++ii) {
                            int i = I * r + ii, j = J * r + jj, k = K * r + kk;
                            size_t c = CIDX(g, i, j, k);
                            mr += S->rho[c];
                            mt += S->rt[c];
                            double uc = 0.5 * (u[c] + cget(g, u, i + 1, j, k));
                            double vc = 0.5 * (v[c] + cget(g, v, i, j + 1, k));
                            double wc = 0.5 * (w[c] + w[CIDX(g, i, j, k + 1)]);
                            double t = th[c];
                            su[0] += uc; su[1] += vc; su[2] += wc; sth += t;
                            suu[0] += uc * uc; suu[1] += vc * vc; suu[2] += wc * wc;
                            suu[3] += uc * vc; suu[4] += uc * wc; suu[5] += vc * wc;
                            sut[0] += uc * t; sut[1] += vc * t; sut[2] += wc * t;
                            if (fsgs)
                                for (int o = 0; o < MO; ++o) ssg[o] += fsgs[c * MO + o];
                        }
                C->rho[cc] = mr / r3;
                C->rt[cc] = mt / r3;
                double mu_[3] = {su[0] / r3, su[1] / r3, su[2] / r3}, mth = sth / r3;
                double *tg = targets + cc * 9;
                tg[0] = suu[0] / r3 - mu_[0] * mu_[0];
                tg[1] = suu[1] / r3 - mu_[1] * mu_[1];
                tg[2] = suu[2] / r3 - mu_[2] * mu_[2];
                tg[3] = suu[3] / r3 - mu_[0] * mu_[1];
                tg[4] = suu[4] / r3 - mu_[0] * mu_[2];
                tg[5] = suu[5] / r3 - mu_[1] * mu_[2];
                tg[6] = sut[0] / r3 - mu_[0] * mth;
                tg[7] = sut[1] / r3 - mu_[1] * mth;
                tg[8] = sut[2] / r3 - mu_[2] * mth;
                for (int o = 0; o < MO; ++o) tg[o] += ssg[o] / r3;
                /* face momenta: mean over the fine faces on the coarse face */
                double fu = 0, fv = 0, fw = 0;
                for (int a = 0; a < r; ++a)
                    for (int b = 0; b < r; ++b) {
                        fu += S->ru[CIDX(g, I * r, J * r + a, K * r + b)];
                        fv += S->rv[CIDX(g, I * r + a, J * r, K * r + b)];
                        fw += S->rw[CIDX(g, I * r + a, J * r + b, K * r)];
                    }
                C->ru[cc] = fu / r2;
                C->rv[cc] = fv / r2;
                C->rw[cc] = (K == 0) ? 0.0 : fw / r2;
            }
    for (int J = 0; J < cy; ++J)
        for (int I = 0; I < cx; ++I) C->rw[CIDX(&cg, I, J, cz)] = 0.0;
    free(th); free(u); free(v); free(w); free(fsgs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* slow right-hand side with the learned closure                            */
/* ------------------------------------------------------------------------ */
int orc_slow_rhs_mlp(const orc_grid *g, const orc_params *P, const orc_base *B, const orc_state *S,
                     const double *params, const double *norm, int bf16, orc_state *R, int64_t *fallback_out)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1);
    if (P->nu_m != 0.0 || P->alpha_m != 0.0) return -5;
    /* resolved terms: the same right-hand side without any stress */
    orc_params Q = *P;
    Q.sgs = 0;
    int rc = orc_slow_rhs(g, &Q, B, S, R);
    if (rc) return rc;
    double *feat = dalloc(n * MI), *xs = dalloc(n * MI), *ys = dalloc(n * MO);
    double *th = dalloc(n), *u = dalloc(n), *v = dalloc(n), *w = dalloc(nw);
    primitives(g, S, th, u, v, w);
    orc_sgs_features(g, S, feat);
    const double *mx = norm, *sx = norm + MI, *my = norm + 2 * MI, *sy = norm + 2 * MI + MO;
    for (size_t c = 0; c < n; ++c)
        for (int f = 0; f < MI; ++f) xs[c * MI + f] = (feat[c * MI + f] - mx[f]) / sx[f];
    orc_mlp_forward(params, xs, (int64_t)n, ys, bf16);
    /* rho tau and rho q at centres, with the per-cell Smagorinsky fallback */
    double *T = dalloc(n * MO);
    int64_t nfb = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                const double *f = feat + c * MI;
                double t[MO];
                int finite = 1;
                for (int o = 0; o < MO; ++o) {
                    t[o] = ys[c * MO + o] * sy[o] + my[o];
                    if (!isfinite(t[o])) finite = 0;
                }
                double s11 = f[0], s22 = f[4], s33 = f[8];
                double s12 = 0.5 * (f[1] + f[3]), s13 = 0.5 * (f[2] + f[6]), s23 = 0.5 * (f[5] + f[7]);
                double dthx = 0.5 * (cget(g, th, i + 1, j, k) - cget(g, th, i - 1, j, k)) / g->dx;
                double dthy = 0.5 * (cget(g, th, i, j + 1, k) - cget(g, th, i, j - 1, k)) / g->dy;
                double ts[MO];
                double diss_smag = centre_smagorinsky(f, dthx, dthy, P->Cs, P->Pr_t, cbrt(g->dx * g->dy * g->dz[k]), ts);
                /* energy transfer to the subgrid scales, -tau:S */
                double pi_mlp = -(t[0] * s11 + t[1] * s22 + t[2] * s33 + 2.0 * (t[3] * s12 + t[4] * s13 + t[5] * s23));
                if (!finite || pi_mlp < -2.0 * diss_smag) {
                    for (int o = 0; o < MO; ++o) t[o] = ts[o];
                    ++nfb;
                }
                for (int o = 0; o < MO; ++o) T[c * MO + o] = S->rho[c] * t[o];
            }
    /* divergence on the staggered points (4-cell means on edges, 2-cell means on faces) */
#define TT(ii, jj, kk, o) (T[CIDX(g, wrap(ii, nx), wrap(jj, ny), kk) * MO + (o)])
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                /* tau_12 on xy-edge (x-face ii, y-face jj) */
#define E12(ii, jj) (0.25 * (TT((ii) - 1, (jj) - 1, k, 3) + TT(ii, (jj) - 1, k, 3) + TT((ii) - 1, jj, k, 3) + TT(ii, jj, k, 3)))
#define E13(ii, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : 0.25 * (TT((ii) - 1, j, (kk) - 1, 4) + TT(ii, j, (kk) - 1, 4) + TT((ii) - 1, j, kk, 4) + TT(ii, j, kk, 4)))
#define E23(jj, kk) (((kk) <= 0 || (kk) >= nz) ? 0.0 : 0.25 * (TT(i, (jj) - 1, (kk) - 1, 5) + TT(i, jj, (kk) - 1, 5) + TT(i, (jj) - 1, kk, 5) + TT(i, jj, kk, 5)))
                R->ru[c] -= (TT(i, j, k, 0) - TT(i - 1, j, k, 0)) / g->dx + (E12(i, j + 1) - E12(i, j)) / g->dy +
                            (E13(i, k + 1) - E13(i, k)) / g->dz[k];
                R->rv[c] -= (E12(i + 1, j) - E12(i, j)) / g->dx + (TT(i, j, k, 1) - TT(i, j - 1, k, 1)) / g->dy +
                            (E23(j, k + 1) - E23(j, k)) / g->dz[k];
                if (k > 0)
                    R->rw[c] -= (E13(i + 1, k) - E13(i, k)) / g->dx + (E23(j + 1, k) - E23(j, k)) / g->dy +
                                (TT(i, j, k, 2) - TT(i, j, k - 1, 2)) / (0.5 * (g->dz[k - 1] + g->dz[k]));
                /* heat: face fluxes as 2-cell means, zero through the lids */
                double hx0 = 0.5 * (TT(i - 1, j, k, 6) + TT(i, j, k, 6)), hx1 = 0.5 * (TT(i, j, k, 6) + TT(i + 1, j, k, 6));
                double hy0 = 0.5 * (TT(i, j - 1, k, 7) + TT(i, j, k, 7)), hy1 = 0.5 * (TT(i, j, k, 7) + TT(i, j + 1, k, 7));
                double hz0 = (k == 0) ? 0.0 : 0.5 * (TT(i, j, k - 1, 8) + TT(i, j, k, 8));
                double hz1 = (k == nz - 1) ? 0.0 : 0.5 * (TT(i, j, k, 8) + TT(i, j, k + 1, 8));
                R->rt[c] -= (hx1 - hx0) / g->dx + (hy1 - hy0) / g->dy + (hz1 - hz0) / g->dz[k];
#undef E12
#undef E13
#undef E23
            }
#undef TT
    if (fallback_out) *fallback_out = nfb;
    free(feat); free(xs); free(ys); free(th); free(u); free(v); free(w); free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Kessler warm-rain microphysics (Sec. 2.4, the scheme of Kessler 1969 in   */
/* the form of Klemp & Wilhelmson 1978), applied after a dynamics step       */
/* ------------------------------------------------------------------------ */
/* Readings (the paper names the scheme, not its constants):
 *  - latent heat of vaporisation 2.5e6 J/kg;
 *  - saturation vapour pressure over water of Bolton (1980), in place of
 *    the polynomial fit the paper cites without its coefficients;
 *    q_vs = (R_d/R_v) e_s / (p - e_s);
 *  - autoconversion k1 (q_c - a)^+ with k1 = 1e-3 1/s, a = 1e-3 kg/kg;
 *    accretion k2 q_c q_r^0.875 with k2 = 2.2 1/s;
 *  - rain evaporation (1 - q_v/q_vs) C (rho q_r)^0.525 / (rho (5.4e5 +
 *    2.55e6 / (p q_vs))), C = 1.6 + 124.9 (rho q_r)^0.2046, with rho in
 *    g/cm^3 and p in hPa, limited by the rain present and by saturation;
 *  - terminal velocity of rain 36.34 (rho q_r)^0.1364 (rho_s / rho)^(1/2)
 *    m/s (rho q_r in g/cm^3, rho_s the base state's lowest density);
 *  - order within a step: rain sedimentation (upwind, sub-stepped at a
 *    fall Courant number of at most 0.8), then autoconversion and
 *    accretion, rain evaporation, and the saturation adjustment of cloud
 *    water; the pressure (hence the Exner function) is that of the state
 *    at the start of the step and is held during it;
 *  - the saturation adjustment solves q_v - d = q_vs(T + L d / c_p, p) for
 *    the condensed amount d by six Newton steps from d = 0, clamped to
 *    [-q_c, q_v] (all cloud evaporates where the air stays subsaturated). */
static const double L_V = 2.5e6;

double orc_esat(double T) { return 611.2 * exp(17.67 * (T - 273.15) / (T - 29.65)); }

double orc_qvsat(double T, double p)
{
    double e = orc_esat(T);
    return (R_D / R_V) * e / (p - e);
}

/* d q_vs / dT at fixed pressure */
static double dqvsat_dT(double T, double p)
{
    double e = orc_esat(T);
    double dlne = 17.67 * (273.15 - 29.65) / ((T - 29.65) * (T - 29.65));
    return (R_D / R_V) * p * e * dlne / ((p - e) * (p - e));
}

/* the condensed amount d of the saturation adjustment (module comment) */
double orc_sat_adjust(double T, double p, double qv, double qc)
{
    if (qc <= 0.0 && qv <= orc_qvsat(T, p)) return 0.0;
    double d = 0.0;
    for (int it = 0; it < 6; ++it) {
        double Tn = T + L_V * d / C_P;
        double f = qv - d - orc_qvsat(Tn, p);
        double df = -1.0 - dqvsat_dT(Tn, p) * L_V / C_P;
        d = d - f / df;
    }
    if (d < -qc) d = -qc;
    if (d > qv) d = qv;
    return d;
}

static double fall_speed(double rho, double qr, double rho_s)
{
    double rqr = 1e-3 * rho * qr;
    return rqr > 0.0 ? 36.34 * pow(rqr, 0.1364) * sqrt(rho_s / rho) : 0.0;
}

int orc_kessler(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S, double dt,
                double *precip)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz, nxy = (size_t)nx * ny;
    if (P->n_scalars < 3 || !S->rq || !(dt > 0.0)) return -1;
    double *rqv = S->rq, *rqc = S->rq + n, *rqr = S->rq + 2 * n;
    double rho_s = B->rho0[0];
#pragma omp parallel for schedule(static)
    for (size_t col = 0; col < nxy; ++col) {
        double *V = dalloc(nz);
        /* 1. sedimentation of rain, flux form, upwind from above */
        double cmax = 0.0;
        for (int k = 0; k < nz; ++k) {
            size_t c = col + (size_t)k * nxy;
            V[k] = fall_speed(S->rho[c], rqr[c] / S->rho[c], rho_s);
            if (V[k] * dt / g->dz[k] > cmax) cmax = V[k] * dt / g->dz[k];
        }
        int nsub = (int)ceil(cmax / 0.8);
        if (nsub < 1) nsub = 1;
        double dts = dt / nsub;
        for (int s = 0; s < nsub; ++s) {
            if (s > 0)
                for (int k = 0; k < nz; ++k) {
                    size_t c = col + (size_t)k * nxy;
                    V[k] = fall_speed(S->rho[c], rqr[c] / S->rho[c], rho_s);
                }
            /* flux out of cell k through its bottom face: (rho q_r)_k V_k */
            double out0 = rqr[col] * V[0];
            for (int k = 0; k < nz; ++k) {
                size_t c = col + (size_t)k * nxy;
                double fin = (k + 1 < nz) ? rqr[c + nxy] * V[k + 1] : 0.0;
                double fout = rqr[c] * V[k];
                rqr[c] = rqr[c] + dts * (fin - fout) / g->dz[k];
            }
            if (precip) precip[col] += dts * out0;
        }
        free(V);
        /* 2-4. the cell processes */
        for (int k = 0; k < nz; ++k) {
            size_t c = col + (size_t)k * nxy;
            double rho = S->rho[c], theta = S->rt[c] / rho;
            double qv = rqv[c] / rho, qc = rqc[c] / rho, qr = rqr[c] / rho;
            double pi = exner(S->rt[c] * (1.0 + EPS_V * qv));
            double p = P_00 * pow(pi, C_P / R_D);
            double T = theta * pi;
            /* autoconversion and accretion */
            double auto_ = qc > 1e-3 ? 1e-3 * (qc - 1e-3) : 0.0;
            double accr = qr > 0.0 ? 2.2 * qc * pow(qr, 0.875) : 0.0;
            double prod = dt * (auto_ + accr);
            if (prod > qc) prod = qc;
            qc -= prod;
            qr += prod;
            /* evaporation of rain into subsaturated air */
            double qvs = orc_qvsat(T, p), ev = 0.0;
            if (qr > 0.0 && qv < qvs) {
                double rg = 1e-3 * rho, rqr_g = rg * qr;
                double cv = 1.6 + 124.9 * pow(rqr_g, 0.2046);
                double er = (1.0 - qv / qvs) * cv * pow(rqr_g, 0.525) / (rg * (5.4e5 + 2.55e6 / (1e-2 * p * qvs)));
                ev = dt * er;
                if (ev > qr) ev = qr;
                if (ev > qvs - qv) ev = qvs - qv;
                qv += ev;
                T -= L_V * ev / C_P;
            }
            /* saturation adjustment of cloud water */
            double d = orc_sat_adjust(T, p, qv, qc);
            /* the state changes by the increments of the three processes, so
             * that a cell where nothing happens keeps its values bit for bit */
            rqv[c] += rho * (ev - d);
            rqc[c] += rho * (d - prod);
            rqr[c] += rho * (prod - ev);
            S->rt[c] += rho * L_V * (d - ev) / (C_P * pi);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* anelastic mode (Sec. 2.2, Sec. 3.2)                                       */
/* ------------------------------------------------------------------------ */
static const double TWO_PI = 6.283185307179586476925286766559;

/* finite-volume divergence of the face momenta, eq. (anelastic) */
int orc_divergence(const orc_grid *g, const double *ru, const double *rv, const double *rw, double *D)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = CIDX(g, i, j, k);
                D[c] = (cget(g, ru, i + 1, j, k) - ru[c]) / g->dx + (cget(g, rv, i, j + 1, k) - rv[c]) / g->dy +
                       (rw[CIDX(g, i, j, k + 1)] - rw[c]) / g->dz[k];
            }
    return 0;
}

/* The discrete Fourier transform by its definition, out_m = sum_t in_t
 * exp(sign 2 pi i m t / n), of n values read with stride s, written to
 * contiguous out arrays; cs/sn hold cos and sin of 2 pi r / n for r < n,
 * indexed by the phase m t reduced modulo n. */
static void dft(int n, int s, const double *re, const double *im, double *ore, double *oim, int sign,
                const double *cs, const double *sn)
{
    for (int m = 0; m < n; ++m) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < n; ++t) {
            long r = ((long)m * t) % n;
            double cr = cs[r], ci = sign * sn[r];
            sr += re[(size_t)t * s] * cr - im[(size_t)t * s] * ci;
            si += re[(size_t)t * s] * ci + im[(size_t)t * s] * cr;
        }
        ore[m] = sr;
        oim[m] = si;
    }
}

/* transform every x-line (dir 0) or y-line (dir 1) of every level in place */
static void dft_lines(const orc_grid *g, double *re, double *im, int dir, int sign)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    int len = dir == 0 ? nx : ny, stride = dir == 0 ? 1 : nx, lines = dir == 0 ? ny : nx;
    double *tr = dalloc(len), *ti = dalloc(len), *cs = dalloc(len), *sn = dalloc(len);
    for (int r = 0; r < len; ++r) {
        cs[r] = cos(TWO_PI * r / len);
        sn[r] = sin(TWO_PI * r / len);
    }
    for (int k = 0; k < nz; ++k)
        for (int l = 0; l < lines; ++l) {
            size_t b = dir == 0 ? CIDX(g, 0, l, k) : CIDX(g, l, 0, k);
            dft(len, stride, re + b, im + b, tr, ti, sign, cs, sn);
            for (int t = 0; t < len; ++t) {
                re[b + (size_t)t * stride] = tr[t];
                im[b + (size_t)t * stride] = ti[t];
            }
        }
    free(tr);
    free(ti);
    free(cs);
    free(sn);
}

int orc_poisson(const orc_grid *g, const double *D, double *phi)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (nx < 1 || ny < 1 || nz < 1) return -2;
    size_t n = (size_t)nx * ny * nz;
    double *re = dalloc(n), *im = dalloc(n);
    memcpy(re, D, n * sizeof(double));
    dft_lines(g, re, im, 0, -1);
    dft_lines(g, re, im, 1, -1);
    /* per horizontal wavenumber (m, l): the x and y second differences act
     * on exp(2 pi i (m x/nx dx + l y/ny dy)) as multiplication by
     * -4 sin^2(pi m/nx)/dx^2 - 4 sin^2(pi l/ny)/dy^2; the z operator stays a
     * tridiagonal matrix, with no flux through the lids */
    double *a = dalloc(nz), *b = dalloc(nz), *c = dalloc(nz), *rr = dalloc(nz), *ri = dalloc(nz);
    double *xr = dalloc(nz), *xi = dalloc(nz);
    for (int l = 0; l < ny; ++l)
        for (int m = 0; m < nx; ++m) {
            double sx = sin(0.5 * TWO_PI * m / nx), sy = sin(0.5 * TWO_PI * l / ny);
            double lam = -4.0 * sx * sx / (g->dx * g->dx) - 4.0 * sy * sy / (g->dy * g->dy);
            for (int k = 0; k < nz; ++k) {
                a[k] = k > 0 ? 1.0 / (g->dz[k] * 0.5 * (g->dz[k - 1] + g->dz[k])) : 0.0;
                c[k] = k < nz - 1 ? 1.0 / (g->dz[k] * 0.5 * (g->dz[k] + g->dz[k + 1])) : 0.0;
                b[k] = -a[k] - c[k] + lam;
                rr[k] = re[CIDX(g, m, l, k)];
                ri[k] = im[CIDX(g, m, l, k)];
            }
            if (m == 0 && l == 0) {
                /* the gauge: this mode's value in the lowest cell is zero */
                b[0] = 1.0;
                c[0] = 0.0;
                rr[0] = 0.0;
                ri[0] = 0.0;
            }
            orc_thomas(nz, a, b, c, rr, xr);
            orc_thomas(nz, a, b, c, ri, xi);
            for (int k = 0; k < nz; ++k) {
                re[CIDX(g, m, l, k)] = xr[k];
                im[CIDX(g, m, l, k)] = xi[k];
            }
        }
    dft_lines(g, re, im, 1, 1);
    dft_lines(g, re, im, 0, 1);
    for (size_t q = 0; q < n; ++q) phi[q] = re[q] / ((double)nx * ny);
    free(re); free(im); free(a); free(b); free(c); free(rr); free(ri); free(xr); free(xi);
    return 0;
}

int orc_project(const orc_grid *g, double *ru, double *rv, double *rw, double dt, double *pp)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    size_t n = (size_t)nx * ny * nz;
    double *D = dalloc(n), *phi = dalloc(n);
    orc_divergence(g, ru, rv, rw, D);
    int rc = orc_poisson(g, D, phi);
    if (rc == 0) {
        /* (rho0 u)^new = (rho0 u)^* - dt grad psi with dt psi = phi */
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t c = CIDX(g, i, j, k);
                    ru[c] -= (phi[c] - cget(g, phi, i - 1, j, k)) / g->dx;
                    rv[c] -= (phi[c] - cget(g, phi, i, j - 1, k)) / g->dy;
                    if (k > 0) rw[c] -= (phi[c] - phi[CIDX(g, i, j, k - 1)]) / (0.5 * (g->dz[k - 1] + g->dz[k]));
                    if (pp) pp[c] += phi[c] / dt;
                }
    }
    free(D);
    free(phi);
    return rc;
}

/* S^* = S^n + dt f(S^n), projected; S^{n+1} = S^n + dt (f(S^n) + f(S^*)) / 2,
 * projected.  The slow right-hand side uses the latest perturbation pressure
 * (lagged in the first stage).  Scalars follow the same two stages with the
 * current momenta as fluxes (continuity is the constraint, so the mixing
 * ratio is rho q / rho0). */
int orc_ssprk2_step(const orc_grid *g, const orc_params *P, const orc_base *B, orc_state *S, double *pp)
{
    if (!P->anelastic || !pp) return -1;
    int nx = g->nx, ny = g->ny, nz = g->nz, nq = P->n_scalars;
    size_t n = (size_t)nx * ny * nz, nw = (size_t)nx * ny * (nz + 1), nqn = (size_t)(nq > 0 ? nq : 0) * n;
    double dt = P->dt;
    orc_params Q = *P;
    Q.p_anel = pp;
    orc_state R1, R2, Ss;
    double *bufs[3][6];
    size_t sz[6] = {n, n, n, n, nw, nqn};
    for (int b = 0; b < 3; ++b)
        for (int f = 0; f < 6; ++f) bufs[b][f] = dalloc(sz[f]);
#define BIND(st, b) st.rho = bufs[b][0], st.rt = bufs[b][1], st.ru = bufs[b][2], st.rv = bufs[b][3], st.rw = bufs[b][4], st.rq = bufs[b][5]
    BIND(R1, 0);
    BIND(R2, 1);
    BIND(Ss, 2);
#undef BIND
    double *tmp = dalloc(nqn);
    int rc = orc_slow_rhs(g, &Q, B, S, &R1);
    if (rc == 0) {
        memcpy(Ss.rho, S->rho, n * 8);
        for (size_t c = 0; c < n; ++c) {
            Ss.rt[c] = S->rt[c] + dt * R1.rt[c];
            Ss.ru[c] = S->ru[c] + dt * R1.ru[c];
            Ss.rv[c] = S->rv[c] + dt * R1.rv[c];
        }
        for (size_t c = 0; c < nw; ++c) Ss.rw[c] = S->rw[c] + dt * R1.rw[c];
        if (nq > 0) rc = orc_scalar_advance(g, &Q, S, S, S->ru, S->rv, S->rw, dt, NULL, Ss.rq);
    }
    if (rc == 0) rc = orc_project(g, Ss.ru, Ss.rv, Ss.rw, dt, pp);
    if (rc == 0) rc = orc_slow_rhs(g, &Q, B, &Ss, &R2);
    if (rc == 0 && nq > 0) rc = orc_scalar_advance(g, &Q, S, &Ss, Ss.ru, Ss.rv, Ss.rw, dt, NULL, tmp);
    if (rc == 0) {
        for (size_t c = 0; c < n; ++c) {
            S->rt[c] = S->rt[c] + 0.5 * dt * (R1.rt[c] + R2.rt[c]);
            S->ru[c] = S->ru[c] + 0.5 * dt * (R1.ru[c] + R2.ru[c]);
            S->rv[c] = S->rv[c] + 0.5 * dt * (R1.rv[c] + R2.rv[c]);
        }
        for (size_t c = 0; c < nw; ++c) S->rw[c] = S->rw[c] + 0.5 * dt * (R1.rw[c] + R2.rw[c]);
        /* (rho q)^n - dt (div^n + div^*)/2 = ((rho q)^* + (rho q)^n - dt div^*)/2 */
        for (size_t c = 0; c < nqn; ++c) S->rq[c] = 0.5 * (Ss.rq[c] + tmp[c]);
        rc = orc_project(g, S->ru, S->rv, S->rw, dt, pp);
    }
    for (int b = 0; b < 3; ++b)
        for (int f = 0; f < 6; ++f) free(bufs[b][f]);
    free(tmp);
    return rc;
}
