// terrain.hip -- terrain-following coordinates on the FP64 path (Sec. 3.4,
// App. A, App. B, App. C): the slow right-hand side and one RK stage of
// acoustic substeps with the metric terms (and the stage-averaged fluxes of
// the scalars, whose update is k_ter_scalar in scalars.hip), for dry,
// inviscid, compressible contexts.
//
// Geometry (erf_set_terrain, on the host): node heights z = zeta + s(zeta)
// h(x, y) with s = (1 - zeta/z_t)^beta; per column hb, the mean of the cell's
// four corner heights; per level s_k; per cell the physical height Hc = dz_k +
// (s_{k+1} - s_k) hb and the Jacobian h_zeta = Hc / dz_k.  The face metrics
// are tables: h_zeta on x- and y-faces (two-cell means), h_xi on the x-face i
// the difference of the two cells' centre heights over dx, (s_k + s_{k+1})/2
// (hb_i - hb_{i-1}) / dx, and on the z-face k s_k times the fourth-order
// centred difference of hb (App. B); h_eta alike.  The base state is stored
// per cell.  The stencil kernels run on tiles of 64 x 4 cells of one level, so
// that the rows a y-stencil reaches are shared within a block.
//
// Kernels:
//   k_ter_prep  theta, u, v, w, p' and rho Omega = rho w - M on the z-faces,
//               M = h_xi <rho u> + h_eta <rho v> with the horizontal momenta
//               averaged from the four faces around the z-face; the lid
//               faces keep rho w (zero)
//   k_ter_rhs   slow tendencies (four kernels: continuity and theta, x-, y- and
//               z-momentum): horizontal mass fluxes weighted by the face's
//               h_zeta, rho Omega through the z-faces, each divergence divided
//               by its control volume's h_zeta; the pressure gradient
//               p_x = p_xi - h_xi (p_zeta / h_zeta), the last factor the mean
//               of the two cells' centred vertical differences over the
//               physical distance (one-sided in the lowest and highest
//               cells); buoyancy about the per-cell base state; Coriolis; a
//               surface heat flux into the lowest cell over its physical height
//   k_ter_init  S'' = S^n - S^t, theta^t and pi^t
//   k_ter_uv    U'', V'' with the metric correction of the gradient of the
//               predicted Theta''
//   k_ter_m     M(U'', V'') of the new horizontal momenta on every z-face (the
//               next substep reuses it as the old one)
//   k_ter_hat   per cell, the explicit parts of Theta'' and rho'' with
//               Omega'' = W'' - M, the M of the new horizontal momenta moved
//               to the known side
//   k_ter_tri   one thread per column: the tridiagonal W'' rows with the
//               column's physical heights built on the fly, the forward sweep
//               and the back substitution (each level's loads issued three
//               levels ahead), the implicit finish of Theta'' and rho'' fused
//               into the back substitution
//   k_ter_fin   S_out = S^t + S''; with scalars, the stage-averaged fluxes
//               S^t + the substeps' mean, rho Omega vertically (the
//               beta-weighted Omega'' summed in k_ter_tri)
// All arithmetic is FP64, written in the order of the oracle's expressions so
// that the two round alike.
#include "erf_internal.h"

namespace erfk {
namespace {

constexpr int kTB = 256;  // threads per block of the per-cell kernels (64 x 4 tiles for the stencil kernels)
constexpr int kCB = 64;   // columns per block of the column kernel

struct Geo {
    Dims d;
    double dx, dy;
    const double *dz, *Hc, *Jc;
    // face metrics tabulated at set-up (the expressions below, evaluated in
    // the same order on the host): h_zeta on x- and y-faces, h_xi on x-faces,
    // h_eta on y-faces [n]; h_xi, h_eta on z-faces [nw]
    const double *JUt, *JVt, *hxUt, *heVt, *hxWt, *heWt;
    // the physical distance of the centres above and below each cell (one
    // level each way, one-sided in the lowest and highest cells) [n]
    const double *dzcT;

    __device__ __forceinline__ int c(int i, int j, int k) const
    {
        return (k * d.ny + wrap_idx(j, d.ny)) * d.nx + wrap_idx(i, d.nx);
    }
    __device__ __forceinline__ double H(int i, int j, int k) const { return Hc[c(i, j, k)]; }
    // h_zeta = Hc / dz_k, tabulated at set-up
    __device__ __forceinline__ double J(int i, int j, int k) const { return Jc[c(i, j, k)]; }
    // h_zeta on the x-face i: 0.5 (J_{i-1} + J_i); on the y-face j likewise
    __device__ __forceinline__ double JU(int i, int j, int k) const { return JUt[c(i, j, k)]; }
    __device__ __forceinline__ double JV(int i, int j, int k) const { return JVt[c(i, j, k)]; }
    // h_xi on the x-face i: 0.5 (s_k + s_{k+1}) (hb_i - hb_{i-1}) / dx; h_eta alike
    __device__ __forceinline__ double hxU(int i, int j, int k) const { return hxUt[c(i, j, k)]; }
    __device__ __forceinline__ double heV(int i, int j, int k) const { return heVt[c(i, j, k)]; }
    // h_xi on the z-face k: s_k ((hb_{i-2} - hb_{i+2}) + 8 (hb_{i+1} - hb_{i-1})) / (12 dx); h_eta alike
    __device__ __forceinline__ double hxW(int i, int j, int k) const { return hxWt[c(i, j, k)]; }
    __device__ __forceinline__ double heW(int i, int j, int k) const { return heWt[c(i, j, k)]; }
    // the metric part M of rho Omega (or of Omega'') on the z-face k; zero on the lids
    __device__ __forceinline__ double M(const double *ru, const double *rv, int i, int j, int k) const
    {
        if (k == 0 || k == d.nz) return 0.0;
        const double su = (ru[c(i, j, k)] + ru[c(i + 1, j, k)]) + (ru[c(i, j, k - 1)] + ru[c(i + 1, j, k - 1)]);
        const double sv = (rv[c(i, j, k)] + rv[c(i, j + 1, k)]) + (rv[c(i, j, k - 1)] + rv[c(i, j + 1, k - 1)]);
        return 0.25 * hxW(i, j, k) * su + 0.25 * heW(i, j, k) * sv;
    }
    // (f_zeta / h_zeta) of a cell field at a cell (f given per cell index)
    template <typename F>
    __device__ __forceinline__ double fz(F f, int i, int j, int k) const
    {
        const int nz = d.nz;
        if (nz < 2) return 0.0;
        const int kl = k > 0 ? k - 1 : 0, ku = k < nz - 1 ? k + 1 : nz - 1;
        return (f(c(i, j, ku)) - f(c(i, j, kl))) / dzcT[c(i, j, k)];
    }
};

__device__ __forceinline__ void split(const Dims &d, int q, int &i, int &j, int &k)
{
    k = q / d.nxy;
    const int r = q - k * d.nxy;
    j = r / d.nx;
    i = r - j * d.nx;
}

// The stencil kernels' blocks are tiles of 64 x 4 cells of one level
// (blockIdx.x over the tiles of a level, blockIdx.y the level), so that the
// rows a y-stencil reaches are shared within a block.  False for the threads
// of a ragged tile that lie outside the domain.
__device__ __forceinline__ bool tile_cell(const Dims &d, int &i, int &j, int &k, int &q)
{
    const int ntx = (d.nx + 63) >> 6;
    const int ty = blockIdx.x / ntx, tx = blockIdx.x - ty * ntx;
    i = (tx << 6) + (threadIdx.x & 63);
    j = (ty << 2) + (threadIdx.x >> 6);
    k = blockIdx.y;
    q = (k * d.ny + j) * d.nx + i;
    return i < d.nx && j < d.ny;
}
inline dim3 tile_grid(const Dims &d, int levels) { return dim3(((d.nx + 63) / 64) * ((d.ny + 3) / 4), levels); }

// ---------------------------------------------------------------------------
// slow right-hand side
// ---------------------------------------------------------------------------
struct RhsA {
    Geo G;
    double g, f_cor, Ug, Vg;
    double qs;  // prescribed kinematic surface heat flux (per unit horizontal area)
    int oh, ov;
    const double *rho0, *Theta0, *p0;
    const double *rho, *rt, *ru, *rv, *rw;
    double *th, *u, *v, *w, *pp, *om;
    double *Rr, *Rt, *Ru, *Rv, *Rw;
};

__global__ void __launch_bounds__(kTB) k_ter_prep(RhsA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    int i, j, k, q;
    if (!tile_cell(d, i, j, k, q)) return;
    if (k < d.nz) {
        const double r = a.rho[q];
        a.th[q] = a.rt[q] / r;
        a.u[q] = a.ru[q] / (0.5 * (a.rho[G.c(i - 1, j, k)] + r));
        a.v[q] = a.rv[q] / (0.5 * (a.rho[G.c(i, j - 1, k)] + r));
        a.pp[q] = a.p0[q] * expm1(kGamma * log1p((a.rt[q] - a.Theta0[q]) / a.Theta0[q]));
    }
    const bool lid = k == 0 || k == d.nz;
    a.w[q] = lid ? 0.0 : a.rw[q] / (0.5 * (a.rho[q - d.nxy] + a.rho[q]));
    a.om[q] = lid ? a.rw[q] : a.rw[q] - G.M(a.ru, a.rv, i, j, k);
}

// face value q_{m-1/2} of a cell (or horizontal-face) field along x, y, z, and
// of a z-face field along x, y (periodic) and z (odd about the lids)
__device__ __forceinline__ double ix(const Geo &G, const double *f, int i, int j, int k, int o, double sg)
{
    return face_interp<double>(o, f[G.c(i - 3, j, k)], f[G.c(i - 2, j, k)], f[G.c(i - 1, j, k)], f[G.c(i, j, k)],
                               f[G.c(i + 1, j, k)], f[G.c(i + 2, j, k)], sg);
}
__device__ __forceinline__ double iy(const Geo &G, const double *f, int i, int j, int k, int o, double sg)
{
    return face_interp<double>(o, f[G.c(i, j - 3, k)], f[G.c(i, j - 2, k)], f[G.c(i, j - 1, k)], f[G.c(i, j, k)],
                               f[G.c(i, j + 1, k)], f[G.c(i, j + 2, k)], sg);
}
__device__ __forceinline__ double izc(const Geo &G, const double *f, int i, int j, int k, int o, double sg)
{
    const int nz = G.d.nz;
    double q[6];
    for (int m = 0; m < 6; ++m) q[m] = f[G.c(i, j, refl_centre(k - 3 + m, nz))];
    return face_interp<double>(o, q[0], q[1], q[2], q[3], q[4], q[5], sg);
}
__device__ __forceinline__ double izw(const Geo &G, const double *f, int i, int j, int k, int o, double sg)
{
    const int nz = G.d.nz;
    double q[6];
    for (int m = 0; m < 6; ++m) {
        double sgn;
        const int kk = refl_face(k - 3 + m, nz, sgn);
        q[m] = sgn * f[G.c(i, j, kk)];
    }
    return face_interp<double>(o, q[0], q[1], q[2], q[3], q[4], q[5], sg);
}

// P selects the equations of one launch: 0 continuity and potential
// temperature, 1 x-momentum, 2 y-momentum, 3 z-momentum (four smaller kernels
// keep more wavefronts resident than one that evaluates all five)
template <int P>
__global__ void __launch_bounds__(kTB) k_ter_rhs(RhsA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    int i, j, k, q;
    if (!tile_cell(d, i, j, k, q)) return;
    const int nz = d.nz, oh = a.oh, ov = a.ov;
    const double dx = G.dx, dy = G.dy;
    const double *ru = a.ru, *rv = a.rv, *om = a.om, *pp = a.pp;
    if (P < 3) {
        if (k >= nz) return;
        const int c = q;
        // continuity and potential temperature
        if (P == 0) {
            const double U0 = G.JU(i, j, k) * ru[c], U1 = G.JU(i + 1, j, k) * ru[G.c(i + 1, j, k)];
            const double V0 = G.JV(i, j, k) * rv[c], V1 = G.JV(i, j + 1, k) * rv[G.c(i, j + 1, k)];
            const double W0 = om[c], W1 = om[c + d.nxy];
            const double Jc = G.J(i, j, k);
            a.Rr[c] = -((U1 - U0) / dx + (V1 - V0) / dy + (W1 - W0) / G.dz[k]) / Jc;
            const double fx0 = U0 * ix(G, a.th, i, j, k, oh, sign_of(U0));
            const double fx1 = U1 * ix(G, a.th, i + 1, j, k, oh, sign_of(U1));
            const double fy0 = V0 * iy(G, a.th, i, j, k, oh, sign_of(V0));
            const double fy1 = V1 * iy(G, a.th, i, j + 1, k, oh, sign_of(V1));
            const double fz0 = (k == 0) ? 0.0 : W0 * izc(G, a.th, i, j, k, ov, sign_of(W0));
            const double fz1 = (k == nz - 1) ? 0.0 : W1 * izc(G, a.th, i, j, k + 1, ov, sign_of(W1));
            double rt = -((fx1 - fx0) / dx + (fy1 - fy0) / dy + (fz1 - fz0) / G.dz[k]) / Jc;
            // the surface heat flux enters the lowest cell over its physical height
            if (k == 0 && a.qs != 0.0) rt += a.rho[c] * a.qs / G.Hc[c];
            a.Rt[c] = rt;
        }
        const auto pf = [&](int cc) { return pp[cc]; };
        // x-momentum on the x-face i
        if (P == 1) {
            const double a_r = 0.5 * (G.JU(i, j, k) * ru[c] + G.JU(i + 1, j, k) * ru[G.c(i + 1, j, k)]);
            const double a_l = 0.5 * (G.JU(i - 1, j, k) * ru[G.c(i - 1, j, k)] + G.JU(i, j, k) * ru[c]);
            const double fxx_r = a_r * ix(G, a.u, i + 1, j, k, oh, sign_of(a_r));
            const double fxx_l = a_l * ix(G, a.u, i, j, k, oh, sign_of(a_l));
            const double b_0 = 0.5 * (G.JV(i - 1, j, k) * rv[G.c(i - 1, j, k)] + G.JV(i, j, k) * rv[c]);
            const double b_1 = 0.5 * (G.JV(i - 1, j + 1, k) * rv[G.c(i - 1, j + 1, k)] +
                                      G.JV(i, j + 1, k) * rv[G.c(i, j + 1, k)]);
            const double fxy0 = b_0 * iy(G, a.u, i, j, k, oh, sign_of(b_0));
            const double fxy1 = b_1 * iy(G, a.u, i, j + 1, k, oh, sign_of(b_1));
            const double e_0 = (k == 0) ? 0.0 : 0.5 * (om[G.c(i - 1, j, k)] + om[c]);
            const double e_1 = (k == nz - 1) ? 0.0 : 0.5 * (om[G.c(i - 1, j, k + 1)] + om[c + d.nxy]);
            const double fxz0 = (k == 0) ? 0.0 : e_0 * izc(G, a.u, i, j, k, ov, sign_of(e_0));
            const double fxz1 = (k == nz - 1) ? 0.0 : e_1 * izc(G, a.u, i, j, k + 1, ov, sign_of(e_1));
            const double adv = ((fxx_r - fxx_l) / dx + (fxy1 - fxy0) / dy + (fxz1 - fxz0) / G.dz[k]) / G.JU(i, j, k);
            double pgf = (pp[c] - pp[G.c(i - 1, j, k)]) / dx;
            pgf -= 0.5 * G.hxU(i, j, k) * (G.fz(pf, i, j, k) + G.fz(pf, i - 1, j, k));
            const double rho_f = 0.5 * (a.rho[G.c(i - 1, j, k)] + a.rho[c]);
            const double vbar = 0.25 * (rv[G.c(i - 1, j, k)] + rv[c] + rv[G.c(i - 1, j + 1, k)] + rv[G.c(i, j + 1, k)]);
            const double cor = a.f_cor * (vbar - rho_f * a.Vg);
            a.Ru[c] = -adv - pgf + cor;
        }
        // y-momentum on the y-face j
        if (P == 2) {
            const double b_r = 0.5 * (G.JV(i, j, k) * rv[c] + G.JV(i, j + 1, k) * rv[G.c(i, j + 1, k)]);
            const double b_l = 0.5 * (G.JV(i, j - 1, k) * rv[G.c(i, j - 1, k)] + G.JV(i, j, k) * rv[c]);
            const double fyy_r = b_r * iy(G, a.v, i, j + 1, k, oh, sign_of(b_r));
            const double fyy_l = b_l * iy(G, a.v, i, j, k, oh, sign_of(b_l));
            const double a_0 = 0.5 * (G.JU(i, j - 1, k) * ru[G.c(i, j - 1, k)] + G.JU(i, j, k) * ru[c]);
            const double a_1 = 0.5 * (G.JU(i + 1, j - 1, k) * ru[G.c(i + 1, j - 1, k)] +
                                      G.JU(i + 1, j, k) * ru[G.c(i + 1, j, k)]);
            const double fyx0 = a_0 * ix(G, a.v, i, j, k, oh, sign_of(a_0));
            const double fyx1 = a_1 * ix(G, a.v, i + 1, j, k, oh, sign_of(a_1));
            const double e_0 = (k == 0) ? 0.0 : 0.5 * (om[G.c(i, j - 1, k)] + om[c]);
            const double e_1 = (k == nz - 1) ? 0.0 : 0.5 * (om[G.c(i, j - 1, k + 1)] + om[c + d.nxy]);
            const double fyz0 = (k == 0) ? 0.0 : e_0 * izc(G, a.v, i, j, k, ov, sign_of(e_0));
            const double fyz1 = (k == nz - 1) ? 0.0 : e_1 * izc(G, a.v, i, j, k + 1, ov, sign_of(e_1));
            const double adv = ((fyx1 - fyx0) / dx + (fyy_r - fyy_l) / dy + (fyz1 - fyz0) / G.dz[k]) / G.JV(i, j, k);
            double pgf = (pp[c] - pp[G.c(i, j - 1, k)]) / dy;
            pgf -= 0.5 * G.heV(i, j, k) * (G.fz(pf, i, j, k) + G.fz(pf, i, j - 1, k));
            const double rho_f = 0.5 * (a.rho[G.c(i, j - 1, k)] + a.rho[c]);
            const double ubar = 0.25 * (ru[G.c(i, j - 1, k)] + ru[G.c(i + 1, j - 1, k)] + ru[c] + ru[G.c(i + 1, j, k)]);
            const double cor = -a.f_cor * (ubar - rho_f * a.Ug);
            a.Rv[c] = -adv - pgf + cor;
        }
        return;
    }
    // z-momentum on the z-face k (zero on the lids)
    if (k == 0 || k == nz) {
        a.Rw[q] = 0.0;
        return;
    }
    const int c = q, cm = q - d.nxy;
    const double dzf = 0.5 * (G.dz[k - 1] + G.dz[k]);
    const double dzp = 0.5 * (G.H(i, j, k - 1) + G.H(i, j, k));
    const double JW = dzp / dzf;
    const double a_0 = 0.5 * (G.JU(i, j, k - 1) * ru[cm] + G.JU(i, j, k) * ru[c]);
    const double a_1 = 0.5 * (G.JU(i + 1, j, k - 1) * ru[G.c(i + 1, j, k - 1)] + G.JU(i + 1, j, k) * ru[G.c(i + 1, j, k)]);
    const double fzx0 = a_0 * ix(G, a.w, i, j, k, oh, sign_of(a_0));
    const double fzx1 = a_1 * ix(G, a.w, i + 1, j, k, oh, sign_of(a_1));
    const double b_0 = 0.5 * (G.JV(i, j, k - 1) * rv[cm] + G.JV(i, j, k) * rv[c]);
    const double b_1 = 0.5 * (G.JV(i, j + 1, k - 1) * rv[G.c(i, j + 1, k - 1)] + G.JV(i, j + 1, k) * rv[G.c(i, j + 1, k)]);
    const double fzy0 = b_0 * iy(G, a.w, i, j, k, oh, sign_of(b_0));
    const double fzy1 = b_1 * iy(G, a.w, i, j + 1, k, oh, sign_of(b_1));
    const double Om = om[c];
    const double e_u = 0.5 * (Om + om[c + d.nxy]);
    const double e_d = 0.5 * (om[cm] + Om);
    const double fzz_u = e_u * izw(G, a.w, i, j, k + 1, ov, sign_of(e_u));
    const double fzz_d = e_d * izw(G, a.w, i, j, k, ov, sign_of(e_d));
    const double adv = ((fzx1 - fzx0) / dx + (fzy1 - fzy0) / dy + (fzz_u - fzz_d) / dzf) / JW;
    const double pgf = (pp[c] - pp[cm]) / dzp;
    const double buoy = -a.g * 0.5 * ((a.rho[c] - a.rho0[c]) + (a.rho[cm] - a.rho0[cm]));
    a.Rw[q] = -adv - pgf + buoy;
}

// ---------------------------------------------------------------------------
// acoustic substeps
// ---------------------------------------------------------------------------
struct StA {
    Geo G;
    double g, dtau, b1, b2, bd;
    const double *rho0, *pi0;
    const double *n_r, *n_t, *n_u, *n_v, *n_w;  // S^n
    const double *t_r, *t_t, *t_u, *t_v, *t_w;  // S^t
    const double *R_r, *R_t, *R_u, *R_v, *R_w;  // R^t
    double *tht, *pit;
    double *t2, *t2p, *u2, *v2, *un, *vn, *r2, *w2, *rh, *cp, *dp;
    double *mo, *mn;  // M of the old and of the new horizontal momenta on z-faces
    // scalars: running sums of U'', V'' and of the beta-weighted Omega'' (null:
    // no sums kept), the substep count and the stage-averaged fluxes written
    // by k_ter_fin (rho Omega vertically)
    double *su, *sv, *sw;
    int nsub;
    double *o_fu, *o_fv, *o_fw;
    double *o_r, *o_t, *o_u, *o_v, *o_w;
};

__global__ void __launch_bounds__(kTB) k_ter_init(StA a)
{
    const Dims &d = a.G.d;
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.nw) return;
    if (q < d.n) {
        const double Tt = a.t_t[q];
        a.tht[q] = Tt / a.t_r[q];
        a.pit[q] = pow(kRd * Tt / kP00, kGamma - 1.0);
        a.u2[q] = a.n_u[q] - a.t_u[q];
        a.v2[q] = a.n_v[q] - a.t_v[q];
        const double T2 = a.n_t[q] - Tt;
        a.t2[q] = T2;
        a.t2p[q] = T2;
        a.r2[q] = a.n_r[q] - a.t_r[q];
        if (a.su) {
            a.su[q] = 0.0;
            a.sv[q] = 0.0;
        }
    }
    a.w2[q] = a.n_w[q] - a.t_w[q];
    if (a.su) a.sw[q] = 0.0;
}

__global__ void __launch_bounds__(kTB) k_ter_uv(StA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    int i, j, k, q;
    if (!tile_cell(d, i, j, k, q)) return;
    const double bd = a.bd;
    // Theta'' predicted forward by beta_d (divergence damping)
    const auto tt = [&](int cc) { return a.t2[cc] + bd * (a.t2[cc] - a.t2p[cc]); };
    const int cw = G.c(i - 1, j, k), cs = G.c(i, j - 1, k);
    const double tt_c = tt(q), tt_w = tt(cw), tt_s = tt(cs);
    const double pfx = 0.5 * (a.pit[cw] + a.pit[q]);
    const double pfy = 0.5 * (a.pit[cs] + a.pit[q]);
    const double fzc = G.fz(tt, i, j, k);
    const double cx = 0.5 * G.hxU(i, j, k) * (fzc + G.fz(tt, i - 1, j, k));
    const double cy = 0.5 * G.heV(i, j, k) * (fzc + G.fz(tt, i, j - 1, k));
    const double un = a.u2[q] + a.dtau * (-kGamma * kRd * pfx * (tt_c - tt_w) / G.dx + kGamma * kRd * pfx * cx + a.R_u[q]);
    const double vn = a.v2[q] + a.dtau * (-kGamma * kRd * pfy * (tt_c - tt_s) / G.dy + kGamma * kRd * pfy * cy + a.R_v[q]);
    a.un[q] = un;
    a.vn[q] = vn;
    if (a.su) {
        a.su[q] += un;
        a.sv[q] += vn;
    }
}

// M(ru, rv) on every z-face (zero on the lids)
__global__ void __launch_bounds__(kTB) k_ter_m(StA a, const double *ru, const double *rv, double *out)
{
    const Geo &G = a.G;
    int i, j, k, q;
    if (!tile_cell(G.d, i, j, k, q)) return;
    out[q] = G.M(ru, rv, i, j, k);
}

__global__ void __launch_bounds__(kTB) k_ter_hat(StA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    int i, j, k, c;
    if (!tile_cell(d, i, j, k, c)) return;
    const int nz = d.nz, nxy = d.nxy;
    const double dtau = a.dtau, b1 = a.b1, b2 = a.b2;
    const double *tht = a.tht;
    const double thc = tht[c];
    const double thx0 = 0.5 * (tht[G.c(i - 1, j, k)] + thc);
    const double thx1 = 0.5 * (thc + tht[G.c(i + 1, j, k)]);
    const double thy0 = 0.5 * (tht[G.c(i, j - 1, k)] + thc);
    const double thy1 = 0.5 * (thc + tht[G.c(i, j + 1, k)]);
    const double Ue = G.JU(i + 1, j, k) * a.un[G.c(i + 1, j, k)], Uw = G.JU(i, j, k) * a.un[c];
    const double Vn_ = G.JV(i, j + 1, k) * a.vn[G.c(i, j + 1, k)], Vs = G.JV(i, j, k) * a.vn[c];
    const double Wt = a.w2[c + nxy] - a.mo[c + nxy], Wb = a.w2[c] - a.mo[c];
    const double Jc = G.J(i, j, k), Hk = G.Hc[c];
    const double hdiv_t = (Ue * thx1 - Uw * thx0) / G.dx + (Vn_ * thy1 - Vs * thy0) / G.dy;
    const double hdiv_r = (Ue - Uw) / G.dx + (Vn_ - Vs) / G.dy;
    // face theta^t above and below the cell (zero on the lids)
    const double tz1 = (k + 1 >= nz) ? 0.0 : 0.5 * (thc + tht[c + nxy]);
    const double tz0 = (k <= 0) ? 0.0 : 0.5 * (tht[c - nxy] + thc);
    double th_hat = a.t2[c] + dtau * (-hdiv_t / Jc - b1 * (Wt * tz1 - Wb * tz0) / Hk + a.R_t[c]);
    double rh_hat = a.r2[c] + dtau * (-hdiv_r / Jc - b1 * (Wt - Wb) / Hk + a.R_r[c]);
    const double Mn1 = a.mn[c + nxy], Mn0 = a.mn[c];
    th_hat += dtau * b2 * (Mn1 * tz1 - Mn0 * tz0) / Hk;
    rh_hat += dtau * b2 * (Mn1 - Mn0) / Hk;
    a.t2p[c] = th_hat;
    a.rh[c] = rh_hat;
}

// The per-level values of the forward sweep at one level of one column.
struct TriLv {
    double H, pit, r0, pi0, tt, th, t2, hat, r2, rh, w2, Rw;
};

// one thread per column; the Thomas factors go through cp, dp (own column)
__global__ void __launch_bounds__(kCB) k_ter_tri(StA a)
{
    const Dims &d = a.G.d;
    const int col = blockIdx.x * kCB + threadIdx.x;
    if (col >= d.nxy) return;
    const int nz = d.nz, nxy = d.nxy, m = nz - 1;
    const double dtau = a.dtau, b1 = a.b1, b2 = a.b2, gr = a.g;
    const double *__restrict__ Hc = a.G.Hc;
    const double *__restrict__ pit = a.pit;
    const double *__restrict__ rho0 = a.rho0;
    const double *__restrict__ pi0 = a.pi0;
    const double *__restrict__ t_t = a.t_t;
    const double *__restrict__ tht = a.tht;
    const double *__restrict__ t2 = a.t2;
    const double *__restrict__ R_w = a.R_w;
    double *__restrict__ hat = a.t2p;
    double *__restrict__ r2 = a.r2;
    double *__restrict__ rh = a.rh;
    double *__restrict__ w2 = a.w2;
    double *__restrict__ cp = a.cp;
    double *__restrict__ dp = a.dp;
    const auto load = [&](int k) {
        const int c = col + k * nxy;
        TriLv v;
        v.H = Hc[c], v.pit = pit[c], v.r0 = rho0[c], v.pi0 = pi0[c], v.tt = t_t[c], v.th = tht[c];
        v.t2 = t2[c], v.hat = hat[c], v.r2 = r2[c], v.rh = rh[c], v.w2 = w2[c], v.Rw = R_w[c];
        return v;
    };
    const double D = dtau * dtau * b2 * b2;
    // Levels k-1 .. k+2 sit in a ring of four (slot = level & 3) while face k
    // is eliminated, and the slot of level k-1 is refilled with level k+3: the
    // loads of a level are issued three levels before their use (one
    // wavefront per SIMD here, so only loads in flight hide the latency).
    TriLv L[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (u < nz) L[u] = load(u);
    double tfm = 0.0, cpm = 0.0, dpm = 0.0;  // face theta^t below, previous factors
    for (int k0 = 1; k0 <= m; k0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u;  // k0 = 1 mod 4: level k is in slot (u + 1) & 3
            if (k > m) break;
            TriLv &lo = L[u & 3];
            const TriLv &up = L[(u + 1) & 3], &nx = L[(u + 2) & 3];
            const int c = col + k * nxy;
            const double dzf = 0.5 * (lo.H + up.H);
            const double pif = 0.5 * (lo.pit + up.pit);
            const double A = kGamma * kRd * (0.5 * (lo.pit + up.pit));
            const double Cc = gr * 0.5 * (lo.r0 + up.r0) * (kRd / kCv) * (pif / (0.5 * (lo.pi0 + up.pi0))) /
                              (0.5 * (lo.tt + up.tt));
            const double idzm = 1.0 / lo.H, idz = 1.0 / up.H;
            const double tf = 0.5 * (lo.th + up.th), tfp = (k + 1 < nz) ? 0.5 * (up.th + nx.th) : 0.0;
            const double ta = (k == 1) ? 0.0 : -D * (A * tfm * idzm / dzf + 0.5 * Cc * tfm * idzm - 0.5 * gr * idzm);
            const double tc = (k == m) ? 0.0 : -D * (A * tfp * idz / dzf - 0.5 * Cc * tfp * idz + 0.5 * gr * idz);
            const double tb =
                1.0 + D * (A * tf * (idz + idzm) / dzf + 0.5 * Cc * tf * (idzm - idz) - 0.5 * gr * (idzm - idz));
            const double tbk = b1 * up.t2 + b2 * up.hat, tbm = b1 * lo.t2 + b2 * lo.hat;
            const double rbk = b1 * up.r2 + b2 * up.rh, rbm = b1 * lo.r2 + b2 * lo.rh;
            const double tr =
                up.w2 + dtau * (-A * (tbk - tbm) / dzf + 0.5 * Cc * (tbk + tbm) - 0.5 * gr * (rbk + rbm) + up.Rw);
            double cpk, dpk;
            if (k == 1) {
                cpk = tc / tb;
                dpk = tr / tb;
            } else {
                const double den = tb - ta * cpm;
                cpk = tc / den;
                dpk = (tr - ta * dpm) / den;
            }
            cp[c] = cpk;
            dp[c] = dpk;
            cpm = cpk, dpm = dpk;
            tfm = tf;
            if (k + 3 < nz) lo = load(k + 3);
        }
    }
    // back substitution (faces m .. 1) with the implicit finish of the cell
    // above each face; the lids carry W'' = 0.  The values of level k (the
    // factors of face k, theta^t below it and the cell's explicit Theta'',
    // rho'' and height) come from a ring of four filled three levels ahead.
    w2[col] = 0.0;
    w2[col + nz * nxy] = 0.0;
    struct BkLv {
        double cp, dp, thl, hat, rh, H;
    };
    const auto bload = [&](int k) {
        const int c = col + k * nxy;
        BkLv v;
        v.cp = k >= 1 ? cp[c] : 0.0;
        v.dp = k >= 1 ? dp[c] : 0.0;
        v.thl = k >= 1 ? tht[c - nxy] : 0.0;
        v.hat = hat[c], v.rh = rh[c], v.H = Hc[c];
        return v;
    };
    const auto finish = [&](int k, const BkLv &v, double Wt, double Wb, double tz1, double tz0) {
        const int c = col + k * nxy;
        hat[c] = v.hat - dtau * b2 * (Wt * tz1 - Wb * tz0) / v.H;
        r2[c] = v.rh - dtau * b2 * (Wt - Wb) / v.H;
    };
    BkLv B[4];  // slot = (m - k) & 3
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (m - u >= 0) B[u] = bload(m - u);
    double xup = 0.0, thu = tht[col + m * nxy], tzu = 0.0;  // W'' above, theta^t of cell k, face theta above
    for (int k0 = m; k0 >= 1; k0 -= 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 - u;  // slot (m - k) & 3 = u, since k0 = m mod 4
            if (k < 1) break;
            BkLv &v = B[u];
            const int c = col + k * nxy;
            const double x = (k == m) ? v.dp : v.dp - v.cp * xup;
            // scalars: Omega'' of this substep with the beta weights
            if (a.sw) a.sw[c] += b1 * (w2[c] - a.mo[c]) + b2 * (x - a.mn[c]);
            w2[c] = x;
            const double tz = 0.5 * (v.thl + thu);
            finish(k, v, xup, x, tzu, tz);
            xup = x;
            tzu = tz;
            thu = v.thl;
            if (k - 4 >= 0) v = bload(k - 4);
        }
    }
    // cell 0: its values are in slot m & 3 (chosen by constant indices, so
    // the ring stays in registers)
    BkLv v0;
    switch (m & 3) {
    case 0: v0 = B[0]; break;
    case 1: v0 = B[1]; break;
    case 2: v0 = B[2]; break;
    default: v0 = B[3]; break;
    }
    finish(0, v0, xup, 0.0, tzu, 0.0);
}

__global__ void __launch_bounds__(kTB) k_ter_fin(StA a)
{
    const Dims &d = a.G.d;
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.nw) return;
    // the stage-averaged fluxes first: o_* may alias S^n, never S^t
    if (a.su) {
        int i, j, k;
        split(d, q, i, j, k);
        const bool lid = k == 0 || k == d.nz;
        const double Om = lid ? a.t_w[q] : a.t_w[q] - a.G.M(a.t_u, a.t_v, i, j, k);
        a.o_fw[q] = Om + a.sw[q] / a.nsub;
        if (q < d.n) {
            a.o_fu[q] = a.t_u[q] + a.su[q] / a.nsub;
            a.o_fv[q] = a.t_v[q] + a.sv[q] / a.nsub;
        }
    }
    if (q < d.n) {
        a.o_r[q] = a.t_r[q] + a.r2[q];
        a.o_t[q] = a.t_t[q] + a.t2[q];
        a.o_u[q] = a.t_u[q] + a.u2[q];
        a.o_v[q] = a.t_v[q] + a.v2[q];
    }
    a.o_w[q] = a.t_w[q] + a.w2[q];
}

Geo geo_of(const erf_ctx *cx)
{
    Geo G;
    G.d = cx->d;
    G.dx = cx->grid.dx;
    G.dy = cx->grid.dy;
    G.dz = cx->base.dz;
    G.Hc = cx->ter.Hc;
    G.Jc = cx->ter.J;
    G.JUt = cx->ter.JU;
    G.JVt = cx->ter.JV;
    G.hxUt = cx->ter.hxU;
    G.heVt = cx->ter.heV;
    G.hxWt = cx->ter.hxW;
    G.heWt = cx->ter.heW;
    G.dzcT = cx->ter.dzc;
    return G;
}

}  // namespace

hipError_t launch_terrain_rhs(erf_ctx *cx, const void *const S[5], void *const R[5])
{
    const Workspace &w = cx->ws;
    RhsA a;
    a.G = geo_of(cx);
    a.g = cx->prm.grav;
    a.f_cor = cx->prm.f_cor;
    a.Ug = cx->prm.Ug;
    a.Vg = cx->prm.Vg;
    a.qs = cx->prm.surf_heat_flux;
    a.oh = cx->prm.adv_order_h;
    a.ov = cx->prm.adv_order_v;
    a.rho0 = cx->ter.rho0;
    a.Theta0 = cx->ter.Theta0;
    a.p0 = cx->ter.p0;
    a.rho = (const double *)S[0];
    a.rt = (const double *)S[1];
    a.ru = (const double *)S[2];
    a.rv = (const double *)S[3];
    a.rw = (const double *)S[4];
    a.th = (double *)w.th;
    a.u = (double *)w.u;
    a.v = (double *)w.v;
    a.w = (double *)w.w;
    a.pp = (double *)w.pp;
    a.om = cx->ter.om;
    a.Rr = (double *)R[0];
    a.Rt = (double *)R[1];
    a.Ru = (double *)R[2];
    a.Rv = (double *)R[3];
    a.Rw = (double *)R[4];
    const dim3 grc = tile_grid(cx->d, cx->d.nz), grw = tile_grid(cx->d, cx->d.nz + 1);
    k_ter_prep<<<grw, kTB, 0, cx->stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_start(cx, K_TER_RHS);
    k_ter_rhs<0><<<grc, kTB, 0, cx->stream>>>(a);
    k_ter_rhs<1><<<grc, kTB, 0, cx->stream>>>(a);
    k_ter_rhs<2><<<grc, kTB, 0, cx->stream>>>(a);
    k_ter_rhs<3><<<grw, kTB, 0, cx->stream>>>(a);
    timing_stop(cx, K_TER_RHS);
    return hipGetLastError();
}

hipError_t launch_terrain_stage(erf_ctx *cx, const void *const Sn[5], const void *const St[5],
                                const void *const Rt[5], int n_sub, double dtau, void *const Sout[5],
                                void *Fu, void *Fv, void *Fw)
{
    const Workspace &w = cx->ws;
    StA a;
    a.G = geo_of(cx);
    a.g = cx->prm.grav;
    a.dtau = dtau;
    a.b1 = 0.5 * (1.0 - cx->prm.beta_s);
    a.b2 = 0.5 * (1.0 + cx->prm.beta_s);
    a.bd = cx->prm.beta_d;
    a.rho0 = cx->ter.rho0;
    a.pi0 = cx->ter.pi0;
    const double *const *sn = (const double *const *)Sn;
    const double *const *st = (const double *const *)St;
    const double *const *rt = (const double *const *)Rt;
    a.n_r = sn[0], a.n_t = sn[1], a.n_u = sn[2], a.n_v = sn[3], a.n_w = sn[4];
    a.t_r = st[0], a.t_t = st[1], a.t_u = st[2], a.t_v = st[3], a.t_w = st[4];
    a.R_r = rt[0], a.R_t = rt[1], a.R_u = rt[2], a.R_v = rt[3], a.R_w = rt[4];
    a.tht = cx->ter.tht;
    a.pit = (double *)w.pit;
    a.t2 = (double *)w.t2[0];
    a.t2p = (double *)w.t2[1];
    a.u2 = (double *)w.u2[0];
    a.un = (double *)w.u2[1];
    a.v2 = (double *)w.v2[0];
    a.vn = (double *)w.v2[1];
    a.r2 = (double *)w.r2;
    a.w2 = (double *)w.w2;
    a.rh = cx->ter.rh;
    a.cp = cx->ter.cp;
    a.dp = cx->ter.dp;
    a.mo = cx->ter.mo;
    a.mn = cx->ter.mn;
    double *const *so = (double *const *)Sout;
    a.o_r = so[0], a.o_t = so[1], a.o_u = so[2], a.o_v = so[3], a.o_w = so[4];
    const bool sums = Fu && Fv && Fw;
    a.su = sums ? (double *)w.su : nullptr;
    a.sv = sums ? (double *)w.sv : nullptr;
    a.sw = sums ? (double *)w.sw : nullptr;
    a.nsub = n_sub;
    a.o_fu = (double *)Fu, a.o_fv = (double *)Fv, a.o_fw = (double *)Fw;
    const dim3 gw((cx->d.nw + kTB - 1) / kTB), gcol((cx->d.nxy + kCB - 1) / kCB);
    const dim3 tc = tile_grid(cx->d, cx->d.nz), tw = tile_grid(cx->d, cx->d.nz + 1);
    k_ter_init<<<gw, kTB, 0, cx->stream>>>(a);
    k_ter_m<<<tw, kTB, 0, cx->stream>>>(a, a.u2, a.v2, a.mo);
    hipError_t e = hipGetLastError();
    for (int s = 0; s < n_sub && e == hipSuccess; ++s) {
        timing_start(cx, K_TER_UV);
        k_ter_uv<<<tc, kTB, 0, cx->stream>>>(a);
        timing_stop(cx, K_TER_UV);
        timing_start(cx, K_TER_M);
        k_ter_m<<<tw, kTB, 0, cx->stream>>>(a, a.un, a.vn, a.mn);
        timing_stop(cx, K_TER_M);
        timing_start(cx, K_TER_HAT);
        k_ter_hat<<<tc, kTB, 0, cx->stream>>>(a);
        timing_stop(cx, K_TER_HAT);
        timing_start(cx, K_TER_COL);
        k_ter_tri<<<gcol, kCB, 0, cx->stream>>>(a);
        timing_stop(cx, K_TER_COL);
        e = hipGetLastError();
        // the new Theta'' is in t2p, the new U'', V'' in un, vn and their M in
        // mn (the next substep's old M)
        double *t = a.mo;
        a.mo = a.mn;
        a.mn = t;
        t = a.t2;
        a.t2 = a.t2p;
        a.t2p = t;
        t = a.u2;
        a.u2 = a.un;
        a.un = t;
        t = a.v2;
        a.v2 = a.vn;
        a.vn = t;
    }
    if (e != hipSuccess) return e;
    k_ter_fin<<<gw, kTB, 0, cx->stream>>>(a);
    return hipGetLastError();
}

}  // namespace erfk
