// terrain.hip -- terrain-following coordinates on the FP64 path (Sec. 3.4,
// App. A, App. B, App. C): the slow right-hand side and one RK stage of
// acoustic substeps with the metric terms, for dry, inviscid, compressible
// contexts.
//
// Geometry (erf_set_terrain): node heights z = zeta + s(zeta) h(x, y) with
// s = (1 - zeta/z_t)^beta; per column hb, the mean of the cell's four corner
// heights; per level s_k; per cell the physical height Hc = dz_k + (s_{k+1} -
// s_k) hb and the Jacobian h_zeta = Hc / dz_k.  Face metrics are recomputed
// where they are used: h_xi on the x-face i is the difference of the two
// cells' centre heights over dx, (s_k + s_{k+1})/2 (hb_i - hb_{i-1}) / dx; on
// the z-face k it is s_k times the fourth-order centred difference of hb
// (App. B); h_eta alike.  The base state is stored per cell.
//
// Kernels:
//   k_ter_prep  theta, u, v, w, p' and rho Omega = rho w - M on the z-faces,
//               M = h_xi <rho u> + h_eta <rho v> with the horizontal momenta
//               averaged from the four faces around the z-face; the lid
//               faces keep rho w (zero)
//   k_ter_rhs   slow tendencies: horizontal mass fluxes weighted by the face's
//               h_zeta, rho Omega through the z-faces, each divergence divided
//               by its control volume's h_zeta; the pressure gradient
//               p_x = p_xi - h_xi (p_zeta / h_zeta), the last factor the mean
//               of the two cells' centred vertical differences over the
//               physical distance (one-sided in the lowest and highest
//               cells); buoyancy about the per-cell base state; Coriolis
//   k_ter_init  S'' = S^n - S^t, theta^t and pi^t
//   k_ter_uv    U'', V'' with the metric correction of the gradient of the
//               predicted Theta''
//   k_ter_col   one thread per column: explicit parts of Theta'' and rho''
//               with Omega'' = W'' - M(U'', V''), the M of the new horizontal
//               momenta moved to the known side, the tridiagonal W'' rows with
//               the column's physical heights, Thomas sweeps, finish
//   k_ter_fin   S_out = S^t + S''
// All arithmetic is FP64, written in the order of the oracle's expressions so
// that the two round alike.
#include "erf_internal.h"

namespace erfk {
namespace {

constexpr int kTB = 256;  // threads per block of the per-cell kernels
constexpr int kCB = 64;   // columns per block of the column kernel

struct Geo {
    Dims d;
    double dx, dy;
    const double *dz, *s, *hb, *Hc;

    __device__ __forceinline__ int c(int i, int j, int k) const
    {
        return (k * d.ny + wrap_idx(j, d.ny)) * d.nx + wrap_idx(i, d.nx);
    }
    __device__ __forceinline__ double hbar(int i, int j) const
    {
        return hb[wrap_idx(j, d.ny) * d.nx + wrap_idx(i, d.nx)];
    }
    __device__ __forceinline__ double H(int i, int j, int k) const { return Hc[c(i, j, k)]; }
    __device__ __forceinline__ double J(int i, int j, int k) const { return H(i, j, k) / dz[k]; }
    __device__ __forceinline__ double JU(int i, int j, int k) const { return 0.5 * (J(i - 1, j, k) + J(i, j, k)); }
    __device__ __forceinline__ double JV(int i, int j, int k) const { return 0.5 * (J(i, j - 1, k) + J(i, j, k)); }
    __device__ __forceinline__ double hxU(int i, int j, int k) const
    {
        return 0.5 * (s[k] + s[k + 1]) * (hbar(i, j) - hbar(i - 1, j)) / dx;
    }
    __device__ __forceinline__ double heV(int i, int j, int k) const
    {
        return 0.5 * (s[k] + s[k + 1]) * (hbar(i, j) - hbar(i, j - 1)) / dy;
    }
    __device__ __forceinline__ double hxW(int i, int j, int k) const
    {
        return s[k] * ((hbar(i - 2, j) - hbar(i + 2, j)) + 8.0 * (hbar(i + 1, j) - hbar(i - 1, j))) / (12.0 * dx);
    }
    __device__ __forceinline__ double heW(int i, int j, int k) const
    {
        return s[k] * ((hbar(i, j - 2) - hbar(i, j + 2)) + 8.0 * (hbar(i, j + 1) - hbar(i, j - 1))) / (12.0 * dy);
    }
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
        double dzc = 0.5 * H(i, j, kl) + 0.5 * H(i, j, ku);
        for (int m = kl + 1; m < ku; ++m) dzc += H(i, j, m);
        return (f(c(i, j, ku)) - f(c(i, j, kl))) / dzc;
    }
};

__device__ __forceinline__ void split(const Dims &d, int q, int &i, int &j, int &k)
{
    k = q / d.nxy;
    const int r = q - k * d.nxy;
    j = r / d.nx;
    i = r - j * d.nx;
}

// ---------------------------------------------------------------------------
// slow right-hand side
// ---------------------------------------------------------------------------
struct RhsA {
    Geo G;
    double g, f_cor, Ug, Vg;
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
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.nw) return;
    int i, j, k;
    split(d, q, i, j, k);
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

__global__ void __launch_bounds__(kTB) k_ter_rhs(RhsA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.nw) return;
    int i, j, k;
    split(d, q, i, j, k);
    const int nz = d.nz, oh = a.oh, ov = a.ov;
    const double dx = G.dx, dy = G.dy;
    const double *ru = a.ru, *rv = a.rv, *om = a.om, *pp = a.pp;
    if (k < nz) {
        const int c = q;
        // continuity and potential temperature
        {
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
            a.Rt[c] = -((fx1 - fx0) / dx + (fy1 - fy0) / dy + (fz1 - fz0) / G.dz[k]) / Jc;
        }
        const auto pf = [&](int cc) { return pp[cc]; };
        // x-momentum on the x-face i
        {
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
        {
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
    }
    a.w2[q] = a.n_w[q] - a.t_w[q];
}

__global__ void __launch_bounds__(kTB) k_ter_uv(StA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.n) return;
    int i, j, k;
    split(d, q, i, j, k);
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
    a.un[q] = a.u2[q] + a.dtau * (-kGamma * kRd * pfx * (tt_c - tt_w) / G.dx + kGamma * kRd * pfx * cx + a.R_u[q]);
    a.vn[q] = a.v2[q] + a.dtau * (-kGamma * kRd * pfy * (tt_c - tt_s) / G.dy + kGamma * kRd * pfy * cy + a.R_v[q]);
}

// one thread per column; the column's per-level values go through the global
// arrays (t2p receives the explicit Theta'', rh the explicit rho'', cp and dp
// the Thomas factors), each thread touching only its own column there
__global__ void __launch_bounds__(kCB) k_ter_col(StA a)
{
    const Geo &G = a.G;
    const Dims &d = G.d;
    const int col = blockIdx.x * kCB + threadIdx.x;
    if (col >= d.nxy) return;
    const int j = col / d.nx, i = col - j * d.nx, nz = d.nz, nxy = d.nxy;
    const double dtau = a.dtau, b1 = a.b1, b2 = a.b2, gr = a.g;
    const double *tht = a.tht;
    // face theta^t of this column (zero on the lids, where W is zero)
    const auto THZ = [&](int kk) {
        return (kk <= 0 || kk >= nz) ? 0.0 : 0.5 * (tht[col + (kk - 1) * nxy] + tht[col + kk * nxy]);
    };
    double Mo_k = 0.0, Mn_k = 0.0;
    for (int k = 0; k < nz; ++k) {
        const int c = col + k * nxy;
        const double thx0 = 0.5 * (tht[G.c(i - 1, j, k)] + tht[c]);
        const double thx1 = 0.5 * (tht[c] + tht[G.c(i + 1, j, k)]);
        const double thy0 = 0.5 * (tht[G.c(i, j - 1, k)] + tht[c]);
        const double thy1 = 0.5 * (tht[c] + tht[G.c(i, j + 1, k)]);
        const double Ue = G.JU(i + 1, j, k) * a.un[G.c(i + 1, j, k)], Uw = G.JU(i, j, k) * a.un[c];
        const double Vn_ = G.JV(i, j + 1, k) * a.vn[G.c(i, j + 1, k)], Vs = G.JV(i, j, k) * a.vn[c];
        const double Mo_kp = G.M(a.u2, a.v2, i, j, k + 1), Mn_kp = G.M(a.un, a.vn, i, j, k + 1);
        const double Wt = a.w2[c + nxy] - Mo_kp, Wb = a.w2[c] - Mo_k;
        const double Jc = G.J(i, j, k), Hk = a.G.Hc[c];
        const double hdiv_t = (Ue * thx1 - Uw * thx0) / G.dx + (Vn_ * thy1 - Vs * thy0) / G.dy;
        const double hdiv_r = (Ue - Uw) / G.dx + (Vn_ - Vs) / G.dy;
        const double tz1 = THZ(k + 1), tz0 = THZ(k);
        double th_hat = a.t2[c] + dtau * (-hdiv_t / Jc - b1 * (Wt * tz1 - Wb * tz0) / Hk + a.R_t[c]);
        double rh_hat = a.r2[c] + dtau * (-hdiv_r / Jc - b1 * (Wt - Wb) / Hk + a.R_r[c]);
        th_hat += dtau * b2 * (Mn_kp * tz1 - Mn_k * tz0) / Hk;
        rh_hat += dtau * b2 * (Mn_kp - Mn_k) / Hk;
        a.t2p[c] = th_hat;
        a.rh[c] = rh_hat;
        Mo_k = Mo_kp;
        Mn_k = Mn_kp;
    }
    // W'' at the interior faces: rows k = 1 .. nz-1, forward elimination
    const double D = dtau * dtau * b2 * b2;
    const int m = nz - 1;
    for (int k = 1; k < nz; ++k) {
        const int c = col + k * nxy, cm = c - nxy;
        const double Hm = a.G.Hc[cm], Hk = a.G.Hc[c];
        const double dzf = 0.5 * (Hm + Hk);
        const double pif = 0.5 * (a.pit[cm] + a.pit[c]);
        const double A = kGamma * kRd * (0.5 * (a.pit[cm] + a.pit[c]));
        const double Cc = gr * 0.5 * (a.rho0[cm] + a.rho0[c]) * (kRd / kCv) * (pif / (0.5 * (a.pi0[cm] + a.pi0[c]))) /
                          (0.5 * (a.t_t[cm] + a.t_t[c]));
        const double idzm = 1.0 / Hm, idz = 1.0 / Hk;
        const double tfm = THZ(k - 1), tf = THZ(k), tfp = THZ(k + 1);
        const double ta = (k == 1) ? 0.0 : -D * (A * tfm * idzm / dzf + 0.5 * Cc * tfm * idzm - 0.5 * gr * idzm);
        const double tc = (k == m) ? 0.0 : -D * (A * tfp * idz / dzf - 0.5 * Cc * tfp * idz + 0.5 * gr * idz);
        const double tb = 1.0 + D * (A * tf * (idz + idzm) / dzf + 0.5 * Cc * tf * (idzm - idz) - 0.5 * gr * (idzm - idz));
        const double tbk = b1 * a.t2[c] + b2 * a.t2p[c], tbm = b1 * a.t2[cm] + b2 * a.t2p[cm];
        const double rbk = b1 * a.r2[c] + b2 * a.rh[c], rbm = b1 * a.r2[cm] + b2 * a.rh[cm];
        const double tr = a.w2[c] + dtau * (-A * (tbk - tbm) / dzf + 0.5 * Cc * (tbk + tbm) - 0.5 * gr * (rbk + rbm) + a.R_w[c]);
        if (k == 1) {
            a.cp[c] = tc / tb;
            a.dp[c] = tr / tb;
        } else {
            const double den = tb - ta * a.cp[cm];
            a.cp[c] = tc / den;
            a.dp[c] = (tr - ta * a.dp[cm]) / den;
        }
    }
    // back substitution into W'' (lids zero)
    a.w2[col] = 0.0;
    a.w2[col + nz * nxy] = 0.0;
    double x = 0.0;
    for (int k = m; k >= 1; --k) {
        const int c = col + k * nxy;
        x = (k == m) ? a.dp[c] : a.dp[c] - a.cp[c] * x;
        a.w2[c] = x;
    }
    // implicit finish of Theta'' (into t2p, the new level) and rho''
    for (int k = 0; k < nz; ++k) {
        const int c = col + k * nxy;
        const double Wt = a.w2[c + nxy], Wb = a.w2[c], Hk = a.G.Hc[c];
        a.t2p[c] = a.t2p[c] - dtau * b2 * (Wt * THZ(k + 1) - Wb * THZ(k)) / Hk;
        a.r2[c] = a.rh[c] - dtau * b2 * (Wt - Wb) / Hk;
    }
}

__global__ void __launch_bounds__(kTB) k_ter_fin(StA a)
{
    const Dims &d = a.G.d;
    const int q = blockIdx.x * kTB + threadIdx.x;
    if (q >= d.nw) return;
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
    G.s = cx->ter.s;
    G.hb = cx->ter.hb;
    G.Hc = cx->ter.Hc;
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
    const dim3 grd((cx->d.nw + kTB - 1) / kTB);
    k_ter_prep<<<grd, kTB, 0, cx->stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_start(cx, K_TER_RHS);
    k_ter_rhs<<<grd, kTB, 0, cx->stream>>>(a);
    timing_stop(cx, K_TER_RHS);
    return hipGetLastError();
}

hipError_t launch_terrain_stage(erf_ctx *cx, const void *const Sn[5], const void *const St[5],
                                const void *const Rt[5], int n_sub, double dtau, void *const Sout[5])
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
    double *const *so = (double *const *)Sout;
    a.o_r = so[0], a.o_t = so[1], a.o_u = so[2], a.o_v = so[3], a.o_w = so[4];
    const dim3 gw((cx->d.nw + kTB - 1) / kTB), gc((cx->d.n + kTB - 1) / kTB), gcol((cx->d.nxy + kCB - 1) / kCB);
    k_ter_init<<<gw, kTB, 0, cx->stream>>>(a);
    hipError_t e = hipGetLastError();
    for (int s = 0; s < n_sub && e == hipSuccess; ++s) {
        timing_start(cx, K_TER_UV);
        k_ter_uv<<<gc, kTB, 0, cx->stream>>>(a);
        timing_stop(cx, K_TER_UV);
        timing_start(cx, K_TER_COL);
        k_ter_col<<<gcol, kCB, 0, cx->stream>>>(a);
        timing_stop(cx, K_TER_COL);
        e = hipGetLastError();
        // the new Theta'' is in t2p; the new U'', V'' in un, vn
        double *t = a.t2;
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
