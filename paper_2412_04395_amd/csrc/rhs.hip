// rhs.hip -- slow right-hand side f(S) of the compressible equations
// (eqs. con, mom, theta of Sec. 2.1) on the C-grid, FP64.
//
// Three passes per call:
//   k_prep    primitive fields at centres / faces: theta, p', Exner, u, v, w
//   k_mut     Smagorinsky eddy viscosity at centres (only with the SGS model)
//   k_rhs     one thread per (i,j,k): R_rho, R_Theta at the cell, R_U, R_V at
//             its x- and y-face, R_W at its z-face
// Neighbours are read through the cache hierarchy; the x-fastest thread layout
// keeps every stencil load of a wavefront on consecutive addresses.
#include "erf_internal.h"

namespace erfk {
namespace {

struct RhsArgs {
    Dims d;
    double dx, dy, idx, idy;
    const double *dz;
    int oh, ov;
    int sgs;
    double Cs, Pr_t, nu, alpha, f, Ug, Vg, Qs, g;
    // state
    const double *rho, *rt, *ru, *rv, *rw;
    // base state
    const double *rho0, *Theta0, *p0;
    // primitives
    const double *th, *pp, *u, *v, *w, *mut;
    // outputs
    double *Rr, *Rt, *Ru, *Rv, *Rw;
};

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

// centre-located or horizontal-face quantity: periodic in x, y; even ghosts in z
__device__ __forceinline__ double ldc(const double *f, const Dims &d, int i, int j, int k)
{
    return f[cidx(d, wrap_idx(i, d.nx), wrap_idx(j, d.ny), refl_centre(k, d.nz))];
}

// z-face quantity: periodic in x, y; odd ghosts about the lids
__device__ __forceinline__ double ldw(const double *f, const Dims &d, int i, int j, int k)
{
    double s;
    int kk = refl_face(k, d.nz, s);
    return s * f[cidx(d, wrap_idx(i, d.nx), wrap_idx(j, d.ny), kk)];
}

__device__ __forceinline__ double interp_x(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldc(f, d, i - 3, j, k), ldc(f, d, i - 2, j, k), ldc(f, d, i - 1, j, k),
                       ldc(f, d, i, j, k), ldc(f, d, i + 1, j, k), ldc(f, d, i + 2, j, k), s);
}
__device__ __forceinline__ double interp_y(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldc(f, d, i, j - 3, k), ldc(f, d, i, j - 2, k), ldc(f, d, i, j - 1, k),
                       ldc(f, d, i, j, k), ldc(f, d, i, j + 1, k), ldc(f, d, i, j + 2, k), s);
}
__device__ __forceinline__ double interp_zc(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldc(f, d, i, j, k - 3), ldc(f, d, i, j, k - 2), ldc(f, d, i, j, k - 1),
                       ldc(f, d, i, j, k), ldc(f, d, i, j, k + 1), ldc(f, d, i, j, k + 2), s);
}
__device__ __forceinline__ double interp_zw(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldw(f, d, i, j, k - 3), ldw(f, d, i, j, k - 2), ldw(f, d, i, j, k - 1),
                       ldw(f, d, i, j, k), ldw(f, d, i, j, k + 1), ldw(f, d, i, j, k + 2), s);
}
__device__ __forceinline__ double interp_xw(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldw(f, d, i - 3, j, k), ldw(f, d, i - 2, j, k), ldw(f, d, i - 1, j, k),
                       ldw(f, d, i, j, k), ldw(f, d, i + 1, j, k), ldw(f, d, i + 2, j, k), s);
}
__device__ __forceinline__ double interp_yw(const double *f, const Dims &d, int i, int j, int k, int o, double s)
{
    return face_interp(o, ldw(f, d, i, j - 3, k), ldw(f, d, i, j - 2, k), ldw(f, d, i, j - 1, k),
                       ldw(f, d, i, j, k), ldw(f, d, i, j + 1, k), ldw(f, d, i, j + 2, k), s);
}

// ---------------------------------------------------------------------------
// primitives
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep(RhsArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    double r = a.rho[c], T = a.rt[c];
    double T0 = a.Theta0[k];
    double *th = const_cast<double *>(a.th), *pp = const_cast<double *>(a.pp);
    double *u = const_cast<double *>(a.u), *v = const_cast<double *>(a.v), *w = const_cast<double *>(a.w);
    th[c] = T / r;
    // p' = p0 ((Theta/Theta0)^gamma - 1) without cancellation (EOS, Sec. 2.1)
    pp[c] = a.p0[k] * expm1(kGamma * log1p((T - T0) / T0));
    u[c] = a.ru[c] / (0.5 * (a.rho[cidx(d, wrap_idx(i - 1, d.nx), j, k)] + r));
    v[c] = a.rv[c] / (0.5 * (a.rho[cidx(d, i, wrap_idx(j - 1, d.ny), k)] + r));
    w[c] = (k == 0) ? 0.0 : a.rw[c] / (0.5 * (a.rho[c - d.nxy] + r));
    if (k == d.nz - 1) w[c + d.nxy] = 0.0;
}

// ---------------------------------------------------------------------------
// strain rates (Sec. 2.3): diagonal at centres, off-diagonal on edges
// ---------------------------------------------------------------------------
__device__ __forceinline__ double s11(const RhsArgs &a, int i, int j, int k)
{
    return (ldc(a.u, a.d, i + 1, j, k) - ldc(a.u, a.d, i, j, k)) / a.dx;
}
__device__ __forceinline__ double s22(const RhsArgs &a, int i, int j, int k)
{
    return (ldc(a.v, a.d, i, j + 1, k) - ldc(a.v, a.d, i, j, k)) / a.dy;
}
__device__ __forceinline__ double s33(const RhsArgs &a, int i, int j, int k)
{
    // k is an interior centre index here
    return (a.w[cidx(a.d, wrap_idx(i, a.d.nx), wrap_idx(j, a.d.ny), k + 1)] -
            a.w[cidx(a.d, wrap_idx(i, a.d.nx), wrap_idx(j, a.d.ny), k)]) / a.dz[k];
}
// edge of x-face i and y-face j at level k
__device__ __forceinline__ double s12(const RhsArgs &a, int i, int j, int k)
{
    return 0.5 * ((ldc(a.u, a.d, i, j, k) - ldc(a.u, a.d, i, j - 1, k)) / a.dy +
                  (ldc(a.v, a.d, i, j, k) - ldc(a.v, a.d, i - 1, j, k)) / a.dx);
}
// edge of x-face i and z-face k (zero on the free-slip lids)
__device__ __forceinline__ double s13(const RhsArgs &a, int i, int j, int k)
{
    if (k <= 0 || k >= a.d.nz) return 0.0;
    double dzf = 0.5 * (a.dz[k - 1] + a.dz[k]);
    return 0.5 * ((ldc(a.u, a.d, i, j, k) - ldc(a.u, a.d, i, j, k - 1)) / dzf +
                  (ldw(a.w, a.d, i, j, k) - ldw(a.w, a.d, i - 1, j, k)) / a.dx);
}
__device__ __forceinline__ double s23(const RhsArgs &a, int i, int j, int k)
{
    if (k <= 0 || k >= a.d.nz) return 0.0;
    double dzf = 0.5 * (a.dz[k - 1] + a.dz[k]);
    return 0.5 * ((ldc(a.v, a.d, i, j, k) - ldc(a.v, a.d, i, j, k - 1)) / dzf +
                  (ldw(a.w, a.d, i, j, k) - ldw(a.w, a.d, i, j - 1, k)) / a.dy);
}

// Smagorinsky eddy viscosity mu_t = rho (Cs Delta)^2 sqrt(2 S:S), Delta = (dx dy dz)^(1/3)
__global__ __launch_bounds__(256) void k_mut(RhsArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    double e11 = s11(a, i, j, k), e22 = s22(a, i, j, k), e33 = s33(a, i, j, k);
    double a12 = 0.25 * (s12(a, i, j, k) + s12(a, i + 1, j, k) + s12(a, i, j + 1, k) + s12(a, i + 1, j + 1, k));
    double a13 = 0.25 * (s13(a, i, j, k) + s13(a, i + 1, j, k) + s13(a, i, j, k + 1) + s13(a, i + 1, j, k + 1));
    double a23 = 0.25 * (s23(a, i, j, k) + s23(a, i, j + 1, k) + s23(a, i, j, k + 1) + s23(a, i, j + 1, k + 1));
    double ss = 2.0 * (e11 * e11 + e22 * e22 + e33 * e33) + 4.0 * (a12 * a12 + a13 * a13 + a23 * a23);
    double cd = a.Cs * cbrt(a.dx * a.dy * a.dz[k]);
    const_cast<double *>(a.mut)[c] = a.rho[c] * cd * cd * sqrt(ss);
}

__device__ __forceinline__ double mu_tot(const RhsArgs &a, int i, int j, int k)
{
    int c = cidx(a.d, wrap_idx(i, a.d.nx), wrap_idx(j, a.d.ny), k);
    return a.rho[c] * a.nu + (a.sgs ? a.mut[c] : 0.0);
}
__device__ __forceinline__ double kappa(const RhsArgs &a, int c)
{
    return a.rho[c] * a.alpha + (a.sgs ? a.mut[c] / a.Pr_t : 0.0);
}
// deviatoric normal stresses at a centre
__device__ __forceinline__ void tau_diag(const RhsArgs &a, int i, int j, int k, double &t11, double &t22, double &t33)
{
    double e11 = s11(a, i, j, k), e22 = s22(a, i, j, k), e33 = s33(a, i, j, k);
    double dd = (e11 + e22 + e33) / 3.0;
    double m = mu_tot(a, i, j, k);
    t11 = -2.0 * m * (e11 - dd);
    t22 = -2.0 * m * (e22 - dd);
    t33 = -2.0 * m * (e33 - dd);
}
__device__ __forceinline__ double tau12(const RhsArgs &a, int i, int j, int k)
{
    double me = 0.25 * (mu_tot(a, i - 1, j - 1, k) + mu_tot(a, i, j - 1, k) + mu_tot(a, i - 1, j, k) + mu_tot(a, i, j, k));
    return -2.0 * me * s12(a, i, j, k);
}
__device__ __forceinline__ double tau13(const RhsArgs &a, int i, int j, int k)
{
    if (k <= 0 || k >= a.d.nz) return 0.0;
    double me = 0.25 * (mu_tot(a, i - 1, j, k - 1) + mu_tot(a, i, j, k - 1) + mu_tot(a, i - 1, j, k) + mu_tot(a, i, j, k));
    return -2.0 * me * s13(a, i, j, k);
}
__device__ __forceinline__ double tau23(const RhsArgs &a, int i, int j, int k)
{
    if (k <= 0 || k >= a.d.nz) return 0.0;
    double me = 0.25 * (mu_tot(a, i, j - 1, k - 1) + mu_tot(a, i, j, k - 1) + mu_tot(a, i, j - 1, k) + mu_tot(a, i, j, k));
    return -2.0 * me * s23(a, i, j, k);
}

// ---------------------------------------------------------------------------
// tendencies
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rhs(RhsArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const int nz = d.nz, oh = a.oh, ov = a.ov;
    const int c = cidx(d, i, j, k);
    const int ip = wrap_idx(i + 1, d.nx), im = wrap_idx(i - 1, d.nx);
    const int jp = wrap_idx(j + 1, d.ny), jm = wrap_idx(j - 1, d.ny);
    const double dzk = a.dz[k];
    const bool visc = a.sgs != 0 || a.nu != 0.0 || a.alpha != 0.0;

    // ---------------- cell: continuity and rho*theta ----------------
    {
        double U0 = a.ru[c], U1 = a.ru[cidx(d, ip, j, k)];
        double V0 = a.rv[c], V1 = a.rv[cidx(d, i, jp, k)];
        double W0 = a.rw[c], W1 = a.rw[c + d.nxy];
        a.Rr[c] = -((U1 - U0) / a.dx + (V1 - V0) / a.dy + (W1 - W0) / dzk);
        double fx0 = U0 * interp_x(a.th, d, i, j, k, oh, sign_of(U0));
        double fx1 = U1 * interp_x(a.th, d, i + 1, j, k, oh, sign_of(U1));
        double fy0 = V0 * interp_y(a.th, d, i, j, k, oh, sign_of(V0));
        double fy1 = V1 * interp_y(a.th, d, i, j + 1, k, oh, sign_of(V1));
        double fz0 = (k == 0) ? 0.0 : W0 * interp_zc(a.th, d, i, j, k, ov, sign_of(W0));
        double fz1 = (k == nz - 1) ? 0.0 : W1 * interp_zc(a.th, d, i, j, k + 1, ov, sign_of(W1));
        double r = -((fx1 - fx0) / a.dx + (fy1 - fy0) / a.dy + (fz1 - fz0) / dzk);
        if (visc) {
            const double *th = a.th;
            double kc = kappa(a, c);
            double hx0 = -0.5 * (kappa(a, cidx(d, im, j, k)) + kc) * (th[c] - th[cidx(d, im, j, k)]) / a.dx;
            double hx1 = -0.5 * (kc + kappa(a, cidx(d, ip, j, k))) * (th[cidx(d, ip, j, k)] - th[c]) / a.dx;
            double hy0 = -0.5 * (kappa(a, cidx(d, i, jm, k)) + kc) * (th[c] - th[cidx(d, i, jm, k)]) / a.dy;
            double hy1 = -0.5 * (kc + kappa(a, cidx(d, i, jp, k))) * (th[cidx(d, i, jp, k)] - th[c]) / a.dy;
            double hz0 = 0.0, hz1 = 0.0;
            if (k > 0)
                hz0 = -0.5 * (kappa(a, c - d.nxy) + kc) * (th[c] - th[c - d.nxy]) / (0.5 * (a.dz[k - 1] + dzk));
            if (k < nz - 1)
                hz1 = -0.5 * (kc + kappa(a, c + d.nxy)) * (th[c + d.nxy] - th[c]) / (0.5 * (dzk + a.dz[k + 1]));
            r -= (hx1 - hx0) / a.dx + (hy1 - hy0) / a.dy + (hz1 - hz0) / dzk;
        }
        if (k == 0 && a.Qs != 0.0) r += a.rho[c] * a.Qs / dzk;
        a.Rt[c] = r;
    }

    // ---------------- x-momentum on x-face (i, j, k) ----------------
    {
        double Uc = a.ru[c];
        double ar = 0.5 * (Uc + a.ru[cidx(d, ip, j, k)]);
        double al = 0.5 * (a.ru[cidx(d, im, j, k)] + Uc);
        double fxx_r = ar * interp_x(a.u, d, i + 1, j, k, oh, sign_of(ar));
        double fxx_l = al * interp_x(a.u, d, i, j, k, oh, sign_of(al));
        double b0 = 0.5 * (a.rv[cidx(d, im, j, k)] + a.rv[c]);
        double b1 = 0.5 * (a.rv[cidx(d, im, jp, k)] + a.rv[cidx(d, i, jp, k)]);
        double fxy0 = b0 * interp_y(a.u, d, i, j, k, oh, sign_of(b0));
        double fxy1 = b1 * interp_y(a.u, d, i, j + 1, k, oh, sign_of(b1));
        double fxz0 = 0.0, fxz1 = 0.0;
        if (k > 0) {
            double e0 = 0.5 * (a.rw[cidx(d, im, j, k)] + a.rw[c]);
            fxz0 = e0 * interp_zc(a.u, d, i, j, k, ov, sign_of(e0));
        }
        if (k < nz - 1) {
            double e1 = 0.5 * (a.rw[cidx(d, im, j, k + 1)] + a.rw[c + d.nxy]);
            fxz1 = e1 * interp_zc(a.u, d, i, j, k + 1, ov, sign_of(e1));
        }
        double adv = (fxx_r - fxx_l) / a.dx + (fxy1 - fxy0) / a.dy + (fxz1 - fxz0) / dzk;
        double pgf = (a.pp[c] - a.pp[cidx(d, im, j, k)]) / a.dx;
        double rho_f = 0.5 * (a.rho[cidx(d, im, j, k)] + a.rho[c]);
        double vbar = 0.25 * (a.rv[cidx(d, im, j, k)] + a.rv[c] + a.rv[cidx(d, im, jp, k)] + a.rv[cidx(d, i, jp, k)]);
        double r = -adv - pgf + a.f * (vbar - rho_f * a.Vg);
        if (visc) {
            double t11c, t22c, t33c, t11w, t22w, t33w;
            tau_diag(a, i, j, k, t11c, t22c, t33c);
            tau_diag(a, i - 1, j, k, t11w, t22w, t33w);
            r -= (t11c - t11w) / a.dx + (tau12(a, i, j + 1, k) - tau12(a, i, j, k)) / a.dy +
                 (tau13(a, i, j, k + 1) - tau13(a, i, j, k)) / dzk;
        }
        a.Ru[c] = r;
    }

    // ---------------- y-momentum on y-face (i, j, k) ----------------
    {
        double Vc = a.rv[c];
        double br = 0.5 * (Vc + a.rv[cidx(d, i, jp, k)]);
        double bl = 0.5 * (a.rv[cidx(d, i, jm, k)] + Vc);
        double fyy_r = br * interp_y(a.v, d, i, j + 1, k, oh, sign_of(br));
        double fyy_l = bl * interp_y(a.v, d, i, j, k, oh, sign_of(bl));
        double a0 = 0.5 * (a.ru[cidx(d, i, jm, k)] + a.ru[c]);
        double a1 = 0.5 * (a.ru[cidx(d, ip, jm, k)] + a.ru[cidx(d, ip, j, k)]);
        double fyx0 = a0 * interp_x(a.v, d, i, j, k, oh, sign_of(a0));
        double fyx1 = a1 * interp_x(a.v, d, i + 1, j, k, oh, sign_of(a1));
        double fyz0 = 0.0, fyz1 = 0.0;
        if (k > 0) {
            double e0 = 0.5 * (a.rw[cidx(d, i, jm, k)] + a.rw[c]);
            fyz0 = e0 * interp_zc(a.v, d, i, j, k, ov, sign_of(e0));
        }
        if (k < nz - 1) {
            double e1 = 0.5 * (a.rw[cidx(d, i, jm, k + 1)] + a.rw[c + d.nxy]);
            fyz1 = e1 * interp_zc(a.v, d, i, j, k + 1, ov, sign_of(e1));
        }
        double adv = (fyx1 - fyx0) / a.dx + (fyy_r - fyy_l) / a.dy + (fyz1 - fyz0) / dzk;
        double pgf = (a.pp[c] - a.pp[cidx(d, i, jm, k)]) / a.dy;
        double rho_f = 0.5 * (a.rho[cidx(d, i, jm, k)] + a.rho[c]);
        double ubar = 0.25 * (a.ru[cidx(d, i, jm, k)] + a.ru[cidx(d, ip, jm, k)] + a.ru[c] + a.ru[cidx(d, ip, j, k)]);
        double r = -adv - pgf - a.f * (ubar - rho_f * a.Ug);
        if (visc) {
            double t11c, t22c, t33c, t11s, t22s, t33s;
            tau_diag(a, i, j, k, t11c, t22c, t33c);
            tau_diag(a, i, j - 1, k, t11s, t22s, t33s);
            r -= (tau12(a, i + 1, j, k) - tau12(a, i, j, k)) / a.dx + (t22c - t22s) / a.dy +
                 (tau23(a, i, j, k + 1) - tau23(a, i, j, k)) / dzk;
        }
        a.Rv[c] = r;
    }

    // ---------------- z-momentum on z-face (i, j, k) ----------------
    if (k == 0) {
        a.Rw[c] = 0.0;
        a.Rw[c + nz * d.nxy] = 0.0;
    } else {
        const int cm = c - d.nxy;
        double dzf = 0.5 * (a.dz[k - 1] + dzk);
        double a0 = 0.5 * (a.ru[cm] + a.ru[c]);
        double a1 = 0.5 * (a.ru[cidx(d, ip, j, k - 1)] + a.ru[cidx(d, ip, j, k)]);
        double fzx0 = a0 * interp_xw(a.w, d, i, j, k, oh, sign_of(a0));
        double fzx1 = a1 * interp_xw(a.w, d, i + 1, j, k, oh, sign_of(a1));
        double b0 = 0.5 * (a.rv[cm] + a.rv[c]);
        double b1 = 0.5 * (a.rv[cidx(d, i, jp, k - 1)] + a.rv[cidx(d, i, jp, k)]);
        double fzy0 = b0 * interp_yw(a.w, d, i, j, k, oh, sign_of(b0));
        double fzy1 = b1 * interp_yw(a.w, d, i, j + 1, k, oh, sign_of(b1));
        double eu = 0.5 * (a.rw[c] + a.rw[c + d.nxy]);
        double ed = 0.5 * (a.rw[cm] + a.rw[c]);
        double fzz_u = eu * interp_zw(a.w, d, i, j, k + 1, ov, sign_of(eu));
        double fzz_d = ed * interp_zw(a.w, d, i, j, k, ov, sign_of(ed));
        double adv = (fzx1 - fzx0) / a.dx + (fzy1 - fzy0) / a.dy + (fzz_u - fzz_d) / dzf;
        double pgf = (a.pp[c] - a.pp[cm]) / dzf;
        // buoyancy B = -(rho - rho0) g on the face; heavier air sinks
        double buoy = -a.g * 0.5 * ((a.rho[c] - a.rho0[k]) + (a.rho[cm] - a.rho0[k - 1]));
        double r = -adv - pgf + buoy;
        if (visc) {
            double t11c, t22c, t33c, t11b, t22b, t33b;
            tau_diag(a, i, j, k, t11c, t22c, t33c);
            tau_diag(a, i, j, k - 1, t11b, t22b, t33b);
            r -= (tau13(a, i + 1, j, k) - tau13(a, i, j, k)) / a.dx + (tau23(a, i, j + 1, k) - tau23(a, i, j, k)) / a.dy +
                 (t33c - t33b) / dzf;
        }
        a.Rw[c] = r;
    }
}

}  // namespace

hipError_t launch_slow_rhs(erf_ctx *cx, const double *rho, const double *rt, const double *ru,
                           const double *rv, const double *rw, double *Rr, double *Rt, double *Ru,
                           double *Rv, double *Rw)
{
    const erf_params &p = cx->prm;
    RhsArgs a{};
    a.d = cx->d;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.idx = 1.0 / a.dx;
    a.idy = 1.0 / a.dy;
    a.dz = cx->base.dz;
    a.oh = p.adv_order_h;
    a.ov = p.adv_order_v;
    a.sgs = p.sgs;
    a.Cs = p.Cs;
    a.Pr_t = p.Pr_t;
    a.nu = p.nu_m;
    a.alpha = p.alpha_m;
    a.f = p.f_cor;
    a.Ug = p.Ug;
    a.Vg = p.Vg;
    a.Qs = p.surf_heat_flux;
    a.g = p.grav;
    a.rho = rho;
    a.rt = rt;
    a.ru = ru;
    a.rv = rv;
    a.rw = rw;
    a.rho0 = cx->base.rho0;
    a.Theta0 = cx->base.Theta0;
    a.p0 = cx->base.p0;
    a.th = cx->ws.th;
    a.pp = cx->ws.pp;
    a.u = cx->ws.u;
    a.v = cx->ws.v;
    a.w = cx->ws.w;
    a.mut = cx->ws.mut;
    a.Rr = Rr;
    a.Rt = Rt;
    a.Ru = Ru;
    a.Rv = Rv;
    a.Rw = Rw;
    const Dims &d = cx->d;
    dim3 blk(64, 4, 1), grd((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
    timing_start(cx, K_PREP); hipLaunchKernelGGL(k_prep, grd, blk, 0, cx->stream, a); timing_stop(cx, K_PREP);
    if (p.sgs) { timing_start(cx, K_MUT); hipLaunchKernelGGL(k_mut, grd, blk, 0, cx->stream, a); timing_stop(cx, K_MUT); }
    timing_start(cx, K_RHS); hipLaunchKernelGGL(k_rhs, grd, blk, 0, cx->stream, a); timing_stop(cx, K_RHS);
    return hipGetLastError();
}

}  // namespace erfk
