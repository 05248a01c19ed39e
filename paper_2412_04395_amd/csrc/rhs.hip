// rhs.hip -- slow right-hand side f(S) of the compressible equations
// (eqs. con, mom, theta of Sec. 2.1) on the C-grid.  Fields are stored as T
// (double, or float holding perturbations of rho and rho*theta about the base
// state).  Arithmetic is in T as well: FP64 for the FP64 path, FP32 for the
// FP32 path (base-state values enter as small level differences).
//
// Passes per call:
//   k_prep    primitive fields: theta, p' at centres, u, v, w on faces (moist:
//             also 1 + q_v + q_c and the total-density departure)
//   k_most    Monin-Obukhov surface layer (Sec. 3.8): per column the friction
//             velocity and the surface stresses (with a roughness length only)
//   k_mut     eddy viscosity at centres: Smagorinsky, or the Deardorff TKE
//             closure (Sec. 2.3) with its heat diffusivity and the local
//             source of rho e; k_tke adds that source's diffusion
//   k_stress  stress tensor of eq. (stresstensor) at its staggered points
//             (normal stresses at centres, shear stresses on edges) and the
//             heat diffusivity (any viscous run)
//   k_rhs     one thread per (i, j, k): R_rho, R_Theta of the cell, R_U, R_V
//             of its x- and y-face, R_W of its z-face: flux-form advection
//             with the interpolants of Sec. 3.6, pressure gradient, buoyancy,
//             Coriolis, surface heat flux and the divergence of the stresses.
// Every thread resolves the periodic wrap in x and y and the lid reflections in
// z as offsets from its cell (selects, not branches, on domains at least 3
// cells wide), so the stencil loads are base + offset and can all be issued
// ahead of the arithmetic.  The interpolation order is a template parameter for
// the orders the workloads use.
// In the FP32 storage theta is kept as theta - theta0(z); the FP32 flux of
// rho theta is U theta0(k) plus U times the interpolant of theta - theta0(k).
#include "erf_internal.h"

namespace erfk {
namespace {

template <typename T>
struct RhsArgs {
    Dims d;
    double dx, dy, idx, idy;
    const double *dz, *idz, *idzf, *cs2;
    int oh, ov;
    int ntx, nty;  // tiles per level (blockDim.x x blockDim.y cells each)
    int kch;       // levels per block of the z-marching tendency kernel
    int sgs, visc;
    // anelastic equation set: p' is the projections' (read, not written) and
    // the buoyancy is g rho0 (theta - theta0) / theta0 (Sec. 2.2)
    int anel;
    double Cs, Pr_t, nu, alpha, f, Ug, Vg, Qs, g;
    // state
    const T *rho, *rt, *ru, *rv, *rw;
    // base state
    const double *rho0, *Theta0, *theta0, *p0, *qv0;
    // moist: rho q_v, rho q_c, rho q_r (components 0..2 of the scalars, n apart)
    const T *rq;
    // primitives and stresses (workspace); moist: 1 + q_v + q_c and the
    // total-density departure at centres
    T *th, *pp, *u, *v, *w, *mut, *qf, *bm;
    T *t11, *t22, *t33, *t12, *t13, *t23, *kap;
    // Deardorff closure: the source of rho e (scalar 0 of rq); surface layer:
    // per column the surface stresses tau_13, tau_23 at the cell centre
    // ([2][ny][nx], null without one) and the roughness length
    T *esrc, *most;
    double z0;
    // outputs
    T *Rr, *Rt, *Ru, *Rv, *Rw;
};

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

// equation sets of the tendency kernel
constexpr int kDryEq = 0, kMoistEq = 1, kAnelEq = 2;
// wavefronts per SIMD the tendency kernel is compiled for: 3 in FP64 (its
// registers hold all of a section's gathers), 4 in FP32 (measured at
// 256 x 256 x 128: 284 against 316 us per launch at 3; FP64 is the same at 3
// and 4, slower at 2)
template <typename T>
constexpr int kRhsWaves = sizeof(T) == 4 ? 4 : 3;
// compute units of an MI355X (the z-marching kernel's chunking aims at two
// blocks per unit; the results do not depend on it)
constexpr int kNumCUs = 256;

// ---------------------------------------------------------------------------
// primitives
// ---------------------------------------------------------------------------
// Arithmetic type R = T: double for the FP64 path, float for the FP32 path
// (bulk stencil arithmetic in FP32; base-state values enter rounded to float,
// and only as the small differences between levels where they are subtracted).
template <typename T, bool kMoist>
__device__ __forceinline__ void k_prep_body(RhsArgs<T> a, VBlock vb)
{
    using R = T;
    const Dims &d = a.d;
    const TileIdx t = tile_cell(vb, a.ntx, a.nty);
    const int i = t.i, j = t.j, k = t.k;
    if (i >= d.nx || j >= d.ny) return;
    const int c = cidx(d, i, j, k);
    // every load first (neighbour indices clamped, so all are valid), then the stores
    const int cw = cidx(d, i == 0 ? d.nx - 1 : i - 1, j, k), cs = cidx(d, i, j == 0 ? d.ny - 1 : j - 1, k);
    const int kb = k > 0 ? k - 1 : 0, cb = c - (k - kb) * d.nxy;
    const double r0 = a.rho0[k], T0 = a.Theta0[k], r0b = a.rho0[kb], p0k = a.p0[k];
    const R r = full_in(a.rho, c, r0), rw_ = full_in(a.rho, cw, r0), rs = full_in(a.rho, cs, r0);
    const R rb = full_in(a.rho, cb, r0b);
    const R Tp = pert_in(a.rt, c, T0);
    const R U = a.ru[c], V = a.rv[c], Wc = a.rw[c];
    const R w = (k == 0) ? R(0) : Wc / (R(0.5) * (rb + r));
    // outputs are read by later launches only: streaming stores, so that no
    // dirty lines are left in the caches for the next kernel to write back.
    // The divisions are stored before the EOS, whose library calls branch:
    // a store keeps every load of the thread ahead of it.
    if constexpr (kPert<T>) {
        // theta - theta0 = (Theta' - theta0 rho') / rho, formed from the two
        // perturbations (no cancellation against the base values in float)
        st_stream(a.th + c, (T)((Tp - (R)a.theta0[k] * a.rho[c]) / r));
    } else {
        st_stream(a.th + c, (T)(full_of(a.rt, c, T0) / r));
    }
    st_stream(a.u + c, (T)(U / (R(0.5) * (rw_ + r))));
    st_stream(a.v + c, (T)(V / (R(0.5) * (rs + r))));
    st_stream(a.w + c, (T)w);
    if (k == d.nz - 1) a.w[c + d.nxy] = 0.0;
    if constexpr (kMoist) {
        // Moist EOS (Sec. 2.1): water vapour scales rho theta by 1 + (R_v/R_d) q_v.
        // With X = Theta (1 + eps q_v) and X0 = Theta0 (1 + eps qv0),
        // p' = p0 ((X/X0)^gamma - 1) and X - X0 = (Theta - Theta0)(1 + eps q_v)
        // + eps Theta0 (q_v - qv0): the small differences stay apart from the
        // large values.
        const R rqv = a.rq[c], rqc = a.rq[c + d.n], rqr = a.rq[c + 2 * d.n];
        const R qv0 = (R)a.qv0[k], eps = (R)kEpsV, T0r = (R)T0;
        const R qv = rqv / r, qc = rqc / r;
        const R x = (Tp * (R(1) + eps * qv) + eps * T0r * (qv - qv0)) / (T0r * (R(1) + eps * qv0));
        // the momentum equation's 1 + q_v + q_c and the departure of the total
        // density rho (1 + q_v + q_c + q_r) from the base state's rho0 (1 + qv0)
        st_stream(a.qf + c, (T)(R(1) + qv + qc));
        st_stream(a.bm + c, (T)(pert_in(a.rho, c, r0) + (rqv + rqc + rqr) - (R)r0 * qv0));
        st_stream(a.pp + c, (T)((R)p0k * expm1(R(kGamma) * log1p(x))));
    } else if (!a.anel) {
        // p' = p0 ((Theta/Theta0)^gamma - 1) without cancellation (EOS, Sec. 2.1)
        st_stream(a.pp + c, (T)((R)p0k * expm1(R(kGamma) * log1p(Tp / (R)T0))));
    }
}
template <typename T, bool kMoist>
__global__ __launch_bounds__(256) void k_prep(RhsArgs<T> a)
{
    k_prep_body<T, kMoist>(a, hw_block());
}
template <typename T, bool kMoist>
__global__ __launch_bounds__(256) void k_prep_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_prep_body<T, kMoist>(args[m], vb);
}

// ---------------------------------------------------------------------------
// strain rates and stresses (Sec. 2.3)
// ---------------------------------------------------------------------------
// Smagorinsky eddy viscosity mu_t = rho (Cs Delta)^2 sqrt(2 S:S), Delta = (dx dy dz)^(1/3);
// off-diagonal strains are averaged from the four edges around the centre.
// Branch-free: neighbours by selects, vertical neighbours clamped; the lid
// edges drop out because 2/(dz_{k-1} + dz_k) is zero on the lids and w is zero
// on the lid faces.
template <typename T, bool kTke>
__device__ __forceinline__ void k_mut_body(RhsArgs<T> a, VBlock vb)
{
    using R = T;
    const Dims &d = a.d;
    const TileIdx t = tile_cell(vb, a.ntx, a.nty);
    const int i = t.i, j = t.j, k = t.k;
    if (i >= d.nx || j >= d.ny) return;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int rj = j * nx, rjm = (j == 0 ? ny - 1 : j - 1) * nx, rjp = (j == ny - 1 ? 0 : j + 1) * nx;
    const int lk = k * P, lkm = (k > 0 ? k - 1 : 0) * P, lkp = (k < nz - 1 ? k + 1 : nz - 1) * P, lk1 = (k + 1) * P;
    auto U = [&](int ii, int r, int l) { return (R)a.u[l + r + ii]; };
    auto V = [&](int ii, int r, int l) { return (R)a.v[l + r + ii]; };
    auto Wf = [&](int ii, int r, int l) { return (R)a.w[l + r + ii]; };
    const R idx = (R)a.idx, idy = (R)a.idy;
    const R gz0 = (R)a.idzf[k], gz1 = (R)a.idzf[k + 1];
    const R u_c = U(i, rj, lk), u_e = U(ip, rj, lk), u_s = U(i, rjm, lk), u_se = U(ip, rjm, lk);
    const R u_n = U(i, rjp, lk), u_ne = U(ip, rjp, lk);
    const R u_b = U(i, rj, lkm), u_be = U(ip, rj, lkm), u_t = U(i, rj, lkp), u_te = U(ip, rj, lkp);
    const R v_c = V(i, rj, lk), v_n = V(i, rjp, lk), v_w = V(im, rj, lk), v_e = V(ip, rj, lk);
    const R v_nw = V(im, rjp, lk), v_ne = V(ip, rjp, lk);
    const R v_b = V(i, rj, lkm), v_bn = V(i, rjp, lkm), v_t = V(i, rj, lkp), v_tn = V(i, rjp, lkp);
    const R w_c = Wf(i, rj, lk), w_u = Wf(i, rj, lk1), w_w = Wf(im, rj, lk), w_e = Wf(ip, rj, lk);
    const R w_wu = Wf(im, rj, lk1), w_eu = Wf(ip, rj, lk1), w_s = Wf(i, rjm, lk), w_n = Wf(i, rjp, lk);
    const R w_su = Wf(i, rjm, lk1), w_nu = Wf(i, rjp, lk1);
    const R rc = full_in(a.rho, lk + rj + i, a.rho0[k]);
    const R e11 = (u_e - u_c) * idx, e22 = (v_n - v_c) * idy, e33 = (w_u - w_c) * (R)a.idz[k];
    const R h = R(0.5), q4 = R(0.25);
    // S12 on the four xy-edges; S13 on the x-face edges of faces k, k+1; S23 likewise
    const R a12 = q4 * (h * ((u_c - u_s) * idy + (v_c - v_w) * idx) + h * ((u_e - u_se) * idy + (v_e - v_c) * idx) +
                        h * ((u_n - u_c) * idy + (v_n - v_nw) * idx) + h * ((u_ne - u_e) * idy + (v_ne - v_n) * idx));
    const R a13 = q4 * (h * ((u_c - u_b) * gz0 + (w_c - w_w) * idx) + h * ((u_e - u_be) * gz0 + (w_e - w_c) * idx) +
                        h * ((u_t - u_c) * gz1 + (w_u - w_wu) * idx) + h * ((u_te - u_e) * gz1 + (w_eu - w_u) * idx));
    const R a23 = q4 * (h * ((v_c - v_b) * gz0 + (w_c - w_s) * idy) + h * ((v_n - v_bn) * gz0 + (w_n - w_c) * idy) +
                        h * ((v_t - v_c) * gz1 + (w_u - w_su) * idy) + h * ((v_tn - v_n) * gz1 + (w_nu - w_u) * idy));
    const R ss = R(2) * (e11 * e11 + e22 * e22 + e33 * e33) + R(4) * (a12 * a12 + a13 * a13 + a23 * a23);
    const int c = lk + rj + i;
    if constexpr (!kTke) {
        st_stream(a.mut + c, (T)(rc * (R)a.cs2[k] * sqrt(ss)));  // read by a later launch only
    } else {
        // Deardorff (1980) 1.5-order closure, coefficients of Moeng (1984):
        // l = Delta, or 0.76 sqrt(e)/N where smaller in stable air;
        // K_m = 0.1 l sqrt(e), K_h = (1 + 2 l/Delta) K_m; source of rho e
        // rho (K_m 2 S:S - K_h N^2 - C_eps e^(3/2)/l), C_eps = 0.19 + 0.51 l/Delta;
        // N^2 = g/theta0 dtheta/dz with dtheta/dz the mean of the two face
        // differences (zero through the lids)
        R e = (R)a.rq[c] / rc;
        e = e < R(0) ? R(0) : e;
        const R dth0u = k < nz - 1 ? (R)(a.theta0[k + 1] - a.theta0[k]) : R(0);
        const R dth0d = k > 0 ? (R)(a.theta0[k] - a.theta0[k - 1]) : R(0);
        const R thc = (R)a.th[c], thu = (R)a.th[lkp + rj + i], thd = (R)a.th[lkm + rj + i];
        // FP32 storage holds theta - theta0(k): the base difference is added
        const R up = k < nz - 1 ? ((thu - thc) + (kPert<T> ? dth0u : R(0))) * gz1 : R(0);
        const R dn = k > 0 ? ((thc - thd) + (kPert<T> ? dth0d : R(0))) * gz0 : R(0);
        const R N2 = (R)a.g / (R)a.theta0[k] * (h * (up + dn));
        const R delta = (R)cbrt(a.dx * a.dy * a.dz[k]);
        const R se = sqrt(e), sn = sqrt(N2 > R(0) ? N2 : R(0));
        const bool limited = N2 > R(0) && R(0.76) * se / sn < delta;
        const R l = limited ? R(0.76) * se / sn : delta;
        const R Km = R(0.1) * l * se, Kh = (R(1) + R(2) * l / delta) * Km;
        const R ceps = R(0.19) + R(0.51) * l / delta;
        // e^(3/2)/l, written as e N/0.76 where l is the stable length
        const R eps = limited ? ceps * e * sn / R(0.76) : ceps * e * se / delta;
        st_stream(a.mut + c, (T)(rc * Km));
        st_stream(a.kap + c, (T)(rc * (R)a.alpha + rc * Kh));
        a.esrc[c] = (T)(rc * (Km * ss - Kh * N2 - eps));
    }
}
template <typename T, bool kTke>
__global__ __launch_bounds__(256) void k_mut(RhsArgs<T> a)
{
    k_mut_body<T, kTke>(a, hw_block());
}
template <typename T, bool kTke>
__global__ __launch_bounds__(256) void k_mut_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_mut_body<T, kTke>(args[m], vb);
}

// The diffusion of rho e, div(2 rho K_m grad e) with rho K_m = mu_t, face
// coefficients the mean of the two cells, no flux through the lids, added to
// the local source of k_mut.
template <typename T>
__device__ __forceinline__ void k_tke_body(RhsArgs<T> a, VBlock vb)
{
    using R = T;
    const Dims &d = a.d;
    const TileIdx t = tile_cell(vb, a.ntx, a.nty);
    const int i = t.i, j = t.j, k = t.k;
    if (i >= d.nx || j >= d.ny) return;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int c = (k * ny + j) * nx + i;
    const int cw = c + (i == 0 ? nx - 1 : -1), ce = c + (i == nx - 1 ? 1 - nx : 1);
    const int cs = c + (j == 0 ? (ny - 1) * nx : -nx), cn = c + (j == ny - 1 ? (1 - ny) * nx : nx);
    const int cb = k > 0 ? c - P : c, ct = k < nz - 1 ? c + P : c;
    const int kb = k > 0 ? k - 1 : 0, kt = k < nz - 1 ? k + 1 : nz - 1;
    auto ev = [&](int cc, int kk) {
        const R r = full_in(a.rho, cc, a.rho0[kk]);
        const R e = (R)a.rq[cc] / r;
        return e < R(0) ? R(0) : e;
    };
    const R e_c = ev(c, k), e_w = ev(cw, k), e_e = ev(ce, k), e_s = ev(cs, k), e_n = ev(cn, k);
    const R e_b = ev(cb, kb), e_t = ev(ct, kt);
    const R m_c = a.mut[c], m_w = a.mut[cw], m_e = a.mut[ce], m_s = a.mut[cs], m_n = a.mut[cn];
    const R m_b = a.mut[cb], m_t = a.mut[ct];
    const R idx = (R)a.idx, idy = (R)a.idy;
    const R fx0 = -(m_w + m_c) * (e_c - e_w) * idx, fx1 = -(m_c + m_e) * (e_e - e_c) * idx;
    const R fy0 = -(m_s + m_c) * (e_c - e_s) * idy, fy1 = -(m_c + m_n) * (e_n - e_c) * idy;
    const R fz0 = k > 0 ? -(m_b + m_c) * (e_c - e_b) * (R)a.idzf[k] : R(0);
    const R fz1 = k < nz - 1 ? -(m_c + m_t) * (e_t - e_c) * (R)a.idzf[k + 1] : R(0);
    const R src = (R)a.esrc[c];
    a.esrc[c] = (T)(src - ((fx1 - fx0) * idx + (fy1 - fy0) * idy + (fz1 - fz0) * (R)a.idz[k]));
}
template <typename T>
__global__ __launch_bounds__(256) void k_tke(RhsArgs<T> a)
{
    k_tke_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(256) void k_tke_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_tke_body<T>(args[m], vb);
}

// Monin-Obukhov surface layer (Sec. 3.8), one thread per column: von Karman
// constant 0.4, Businger-Dyer psi_m (x = (1 - 16 zeta)^(1/4) for zeta < 0,
// -5 zeta otherwise), zeta = z1/L with L = -u*^3 theta_1/(kappa g Qs) clamped
// to [-5, 1], u* from the log law by twenty fixed-point steps from the
// neutral value; the surface stresses -rho u*^2 (u, v)/U at the lowest cell
// centre from its centre wind (U at least 0.1 m/s), in FP64.
__device__ __forceinline__ double most_psi_m(double zeta)
{
    if (zeta >= 0.0) return -5.0 * zeta;
    const double x = pow(1.0 - 16.0 * zeta, 0.25);
    return 2.0 * log(0.5 * (1.0 + x)) + log(0.5 * (1.0 + x * x)) - 2.0 * atan(x) + 2.0 * atan(1.0);
}
template <typename T>
__device__ __forceinline__ void k_most_body(RhsArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    const int col = vb.x * blockDim.x + threadIdx.x;
    if (col >= d.nxy) return;
    const int j = col / d.nx, i = col - j * d.nx;
    const int ce = col + (i == d.nx - 1 ? 1 - d.nx : 1), cn = col + (j == d.ny - 1 ? (1 - d.ny) * d.nx : d.nx);
    const double u1 = 0.5 * ((double)a.u[col] + (double)a.u[ce]);
    const double v1 = 0.5 * ((double)a.v[col] + (double)a.v[cn]);
    double U = sqrt(u1 * u1 + v1 * v1);
    if (U < 0.1) U = 0.1;
    const double th1 = kPert<T> ? (double)a.th[col] + a.theta0[0] : (double)a.th[col];
    const double rho1 = kPert<T> ? a.rho0[0] + (double)a.rho[col] : (double)a.rho[col];
    const double z1 = 0.5 * a.dz[0], lnz = log(z1 / a.z0), kap = 0.4;
    double ust = kap * U / lnz;
    for (int it = 0; it < 20; ++it) {
        double zeta = 0.0;
        if (a.Qs != 0.0) {
            zeta = -z1 * kap * a.g * a.Qs / (ust * ust * ust * th1);
            zeta = zeta < -5.0 ? -5.0 : (zeta > 1.0 ? 1.0 : zeta);
        }
        ust = kap * U / (lnz - most_psi_m(zeta));
    }
    a.most[col] = (T)(-rho1 * ust * ust * u1 / U);
    a.most[d.nxy + col] = (T)(-rho1 * ust * ust * v1 / U);
}
template <typename T>
__global__ __launch_bounds__(64) void k_most(RhsArgs<T> a)
{
    k_most_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(64) void k_most_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_most_body<T>(args[m], vb);
}

// Stresses tau = -2 mu (S - D) at their points, mu = rho nu_m + mu_t averaged
// from the four cells around an edge; heat diffusivity rho alpha_m + mu_t/Pr_t.
// z runs to nz for the shear stresses on the top faces (zero: free slip).
// (at most 4 wavefronts per SIMD: the register budget lets the scheduler issue
// all 27 gathers at once instead of in two dependent groups)
template <typename T>
__device__ __forceinline__ void k_stress_body(RhsArgs<T> a, VBlock vb)
{
    using R = T;
    const Dims &d = a.d;
    const TileIdx t = tile_cell(vb, a.ntx, a.nty);
    const int i = t.i, j = t.j, k = t.k;  // k = 0..nz: face k and, below the top, cell k
    if (i >= d.nx || j >= d.ny) return;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int rj = j * nx, rjm = (j == 0 ? ny - 1 : j - 1) * nx, rjp = (j == ny - 1 ? 0 : j + 1) * nx;
    // every load first, from indices clamped into the arrays: the cell level
    // kc (k, or nz-1 for the top face) and the level below the face kb
    const int kc = k < nz ? k : nz - 1, kb = k > 0 ? k - 1 : 0;
    const int lc = kc * P, lb = kb * P, lf = k * P, lc1 = (kc + 1) * P;
    const double rc0 = a.rho0[kc], rb0 = a.rho0[kb];
    const bool sgs = a.sgs != 0;
    const R nu = (R)a.nu, idx = (R)a.idx, idy = (R)a.idy, q4 = R(0.25), h = R(0.5), m2 = R(-2);
    // mu = rho nu_m + mu_t (mu_t read always and used only with the SGS model)
    auto mu = [&](int cc, double r0) {
        const R mt = (R)a.mut[cc];
        return full_in(a.rho, cc, r0) * nu + (sgs ? mt : R(0));
    };
    const R u_f = a.u[lc + rj + i], u_fb = a.u[lb + rj + i];
    const R v_f = a.v[lc + rj + i], v_fb = a.v[lb + rj + i];
    const R w_f = a.w[lf + rj + i], w_fw = a.w[lf + rj + im], w_fs = a.w[lf + rjm + i];
    const R m_c = mu(lc + rj + i, rc0), m_w = mu(lc + rj + im, rc0), m_s = mu(lc + rjm + i, rc0);
    const R m_ws = mu(lc + rjm + im, rc0);
    const R m_b = mu(lb + rj + i, rb0), m_bw = mu(lb + rj + im, rb0), m_bs = mu(lb + rjm + i, rb0);
    const R u_e = a.u[lc + rj + ip], u_s = a.u[lc + rjm + i];
    const R v_n = a.v[lc + rjp + i], v_w = a.v[lc + rj + im];
    const R w_u = a.w[lc1 + rj + i], w_c = a.w[lc + rj + i];
    const R rc = full_in(a.rho, lc + rj + i, rc0), mtc = (R)a.mut[lc + rj + i];
    // shear stresses on the z-face edges of face k (zero on the lids)
    const bool inner = k > 0 && k < nz;
    const R idzf = (R)a.idzf[k];
    const R s13 = h * ((u_f - u_fb) * idzf + (w_f - w_fw) * idx);
    const R s23 = h * ((v_f - v_fb) * idzf + (w_f - w_fs) * idy);
    const R mxz = q4 * (m_bw + m_b + m_w + m_c);
    const R myz = q4 * (m_bs + m_b + m_s + m_c);
    // centre values of the level (the top face plane computes them for
    // level nz - 1 again and does not store them)
    const R idz = (R)a.idz[kc];
    const R e11 = (u_e - u_f) * idx;
    const R e22 = (v_n - v_f) * idy;
    const R e33 = (w_u - w_c) * idz;
    const R dd = (e11 + e22 + e33) / R(3);
    const R s12 = h * ((u_f - u_s) * idy + (v_f - v_w) * idx);
    const R me = q4 * (m_ws + m_s + m_w + m_c);
    // the bottom faces carry the surface layer's stresses (means of the two
    // columns beside the edge), else zero as the top's
    R s13b = R(0), s23b = R(0);
    if (k == 0 && a.most) {
        s13b = h * ((R)a.most[rj + im] + (R)a.most[rj + i]);
        s23b = h * ((R)a.most[P + rjm + i] + (R)a.most[P + rj + i]);
    }
    st_stream(a.t13 + lf + rj + i, (T)(inner ? m2 * mxz * s13 : s13b));
    st_stream(a.t23 + lf + rj + i, (T)(inner ? m2 * myz * s23 : s23b));
    if (k < nz) {
        const int c = lc + rj + i;
        st_stream(a.t11 + c, (T)(m2 * m_c * (e11 - dd)));
        st_stream(a.t22 + c, (T)(m2 * m_c * (e22 - dd)));
        st_stream(a.t33 + c, (T)(m2 * m_c * (e33 - dd)));
        st_stream(a.t12 + c, (T)(m2 * me * s12));
        // (the Deardorff closure's diffusivity is k_mut's)
        if (a.sgs != 3) st_stream(a.kap + c, (T)(rc * (R)a.alpha + (sgs ? mtc / (R)a.Pr_t : R(0))));
    }
}
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4))) void k_stress(RhsArgs<T> a)
{
    k_stress_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4))) void k_stress_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_stress_body<T>(args[m], vb);
}

// ---------------------------------------------------------------------------
// interpolants (Sec. 3.6), order fixed at compile time (O = 0: runtime order)
// ---------------------------------------------------------------------------
// q holds q_{-3..3} around the thread's point; the face value q_{m-1/2} uses
// q_{m-3..m+2}: o = 0 for the face on the low side of the point, o = 1 for the
// face on the high side.  s is a sign (-1, 0 or 1), so s * (1/12) and
// s * (1/60) are exactly s / 12 and s / 60, without a division.
template <int O, typename R>
__device__ __forceinline__ R interp(int order, const R (&q)[7], int o, R s)
{
    const R qm3 = q[o], qm2 = q[o + 1], qm1 = q[o + 2], q0 = q[o + 3], qp1 = q[o + 4], qp2 = q[o + 5];
    const int ord = O ? O : order;
    if (ord == 2) return R(0.5) * (q0 + qm1);
    if (ord == 3 || ord == 4) {
        const R c4 = R(7.0 / 12.0) * (q0 + qm1) - R(1.0 / 12.0) * (qp1 + qm2);
        return ord == 4 ? c4 : c4 + s * R(1.0 / 12.0) * ((qp1 - qm2) - R(3) * (q0 - qm1));
    }
    const R c6 = R(37.0 / 60.0) * (q0 + qm1) - R(2.0 / 15.0) * (qp1 + qm2) + R(1.0 / 60.0) * (qp2 + qm3);
    return ord == 6 ? c6 : c6 - s * R(1.0 / 60.0) * ((qp2 - qm3) - R(5) * (qp1 - qm2) + R(10) * (q0 - qm1));
}

// What k_rhs takes from the thread's own column at levels other than its
// own, and the values of its own level that the next level needs again: the
// vertical stencils of theta, u, v and w over levels k-3..k+3 (reflected at
// the lids, w with the sign of its odd reflection) and the momenta, pressure,
// density, stresses and diffusivity of the neighbouring levels.  The
// single-level kernel loads them for each cell; the z-marching kernel takes
// them from its LDS planes or carries them in registers from level to level.
template <typename T>
struct RhsCol {
    T th[7], u[7], v[7], w[7];  // levels (faces for w) k-3 .. k+3
    T U0, U1, V0, V1;           // ru at x-faces i, i+1 and rv at y-faces j, j+1 of level k
    T Um, U1m, Vm, V1m;         // the same at level k-1 (level 0: its own)
    T W0, W1, Wm;               // rw on faces k, k+1, k-1 (face 0: its own)
    T Wx0, Wx1, Wy0, Wy1;       // rw on faces k, k+1 of the columns i-1 and j-1
    T rho, rhom, pp, ppm;       // stored rho and p' of levels k and k-1 (level 0: its own)
    T qf, qfm, bm, bmm;         // moist: 1 + q_v + q_c and the density departure, k and k-1
    T t33, t33m;                // tau_33 of levels k and k-1
    T t13, t13p, t23, t23p;     // tau_13, tau_23 on faces k and k+1
    T kb, kc, ka;               // heat diffusivity of levels k-1, k, k+1 (clamped at the lids)
};

// kNear: the domain is at least 3 cells wide and 3 levels high, so that one
// conditional add or reflection brings any stencil offset (at most 3) back
// into it; the periodic and reflected indices are then selects instead of
// branches, and every load of a section can be issued before its arithmetic.
// kVisc: the viscous and diffusive terms (stress and diffusivity arrays).
// kEq: the equation set (kDryEq, kMoistEq, kAnelEq).
// kMoistEq: the pressure gradient and the buoyancy are divided by the face mean of
// 1 + q_v + q_c, and the buoyancy is that of the total density (eq. mom).
template <bool kNear>
__device__ __forceinline__ int rhs_wrap(int v, int n)
{
    return kNear ? v + (v < 0 ? n : 0) - (v >= n ? n : 0) : wrap_idx(v, n);
}
// (two plain selects each rather than nested conditionals, which the
// compiler turns into branches)
template <bool kNear>
__device__ __forceinline__ int rhs_reflc(int kk, int nz)
{
    if constexpr (!kNear) return refl_centre(kk, nz);
    const int r = kk < 0 ? -1 - kk : kk;
    return r >= nz ? 2 * nz - 1 - r : r;
}
template <bool kNear>
__device__ __forceinline__ int rhs_reflf(int kk, int nz, double &sg)
{
    if constexpr (!kNear) return refl_face(kk, nz, sg);
    sg = ((kk < 0) | (kk > nz)) ? -1.0 : 1.0;
    const int r = kk < 0 ? -kk : kk;
    return r > nz ? 2 * nz - r : r;
}

// slot t (0..6) of the vertical windows: level (face) L = k + t - 3 of the
// column col
template <typename T, bool kNear>
__device__ __forceinline__ void rhs_window_load(const RhsArgs<T> &a, RhsCol<T> &z, int col, int t, int L)
{
    const int nz = a.d.nz, P = a.d.nxy;
    const int lc = rhs_reflc<kNear>(L, nz) * P + col;
    double sg;
    const int lf = rhs_reflf<kNear>(L, nz, sg) * P + col;
    z.th[t] = a.th[lc];
    z.u[t] = a.u[lc];
    z.v[t] = a.v[lc];
    z.w[t] = (T)sg * a.w[lf];
}

// the single-level kernel's loads of level k and face k+1 (oxp, oym...: the
// offsets of the neighbouring columns)
template <typename T, bool kVisc, int kEq>
__device__ __forceinline__ void rhs_level_load(const RhsArgs<T> &a, RhsCol<T> &z, int c, int k, int oxm, int oxp,
                                               int oym, int oyp)
{
    const int nz = a.d.nz, P = a.d.nxy;
    z.U0 = a.ru[c];
    z.U1 = a.ru[c + oxp];
    z.V0 = a.rv[c];
    z.V1 = a.rv[c + oyp];
    z.W1 = a.rw[c + P];
    z.Wx1 = a.rw[c + oxm + P];
    z.Wy1 = a.rw[c + oym + P];
    z.rho = a.rho[c];
    z.pp = a.pp[c];
    if constexpr (kEq == kMoistEq) {
        z.qf = a.qf[c];
        z.bm = a.bm[c];
    }
    if constexpr (kVisc) {
        z.t33 = a.t33[c];
        z.t13p = a.t13[c + P];
        z.t23p = a.t23[c + P];
        z.ka = a.kap[c + (k < nz - 1 ? P : 0)];
    }
}

// the single-level kernel's loads of level k-1 (level 0: of level 0) and of
// face k
template <typename T, bool kVisc, int kEq>
__device__ __forceinline__ void rhs_carry_load(const RhsArgs<T> &a, RhsCol<T> &z, int col, int k, int oxm, int oxp,
                                               int oym, int oyp)
{
    const int P = a.d.nxy;
    const int c = col + k * P, cm = col + (k > 0 ? k - 1 : 0) * P;
    z.W0 = a.rw[c];
    z.Wx0 = a.rw[c + oxm];
    z.Wy0 = a.rw[c + oym];
    z.Um = a.ru[cm];
    z.U1m = a.ru[cm + oxp];
    z.Vm = a.rv[cm];
    z.V1m = a.rv[cm + oyp];
    z.Wm = a.rw[cm];
    z.rhom = a.rho[cm];
    z.ppm = a.pp[cm];
    if constexpr (kEq == kMoistEq) {
        z.qfm = a.qf[cm];
        z.bmm = a.bm[cm];
    }
    if constexpr (kVisc) {
        z.t33m = a.t33[cm];
        z.t13 = a.t13[c];
        z.t23 = a.t23[c];
        z.kb = a.kap[cm];
        z.kc = a.kap[c];
    }
}

// from level k to level k+1: the windows move up one slot, this level's
// values become the level-below values and the face-(k+1) values this level's
template <typename T>
__device__ __forceinline__ void rhs_carry_up(RhsCol<T> &z)
{
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        z.th[t] = z.th[t + 1];
        z.u[t] = z.u[t + 1];
        z.v[t] = z.v[t + 1];
        z.w[t] = z.w[t + 1];
    }
    z.Um = z.U0;
    z.U1m = z.U1;
    z.Vm = z.V0;
    z.V1m = z.V1;
    z.Wm = z.W0;
    z.W0 = z.W1;
    z.Wx0 = z.Wx1;
    z.Wy0 = z.Wy1;
    z.rhom = z.rho;
    z.ppm = z.pp;
    z.qfm = z.qf;
    z.bmm = z.bm;
    z.t33m = z.t33;
    z.t13 = z.t13p;
    z.t23 = z.t23p;
    z.kb = z.kc;
    z.kc = z.ka;
}

// full value from a stored one (FP32 storage: a perturbation of base)
template <typename T>
__device__ __forceinline__ T full_v(T stored, double base)
{
    if constexpr (kPert<T>)
        return (T)base + stored;
    else
        return stored;
}

// Horizontal neighbours of level k (and of face k for w, rw, tau_13,
// tau_23) at offsets (dx, dy) from the thread's cell, read from the arrays
// in memory: x and y periodic, the offsets computed where used (cheap integer
// work instead of registers).
template <typename T, bool kNear>
struct GlobalNbr {
    const RhsArgs<T> &a;
    int i, j, c;
    __device__ __forceinline__ int off(int dx, int dy) const
    {
        const Dims &d = a.d;
        return (rhs_wrap<kNear>(i + dx, d.nx) - i) + (rhs_wrap<kNear>(j + dy, d.ny) - j) * d.nx;
    }
    __device__ __forceinline__ T th(int dx, int dy) const { return a.th[c + off(dx, dy)]; }
    __device__ __forceinline__ T u(int dx, int dy) const { return a.u[c + off(dx, dy)]; }
    __device__ __forceinline__ T v(int dx, int dy) const { return a.v[c + off(dx, dy)]; }
    __device__ __forceinline__ T w(int dx, int dy) const { return a.w[c + off(dx, dy)]; }
    __device__ __forceinline__ T ru(int dx, int dy) const { return a.ru[c + off(dx, dy)]; }
    __device__ __forceinline__ T rv(int dx, int dy) const { return a.rv[c + off(dx, dy)]; }
    __device__ __forceinline__ T rho(int dx, int dy) const { return a.rho[c + off(dx, dy)]; }
    __device__ __forceinline__ T pp(int dx, int dy) const { return a.pp[c + off(dx, dy)]; }
    __device__ __forceinline__ T qf(int dx, int dy) const { return a.qf[c + off(dx, dy)]; }
    __device__ __forceinline__ T kap(int dx, int dy) const { return a.kap[c + off(dx, dy)]; }
    __device__ __forceinline__ T t11(int dx, int dy) const { return a.t11[c + off(dx, dy)]; }
    __device__ __forceinline__ T t12(int dx, int dy) const { return a.t12[c + off(dx, dy)]; }
    __device__ __forceinline__ T t22(int dx, int dy) const { return a.t22[c + off(dx, dy)]; }
    __device__ __forceinline__ T t13(int dx, int dy) const { return a.t13[c + off(dx, dy)]; }
    __device__ __forceinline__ T t23(int dx, int dy) const { return a.t23[c + off(dx, dy)]; }
};

// The five tendencies of cell (i, j, k) (c its index) from the column values
// z and the horizontal neighbours H of level k (GlobalNbr or LdsNbr).
template <typename T, int OH, int OV, bool kNear, bool kVisc, int kEq, typename Nbr>
__device__ __forceinline__ void rhs_level(const RhsArgs<T> &a, const RhsCol<T> &z, const Nbr &H, int k, int c)
{
    constexpr bool kMoist = kEq == kMoistEq;
    using R = T;
    const Dims &d = a.d;
    const int nz = d.nz, P = d.nxy;
    // FP32 storage: theta0 of the level k + t - 3 relative to level k (the
    // base-state difference formed in double, then rounded)
    auto dthz0 = [&](int t) { return (R)(a.theta0[rhs_reflc<kNear>(k + t - 3, nz)] - a.theta0[k]); };
    // 1 away from the bottom (top) lid, 0 on it: the lid fluxes are masked by
    // a product rather than a conditional, which the compiler would make a
    // branch with part of the stencil loads behind it
    const R not_bot = (R)(k > 0), not_top = (R)(k < nz - 1);
    const R idx = (R)a.idx, idy = (R)a.idy, idz = (R)a.idz[k], h = R(0.5), q4 = R(0.25);
    const int oh = a.oh, ov = a.ov;
    const int kb = k > 0 ? k - 1 : 0;
    R q[7];
    // the five tendencies, stored together at the end: a store between the
    // sections would keep every later load behind it (the compiler cannot
    // rule out that it aliases them)
    R out_r, out_t, out_u, out_v, out_w;

    // ---------------- cell: continuity and rho*theta ----------------
    const R U0 = z.U0, U1 = z.U1, V0 = z.V0, V1 = z.V1, W0 = z.W0, W1 = z.W1;
    const double r0k = a.rho0[k];
    const R rc = kPert<T> ? (R)r0k + z.rho : z.rho;
    {
        out_r = -((U1 - U0) * idx + (V1 - V0) * idy + (W1 - W0) * idz);
        R r;
        if constexpr (kPert<T>) {
            // FP32: the flux U theta^ split as U theta0(k) + U (theta^ - theta0(k)),
            // theta^ - theta0(k) interpolated from theta - theta0(k) (horizontally
            // the stored perturbation, vertically plus the base-state difference
            // of the levels), so that no float sum carries theta0 ~ 300 K
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = H.th(t - 3, 0);
            const R fx0 = U0 * interp<OH>(oh, q, 0, sign_of(U0)), fx1 = U1 * interp<OH>(oh, q, 1, sign_of(U1));
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = H.th(0, t - 3);
            const R fy0 = V0 * interp<OH>(oh, q, 0, sign_of(V0)), fy1 = V1 * interp<OH>(oh, q, 1, sign_of(V1));
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = dthz0(t) + z.th[t];
            const R fz0 = W0 * interp<OV>(ov, q, 0, sign_of(W0)) * not_bot;
            const R fz1 = W1 * interp<OV>(ov, q, 1, sign_of(W1)) * not_top;
            r = (R)a.theta0[k] * out_r - ((fx1 - fx0) * idx + (fy1 - fy0) * idy + (fz1 - fz0) * idz);
        } else {
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = H.th(t - 3, 0);
            const R fx0 = U0 * interp<OH>(oh, q, 0, sign_of(U0)), fx1 = U1 * interp<OH>(oh, q, 1, sign_of(U1));
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = H.th(0, t - 3);
            const R fy0 = V0 * interp<OH>(oh, q, 0, sign_of(V0)), fy1 = V1 * interp<OH>(oh, q, 1, sign_of(V1));
#pragma unroll
            for (int t = 0; t < 7; ++t) q[t] = z.th[t];
            const R fz0 = W0 * interp<OV>(ov, q, 0, sign_of(W0)) * not_bot;
            const R fz1 = W1 * interp<OV>(ov, q, 1, sign_of(W1)) * not_top;
            r = -((fx1 - fx0) * idx + (fy1 - fy0) * idy + (fz1 - fz0) * idz);
        }
        if constexpr (kVisc) {
            const R kc = z.kc, thc = z.th[3];
            // differences of theta: on one level the base value cancels; across
            // levels (FP32 storage) the base-state difference is added
            const R dzb = kPert<T> ? dthz0(2) : R(0), dza = kPert<T> ? dthz0(4) : R(0);
            const R hx0 = -h * (H.kap(-1, 0) + kc) * (thc - (R)H.th(-1, 0)) * idx;
            const R hx1 = -h * (kc + H.kap(1, 0)) * ((R)H.th(1, 0) - thc) * idx;
            const R hy0 = -h * (H.kap(0, -1) + kc) * (thc - (R)H.th(0, -1)) * idy;
            const R hy1 = -h * (kc + H.kap(0, 1)) * ((R)H.th(0, 1) - thc) * idy;
            // the levels below and above (clamped at the lids: the cell itself)
            const R hz0 = -h * (z.kb + kc) * (thc - (dzb + z.th[2])) * (R)a.idzf[k] * not_bot;
            const R hz1 = -h * (kc + z.ka) * ((dza + z.th[4]) - thc) * (R)a.idzf[k + 1] * not_top;
            r -= (hx1 - hx0) * idx + (hy1 - hy0) * idy + (hz1 - hz0) * idz;
        }
        if (k == 0 && a.Qs != 0.0) r += rc * (R)a.Qs * idz;
        out_t = r;
    }

    // ---------------- x-momentum on x-face (i, j, k) ----------------
    {
        const R Um = H.ru(-1, 0);
        const R ar = h * (U0 + U1), al = h * (Um + U0);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.u(t - 3, 0);
        const R fxx_r = ar * interp<OH>(oh, q, 1, sign_of(ar)), fxx_l = al * interp<OH>(oh, q, 0, sign_of(al));
        const R Vw = H.rv(-1, 0), Vwn = H.rv(-1, 1);
        const R b0 = h * (Vw + V0), b1 = h * (Vwn + V1);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.u(0, t - 3);
        const R fxy0 = b0 * interp<OH>(oh, q, 0, sign_of(b0)), fxy1 = b1 * interp<OH>(oh, q, 1, sign_of(b1));
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = z.u[t];
        // z-face momenta (faces 0..nz all exist; the lid fluxes are zero)
        const R e0 = h * (z.Wx0 + W0), e1 = h * (z.Wx1 + W1);
        const R fxz0 = e0 * interp<OV>(ov, q, 0, sign_of(e0)) * not_bot;
        const R fxz1 = e1 * interp<OV>(ov, q, 1, sign_of(e1)) * not_top;
        const R adv = (fxx_r - fxx_l) * idx + (fxy1 - fxy0) * idy + (fxz1 - fxz0) * idz;
        R pgf = (z.pp - (R)H.pp(-1, 0)) * idx;
        if constexpr (kMoist) pgf = pgf / (h * ((R)H.qf(-1, 0) + z.qf));
        const R rho_f = h * (full_v<T>(H.rho(-1, 0), r0k) + rc);
        const R vbar = q4 * (Vw + V0 + Vwn + V1);
        R r = -adv - pgf + (R)a.f * (vbar - rho_f * (R)a.Vg);
        if constexpr (kVisc)
            r -= ((R)H.t11(0, 0) - (R)H.t11(-1, 0)) * idx + ((R)H.t12(0, 1) - (R)H.t12(0, 0)) * idy +
                 (z.t13p - z.t13) * idz;
        out_u = r;
    }

    // ---------------- y-momentum on y-face (i, j, k) ----------------
    {
        const R Vs = H.rv(0, -1);
        const R br = h * (V0 + V1), bl = h * (Vs + V0);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.v(0, t - 3);
        const R fyy_r = br * interp<OH>(oh, q, 1, sign_of(br)), fyy_l = bl * interp<OH>(oh, q, 0, sign_of(bl));
        const R Us = H.ru(0, -1), Use = H.ru(1, -1);
        const R a0 = h * (Us + U0), a1 = h * (Use + U1);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.v(t - 3, 0);
        const R fyx0 = a0 * interp<OH>(oh, q, 0, sign_of(a0)), fyx1 = a1 * interp<OH>(oh, q, 1, sign_of(a1));
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = z.v[t];
        const R e0 = h * (z.Wy0 + W0), e1 = h * (z.Wy1 + W1);
        const R fyz0 = e0 * interp<OV>(ov, q, 0, sign_of(e0)) * not_bot;
        const R fyz1 = e1 * interp<OV>(ov, q, 1, sign_of(e1)) * not_top;
        const R adv = (fyx1 - fyx0) * idx + (fyy_r - fyy_l) * idy + (fyz1 - fyz0) * idz;
        R pgf = (z.pp - (R)H.pp(0, -1)) * idy;
        if constexpr (kMoist) pgf = pgf / (h * ((R)H.qf(0, -1) + z.qf));
        const R rho_f = h * (full_v<T>(H.rho(0, -1), r0k) + rc);
        const R ubar = q4 * (Us + Use + U0 + U1);
        R r = -adv - pgf - (R)a.f * (ubar - rho_f * (R)a.Ug);
        if constexpr (kVisc)
            r -= ((R)H.t12(1, 0) - (R)H.t12(0, 0)) * idx + ((R)H.t22(0, 0) - (R)H.t22(0, -1)) * idy +
                 (z.t23p - z.t23) * idz;
        out_v = r;
    }

    // ---------------- z-momentum on z-face (i, j, k) ----------------
    // the lid faces carry W = 0: the bottom face's tendency is computed from
    // the level's own values in place of the level below and stored as zero
    {
        const R idzf = (R)a.idzf[k];
        const R a0 = h * (z.Um + U0), a1 = h * (z.U1m + U1);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.w(t - 3, 0);
        const R fzx0 = a0 * interp<OH>(oh, q, 0, sign_of(a0)), fzx1 = a1 * interp<OH>(oh, q, 1, sign_of(a1));
        const R b0 = h * (z.Vm + V0), b1 = h * (z.V1m + V1);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = H.w(0, t - 3);
        const R fzy0 = b0 * interp<OH>(oh, q, 0, sign_of(b0)), fzy1 = b1 * interp<OH>(oh, q, 1, sign_of(b1));
        const R eu = h * (W0 + W1), ed = h * (z.Wm + W0);
#pragma unroll
        for (int t = 0; t < 7; ++t) q[t] = z.w[t];
        const R fzz_u = eu * interp<OV>(ov, q, 1, sign_of(eu)), fzz_d = ed * interp<OV>(ov, q, 0, sign_of(ed));
        const R adv = (fzx1 - fzx0) * idx + (fzy1 - fzy0) * idy + (fzz_u - fzz_d) * idzf;
        const R pgf = (z.pp - z.ppm) * idzf;
        R r;
        if constexpr (kMoist) {
            // B = -g (rho_m - rho_m0) from the total densities; -grad p' + B over
            // the face mean of 1 + q_v + q_c
            const R buoy = -(R)a.g * h * (z.bm + z.bmm);
            const R qfm = h * (z.qfm + z.qf);
            r = -adv - pgf / qfm + buoy / qfm;
        } else if constexpr (kEq == kAnelEq) {
            // anelastic buoyancy g rho0 (theta - theta0) / theta0, the mean of
            // the two cells on the face
            const R tu = kPert<T> ? z.th[3] : z.th[3] - (R)a.theta0[k];
            const R td = kPert<T> ? z.th[2] : z.th[2] - (R)a.theta0[kb];
            const R bu = (R)a.rho0[k] * tu / (R)a.theta0[k], bd = (R)a.rho0[kb] * td / (R)a.theta0[kb];
            r = -adv - pgf + (R)a.g * h * (bu + bd);
        } else {
            // buoyancy B = -(rho - rho0) g on the face; heavier air sinks
            const R pu = kPert<T> ? z.rho : z.rho - (R)r0k;
            const R pd = kPert<T> ? z.rhom : z.rhom - (R)a.rho0[kb];
            const R buoy = -(R)a.g * h * (pu + pd);
            r = -adv - pgf + buoy;
        }
        if constexpr (kVisc)
            r -= ((R)H.t13(1, 0) - z.t13) * idx + ((R)H.t23(0, 1) - z.t23) * idy + (z.t33 - z.t33m) * idzf;
        out_w = k > 0 ? r : R(0);
    }
    // tendencies are read by later launches only: streaming stores
    st_stream(a.Rr + c, (T)out_r);
    st_stream(a.Rt + c, (T)out_t);
    st_stream(a.Ru + c, (T)out_u);
    st_stream(a.Rv + c, (T)out_v);
    st_stream(a.Rw + c, (T)out_w);
    if (k == 0) a.Rw[c + nz * P] = 0.0;
}

// One thread per cell (i, j, k): every column value loaded for the cell.
// The general kernel (domains narrower than the stencil), and the ensemble
// members' batched launches.
template <typename T, int OH, int OV, bool kNear, bool kVisc, int kEq>
__device__ __forceinline__ void k_rhs_body(RhsArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    const TileIdx tc = tile_cell(vb, a.ntx, a.nty);
    const int i = tc.i, j = tc.j, k = tc.k;
    if (i >= d.nx || j >= d.ny) return;
    const int col = j * d.nx + i, c = col + k * d.nxy;
    const int oxm = rhs_wrap<kNear>(i - 1, d.nx) - i, oxp = rhs_wrap<kNear>(i + 1, d.nx) - i;
    const int oym = (rhs_wrap<kNear>(j - 1, d.ny) - j) * d.nx, oyp = (rhs_wrap<kNear>(j + 1, d.ny) - j) * d.nx;
    RhsCol<T> z{};
#pragma unroll
    for (int t = 0; t < 7; ++t) rhs_window_load<T, kNear>(a, z, col, t, k + t - 3);
    rhs_carry_load<T, kVisc, kEq>(a, z, col, k, oxm, oxp, oym, oyp);
    rhs_level_load<T, kVisc, kEq>(a, z, c, k, oxm, oxp, oym, oyp);
    rhs_level<T, OH, OV, kNear, kVisc, kEq>(a, z, GlobalNbr<T, kNear>{a, i, j, c}, k, c);
}

// ---------------------------------------------------------------------------
// z-marching tendency kernel with the horizontal neighbours staged in LDS
// ---------------------------------------------------------------------------
// A block owns a 64 x 4 tile of columns and marches up a chunk of levels.  Per
// level it writes the planes of the tile with their halos into LDS -- theta,
// u, v, w with three cells on each side, the other fields with one -- and
// computes every cell of the level from LDS.  The planes of level k+1 are
// read from memory into registers while level k is computed; that phase
// issues no memory loads of its own, so no wait for the memory counter holds
// it behind them.  Face fields (rw, tau_13, tau_23) and the heat diffusivity
// are kept for two faces (levels) in a ring of two slots; the vertical
// stencils of the thread's own column stay in registers.
constexpr int kLX = 64, kLY = 4;                        // tile
constexpr int kBW = kLX + 6, kBH = kLY + 6;             // planes with 3-cell halos
constexpr int kBN = kBW * kBH;                          // 700
constexpr int kSW = kLX + 2, kSH = kLY + 2;             // planes with 1-cell halos
constexpr int kSN = kSW * kSH;                          // 396
constexpr int kBLoads = (kBN + 255) / 256, kSLoads = (kSN + 255) / 256;

// plane indices
constexpr int kPlRu = 0, kPlRv = 1, kPlRho = 2, kPlPp = 3, kPlT11 = 4, kPlT22 = 5, kPlT12 = 6;
template <bool kVisc>
constexpr int kPlQf = kVisc ? 7 : 4;
template <bool kVisc, bool kMoist>
constexpr int kNSmall = 4 + (kVisc ? 3 : 0) + (kMoist ? 1 : 0);
constexpr int kRgRw = 0, kRgT13 = 1, kRgT23 = 2, kRgKap = 3;
template <bool kVisc>
constexpr int kNRing = kVisc ? 4 : 1;
template <typename T, bool kVisc, bool kMoist>
constexpr size_t kLdsBytes = sizeof(T) * (4 * kBN + kNSmall<kVisc, kMoist> * kSN + 2 * kNRing<kVisc> * kSN);

// Neighbours from the LDS planes: b = the big planes (theta, u, v, w), s = the
// small ones, r0 = the ring slot of level (face) k, p3 and p1 the thread's
// centre in the two plane shapes.
template <typename T, bool kVisc>
struct LdsNbr {
    const T *b, *s, *r0;
    int p3, p1;
    __device__ __forceinline__ T big(int f, int dx, int dy) const { return b[f * kBN + p3 + dy * kBW + dx]; }
    __device__ __forceinline__ T sml(int f, int dx, int dy) const { return s[f * kSN + p1 + dy * kSW + dx]; }
    __device__ __forceinline__ T rng(int f, int dx, int dy) const { return r0[f * kSN + p1 + dy * kSW + dx]; }
    __device__ __forceinline__ T th(int dx, int dy) const { return big(0, dx, dy); }
    __device__ __forceinline__ T u(int dx, int dy) const { return big(1, dx, dy); }
    __device__ __forceinline__ T v(int dx, int dy) const { return big(2, dx, dy); }
    __device__ __forceinline__ T w(int dx, int dy) const { return big(3, dx, dy); }
    __device__ __forceinline__ T ru(int dx, int dy) const { return sml(kPlRu, dx, dy); }
    __device__ __forceinline__ T rv(int dx, int dy) const { return sml(kPlRv, dx, dy); }
    __device__ __forceinline__ T rho(int dx, int dy) const { return sml(kPlRho, dx, dy); }
    __device__ __forceinline__ T pp(int dx, int dy) const { return sml(kPlPp, dx, dy); }
    __device__ __forceinline__ T qf(int dx, int dy) const { return sml(kPlQf<kVisc>, dx, dy); }
    __device__ __forceinline__ T t11(int dx, int dy) const { return sml(kPlT11, dx, dy); }
    __device__ __forceinline__ T t22(int dx, int dy) const { return sml(kPlT22, dx, dy); }
    __device__ __forceinline__ T t12(int dx, int dy) const { return sml(kPlT12, dx, dy); }
    __device__ __forceinline__ T kap(int dx, int dy) const { return rng(kRgKap, dx, dy); }
    __device__ __forceinline__ T t13(int dx, int dy) const { return rng(kRgT13, dx, dy); }
    __device__ __forceinline__ T t23(int dx, int dy) const { return rng(kRgT23, dx, dy); }
};

// offset within a level of plane element e of a plane of width pw whose
// corner is (x0, y0): periodic in x and y (any number of wraps)
__device__ __forceinline__ int plane_off(const Dims &d, int e, int pw, int x0, int y0)
{
    const int gx = x0 + e % pw, gy = y0 + e / pw;
    const int wx = ((gx % d.nx) + d.nx) % d.nx, wy = ((gy % d.ny) + d.ny) % d.ny;
    return wy * d.nx + wx;
}

template <typename T, int OH, int OV, bool kVisc, int kEq>
__device__ __forceinline__ void k_rhs_lds_body(const RhsArgs<T> &a, VBlock vb, T *lds)
{
    constexpr bool kMoist = kEq == kMoistEq;
    constexpr int NS = kNSmall<kVisc, kMoist>, NR = kNRing<kVisc>;
    const Dims &d = a.d;
    const int nz = d.nz, P = d.nxy;
    const TileIdx tc = tile_cell(vb, a.ntx, a.nty);  // blockDim = (64, 4)
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kLX + tx;
    const int i = tc.i, j = tc.j, i0 = i - tx, j0 = j - ty;
    const bool active = i < d.nx && j < d.ny;
    const int k0 = tc.k * a.kch, k1 = min(k0 + a.kch, nz);
    T *big = lds, *sml = lds + 4 * kBN, *ring = sml + NS * kSN;
    // plane elements this thread loads, as offsets within a level (the same
    // on every level)
    int ob[kBLoads], os[kSLoads];
#pragma unroll
    for (int r = 0; r < kBLoads; ++r) ob[r] = tid + 256 * r < kBN ? plane_off(d, tid + 256 * r, kBW, i0 - 3, j0 - 3) : 0;
#pragma unroll
    for (int r = 0; r < kSLoads; ++r) os[r] = tid + 256 * r < kSN ? plane_off(d, tid + 256 * r, kSW, i0 - 1, j0 - 1) : 0;
    const T *const bsrc[4] = {a.th, a.u, a.v, a.w};
    const T *ssrc[NS];
    ssrc[kPlRu] = a.ru;
    ssrc[kPlRv] = a.rv;
    ssrc[kPlRho] = a.rho;
    ssrc[kPlPp] = a.pp;
    if constexpr (kVisc) {
        ssrc[kPlT11] = a.t11;
        ssrc[kPlT22] = a.t22;
        ssrc[kPlT12] = a.t12;
    }
    if constexpr (kMoist) ssrc[kPlQf<kVisc>] = a.qf;
    const T *rsrc[NR];
    rsrc[kRgRw] = a.rw;
    if constexpr (kVisc) {
        rsrc[kRgT13] = a.t13;
        rsrc[kRgT23] = a.t23;
        rsrc[kRgKap] = a.kap;
    }
    // ring slot s: the planes of face (level) l; the diffusivity of level
    // min(l, nz - 1)
    auto load_ring = [&](T (&v)[NR][kSLoads], int l) {
#pragma unroll
        for (int f = 0; f < NR; ++f) {
            const int L = (kVisc && f == kRgKap) ? min(l, nz - 1) : l;
#pragma unroll
            for (int r = 0; r < kSLoads; ++r) v[f][r] = rsrc[f][L * P + os[r]];
        }
    };
    auto store_ring = [&](const T (&v)[NR][kSLoads], int l) {
        T *dst = ring + (l & 1) * NR * kSN;
#pragma unroll
        for (int f = 0; f < NR; ++f)
#pragma unroll
            for (int r = 0; r < kSLoads; ++r)
                if (tid + 256 * r < kSN) dst[f * kSN + tid + 256 * r] = v[f][r];
    };
    const int col = j * d.nx + i;
    const int oxp = rhs_wrap<true>(i + 1, d.nx) - i, oyp = (rhs_wrap<true>(j + 1, d.ny) - j) * d.nx;
    RhsCol<T> z{};
    // the start of the chunk: windows of levels k0-3 .. k0+2 and the values of
    // level k0-1 (own column), the ring slot of face k0
    if (active) {
#pragma unroll
        for (int t = 0; t < 6; ++t) rhs_window_load<T, true>(a, z, col, t, k0 + t - 3);
        const int cm = col + (k0 > 0 ? k0 - 1 : 0) * P;
        z.Um = a.ru[cm];
        z.U1m = a.ru[cm + oxp];
        z.Vm = a.rv[cm];
        z.V1m = a.rv[cm + oyp];
        z.Wm = a.rw[cm];
        z.rhom = a.rho[cm];
        z.ppm = a.pp[cm];
        if constexpr (kMoist) {
            z.qfm = a.qf[cm];
            z.bmm = a.bm[cm];
        }
        if constexpr (kVisc) {
            z.t33m = a.t33[cm];
            z.kb = a.kap[cm];
        }
    }
    {
        T v[NR][kSLoads];
        load_ring(v, k0);
        store_ring(v, k0);
    }
    const int p3 = (ty + 3) * kBW + tx + 3, p1 = (ty + 1) * kSW + tx + 1;
    // Level k's planes, the ring slot of face (level) k+1 and the own column's
    // values that no plane holds, read into registers one level ahead: the
    // loads of level k+1 are in flight while level k is computed from LDS
    // (whose phase issues no memory loads of its own).
    T vb_[4][kBLoads], vs[NS][kSLoads], vr[NR][kSLoads];
    T w6th = 0, w6u = 0, w6v = 0, w6w = 0, t33 = 0, bm = 0;
    auto load_level = [&](int k) {
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int r = 0; r < kBLoads; ++r) vb_[f][r] = bsrc[f][k * P + ob[r]];
#pragma unroll
        for (int f = 0; f < NS; ++f)
#pragma unroll
            for (int r = 0; r < kSLoads; ++r) vs[f][r] = ssrc[f][k * P + os[r]];
        load_ring(vr, k + 1);
        if (active) {
            RhsCol<T> w6{};
            rhs_window_load<T, true>(a, w6, col, 6, k + 3);
            w6th = w6.th[6];
            w6u = w6.u[6];
            w6v = w6.v[6];
            w6w = w6.w[6];
            if constexpr (kVisc) t33 = a.t33[col + k * P];
            if constexpr (kMoist) bm = a.bm[col + k * P];
        }
    };
    load_level(k0);
    for (int k = k0; k < k1; ++k) {
        __syncthreads();  // level k-1 computed: its planes and slot (k+1)&1 are free
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int r = 0; r < kBLoads; ++r)
                if (tid + 256 * r < kBN) big[f * kBN + tid + 256 * r] = vb_[f][r];
#pragma unroll
        for (int f = 0; f < NS; ++f)
#pragma unroll
            for (int r = 0; r < kSLoads; ++r)
                if (tid + 256 * r < kSN) sml[f * kSN + tid + 256 * r] = vs[f][r];
        store_ring(vr, k + 1);
        z.th[6] = w6th;
        z.u[6] = w6u;
        z.v[6] = w6v;
        z.w[6] = w6w;
        z.t33 = t33;
        z.bm = bm;
        __syncthreads();
        if (k + 1 < k1) load_level(k + 1);
        if (active) {
            const LdsNbr<T, kVisc> H{big, sml, ring + (k & 1) * NR * kSN, p3, p1};
            const T *r1 = ring + ((k + 1) & 1) * NR * kSN;
            z.U0 = H.ru(0, 0);
            z.U1 = H.ru(1, 0);
            z.V0 = H.rv(0, 0);
            z.V1 = H.rv(0, 1);
            z.W0 = H.rng(kRgRw, 0, 0);
            z.Wx0 = H.rng(kRgRw, -1, 0);
            z.Wy0 = H.rng(kRgRw, 0, -1);
            z.W1 = r1[kRgRw * kSN + p1];
            z.Wx1 = r1[kRgRw * kSN + p1 - 1];
            z.Wy1 = r1[kRgRw * kSN + p1 - kSW];
            z.rho = H.rho(0, 0);
            z.pp = H.pp(0, 0);
            if constexpr (kMoist) z.qf = H.qf(0, 0);
            if constexpr (kVisc) {
                z.t13 = H.t13(0, 0);
                z.t23 = H.t23(0, 0);
                z.t13p = r1[kRgT13 * kSN + p1];
                z.t23p = r1[kRgT23 * kSN + p1];
                z.kc = H.kap(0, 0);
                z.ka = r1[kRgKap * kSN + p1];
            }
            rhs_level<T, OH, OV, true, kVisc, kEq>(a, z, H, k, col + k * P);
            rhs_carry_up(z);
        }
    }
}

template <typename T, int OH, int OV, bool kNear, bool kVisc, int kEq>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kRhsWaves<T>, kRhsWaves<T>))) void k_rhs(RhsArgs<T> a)
{
    k_rhs_body<T, OH, OV, kNear, kVisc, kEq>(a, hw_block());
}
// two blocks per compute unit (the LDS of one FP64 viscous block is 68 KiB,
// its registers 255 per lane with the loads of the next level in flight)
template <typename T, int OH, int OV, bool kVisc, int kEq>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_rhs_lds(RhsArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char rhs_lds_raw[];
    k_rhs_lds_body<T, OH, OV, kVisc, kEq>(a, hw_block(), (T *)rhs_lds_raw);
}

// ---------------------------------------------------------------------------
// eddy viscosity and stresses in one z-marching pass (Smagorinsky or none)
// ---------------------------------------------------------------------------
// A block owns a 64 x 4 tile of columns and marches up a chunk of levels.  The
// planes it needs are staged in LDS with two cells around the tile: u and v at
// levels k-1, k, k+1 and w at faces k, k+1 (rings of three and two slots), rho
// at level k.  Per level it first evaluates mu = rho nu_m + mu_t on the tile and
// one cell on its low sides (the Smagorinsky mu_t as k_mut does, expression
// for expression), into a ring of two levels, then the stresses of level k and
// face k and the heat diffusivity as k_stress does.  mu_t itself never goes
// to memory.  Same results as k_mut and k_stress, bit for bit.  FP64 only.
constexpr int kMW = kLX + 4, kMH = kLY + 4, kMN = kMW * kMH;  // planes with 2-cell halos: 68 x 8
constexpr int kMLoads = (kMN + 255) / 256;
// LDS planes: u[3], v[3], w[2], rho, mu[2]
constexpr int kMsPlanes = 11;

template <typename T, bool kSgs>
__device__ __forceinline__ void k_mustress_lds_body(const RhsArgs<T> &a, VBlock vb, T *lds)
{
    using R = T;
    const Dims &d = a.d;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const TileIdx tc = tile_cell(vb, a.ntx, a.nty);  // blockDim = (64, 4)
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kLX + tx;
    const int i = tc.i, j = tc.j, i0 = i - tx, j0 = j - ty;
    const bool active = i < nx && j < ny;
    const int k0 = tc.k * a.kch, k1 = min(k0 + a.kch, nz);
    T *pu = lds, *pv = lds + 3 * kMN, *pw = lds + 6 * kMN, *prho = lds + 8 * kMN, *pmu = lds + 9 * kMN;
    int om[kMLoads];
#pragma unroll
    for (int r = 0; r < kMLoads; ++r) om[r] = tid + 256 * r < kMN ? plane_off(d, tid + 256 * r, kMW, i0 - 2, j0 - 2) : 0;
    auto clampk = [&](int m) { return m < 0 ? 0 : (m > nz - 1 ? nz - 1 : m); };
    auto load = [&](T (&v)[kMLoads], const T *f, int lvl) {
#pragma unroll
        for (int r = 0; r < kMLoads; ++r) v[r] = f[lvl * P + om[r]];
    };
    auto store = [&](T *dst, const T (&v)[kMLoads]) {
#pragma unroll
        for (int r = 0; r < kMLoads - 1; ++r) dst[tid + 256 * r] = v[r];
        if (tid + 256 * (kMLoads - 1) < kMN) dst[tid + 256 * (kMLoads - 1)] = v[kMLoads - 1];
    };
    // plane index of the tile-relative point (x, y)
    auto at = [](int x, int y) { return (y + 2) * kMW + x + 2; };
    const R idx = (R)a.idx, idy = (R)a.idy, h = R(0.5), q4 = R(0.25), m2 = R(-2);
    const R nu = (R)a.nu;
    // mu_t (returned) and mu at the tile-relative point (x, y) of level m, from
    // the planes of levels m-1, m, m+1 (u, v) and faces m, m+1 (w) and rho(m)
    auto mu_at = [&](int x, int y, int m, R &mut_out) -> R {
        const T *uc = pu + ((m + 3) % 3) * kMN, *ub = pu + ((m + 2) % 3) * kMN, *ut = pu + ((m + 4) % 3) * kMN;
        const T *vc = pv + ((m + 3) % 3) * kMN, *vb_ = pv + ((m + 2) % 3) * kMN, *vt = pv + ((m + 4) % 3) * kMN;
        const T *wc = pw + (m & 1) * kMN, *wu = pw + ((m + 1) & 1) * kMN;
        const int q = at(x, y);
        const R rc = full_v<T>(prho[q], a.rho0[m]);
        R mt = R(0);
        if constexpr (kSgs) {
            const R gz0 = (R)a.idzf[m], gz1 = (R)a.idzf[m + 1];
            const R u_c = uc[q], u_e = uc[q + 1], u_s = uc[q - kMW], u_se = uc[q - kMW + 1];
            const R u_n = uc[q + kMW], u_ne = uc[q + kMW + 1];
            const R u_b = ub[q], u_be = ub[q + 1], u_t = ut[q], u_te = ut[q + 1];
            const R v_c = vc[q], v_n = vc[q + kMW], v_w = vc[q - 1], v_e = vc[q + 1];
            const R v_nw = vc[q + kMW - 1], v_ne = vc[q + kMW + 1];
            const R v_b = vb_[q], v_bn = vb_[q + kMW], v_t = vt[q], v_tn = vt[q + kMW];
            const R w_c = wc[q], w_u = wu[q], w_w = wc[q - 1], w_e = wc[q + 1];
            const R w_wu = wu[q - 1], w_eu = wu[q + 1], w_s = wc[q - kMW], w_n = wc[q + kMW];
            const R w_su = wu[q - kMW], w_nu = wu[q + kMW];
            const R e11 = (u_e - u_c) * idx, e22 = (v_n - v_c) * idy, e33 = (w_u - w_c) * (R)a.idz[m];
            const R a12 = q4 * (h * ((u_c - u_s) * idy + (v_c - v_w) * idx) + h * ((u_e - u_se) * idy + (v_e - v_c) * idx) +
                                h * ((u_n - u_c) * idy + (v_n - v_nw) * idx) + h * ((u_ne - u_e) * idy + (v_ne - v_n) * idx));
            const R a13 = q4 * (h * ((u_c - u_b) * gz0 + (w_c - w_w) * idx) + h * ((u_e - u_be) * gz0 + (w_e - w_c) * idx) +
                                h * ((u_t - u_c) * gz1 + (w_u - w_wu) * idx) + h * ((u_te - u_e) * gz1 + (w_eu - w_u) * idx));
            const R a23 = q4 * (h * ((v_c - v_b) * gz0 + (w_c - w_s) * idy) + h * ((v_n - v_bn) * gz0 + (w_n - w_c) * idy) +
                                h * ((v_t - v_c) * gz1 + (w_u - w_su) * idy) + h * ((v_tn - v_n) * gz1 + (w_nu - w_u) * idy));
            const R ss = R(2) * (e11 * e11 + e22 * e22 + e33 * e33) + R(4) * (a12 * a12 + a13 * a13 + a23 * a23);
            mt = (T)(rc * (R)a.cs2[m] * sqrt(ss));  // as stored by k_mut
        }
        mut_out = mt;
        return rc * nu + mt;
    };
    // the planes of step k: u, v at level k+1, w at face k+1 (clamped like
    // k_mut's level k+1), rho at level k
    T lu[kMLoads], lv[kMLoads], lw[kMLoads], lr[kMLoads];
    auto load_step = [&](int k) {
        load(lu, a.u, clampk(k + 1));
        load(lv, a.v, clampk(k + 1));
        load(lw, a.w, k + 1);
        load(lr, a.rho, k);
    };
    // start: levels ks-1 and ks of u, v (clamped) and face ks of w, where ks
    // is the first level whose mu is evaluated (one below the chunk, whose
    // stresses need it)
    const int ks = k0 > 0 ? k0 - 1 : 0;
    {
        T t0[kMLoads];
        load(t0, a.u, clampk(ks - 1));
        store(pu + ((ks - 1 + 3) % 3) * kMN, t0);
        load(t0, a.u, ks);
        store(pu + ((ks + 3) % 3) * kMN, t0);
        load(t0, a.v, clampk(ks - 1));
        store(pv + ((ks - 1 + 3) % 3) * kMN, t0);
        load(t0, a.v, ks);
        store(pv + ((ks + 3) % 3) * kMN, t0);
        load(t0, a.w, ks);
        store(pw + (ks & 1) * kMN, t0);
    }
    load_step(ks);
    for (int k = ks; k < k1; ++k) {
        __syncthreads();  // step k-1 done: the slots of level k-2 and face k-1 are free
        store(pu + ((k + 4) % 3) * kMN, lu);
        store(pv + ((k + 4) % 3) * kMN, lv);
        store(pw + ((k + 1) & 1) * kMN, lw);
        store(prho, lr);
        __syncthreads();
        if (k + 1 < k1) load_step(k + 1);
        // mu of level k on the tile and one cell on its low sides
        T *mu_k = pmu + (k & 1) * kMN;
        R mut_own;
        mu_k[at(tx, ty)] = mu_at(tx, ty, k, mut_own);
        if (tid < kLX + kLY + 1) {
            R unused;
            const int x = tid < kLX ? tid : -1, y = tid < kLX ? -1 : tid - kLX - 1;
            mu_k[at(x, y)] = mu_at(x, y, k, unused);
        }
        __syncthreads();
        if (k < k0 || !active) continue;
        // the stresses of level k and face k (k_stress, expression for expression)
        const int kb = k > 0 ? k - 1 : 0;
        const T *uc = pu + ((k + 3) % 3) * kMN, *ub = pu + ((kb + 3) % 3) * kMN;
        const T *vc = pv + ((k + 3) % 3) * kMN, *vb_ = pv + ((kb + 3) % 3) * kMN;
        const T *wc = pw + (k & 1) * kMN, *wu = pw + ((k + 1) & 1) * kMN;
        const T *mc = pmu + (k & 1) * kMN, *mb = pmu + (kb & 1) * kMN;
        const int q = at(tx, ty);
        const R u_f = uc[q], u_fb = ub[q], v_f = vc[q], v_fb = vb_[q];
        const R w_f = wc[q], w_fw = wc[q - 1], w_fs = wc[q - kMW];
        const R m_c = mc[q], m_w = mc[q - 1], m_s = mc[q - kMW], m_ws = mc[q - kMW - 1];
        const R m_b = mb[q], m_bw = mb[q - 1], m_bs = mb[q - kMW];
        const R u_e = uc[q + 1], u_s = uc[q - kMW], v_n = vc[q + kMW], v_w = vc[q - 1];
        const R w_u = wu[q], w_c = wc[q];
        const R rc = full_v<T>(prho[q], a.rho0[k]);
        const bool inner = k > 0;
        const R idzf = (R)a.idzf[k];
        const R s13 = h * ((u_f - u_fb) * idzf + (w_f - w_fw) * idx);
        const R s23 = h * ((v_f - v_fb) * idzf + (w_f - w_fs) * idy);
        const R mxz = q4 * (m_bw + m_b + m_w + m_c);
        const R myz = q4 * (m_bs + m_b + m_s + m_c);
        const R idz = (R)a.idz[k];
        const R e11 = (u_e - u_f) * idx;
        const R e22 = (v_n - v_f) * idy;
        const R e33 = (w_u - w_c) * idz;
        const R dd = (e11 + e22 + e33) / R(3);
        const R s12 = h * ((u_f - u_s) * idy + (v_f - v_w) * idx);
        const R me = q4 * (m_ws + m_s + m_w + m_c);
        R s13b = R(0), s23b = R(0);
        const int col = j * nx + i;
        if (k == 0 && a.most) {
            const int rj = j * nx, rjm = (j == 0 ? ny - 1 : j - 1) * nx, im = i == 0 ? nx - 1 : i - 1;
            s13b = h * ((R)a.most[rj + im] + (R)a.most[rj + i]);
            s23b = h * ((R)a.most[P + rjm + i] + (R)a.most[P + rj + i]);
        }
        const int c = k * P + col;
        st_stream(a.t13 + c, (T)(inner ? m2 * mxz * s13 : s13b));
        st_stream(a.t23 + c, (T)(inner ? m2 * myz * s23 : s23b));
        st_stream(a.t11 + c, (T)(m2 * m_c * (e11 - dd)));
        st_stream(a.t22 + c, (T)(m2 * m_c * (e22 - dd)));
        st_stream(a.t33 + c, (T)(m2 * m_c * (e33 - dd)));
        st_stream(a.t12 + c, (T)(m2 * me * s12));
        st_stream(a.kap + c, (T)(rc * (R)a.alpha + (kSgs ? mut_own / (R)a.Pr_t : R(0))));
    }
    // the top lid's face: no shear stress
    if (k1 == nz && active) {
        const int c = nz * P + j * nx + i;
        st_stream(a.t13 + c, (T)R(0));
        st_stream(a.t23 + c, (T)R(0));
    }
}
template <typename T, bool kSgs>
__global__ __launch_bounds__(256) void k_mustress_lds(RhsArgs<T> a)
{
    __shared__ T lds[kMsPlanes * kMN];
    k_mustress_lds_body<T, kSgs>(a, hw_block(), lds);
}

template <typename T, int OH, int OV, bool kNear, bool kVisc, int kEq>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kRhsWaves<T>, kRhsWaves<T>))) void k_rhs_batch(const RhsArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_rhs_body<T, OH, OV, kNear, kVisc, kEq>(args[m], vb);
}

}  // namespace

namespace {
// orders 2, 3 and 5 in both directions have their own instances; any other
// combination, and domains narrower than the stencil, take the general one.
// Moist dynamics: 3rd order (the moist workload's) and the general instances.
// The anelastic set (FP64 only): orders 2, 3 and 5 and the general instances.
// FP64 on domains at least 3 cells wide and 3 levels high takes the
// LDS-staged z-marching kernel (al: its 64 x 4 tiles and chunks of al.kch
// levels, grid grdl); FP32, narrower domains and ensemble members take the
// single-level kernel (a, grd: tiles x levels).  Both give the same results
// bit for bit.  At 256 x 256 x 128 the FP64 single-level kernel re-reads its
// stencil operands from HBM (2.85 times its compulsory bytes: its FP64
// footprint outgrows the caches) and takes 704 us per launch, the z-march
// 467 us; in FP32 the single-level kernel's operands fit the caches (1.06
// times) and its four wavefronts per SIMD make it the faster one (290 us
// against 324).  Inside the ensemble's graphs the z-marching kernel is not
// used.
template <typename T, int OH, int OV, bool kNear, bool kVisc, int kEq>
hipError_t rhs_one(erf_ctx *cx, const RhsArgs<T> &a, const RhsArgs<T> &al, dim3 grd, dim3 grdl, dim3 blk)
{
    if constexpr (kNear && sizeof(T) == 8) {
        if (!cx->member && !cx->rec) {
            constexpr size_t lds = kLdsBytes<T, kVisc, kEq == kMoistEq>;
            const void *fn = (const void *)k_rhs_lds<T, OH, OV, kVisc, kEq>;
            if (lds > 64 * 1024) {
                const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return e;
            }
            void *argv[] = {(void *)&al};
            return hipLaunchKernel(fn, grdl, dim3(kLX, kLY, 1), argv, lds, cx->stream);
        }
    }
    run<RhsArgs<T>, k_rhs<T, OH, OV, kNear, kVisc, kEq>, k_rhs_batch<T, OH, OV, kNear, kVisc, kEq>>(cx, grd, blk, 0, a);
    return hipSuccess;
}
template <typename T, bool kVisc, int kEq>
hipError_t launch_rhs_eq(erf_ctx *cx, const RhsArgs<T> &a, const RhsArgs<T> &al, dim3 grd, dim3 grdl, dim3 blk)
{
    const bool near = a.d.nx >= 3 && a.d.ny >= 3 && a.d.nz >= 3;
    if (near && a.oh == 5 && a.ov == 5)
        return rhs_one<T, 5, 5, true, kVisc, kEq>(cx, a, al, grd, grdl, blk);
    else if (near && a.oh == 3 && a.ov == 3)
        return rhs_one<T, 3, 3, true, kVisc, kEq>(cx, a, al, grd, grdl, blk);
    else if (near && a.oh == 2 && a.ov == 2)
        return rhs_one<T, 2, 2, true, kVisc, kEq>(cx, a, al, grd, grdl, blk);
    else if (near)
        return rhs_one<T, 0, 0, true, kVisc, kEq>(cx, a, al, grd, grdl, blk);
    else
        return rhs_one<T, 0, 0, false, kVisc, kEq>(cx, a, al, grd, grdl, blk);
}
template <typename T, bool kVisc>
hipError_t launch_rhs(erf_ctx *cx, const RhsArgs<T> &a, const RhsArgs<T> &al, bool moist, dim3 grd, dim3 grdl,
                      dim3 blk)
{
    const bool near = a.d.nx >= 3 && a.d.ny >= 3 && a.d.nz >= 3;
    if (moist) {
        if (near && a.oh == 3 && a.ov == 3)
            return rhs_one<T, 3, 3, true, kVisc, kMoistEq>(cx, a, al, grd, grdl, blk);
        else if (near)
            return rhs_one<T, 0, 0, true, kVisc, kMoistEq>(cx, a, al, grd, grdl, blk);
        else
            return rhs_one<T, 0, 0, false, kVisc, kMoistEq>(cx, a, al, grd, grdl, blk);
    } else if constexpr (std::is_same_v<T, double>) {
        if (a.anel)
            return launch_rhs_eq<T, kVisc, kAnelEq>(cx, a, al, grd, grdl, blk);
        else
            return launch_rhs_eq<T, kVisc, kDryEq>(cx, a, al, grd, grdl, blk);
    } else {
        return launch_rhs_eq<T, kVisc, kDryEq>(cx, a, al, grd, grdl, blk);
    }
}

template <typename T>
hipError_t slow_rhs_t(erf_ctx *cx, const void *const S[5], const void *rq, void *const R[5], bool prep_only)
{
    const erf_params &p = cx->prm;
    Workspace &ws = cx->ws;
    RhsArgs<T> a{};
    a.d = cx->d;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.idx = 1.0 / a.dx;
    a.idy = 1.0 / a.dy;
    a.dz = cx->base.dz;
    a.idz = cx->base.idz();
    a.idzf = cx->base.idzf();
    a.cs2 = cx->base.cs2();
    a.oh = p.adv_order_h;
    a.ov = p.adv_order_v;
    // the learned closure adds its own stress divergence after k_rhs
    const bool mlp = p.sgs == ERF_SGS_MLP;
    a.sgs = mlp ? 0 : p.sgs;
    a.visc = (a.sgs != 0 || p.nu_m != 0.0 || p.alpha_m != 0.0 || p.most_z0 > 0.0) ? 1 : 0;
    a.z0 = p.most_z0;
    a.most = p.most_z0 > 0.0 ? (T *)ws.most : nullptr;
    a.esrc = (T *)ws.esrc;
    a.Cs = p.Cs;
    a.Pr_t = p.Pr_t;
    a.nu = p.nu_m;
    a.alpha = p.alpha_m;
    a.f = p.f_cor;
    a.Ug = p.Ug;
    a.Vg = p.Vg;
    a.Qs = p.surf_heat_flux;
    a.g = p.grav;
    a.rho = (const T *)S[0];
    a.rt = (const T *)S[1];
    a.ru = (const T *)S[2];
    a.rv = (const T *)S[3];
    a.rw = (const T *)S[4];
    a.rho0 = cx->base.rho0;
    a.Theta0 = cx->base.Theta0;
    a.theta0 = cx->base.theta0;
    a.p0 = cx->base.p0;
    a.qv0 = cx->base.qv0;
    // moist dynamics need the water species; without them (the closure's
    // feature pass, which uses no pressure) the dry primitives are computed
    const bool moist = p.moist != 0 && rq != nullptr;
    const bool tke = p.sgs == ERF_SGS_DEARDORFF;
    a.rq = (const T *)rq;
    a.qf = (T *)ws.qf;
    a.bm = (T *)ws.bm;
    a.th = (T *)ws.th;
    a.anel = p.anelastic ? 1 : 0;
    a.pp = p.anelastic ? (T *)cx->an.pa : (T *)ws.pp;
    a.u = (T *)ws.u;
    a.v = (T *)ws.v;
    a.w = (T *)ws.w;
    a.mut = (T *)ws.mut;
    a.t11 = (T *)ws.tau[0];
    a.t22 = (T *)ws.tau[1];
    a.t33 = (T *)ws.tau[2];
    a.t12 = (T *)ws.tau[3];
    a.t13 = (T *)ws.tau[4];
    a.t23 = (T *)ws.tau[5];
    a.kap = (T *)ws.kap;
    a.Rr = (T *)R[0];
    a.Rt = (T *)R[1];
    a.Ru = (T *)R[2];
    a.Rv = (T *)R[3];
    a.Rw = (T *)R[4];
    const Dims &d = cx->d;
    // 256-cell tiles per level, rows of 64, 32 or 16 cells (least padding)
    const int tx = tile_width(d.nx, d.ny, 256), ty = 256 / tx;
    a.ntx = (d.nx + tx - 1) / tx;
    a.nty = (d.ny + ty - 1) / ty;
    const int tiles = a.ntx * a.nty;
    dim3 blk(tx, ty, 1), grd(tiles * d.nz), grdw(tiles * (d.nz + 1));
    // the z-marching tendency kernel: 64 x 4 tiles, levels in chunks, enough
    // of them for about two blocks per compute unit, at least 16 levels each
    // (the windows reload 6 levels per chunk)
    RhsArgs<T> al = a;
    al.ntx = (d.nx + kLX - 1) / kLX;
    al.nty = (d.ny + kLY - 1) / kLY;
    const int ltiles = al.ntx * al.nty;
    const int nch = std::max(1, std::min((2 * kNumCUs + ltiles - 1) / ltiles, d.nz / 16));
    al.kch = (d.nz + nch - 1) / nch;
    const dim3 grdl(ltiles * ((d.nz + al.kch - 1) / al.kch));
    timing_start(cx, K_PREP);
    if (moist)
        run<RhsArgs<T>, k_prep<T, true>, k_prep_batch<T, true>>(cx, grd, blk, 0, a);
    else
        run<RhsArgs<T>, k_prep<T, false>, k_prep_batch<T, false>>(cx, grd, blk, 0, a);
    timing_stop(cx, K_PREP);
    if (prep_only) return hipGetLastError();
    if (a.most) {
        timing_start(cx, K_MOST);
        run<RhsArgs<T>, k_most<T>, k_most_batch<T>>(cx, dim3((d.nxy + 63) / 64), dim3(64), 0, a);
        timing_stop(cx, K_MOST);
    }
    // FP64 with Smagorinsky or constant viscosity, outside ensembles: mu_t and
    // the stresses in one z-marching pass (10.65 against 11.05 ms per step at
    // 256 x 256 x 128).  FP32 keeps the two kernels (5.84 against 5.94 ms); the
    // Deardorff closure keeps k_mut, whose mu_t, K_h and source k_tke reads.
    const bool fused = sizeof(T) == 8 && a.visc && !tke && !cx->member && !cx->rec;
    if (a.sgs && !fused) {
        timing_start(cx, K_MUT);
        if (tke)
            run<RhsArgs<T>, k_mut<T, true>, k_mut_batch<T, true>>(cx, grd, blk, 0, a);
        else
            run<RhsArgs<T>, k_mut<T, false>, k_mut_batch<T, false>>(cx, grd, blk, 0, a);
        timing_stop(cx, K_MUT);
    }
    if (tke) {
        timing_start(cx, K_TKE);
        run<RhsArgs<T>, k_tke<T>, k_tke_batch<T>>(cx, grd, blk, 0, a);
        timing_stop(cx, K_TKE);
    }
    if (a.visc) {
        timing_start(cx, K_STRESS);
        if (fused) {
            if constexpr (sizeof(T) == 8) {
                void *argv[] = {(void *)&al};
                const void *fn =
                    a.sgs ? (const void *)k_mustress_lds<T, true> : (const void *)k_mustress_lds<T, false>;
                const hipError_t e = hipLaunchKernel(fn, grdl, dim3(kLX, kLY, 1), argv, 0, cx->stream);
                if (e != hipSuccess) return e;
            }
        } else {
            run<RhsArgs<T>, k_stress<T>, k_stress_batch<T>>(cx, grdw, blk, 0, a);
        }
        timing_stop(cx, K_STRESS);
    }
    timing_start(cx, K_RHS);
    const hipError_t er =
        a.visc ? launch_rhs<T, true>(cx, a, al, moist, grd, grdl, blk) : launch_rhs<T, false>(cx, a, al, moist, grd, grdl, blk);
    timing_stop(cx, K_RHS);
    if (er != hipSuccess) return er;
    if (mlp) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_mlp_closure(cx, S[0], R);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_slow_rhs(erf_ctx *cx, const void *const S[5], const void *rq, void *const R[5])
{
    if (cx->prm.precision == ERF_FP32_MIXED) return slow_rhs_t<float>(cx, S, rq, R, false);
    return slow_rhs_t<double>(cx, S, rq, R, false);
}

hipError_t launch_prep(erf_ctx *cx, const void *const S[5])
{
    void *const none[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    if (cx->prm.precision == ERF_FP32_MIXED) return slow_rhs_t<float>(cx, S, nullptr, none, true);
    return slow_rhs_t<double>(cx, S, nullptr, none, true);
}

}  // namespace erfk
