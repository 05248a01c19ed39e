// acoustic.hip -- one RK stage of semi-implicit acoustic substepping (App. C of
// the ERF paper, Sec. 3.1), FP64.
//
// Kernels of one stage:
//   k_stage_init  S'' = S^n - S^t, frozen theta^t and Exner pi^t, zero sums
//   k_coef        per column: the tridiagonal rows of the implicit W'' equation
//                 (they depend only on S^t and dtau) and their Thomas factors
//   per substep:
//     k_horiz     U'', V'' forward step with the forward-predicted Theta''
//                 (divergence damping), running sums of U'', V''
//     k_column    per column: explicit parts of Theta'', rho''; forward
//                 elimination with the frozen factors; back substitution for
//                 W''; then Theta'', rho'' from the new W''
//   k_finalize    S_out = S^t + S'', stage-averaged momenta
//
// Column kernels map one thread to one (i, j) column with i fastest, so every
// level of the vertical sweep is a coalesced row access across the wavefront.
#include "erf_internal.h"

namespace erfk {
namespace {

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

struct StageArgs {
    Dims d;
    double dx, dy;
    const double *dz;
    double g, b1, b2, bd, dtau;
    const double *rho0, *pi0;
    // S^n, S^t, R^t
    const double *n_r, *n_t, *n_u, *n_v, *n_w;
    const double *t_r, *t_t, *t_u, *t_v, *t_w;
    const double *R_r, *R_t, *R_u, *R_v, *R_w;
    // frozen fields
    double *tht, *pit;
    // perturbations and sums
    double *T2cur, *T2prv, *T2nxt, *r2, *u2, *v2, *w2, *su, *sv, *sw;
    // coefficients on z-faces
    double *ca, *cden, *cc, *cA, *cC;
};

__global__ __launch_bounds__(256) void k_stage_init(StageArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;  // 0..nz (the extra plane handles the top z-face)
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    a.w2[c] = a.n_w[c] - a.t_w[c];
    a.sw[c] = 0.0;
    if (k == d.nz) return;
    double Tt = a.t_t[c];
    a.tht[c] = Tt / a.t_r[c];
    a.pit[c] = pow(kRd * Tt / kP00, kGamma - 1.0);
    a.T2cur[c] = a.n_t[c] - Tt;
    a.r2[c] = a.n_r[c] - a.t_r[c];
    a.u2[c] = a.n_u[c] - a.t_u[c];
    a.v2[c] = a.n_v[c] - a.t_v[c];
    a.su[c] = 0.0;
    a.sv[c] = 0.0;
}

// theta^t on z-face k of a column (lid faces carry W = 0; value unused)
__device__ __forceinline__ double thz(const StageArgs &a, int col, int k)
{
    if (k <= 0 || k >= a.d.nz) return 0.0;
    return 0.5 * (a.tht[col + (k - 1) * a.d.nxy] + a.tht[col + k * a.d.nxy]);
}

// Tridiagonal rows for W'' at interior faces k = 1..nz-1.  With
// Theta''_new = That - dtau b2 delta_z(W theta_f)/dz and rho''_new = Rhat -
// dtau b2 delta_z(W)/dz substituted into the W'' equation of App. C, face k
// couples W_{k-1}, W_k, W_{k+1} with coefficients that only involve the frozen
// state.  Stores a_k, the Thomas pivot den_k and c'_k.
__global__ __launch_bounds__(256) void k_coef(StageArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int col = j * d.nx + i, nxy = d.nxy, nz = d.nz;
    const double D = a.dtau * a.dtau * a.b2 * a.b2, g = a.g;
    double cprev = 0.0;
    for (int k = 1; k < nz; ++k) {
        int c = col + k * nxy, cm = c - nxy;
        double dzf = 0.5 * (a.dz[k - 1] + a.dz[k]);
        double pif = 0.5 * (a.pit[cm] + a.pit[c]);
        double A = kGamma * kRd * pif;
        double C = g * 0.5 * (a.rho0[k - 1] + a.rho0[k]) * (kRd / kCv) * (pif / (0.5 * (a.pi0[k - 1] + a.pi0[k]))) /
                   (0.5 * (a.t_t[cm] + a.t_t[c]));
        double idzm = 1.0 / a.dz[k - 1], idz = 1.0 / a.dz[k];
        double tfm = thz(a, col, k - 1), tf = thz(a, col, k), tfp = thz(a, col, k + 1);
        double lo = (k == 1) ? 0.0 : -D * (A * tfm * idzm / dzf + 0.5 * C * tfm * idzm - 0.5 * g * idzm);
        double up = (k == nz - 1) ? 0.0 : -D * (A * tfp * idz / dzf - 0.5 * C * tfp * idz + 0.5 * g * idz);
        double di = 1.0 + D * (A * tf * (idz + idzm) / dzf + 0.5 * C * tf * (idzm - idz) - 0.5 * g * (idzm - idz));
        double den = (k == 1) ? di : di - lo * cprev;
        double cp = up / den;
        a.ca[c] = lo;
        a.cden[c] = den;
        a.cc[c] = cp;
        a.cA[c] = A;
        a.cC[c] = C;
        cprev = cp;
    }
}

// U'', V'' forward step.  bd = 0 on the first substep of a stage.
__global__ __launch_bounds__(256) void k_horiz(StageArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    int cw = cidx(d, wrap_idx(i - 1, d.nx), j, k), cs = cidx(d, i, wrap_idx(j - 1, d.ny), k);
    const double bd = a.bd;
    double Tc = a.T2cur[c], Tw = a.T2cur[cw], Ts = a.T2cur[cs];
    double ttc = Tc + bd * (Tc - a.T2prv[c]);
    double ttw = Tw + bd * (Tw - a.T2prv[cw]);
    double tts = Ts + bd * (Ts - a.T2prv[cs]);
    double pfx = 0.5 * (a.pit[cw] + a.pit[c]);
    double pfy = 0.5 * (a.pit[cs] + a.pit[c]);
    double un = a.u2[c] + a.dtau * (-kGamma * kRd * pfx * (ttc - ttw) / a.dx + a.R_u[c]);
    double vn = a.v2[c] + a.dtau * (-kGamma * kRd * pfy * (ttc - tts) / a.dy + a.R_v[c]);
    a.u2[c] = un;
    a.v2[c] = vn;
    a.su[c] += un;
    a.sv[c] += vn;
}

// Explicit parts of Theta'' and rho'', the implicit W'' solve, and the update.
// In the forward sweep That and Rhat are stored in T2nxt and r2 (in place) and
// the eliminated right-hand side d'_k in w2 (in place, after W''_k is read).
__global__ __launch_bounds__(256) void k_column(StageArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int nxy = d.nxy, nz = d.nz, col = j * d.nx + i;
    const int ip = wrap_idx(i + 1, d.nx), im = wrap_idx(i - 1, d.nx);
    const int jp = wrap_idx(j + 1, d.ny), jm = wrap_idx(j - 1, d.ny);
    const int o_e = ip - i, o_w = im - i, o_n = (jp - j) * d.nx, o_s = (jm - j) * d.nx;
    const double dt = a.dtau, b1 = a.b1, b2 = a.b2, g = a.g;

    double th_prev = 0.0, rh_prev = 0.0, t2_prev = 0.0, r2_prev = 0.0, dprev = 0.0;
    double w_lo = a.w2[col];  // W''_k (old), carried upward
    for (int k = 0; k < nz; ++k) {
        const int c = col + k * nxy;
        const double tc = a.tht[c];
        const double thx0 = 0.5 * (a.tht[c + o_w] + tc), thx1 = 0.5 * (tc + a.tht[c + o_e]);
        const double thy0 = 0.5 * (a.tht[c + o_s] + tc), thy1 = 0.5 * (tc + a.tht[c + o_n]);
        const double Ue = a.u2[c + o_e], Uw = a.u2[c], Vn = a.v2[c + o_n], Vs = a.v2[c];
        const double w_hi = a.w2[c + nxy];
        const double hdiv_t = (Ue * thx1 - Uw * thx0) / a.dx + (Vn * thy1 - Vs * thy0) / a.dy;
        const double hdiv_r = (Ue - Uw) / a.dx + (Vn - Vs) / a.dy;
        const double t2 = a.T2cur[c], r2 = a.r2[c];
        const double tfk = thz(a, col, k), tfk1 = thz(a, col, k + 1);
        const double th_hat = t2 + dt * (-hdiv_t - b1 * (w_hi * tfk1 - w_lo * tfk) / a.dz[k] + a.R_t[c]);
        const double rh_hat = r2 + dt * (-hdiv_r - b1 * (w_hi - w_lo) / a.dz[k] + a.R_r[c]);
        if (k >= 1) {
            const double dzf = 0.5 * (a.dz[k - 1] + a.dz[k]);
            const double A = a.cA[c], C = a.cC[c];
            const double tbk = b1 * t2 + b2 * th_hat, tbm = b1 * t2_prev + b2 * th_prev;
            const double rbk = b1 * r2 + b2 * rh_hat, rbm = b1 * r2_prev + b2 * rh_prev;
            const double rk = w_lo + dt * (-A * (tbk - tbm) / dzf + 0.5 * C * (tbk + tbm) - 0.5 * g * (rbk + rbm) + a.R_w[c]);
            const double dk = (k == 1) ? rk / a.cden[c] : (rk - a.ca[c] * dprev) / a.cden[c];
            a.w2[c] = dk;
            dprev = dk;
        }
        a.T2nxt[c] = th_hat;
        a.r2[c] = rh_hat;
        th_prev = th_hat;
        rh_prev = rh_hat;
        t2_prev = t2;
        r2_prev = r2;
        w_lo = w_hi;
    }
    // back substitution and the implicit parts of Theta'', rho''
    double w_up = 0.0;  // W at face k+1 (face nz is the lid)
    for (int k = nz - 1; k >= 0; --k) {
        const int c = col + k * nxy;
        double wk = 0.0;
        if (k >= 1) {
            wk = a.w2[c] - a.cc[c] * w_up;
            a.w2[c] = wk;
            a.sw[c] += wk;
        }
        const double tfk = thz(a, col, k), tfk1 = thz(a, col, k + 1);
        a.T2nxt[c] = a.T2nxt[c] - dt * b2 * (w_up * tfk1 - wk * tfk) / a.dz[k];
        a.r2[c] = a.r2[c] - dt * b2 * (w_up - wk) / a.dz[k];
        w_up = wk;
    }
}

struct FinArgs {
    Dims d;
    int n_sub;
    double b1;
    const double *t_r, *t_t, *t_u, *t_v, *t_w, *n_w;
    const double *T2, *r2, *u2, *v2, *w2, *su, *sv, *sw;
    double *o_r, *o_t, *o_u, *o_v, *o_w, *Fu, *Fv, *Fw;
};

// S_out = S^t + S''; stage-averaged momenta.  The W-sum accumulated only the
// new W'' of each substep; the beta-weighted average over substeps is
// b1 W''_0 + W''_1 + ... + W''_{N-1} + b2 W''_N = sum_{s=1..N} W''_s + b1 (W''_0 - W''_N).
__global__ __launch_bounds__(256) void k_finalize(FinArgs a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    double inv = 1.0 / a.n_sub;
    double wt = a.t_w[c], w0 = a.n_w[c] - wt, wN = a.w2[c];
    if (a.Fw) a.Fw[c] = wt + (a.sw[c] + a.b1 * (w0 - wN)) * inv;
    a.o_w[c] = wt + wN;
    if (k == d.nz) return;
    a.o_r[c] = a.t_r[c] + a.r2[c];
    a.o_t[c] = a.t_t[c] + a.T2[c];
    double ut = a.t_u[c], vt = a.t_v[c];
    a.o_u[c] = ut + a.u2[c];
    a.o_v[c] = vt + a.v2[c];
    if (a.Fu) a.Fu[c] = ut + a.su[c] * inv;
    if (a.Fv) a.Fv[c] = vt + a.sv[c] * inv;
}

}  // namespace

hipError_t launch_acoustic_stage(erf_ctx *cx, const double *const Sn[5], const double *const St[5],
                                 const double *const Rt[5], int n_sub, double dtau,
                                 double *const Sout[5], double *Fu, double *Fv, double *Fw)
{
    const Dims &d = cx->d;
    Workspace &w = cx->ws;
    StageArgs a{};
    a.d = d;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.dz = cx->base.dz;
    a.g = cx->prm.grav;
    a.b1 = 0.5 * (1.0 - cx->prm.beta_s);
    a.b2 = 0.5 * (1.0 + cx->prm.beta_s);
    a.dtau = dtau;
    a.rho0 = cx->base.rho0;
    a.pi0 = cx->base.pi0;
    a.n_r = Sn[0]; a.n_t = Sn[1]; a.n_u = Sn[2]; a.n_v = Sn[3]; a.n_w = Sn[4];
    a.t_r = St[0]; a.t_t = St[1]; a.t_u = St[2]; a.t_v = St[3]; a.t_w = St[4];
    a.R_r = Rt[0]; a.R_t = Rt[1]; a.R_u = Rt[2]; a.R_v = Rt[3]; a.R_w = Rt[4];
    a.tht = w.th;
    a.pit = w.pit;
    a.r2 = w.r2; a.u2 = w.u2; a.v2 = w.v2; a.w2 = w.w2;
    a.su = w.su; a.sv = w.sv; a.sw = w.sw;
    a.ca = w.ca; a.cden = w.cb; a.cc = w.cc; a.cA = w.cA; a.cC = w.cC;
    int cur = 0;
    a.T2cur = w.t2[0];
    a.T2prv = w.t2[0];
    a.T2nxt = w.t2[1];

    dim3 blk(64, 4, 1);
    dim3 g3((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz), g3w((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz + 1);
    dim3 g2((d.nx + 63) / 64, (d.ny + 3) / 4, 1);
    timing_start(cx, K_STAGE_INIT); hipLaunchKernelGGL(k_stage_init, g3w, blk, 0, cx->stream, a); timing_stop(cx, K_STAGE_INIT);
    timing_start(cx, K_COEF); hipLaunchKernelGGL(k_coef, g2, blk, 0, cx->stream, a); timing_stop(cx, K_COEF);
    for (int s = 0; s < n_sub; ++s) {
        a.T2cur = w.t2[cur];
        a.T2prv = (s == 0) ? w.t2[cur] : w.t2[cur ^ 1];
        a.T2nxt = w.t2[cur ^ 1];
        a.bd = (s == 0) ? 0.0 : cx->prm.beta_d;
        timing_start(cx, K_HORIZ); hipLaunchKernelGGL(k_horiz, g3, blk, 0, cx->stream, a); timing_stop(cx, K_HORIZ);
        timing_start(cx, K_COLUMN); hipLaunchKernelGGL(k_column, g2, blk, 0, cx->stream, a); timing_stop(cx, K_COLUMN);
        cur ^= 1;
    }
    FinArgs f{};
    f.d = d;
    f.n_sub = n_sub;
    f.b1 = a.b1;
    f.t_r = St[0]; f.t_t = St[1]; f.t_u = St[2]; f.t_v = St[3]; f.t_w = St[4]; f.n_w = Sn[4];
    f.T2 = w.t2[cur]; f.r2 = w.r2; f.u2 = w.u2; f.v2 = w.v2; f.w2 = w.w2;
    f.su = w.su; f.sv = w.sv; f.sw = w.sw;
    f.o_r = Sout[0]; f.o_t = Sout[1]; f.o_u = Sout[2]; f.o_v = Sout[3]; f.o_w = Sout[4];
    f.Fu = Fu; f.Fv = Fv; f.Fw = Fw;
    timing_start(cx, K_FINALIZE); hipLaunchKernelGGL(k_finalize, g3w, blk, 0, cx->stream, f); timing_stop(cx, K_FINALIZE);
    return hipGetLastError();
}

}  // namespace erfk
