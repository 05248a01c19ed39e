// api.hip -- the C-ABI of liberf.so (include/erf.h): context, workspace,
// base state and the RK3 driver that sequences the kernels of the other
// translation units on the context's stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "erf_internal.h"

using namespace erfk;

namespace {

erf_status fail(erf_ctx *c, erf_status s, const char *msg)
{
    if (c) {
        c->err = msg;
        if (s == ERF_E_HIP) c->sticky = ERF_E_HIP;
    }
    return s;
}

erf_status hip_fail(erf_ctx *c, hipError_t e, const char *where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return fail(c, ERF_E_HIP, buf);
}

#define ERF_CHECK_CTX(c)                                                   \
    do {                                                                   \
        if (!(c)) return ERF_E_ARG;                                        \
        if ((c)->sticky != ERF_OK) return (c)->sticky;                     \
    } while (0)

double eos_p(double Theta) { return kP00 * std::pow(kRd * Theta / kP00, kGamma); }
// the moist equation of state: water vapour scales rho theta by 1 + (R_v/R_d) q_v
double eos_p_moist(double Theta, double qv) { return eos_p(Theta * (1.0 + kEpsV * qv)); }

// Newton-Raphson for the hydrostatic base state, level by level upward from
// the surface: p_k = EOS(rho_k theta_k, qv_k), p_0 = p_s - g (dz_0/2) rho_0
// (1 + qv_0) and p_k - p_{k-1} = -g dzf_k (rho_k (1 + qv_k) + rho_{k-1}
// (1 + qv_{k-1})) / 2: rho is the dry density and the vapour adds its weight.
// Without vapour (qv0 NULL) every factor is exactly 1.
erf_status base_state(int nz, const double *dz, const double *theta0, const double *qv0, double ps, double g,
                      double *rho0, double *p0, double *pi0)
{
    if (nz < 1 || !dz || !theta0 || !rho0 || !p0) return ERF_E_ARG;
    double p_prev = ps, rho_prev = 0.0, q_prev = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double q = qv0 ? qv0[k] : 0.0;
        if (!(theta0[k] > 0.0) || !(dz[k] > 0.0) || !(q >= 0.0)) return ERF_E_ARG;
        const double h = (k == 0) ? 0.5 * dz[0] : 0.5 * (dz[k - 1] + dz[k]);
        double rho = (k == 0) ? ps / (kRd * theta0[0] * (1.0 + kEpsV * q)) : rho_prev;
        for (int it = 0; it < 30; ++it) {
            const double p = eos_p_moist(rho * theta0[k], q);
            double f, fp;
            if (k == 0) {
                f = p - p_prev + g * h * (rho * (1.0 + q));
                fp = kGamma * p / rho + g * h * (1.0 + q);
            } else {
                f = p - p_prev + g * h * 0.5 * (rho * (1.0 + q) + rho_prev * (1.0 + q_prev));
                fp = kGamma * p / rho + g * h * 0.5 * (1.0 + q);
            }
            const double step = f / fp;
            rho = rho - step;
            if (std::fabs(step) <= 1e-15 * rho) break;
        }
        rho0[k] = rho;
        p0[k] = eos_p_moist(rho * theta0[k], q);
        if (pi0) pi0[k] = std::pow(p0[k] / kP00, kRd / kCp);
        p_prev = p0[k];
        rho_prev = rho;
        q_prev = q;
    }
    return ERF_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" {

erf_status erf_base_state_host(int32_t nz, const double *dz, const double *theta0, const double *qv0,
                               double p_surface, double grav, double *rho0, double *p0, double *pi0)
{
    return base_state(nz, dz, theta0, qv0, p_surface, grav, rho0, p0, pi0);
}

const char *erf_last_error(const erf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t erf_workspace_bytes(const erf_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

erf_status erf_create(const erf_grid *grid, const erf_params *prm, void *hip_stream, erf_ctx **out)
{
    if (!grid || !prm || !out || !grid->dz) return ERF_E_ARG;
    *out = nullptr;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 2) return ERF_E_SHAPE;
    const int64_t nxy = (int64_t)grid->nx * grid->ny;
    const int64_t nw = nxy * (grid->nz + 1);
    const int64_t nq = prm->n_scalars;
    if (nw * (nq > 1 ? nq : 1) >= ((int64_t)1 << 31)) return ERF_E_SHAPE;
    if (grid->nz > 256) return ERF_E_SHAPE;  // a substep block holds whole columns
    if (!(grid->dx > 0.0) || !(grid->dy > 0.0)) return ERF_E_ARG;
    for (int k = 0; k < grid->nz; ++k)
        if (!(grid->dz[k] > 0.0)) return ERF_E_ARG;
    if (prm->anelastic != 0 && prm->anelastic != 1) return ERF_E_ARG;
    const bool anel = prm->anelastic != 0;
    if (!anel && (prm->n_substeps < 2 || prm->n_substeps % 2 != 0)) return ERF_E_ARG;
    if (anel) {
        // the projection's transforms: powers of two up to 2048 in x and y
        auto pow2 = [](int v) { return v >= 1 && v <= 2048 && (v & (v - 1)) == 0; };
        if (!pow2(grid->nx) || !pow2(grid->ny)) return ERF_E_SHAPE;
        if (prm->precision != ERF_FP64 || prm->moist || prm->sgs == ERF_SGS_MLP) return ERF_E_UNSUPPORTED;
    }
    if (prm->adv_order_h < 2 || prm->adv_order_h > 6 || prm->adv_order_v < 2 || prm->adv_order_v > 6)
        return ERF_E_ARG;
    if (nq < 0 || nq > 8) return ERF_E_ARG;
    if (prm->sgs != ERF_SGS_NONE && prm->sgs != ERF_SGS_SMAGORINSKY && prm->sgs != ERF_SGS_MLP &&
        prm->sgs != ERF_SGS_DEARDORFF)
        return ERF_E_ARG;
    // the Deardorff closure carries rho e as scalar 0 and no other scalar
    if (prm->sgs == ERF_SGS_DEARDORFF && (nq != 1 || prm->moist || prm->anelastic || prm->alpha_m != 0.0))
        return ERF_E_UNSUPPORTED;
    if (!(prm->most_z0 >= 0.0) || (prm->most_z0 > 0.0 && !(prm->most_z0 < 0.5 * grid->dz[0]))) return ERF_E_ARG;
    if (prm->sgs == ERF_SGS_MLP && (prm->nu_m != 0.0 || prm->alpha_m != 0.0)) return ERF_E_UNSUPPORTED;
    if (prm->scalar_scheme != ERF_SCALAR_INTERP && prm->scalar_scheme != ERF_SCALAR_WENO5) return ERF_E_ARG;
    if (prm->precision != ERF_FP64 && prm->precision != ERF_FP32_MIXED) return ERF_E_ARG;
    if (nq > 0 && ((prm->sgs != ERF_SGS_NONE && prm->sgs != ERF_SGS_DEARDORFF) || prm->alpha_m != 0.0))
        return ERF_E_UNSUPPORTED;
    if (prm->moist != 0 && prm->moist != 1) return ERF_E_ARG;
    if (prm->moist && nq < 3) return ERF_E_ARG;  // rho q_v, rho q_c, rho q_r
    if (prm->microphysics != 0 && prm->microphysics != 1) return ERF_E_ARG;
    if (prm->microphysics && !prm->moist) return ERF_E_ARG;
    if (!(prm->dt > 0.0) || !(prm->beta_s >= 0.0 && prm->beta_s <= 1.0)) return ERF_E_ARG;

    erf_ctx *c = new (std::nothrow) erf_ctx();
    if (!c) return ERF_E_NOMEM;
    c->grid = *grid;
    c->prm = *prm;
    c->stream = (hipStream_t)hip_stream;
    c->d.nx = grid->nx;
    c->d.ny = grid->ny;
    c->d.nz = grid->nz;
    c->d.nxy = (int)nxy;
    c->d.n = (int)(nxy * grid->nz);
    c->d.nw = (int)nw;
    c->dz_host = new double[grid->nz];
    std::memcpy(c->dz_host, grid->dz, sizeof(double) * grid->nz);
    c->grid.dz = c->dz_host;
    (void)hipGetDevice(&c->device);

    // one arena for the whole workspace; bulk fields in the context's precision
    const size_t n = (size_t)c->d.n, w = (size_t)nw, q = (size_t)(nq > 0 ? nq : 0) * n;
    const size_t es = prm->precision == ERF_FP32_MIXED ? sizeof(float) : sizeof(double);
    struct Req { void **p; size_t bytes; };
    Workspace &ws = c->ws;
    Base &b = c->base;
    const size_t N = n * es, Wb = w * es, Q = q * es, D = sizeof(double);
    const size_t nzs = (size_t)grid->nz;
    const size_t G = prm->sgs == ERF_SGS_MLP ? N : 0;
    const size_t M = prm->moist ? N : 0;
    const size_t A8 = anel ? n * sizeof(double) : 0, A16 = anel ? n * sizeof(double2) : 0;
    const size_t E = prm->sgs == ERF_SGS_DEARDORFF ? N : 0, MO = prm->most_z0 > 0.0 ? 2 * (size_t)nxy * es : 0;
    Anel &an = c->an;
    Req reqs[] = {
        {&ws.sa[0], N}, {&ws.sa[1], N}, {&ws.sa[2], N}, {&ws.sa[3], N}, {&ws.sa[4], Wb}, {&ws.sa[5], Q},
        {&ws.sb[0], N}, {&ws.sb[1], N}, {&ws.sb[2], N}, {&ws.sb[3], N}, {&ws.sb[4], Wb}, {&ws.sb[5], Q},
        {&ws.R[0], N}, {&ws.R[1], N}, {&ws.R[2], N}, {&ws.R[3], N}, {&ws.R[4], Wb},
        {&ws.th, N}, {&ws.pp, N}, {&ws.pit, N}, {&ws.u, N}, {&ws.v, N}, {&ws.w, Wb}, {&ws.mut, N},
        {&ws.tau[0], N}, {&ws.tau[1], N}, {&ws.tau[2], N}, {&ws.tau[3], N}, {&ws.tau[4], Wb}, {&ws.tau[5], Wb},
        {&ws.kap, N},
        {&ws.t2[0], N}, {&ws.t2[1], N}, {&ws.t2[2], N}, {&ws.r2, N}, {&ws.w2, Wb},
        {&ws.u2[0], N}, {&ws.u2[1], N}, {&ws.v2[0], N}, {&ws.v2[1], N},
        {&ws.su, N}, {&ws.sv, N}, {&ws.sw, Wb},
        {&ws.cC, Wb}, {(void **)&ws.cb, w * D},
        {&ws.q, Q}, {&ws.fu, N}, {&ws.fv, N}, {&ws.fw, Wb},
        {(void **)&ws.diag, diag_slots_needed() * D},
        {&ws.sg[0], G}, {&ws.sg[1], G}, {&ws.sg[2], G}, {&ws.sg[3], G}, {&ws.sg[4], G}, {&ws.sg[5], G},
        {&ws.sg[6], G}, {&ws.sg[7], G}, {&ws.sg[8], G},
        {&ws.qf, M}, {&ws.bm, M}, {&ws.pex, M}, {&ws.rdm, M}, {(void **)&ws.precip, (size_t)nxy * D},
        {&ws.esrc, E}, {&ws.most, MO},
        {(void **)&b.rho0, nzs * D}, {(void **)&b.theta0, nzs * D}, {(void **)&b.Theta0, nzs * D},
        {(void **)&b.p0, nzs * D}, {(void **)&b.pi0, nzs * D}, {(void **)&b.dz, (5 * nzs + 1) * D},
        {(void **)&b.qv0, nzs * D}, {(void **)&b.rho0t, nzs * D},
        {(void **)&an.pa, A8}, {(void **)&an.Z, A16}, {(void **)&an.cp, A8}, {(void **)&an.phi, A8},
        {(void **)&an.twx, anel ? (size_t)(grid->nx / 2) * sizeof(double2) : 0},
        {(void **)&an.twy, anel ? (size_t)(grid->ny / 2) * sizeof(double2) : 0},
    };
    size_t total = 0;
    for (const Req &r : reqs) total += align_up(r.bytes);
    hipError_t e = hipMalloc(&c->arena, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete[] c->dz_host;
        delete c;
        return ERF_E_NOMEM;
    }
    c->ws_bytes = (int64_t)total;
    char *p = (char *)c->arena;
    for (const Req &r : reqs) {
        *r.p = r.bytes ? (void *)p : nullptr;
        p += align_up(r.bytes);
    }
    // dz, centre heights, 1/dz and 2/(dz_{k-1} + dz_k) on the z-faces
    const int nz = grid->nz;
    b.nz = nz;
    double *hz = new double[5 * nz + 1];
    double zc = 0.0;
    for (int k = 0; k < nz; ++k) {
        hz[k] = grid->dz[k];
        hz[nz + k] = zc + 0.5 * grid->dz[k];
        hz[2 * nz + k] = 1.0 / grid->dz[k];
        hz[3 * nz + k] = k == 0 ? 0.0 : 2.0 / (grid->dz[k - 1] + grid->dz[k]);
        zc += grid->dz[k];
    }
    hz[4 * nz] = 0.0;
    // no rain has fallen yet
    e = hipMemset(ws.precip, 0, (size_t)nxy * sizeof(double));
    if (e != hipSuccess) {
        delete[] hz;
        erf_destroy(c);
        return ERF_E_HIP;
    }
    for (int k = 0; k < nz; ++k) {
        const double cd = prm->Cs * std::cbrt(grid->dx * grid->dy * grid->dz[k]);
        hz[4 * nz + 1 + k] = cd * cd;
    }
    e = hipMemcpy(b.dz, hz, (5 * nz + 1) * sizeof(double), hipMemcpyHostToDevice);
    delete[] hz;
    if (e != hipSuccess) {
        erf_destroy(c);
        return ERF_E_HIP;
    }
    if (anel) {
        // twiddle factors exp(-2 pi i t / N), t < N/2, of the two transform lengths
        for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
            const int N = dir == 0 ? grid->nx : grid->ny;
            int lg = 0;
            while ((1 << lg) < N) ++lg;
            (dir == 0 ? an.lgx : an.lgy) = lg;
            if (N < 2) continue;
            std::vector<double2> tw(N / 2);
            const double two_pi = 6.283185307179586476925286766559;
            for (int q = 0; q < N / 2; ++q) tw[q] = make_double2(std::cos(two_pi * q / N), -std::sin(two_pi * q / N));
            e = hipMemcpy(dir == 0 ? an.twx : an.twy, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipMemset(an.pa, 0, n * sizeof(double));
        if (e != hipSuccess) {
            erf_destroy(c);
            return ERF_E_HIP;
        }
    }
    *out = c;
    return ERF_OK;
}

void erf_destroy(erf_ctx *c)
{
    if (!c) return;
    for (auto &x : c->timing_events)
        if (x) (void)hipEventDestroy(x);
    if (c->arena || c->mlp.alloc || c->mlp.talloc) (void)hipStreamSynchronize(c->stream);
    if (c->arena) (void)hipFree(c->arena);
    if (c->mlp.alloc) (void)hipFree(c->mlp.alloc);
    if (c->mlp.talloc) (void)hipFree(c->mlp.talloc);
    if (c->ter.mem) (void)hipFree(c->ter.mem);
    delete[] c->dz_host;
    delete c;
}

erf_status erf_init_base_state(erf_ctx *c, const double *theta0, const double *qv0, double p_surface,
                               double *rho0_out, double *p0_out, double *pi0_out)
{
    ERF_CHECK_CTX(c);
    if (!theta0) return fail(c, ERF_E_ARG, "theta0 is NULL");
    if (qv0 && !c->prm.moist) return fail(c, ERF_E_ARG, "qv0 given to a dry context");
    if (c->ter.on) return fail(c, ERF_E_UNSUPPORTED, "a terrain context takes erf_init_base_state_columns");
    const int nz = c->d.nz;
    double *h = new double[7 * nz];
    double *rho0 = h, *p0 = h + nz, *pi0 = h + 2 * nz, *Th0 = h + 3 * nz, *th0 = h + 4 * nz;
    double *qv = h + 5 * nz, *rho0t = h + 6 * nz;
    erf_status s = base_state(nz, c->dz_host, theta0, qv0, p_surface, c->prm.grav, rho0, p0, pi0);
    if (s != ERF_OK) {
        delete[] h;
        return fail(c, s, "base state: invalid theta0, qv0 or dz");
    }
    for (int k = 0; k < nz; ++k) {
        th0[k] = theta0[k];
        Th0[k] = rho0[k] * theta0[k];
        qv[k] = qv0 ? qv0[k] : 0.0;
        rho0t[k] = rho0[k] * (1.0 + qv[k]);
    }
    hipError_t e = hipMemcpyAsync(c->base.rho0, rho0, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.p0, p0, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.pi0, pi0, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.Theta0, Th0, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.theta0, th0, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.qv0, qv, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->base.rho0t, rho0t, nz * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete[] h;
        return hip_fail(c, e, "uploading the base state");
    }
    if (rho0_out) std::memcpy(rho0_out, rho0, nz * sizeof(double));
    if (p0_out) std::memcpy(p0_out, p0, nz * sizeof(double));
    if (pi0_out) std::memcpy(pi0_out, pi0, nz * sizeof(double));
    delete[] h;
    c->have_base = true;
    return ERF_OK;
}

// ---- terrain-following coordinates (Sec. 3.4, App. A, App. B) ----------------
erf_status erf_set_terrain(erf_ctx *c, const double *h, double beta)
{
    ERF_CHECK_CTX(c);
    if (!h) return fail(c, ERF_E_ARG, "terrain heights are NULL");
    const erf_params &p = c->prm;
    if (p.precision != ERF_FP64 || p.moist || p.anelastic || p.sgs != ERF_SGS_NONE || p.nu_m != 0.0 ||
        p.alpha_m != 0.0 || p.most_z0 > 0.0 || c->member)
        return fail(c, ERF_E_UNSUPPORTED,
                    "terrain needs a dry, inviscid ERF_FP64 compressible context without surface layer");
    if (!(beta >= 1.0 && beta <= 8.0)) return fail(c, ERF_E_ARG, "beta must lie in [1, 8]");
    const int nx = c->d.nx, ny = c->d.ny, nz = c->d.nz, nxy = c->d.nxy;
    const size_t n = (size_t)c->d.n, nw = (size_t)c->d.nw;
    std::vector<double> sl(nz + 1), hb(nxy), Hc(n), zc(n);
    double zt = 0.0;
    for (int k = 0; k < nz; ++k) zt += c->dz_host[k];
    double zeta = 0.0;
    for (int k = 0; k <= nz; ++k) {
        sl[k] = (k == nz) ? 0.0 : std::pow(1.0 - zeta / zt, beta);
        if (k < nz) zeta += c->dz_host[k];
    }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int i1 = (i + 1) % nx, j1 = (j + 1) % ny;
            const double a = h[(size_t)j * nx + i], b = h[(size_t)j * nx + i1];
            const double e = h[(size_t)j1 * nx + i], f = h[(size_t)j1 * nx + i1];
            if (!std::isfinite(a)) return fail(c, ERF_E_ARG, "terrain heights must be finite");
            hb[(size_t)j * nx + i] = 0.25 * ((a + b) + (e + f));
        }
    zeta = 0.0;
    for (int k = 0; k < nz; ++k) {
        for (int q = 0; q < nxy; ++q) {
            const size_t cc = (size_t)k * nxy + q;
            Hc[cc] = c->dz_host[k] + (sl[k + 1] - sl[k]) * hb[q];
            zc[cc] = (zeta + 0.5 * c->dz_host[k]) + 0.5 * (sl[k] + sl[k + 1]) * hb[q];
            if (!(Hc[cc] > 0.0)) return fail(c, ERF_E_ARG, "terrain too high: a cell of non-positive height");
        }
        zeta += c->dz_host[k];
    }
    Terrain &t = c->ter;
    if (!t.mem) {
        const size_t doubles = (size_t)(nz + 1) + nxy + 14 * n + 7 * nw;
        hipError_t e = hipMalloc(&t.mem, doubles * sizeof(double));
        if (e != hipSuccess) {
            t.mem = nullptr;
            return fail(c, ERF_E_NOMEM, "terrain arrays do not fit");
        }
        double *m = (double *)t.mem;
        t.s = m, m += nz + 1;
        t.hb = m, m += nxy;
        t.Hc = m, m += n;
        t.rho0 = m, m += n;
        t.theta0 = m, m += n;
        t.Theta0 = m, m += n;
        t.p0 = m, m += n;
        t.pi0 = m, m += n;
        t.tht = m, m += n;
        t.rh = m, m += n;
        t.om = m, m += nw;
        t.cp = m, m += nw;
        t.dp = m, m += nw;
        t.J = m, m += n;
        t.mo = m, m += nw;
        t.mn = m, m += nw;
        t.JU = m, m += n;
        t.JV = m, m += n;
        t.hxU = m, m += n;
        t.heV = m, m += n;
        t.hxW = m, m += nw;
        t.heW = m, m += nw;
        t.dzc = m;
    }
    std::vector<double> Jc(n);
    for (int k = 0; k < nz; ++k)
        for (int q = 0; q < nxy; ++q) Jc[(size_t)k * nxy + q] = Hc[(size_t)k * nxy + q] / c->dz_host[k];
    // face metrics, in the expressions and order the kernels used to evaluate
    // them (App. B): h_zeta on x-/y-faces as two-cell means, h_xi on x-faces
    // from the centre heights, h_xi on z-faces by the fourth-order difference
    std::vector<double> JU(n), JV(n), hxU(n), heV(n), hxW(nw), heW(nw), dzc(n);
    // the distance of the centres above and below each cell, summed as the
    // kernels summed it (half the outer cells, then the cell between)
    for (int k = 0; k < nz; ++k) {
        const int kl = k > 0 ? k - 1 : 0, ku = k < nz - 1 ? k + 1 : nz - 1;
        for (int q = 0; q < nxy; ++q) {
            double v = 0.5 * Hc[(size_t)kl * nxy + q] + 0.5 * Hc[(size_t)ku * nxy + q];
            for (int mm = kl + 1; mm < ku; ++mm) v += Hc[(size_t)mm * nxy + q];
            dzc[(size_t)k * nxy + q] = v;
        }
    }
    const double dx = c->grid.dx, dy = c->grid.dy;
    const auto H = [&](int i, int j) { return hb[(size_t)((j % ny + ny) % ny) * nx + (i % nx + nx) % nx]; };
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t q = ((size_t)k * ny + j) * nx + i;
                hxW[q] = sl[k] * ((H(i - 2, j) - H(i + 2, j)) + 8.0 * (H(i + 1, j) - H(i - 1, j))) / (12.0 * dx);
                heW[q] = sl[k] * ((H(i, j - 2) - H(i, j + 2)) + 8.0 * (H(i, j + 1) - H(i, j - 1))) / (12.0 * dy);
                if (k == nz) continue;
                const size_t kq = (size_t)k * nxy;
                const double Jw = Jc[kq + (size_t)j * nx + (i + nx - 1) % nx], Js = Jc[kq + (size_t)((j + ny - 1) % ny) * nx + i];
                JU[q] = 0.5 * (Jw + Jc[q]);
                JV[q] = 0.5 * (Js + Jc[q]);
                hxU[q] = 0.5 * (sl[k] + sl[k + 1]) * (H(i, j) - H(i - 1, j)) / dx;
                heV[q] = 0.5 * (sl[k] + sl[k + 1]) * (H(i, j) - H(i, j - 1)) / dy;
            }
    hipError_t e = hipMemcpyAsync(t.s, sl.data(), (nz + 1) * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.hb, hb.data(), nxy * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.Hc, Hc.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.J, Jc.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    const double *tabs[7] = {JU.data(), JV.data(), hxU.data(), heV.data(), dzc.data(), hxW.data(), heW.data()};
    double *devs[7] = {t.JU, t.JV, t.hxU, t.heV, t.dzc, t.hxW, t.heW};
    for (int a = 0; a < 7 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(devs[a], tabs[a], (a < 5 ? n : nw) * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "uploading the terrain geometry");
    t.Hc_host = std::move(Hc);
    t.zc_host = std::move(zc);
    t.beta = beta;
    t.on = true;
    c->have_base = false;
    return ERF_OK;
}

erf_status erf_terrain_heights(const erf_ctx *c, double *Hc, double *zc)
{
    if (!c) return ERF_E_ARG;
    if (!c->ter.on) return ERF_E_STATE;
    const size_t n = (size_t)c->d.n;
    if (Hc) std::memcpy(Hc, c->ter.Hc_host.data(), n * sizeof(double));
    if (zc) std::memcpy(zc, c->ter.zc_host.data(), n * sizeof(double));
    return ERF_OK;
}

erf_status erf_init_base_state_columns(erf_ctx *c, const double *theta0, const double *p_surf, double *rho0_out,
                                       double *p0_out, double *pi0_out)
{
    ERF_CHECK_CTX(c);
    if (!c->ter.on) return fail(c, ERF_E_STATE, "erf_set_terrain must come first");
    if (!theta0 || !p_surf) return fail(c, ERF_E_ARG, "theta0 or p_surf is NULL");
    const int nz = c->d.nz, nxy = c->d.nxy;
    const size_t n = (size_t)c->d.n;
    std::vector<double> rho0(n), p0(n), pi0(n), th(n), Th0(n);
    std::vector<double> hcol(nz), tcol(nz), rc(nz), pc(nz), ic(nz);
    for (int q = 0; q < nxy; ++q) {
        for (int k = 0; k < nz; ++k) {
            hcol[k] = c->ter.Hc_host[(size_t)k * nxy + q];
            tcol[k] = theta0[(size_t)k * nxy + q];
        }
        if (!(p_surf[q] > 0.0)) return fail(c, ERF_E_ARG, "p_surf must be positive");
        erf_status s = base_state(nz, hcol.data(), tcol.data(), nullptr, p_surf[q], c->prm.grav, rc.data(),
                                  pc.data(), ic.data());
        if (s != ERF_OK) return fail(c, s, "base state: invalid theta0");
        for (int k = 0; k < nz; ++k) {
            const size_t cc = (size_t)k * nxy + q;
            rho0[cc] = rc[k];
            p0[cc] = pc[k];
            pi0[cc] = ic[k];
            th[cc] = tcol[k];
            Th0[cc] = rc[k] * tcol[k];
        }
    }
    Terrain &t = c->ter;
    const size_t B = n * sizeof(double);
    hipError_t e = hipMemcpyAsync(t.rho0, rho0.data(), B, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.theta0, th.data(), B, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.Theta0, Th0.data(), B, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.p0, p0.data(), B, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.pi0, pi0.data(), B, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "uploading the base state");
    if (rho0_out) std::memcpy(rho0_out, rho0.data(), B);
    if (p0_out) std::memcpy(p0_out, p0.data(), B);
    if (pi0_out) std::memcpy(pi0_out, pi0.data(), B);
    c->have_base = true;
    return ERF_OK;
}

static bool state_ok(const erf_state *S, bool need_q, int nq)
{
    return S && S->rho && S->rhotheta && S->rhou && S->rhov && S->rhow && (!need_q || nq == 0 || S->rhoq);
}

erf_status erf_slow_rhs(erf_ctx *c, const erf_state *S, erf_state *R)
{
    ERF_CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!state_ok(S, false, 0) || !state_ok(R, false, 0)) return fail(c, ERF_E_ARG, "null field pointer");
    if (c->prm.sgs == ERF_SGS_MLP && !c->mlp.have_weights)
        return fail(c, ERF_E_STATE, "erf_mlp_set_weights must precede the learned closure");
    const bool tke = c->prm.sgs == ERF_SGS_DEARDORFF;
    if ((c->prm.moist || tke) && !S->rhoq) return fail(c, ERF_E_ARG, "this context needs S->rhoq");
    const void *s5[5] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow};
    void *r5[5] = {R->rho, R->rhotheta, R->rhou, R->rhov, R->rhow};
    if (c->ter.on) {
        hipError_t e = launch_terrain_rhs(c, s5, r5);
        return e == hipSuccess ? ERF_OK : hip_fail(c, e, "terrain slow rhs launch");
    }
    hipError_t e = launch_slow_rhs(c, s5, (c->prm.moist || tke) ? S->rhoq : nullptr, r5);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "slow rhs launch");
}

erf_status erf_acoustic_substeps(erf_ctx *c, const erf_state *Sn, const erf_state *St, const erf_state *Rt,
                                 int32_t n_sub, double dtau, erf_state *Sout, erf_state *flux)
{
    ERF_CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!state_ok(Sn, false, 0) || !state_ok(St, false, 0) || !state_ok(Rt, false, 0) || !state_ok(Sout, false, 0))
        return fail(c, ERF_E_ARG, "null field pointer");
    if (c->prm.anelastic) return fail(c, ERF_E_UNSUPPORTED, "an anelastic context has no acoustic substeps");
    if (n_sub < 1 || !(dtau > 0.0)) return fail(c, ERF_E_ARG, "n_sub >= 1 and dtau > 0 required");
    if (c->prm.moist && !St->rhoq) return fail(c, ERF_E_ARG, "a moist context needs S_t->rhoq");
    const void *sn[5] = {Sn->rho, Sn->rhotheta, Sn->rhou, Sn->rhov, Sn->rhow};
    const void *st[5] = {St->rho, St->rhotheta, St->rhou, St->rhov, St->rhow};
    const void *rt[5] = {Rt->rho, Rt->rhotheta, Rt->rhou, Rt->rhov, Rt->rhow};
    void *so[5] = {Sout->rho, Sout->rhotheta, Sout->rhou, Sout->rhov, Sout->rhow};
    if (c->ter.on) {
        if (flux && (!flux->rhou || !flux->rhov || !flux->rhow)) return fail(c, ERF_E_ARG, "null flux pointer");
        hipError_t e = launch_terrain_stage(c, sn, st, rt, n_sub, dtau, so, flux ? flux->rhou : nullptr,
                                            flux ? flux->rhov : nullptr, flux ? flux->rhow : nullptr);
        return e == hipSuccess ? ERF_OK : hip_fail(c, e, "terrain acoustic substeps launch");
    }
    hipError_t e = launch_acoustic_stage(c, sn, st, c->prm.moist ? St->rhoq : nullptr, rt, n_sub, dtau, so,
                                         flux ? flux->rhou : nullptr,
                                         flux ? flux->rhov : nullptr, flux ? flux->rhow : nullptr);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "acoustic substeps launch");
}

erf_status erf_scalar_advance(erf_ctx *c, const erf_state *Sn, const erf_state *St, const erf_state *flux, double dts,
                              void *rhoq_out)
{
    ERF_CHECK_CTX(c);
    if (c->prm.n_scalars == 0) return ERF_OK;
    if (!Sn || !St || !flux || !Sn->rhoq || !St->rhoq || !St->rho || !flux->rhou || !flux->rhov || !flux->rhow ||
        !rhoq_out)
        return fail(c, ERF_E_ARG, "null field pointer");
    hipError_t e = launch_scalar_advance(c, Sn->rhoq, St->rho, St->rhoq, flux->rhou, flux->rhov, flux->rhow, dts,
                                         rhoq_out);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "scalar advance launch");
}

erf_status erf_rk3_step(erf_ctx *c, erf_state *S)
{
    ERF_CHECK_CTX(c);
    if (c->prm.anelastic) return fail(c, ERF_E_UNSUPPORTED, "an anelastic context steps with erf_ssprk2_step");
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    const int nq = c->prm.n_scalars;
    if (!state_ok(S, true, nq)) return fail(c, ERF_E_ARG, "null field pointer");
    Workspace &w = c->ws;
    const double dt = c->prm.dt;
    const int ns = c->prm.n_substeps;
    erf_state A{w.sa[0], w.sa[1], w.sa[2], w.sa[3], w.sa[4], w.sa[5]};
    erf_state B{w.sb[0], w.sb[1], w.sb[2], w.sb[3], w.sb[4], w.sb[5]};
    erf_state R{w.R[0], w.R[1], w.R[2], w.R[3], w.R[4], nullptr};
    erf_state F{nullptr, nullptr, w.fu, w.fv, w.fw, nullptr};
    const erf_state *St = S;
    erf_state *outs[3] = {&A, &B, S};
    for (int stage = 0; stage < 3; ++stage) {
        const double dts = stage == 0 ? dt / 3.0 : (stage == 1 ? dt / 2.0 : dt);
        const int nsub = stage == 0 ? 1 : (stage == 1 ? ns / 2 : ns);
        const double dtau = stage == 0 ? dt / 3.0 : dt / ns;
        erf_status s = erf_slow_rhs(c, St, &R);
        if (s != ERF_OK) return s;
        // the stage-averaged momenta are only needed to transport scalars
        s = erf_acoustic_substeps(c, S, St, &R, nsub, dtau, outs[stage], nq > 0 ? &F : nullptr);
        if (s != ERF_OK) return s;
        if (nq > 0) {
            s = erf_scalar_advance(c, S, St, &F, dts, outs[stage]->rhoq);
            if (s != ERF_OK) return s;
        }
        St = outs[stage];
    }
    // process-split microphysics after the dynamics step (Sec. 2.4)
    if (c->prm.microphysics) {
        hipError_t e = launch_kessler(c, S->rho, S->rhotheta, S->rhoq, dt, w.precip);
        if (e != hipSuccess) return hip_fail(c, e, "microphysics launch");
    }
    return ERF_OK;
}

erf_status erf_project(erf_ctx *c, erf_state *S, double dt)
{
    ERF_CHECK_CTX(c);
    if (!c->prm.anelastic) return fail(c, ERF_E_UNSUPPORTED, "erf_project needs an anelastic context");
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!S || !S->rhou || !S->rhov || !S->rhow) return fail(c, ERF_E_ARG, "null field pointer");
    if (!(dt > 0.0)) return fail(c, ERF_E_ARG, "dt > 0 required");
    if (c->rec) return fail(c, ERF_E_UNSUPPORTED, "anelastic calls are not recorded");
    hipError_t e = launch_project(c, S->rhou, S->rhov, S->rhow, dt);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "projection launch");
}

erf_status erf_ssprk2_step(erf_ctx *c, erf_state *S)
{
    ERF_CHECK_CTX(c);
    if (!c->prm.anelastic) return fail(c, ERF_E_UNSUPPORTED, "erf_ssprk2_step needs an anelastic context");
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    const int nq = c->prm.n_scalars;
    if (!state_ok(S, true, nq)) return fail(c, ERF_E_ARG, "null field pointer");
    if (c->rec) return fail(c, ERF_E_UNSUPPORTED, "anelastic calls are not recorded");
    Workspace &w = c->ws;
    const double dt = c->prm.dt;
    // S* (its density is the state's: rho0), the two stages' tendencies
    erf_state A{S->rho, w.sa[1], w.sa[2], w.sa[3], w.sa[4], w.sa[5]};
    erf_state R1{w.R[0], w.R[1], w.R[2], w.R[3], w.R[4], nullptr};
    erf_state R2{w.sb[0], w.sb[1], w.sb[2], w.sb[3], w.sb[4], nullptr};
    const void *sn[5] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow};
    const void *r1[5] = {R1.rho, R1.rhotheta, R1.rhou, R1.rhov, R1.rhow};
    const void *r2[5] = {R2.rho, R2.rhotheta, R2.rhou, R2.rhov, R2.rhow};
    void *sa[5] = {A.rho, A.rhotheta, A.rhou, A.rhov, A.rhow};
    void *so[5] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow};
    // stage 1 with the lagged pressure
    erf_status s = erf_slow_rhs(c, S, &R1);
    if (s != ERF_OK) return s;
    hipError_t e = launch_ssp_update(c, 1, sn, r1, nullptr, sa, dt);
    if (e != hipSuccess) return hip_fail(c, e, "stage update launch");
    if (nq > 0 && (s = erf_scalar_advance(c, S, S, S, dt, A.rhoq)) != ERF_OK) return s;
    e = launch_project(c, A.rhou, A.rhov, A.rhow, dt);
    if (e != hipSuccess) return hip_fail(c, e, "projection launch");
    // stage 2
    if ((s = erf_slow_rhs(c, &A, &R2)) != ERF_OK) return s;
    if (nq > 0 && (s = erf_scalar_advance(c, S, &A, &A, dt, w.sb[5])) != ERF_OK) return s;
    e = launch_ssp_update(c, 2, sn, r1, r2, so, dt);
    if (e == hipSuccess && nq > 0) e = launch_qavg(c, A.rhoq, w.sb[5], S->rhoq, (int64_t)nq * c->d.n);
    if (e == hipSuccess) e = launch_project(c, S->rhou, S->rhov, S->rhow, dt);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "stage update / projection launch");
}

erf_status erf_anelastic_pressure(erf_ctx *c, void *p, int32_t set)
{
    ERF_CHECK_CTX(c);
    if (!c->prm.anelastic) return fail(c, ERF_E_UNSUPPORTED, "no perturbation pressure in a compressible context");
    if (!p || (set != 0 && set != 1)) return fail(c, ERF_E_ARG, "null buffer or set not 0 / 1");
    const size_t bytes = (size_t)c->d.n * sizeof(double);
    hipError_t e = set ? hipMemcpyAsync(c->an.pa, p, bytes, hipMemcpyDeviceToDevice, c->stream)
                       : hipMemcpyAsync(p, c->an.pa, bytes, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "pressure copy");
}

erf_status erf_kessler(erf_ctx *c, erf_state *S, double dt, double *precip)
{
    ERF_CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!c->prm.moist) return fail(c, ERF_E_UNSUPPORTED, "the microphysics needs a moist context");
    if (!S || !S->rho || !S->rhotheta || !S->rhoq || !(dt > 0.0)) return fail(c, ERF_E_ARG, "S with rhoq and dt > 0");
    hipError_t e = launch_kessler(c, S->rho, S->rhotheta, S->rhoq, dt, precip ? precip : c->ws.precip);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "microphysics launch");
}

erf_status erf_precipitation(erf_ctx *c, double *host_out, int32_t reset)
{
    ERF_CHECK_CTX(c);
    if (!host_out) return fail(c, ERF_E_ARG, "host_out is NULL");
    const size_t bytes = (size_t)c->d.nxy * sizeof(double);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host_out, c->ws.precip, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) e = hipMemsetAsync(c->ws.precip, 0, bytes, c->stream);
    if (e == hipSuccess && reset) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "reading the precipitation");
}

erf_status erf_timing_begin(erf_ctx *c, const char *kernel, int32_t max_launches)
{
    ERF_CHECK_CTX(c);
    if (!kernel || max_launches < 1) return fail(c, ERF_E_ARG, "kernel name and max_launches >= 1 required");
    int id = -1;
    for (int k = 0; k < K_COUNT; ++k)
        if (std::strcmp(kernel, kernel_name(k)) == 0) id = k;
    if (id < 0) return fail(c, ERF_E_ARG, "unknown kernel name");
    int64_t ms = 0;
    double t = 0.0;
    if (c->timed_kernel >= 0) erf_timing_end(c, &t, &ms);
    c->timing_events.assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : c->timing_events) {
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            for (auto &x : c->timing_events)
                if (x) (void)hipEventDestroy(x);
            c->timing_events.clear();
            return fail(c, ERF_E_NOMEM, "hipEventCreate failed");
        }
    }
    c->timed_kernel = id;
    c->timed_count = 0;
    return ERF_OK;
}

erf_status erf_timing_end(erf_ctx *c, double *total_ms, int64_t *launches)
{
    ERF_CHECK_CTX(c);
    double tot = 0.0;
    hipError_t e = hipStreamSynchronize(c->stream);
    for (int i = 0; e == hipSuccess && i < c->timed_count; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->timing_events[2 * i], c->timing_events[2 * i + 1]);
        tot += ms;
    }
    int64_t n = c->timed_count;
    for (auto &x : c->timing_events)
        if (x) (void)hipEventDestroy(x);
    c->timing_events.clear();
    c->timed_kernel = -1;
    c->timed_count = 0;
    if (e != hipSuccess) return hip_fail(c, e, "timing events");
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return ERF_OK;
}

erf_status erf_diagnostics(erf_ctx *c, const erf_state *S, erf_diag *out)
{
    ERF_CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!state_ok(S, true, c->prm.n_scalars) || !out) return fail(c, ERF_E_ARG, "null pointer");
    double h[13];
    const void *s6[6] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow, S->rhoq};
    hipError_t e = launch_diagnostics(c, s6, h);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostics");
    out->mass = h[0];
    out->theta_mass = h[1];
    out->energy = h[2];
    out->max_w = h[3];
    out->nonfinite = (int64_t)h[4];
    for (int s = 0; s < 8; ++s) out->scalar_mass[s] = h[5 + s];
    return out->nonfinite ? ERF_E_NONFINITE : ERF_OK;
}

}  // extern "C"
