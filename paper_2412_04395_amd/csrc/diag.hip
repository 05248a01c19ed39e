// diag.hip -- FP64 budget sums (mass and energy, Sec. 4.1.2) and a non-finite
// count.  Two passes with a fixed reduction tree, so the result does not
// depend on scheduling: per-block partials in a grid-stride loop, then one
// block sums the partials in block order.  Every sum is compensated: each
// partial is a pair (s, c) whose exact value s + c carries the rounding error
// of every addition so far (Neumaier's variant of Kahan summation within a
// thread, Knuth's error-free TwoSum where two pairs are merged), so that long
// FP64 budgets keep contributions far below one ulp of the total.
#include "erf_internal.h"

namespace erfk {
namespace {

constexpr int kSlots = 13;  // mass, theta, energy, maxw, nonfinite, 8 scalars
constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

template <typename T>
struct DiagArgs {
    Dims d;
    int nq;
    double dx, dy, g;
    const double *dz, *zc, *rho0, *Theta0;
    // terrain (null without): physical cell heights [n], corner-mean terrain
    // height per column and s_k = (1 - zeta_k / z_t)^beta [nz + 1]
    const double *Hc, *hb, *sl;
    const T *rho, *rt, *ru, *rv, *rw, *rq;
    double *part;
};

__device__ __forceinline__ bool bad(double x) { return !isfinite(x); }

// A compensated sum: the exact total is s + c.
struct CSum {
    double s, c;
};
// add x (Neumaier): the rounding error of s + x goes to c
__device__ __forceinline__ void cadd(CSum &a, double x)
{
    const double t = a.s + x;
    a.c += fabs(a.s) >= fabs(x) ? (a.s - t) + x : (x - t) + a.s;
    a.s = t;
}
// merge two pairs: TwoSum of the leading parts, the compensations added
__device__ __forceinline__ CSum cmerge(CSum a, CSum b)
{
    const double t = a.s + b.s, bp = t - a.s, e = (a.s - (t - bp)) + (b.s - bp);
    return {t, (a.c + b.c) + e};
}

__device__ __forceinline__ CSum block_sum(CSum v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = cmerge(v, {__shfl_down(v.s, o, 64), __shfl_down(v.c, o, 64)});
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * wv] = v.s;
        sh[2 * wv + 1] = v.c;
    }
    __syncthreads();
    CSum r{0.0, 0.0};
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) r = cmerge(r, {sh[2 * q], sh[2 * q + 1]});
    return r;
}
__device__ __forceinline__ double block_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) r = fmax(r, sh[q]);
    return r;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag_partial(DiagArgs<T> a)
{
    __shared__ double sh[2 * (kThreads / 64)];
    const Dims &d = a.d;
    // slot 3 (max |w|) and slot 4 (a count) use .s only
    CSum acc[kSlots];
    for (int s = 0; s < kSlots; ++s) acc[s] = {0.0, 0.0};
    const int total = d.nw;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < total; c += gridDim.x * kThreads) {
        int k = c / d.nxy, rem = c - k * d.nxy, j = rem / d.nx, i = rem - j * d.nx;
        double W = a.rw[c];
        if (bad(W)) acc[4].s += 1.0;
        // full density on level kk
        auto rh = [&](int cc, int kk) { return full_of(a.rho, cc, a.rho0[kk]); };
        if (k > 0 && k < d.nz) {
            double wv = fabs(W / (0.5 * (rh(c - d.nxy, k - 1) + rh(c, k))));
            acc[3].s = fmax(acc[3].s, wv);
        }
        if (k == d.nz) continue;
        // terrain: the cell's physical volume and its centre's height
        double vol = a.Hc ? a.dx * a.dy * a.Hc[c] : a.dx * a.dy * a.dz[k];
        const double zck = a.Hc ? a.zc[k] + 0.5 * (a.sl[k] + a.sl[k + 1]) * a.hb[rem] : a.zc[k];
        double r = rh(c, k), Tf = full_of(a.rt, c, a.Theta0[k]), U = a.ru[c], V = a.rv[c];
        acc[4].s += (double)bad(r) + (double)bad(Tf) + (double)bad(U) + (double)bad(V);
        cadd(acc[0], r * vol);
        cadd(acc[1], Tf * vol);
        int ip = wrap_idx(i + 1, d.nx), im = wrap_idx(i - 1, d.nx), jp = wrap_idx(j + 1, d.ny), jm = wrap_idx(j - 1, d.ny);
        double uc = 0.5 * (U / (0.5 * (rh(cidx(d, im, j, k), k) + r)) +
                           a.ru[cidx(d, ip, j, k)] / (0.5 * (r + rh(cidx(d, ip, j, k), k))));
        double vc = 0.5 * (V / (0.5 * (rh(cidx(d, i, jm, k), k) + r)) +
                           a.rv[cidx(d, i, jp, k)] / (0.5 * (r + rh(cidx(d, i, jp, k), k))));
        double wb = (k == 0) ? 0.0 : W / (0.5 * (rh(c - d.nxy, k - 1) + r));
        double wt = (k == d.nz - 1) ? 0.0 : a.rw[c + d.nxy] / (0.5 * (r + rh(c + d.nxy, k + 1)));
        double wc = 0.5 * (wb + wt);
        double temp = (Tf / r) * pow(kRd * Tf / kP00, kGamma - 1.0);
        cadd(acc[2], (0.5 * r * (uc * uc + vc * vc + wc * wc) + r * kCv * temp + r * a.g * zck) * vol);
        for (int s = 0; s < a.nq && s < 8; ++s) cadd(acc[5 + s], (double)a.rq[(size_t)s * d.n + c] * vol);
    }
    // partials as (s, c) pairs: slot s of block b at part[(b * kSlots + s) * 2]
    for (int s = 0; s < kSlots; ++s) {
        CSum v{0.0, 0.0};
        if (s == 3)
            v.s = block_max(acc[s].s, sh);
        else if (s == 4)
            v.s = block_sum({acc[s].s, 0.0}, sh).s;  // a count of at most 2^31: exact
        else
            v = block_sum(acc[s], sh);
        if (threadIdx.x == 0) {
            a.part[(blockIdx.x * kSlots + s) * 2] = v.s;
            a.part[(blockIdx.x * kSlots + s) * 2 + 1] = v.c;
        }
    }
}

// the block partials in block order; the result s + c rounded once
__global__ __launch_bounds__(64) void k_diag_final(double *part, int nblocks)
{
    int s = threadIdx.x;
    if (s >= kSlots) return;
    CSum acc{0.0, 0.0};
    for (int b = 0; b < nblocks; ++b) {
        const CSum v{part[(b * kSlots + s) * 2], part[(b * kSlots + s) * 2 + 1]};
        if (s == 3)
            acc.s = fmax(acc.s, v.s);
        else
            acc = cmerge(acc, v);
    }
    part[2 * nblocks * kSlots + s] = acc.s + acc.c;
}

}  // namespace

namespace {
template <typename T>
hipError_t diag_t(erf_ctx *cx, const void *const S[6], double *host_out)
{
    DiagArgs<T> a{};
    a.d = cx->d;
    a.nq = cx->prm.n_scalars;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.g = cx->prm.grav;
    a.dz = cx->base.dz;
    a.zc = cx->base.zc();
    a.rho0 = cx->base.rho0;
    a.Theta0 = cx->base.Theta0;
    a.Hc = cx->ter.on ? cx->ter.Hc : nullptr;
    a.hb = cx->ter.hb;
    a.sl = cx->ter.s;
    a.rho = (const T *)S[0];
    a.rt = (const T *)S[1];
    a.ru = (const T *)S[2];
    a.rv = (const T *)S[3];
    a.rw = (const T *)S[4];
    a.rq = (const T *)S[5];
    a.part = cx->ws.diag;
    int nb = (cx->d.nw + kThreads - 1) / kThreads;
    if (nb > kBlocks) nb = kBlocks;
    hipLaunchKernelGGL(k_diag_partial<T>, dim3(nb), dim3(kThreads), 0, cx->stream, a);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, cx->stream, a.part, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_out, a.part + 2 * (size_t)nb * kSlots, kSlots * sizeof(double), hipMemcpyDeviceToHost,
                       cx->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(cx->stream);
}
}  // namespace

hipError_t launch_diagnostics(erf_ctx *cx, const void *const S[6], double *host_out)
{
    if (cx->prm.precision == ERF_FP32_MIXED) return diag_t<float>(cx, S, host_out);
    return diag_t<double>(cx, S, host_out);
}

size_t diag_slots_needed() { return (size_t)(2 * kBlocks + 1) * kSlots; }

}  // namespace erfk
