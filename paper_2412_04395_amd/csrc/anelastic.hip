// anelastic.hip -- the anelastic equation set (Sec. 2.2) advanced by the
// second-order strong-stability-preserving Runge-Kutta scheme with a
// projection after each stage (Sec. 3.2), FP64.
//
//   k_ssp_update  S* = S^n + dt R1 (stage 1) or S^n + dt (R1 + R2) / 2
//                 (stage 2) for rho theta and the three face momenta; rho
//                 stays rho0
//   k_qavg        the scalars' second stage, ((rho q)^* + (rho q)^n - dt
//                 div(U* q*)) / 2
//   projection    dt div grad psi = div(rho0 u); with phi = dt psi:
//     k_div_fftx  the divergence of the face momenta along one x-line and its
//                 discrete Fourier transform in x, of which the x-wavenumbers
//                 0..nx/2 are kept (the divergence is real: the others are
//                 their complex conjugates)
//     k_ffty      the transform in y of a few adjacent x-wavenumbers per block
//     k_poisson_z per horizontal wavenumber the tridiagonal z solve (Thomas;
//                 real coefficients, complex right-hand side)
//     k_ffty      (inverse), then k_ifftx: the line completed by conjugate
//                 symmetry, the inverse in x and 1/(nx ny)
//     k_project   face momenta minus grad phi; the pressure plus phi / dt
// The half spectrum holds nh = nx/2 + 1 wavenumbers per line ([nz][ny][nh]):
// the y transforms and the z solves run over nh (not nx) columns.
//
// The transforms are radix-2 Stockham passes in LDS (no bit-reversal pass):
// nx and ny are powers of two up to 2048, so that a whole line of complex
// doubles (and its ping-pong copy) fits in 64 KiB of LDS.  Every pass moves
// each value once through HBM; the z solve walks the columns with the
// coefficients of the stretched grid, as the acoustic solve does.
#include "erf_internal.h"

namespace erfk {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct SspArgs {
    int n, nw;
    double dt;
    const double *sn[4], *r1[4], *r2[4];  // rho theta, rho u, rho v, rho w
    double *out[4];
};

template <int kStage>
__global__ __launch_bounds__(256) void k_ssp_update(SspArgs a)
{
    const int f = blockIdx.y;
    const int cnt = f == 3 ? a.nw : a.n;
    const int stride = gridDim.x * blockDim.x;
    const double *sn = a.sn[f], *r1 = a.r1[f];
    double *out = a.out[f];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cnt; c += stride) {
        if constexpr (kStage == 1)
            out[c] = sn[c] + a.dt * r1[c];
        else
            out[c] = sn[c] + 0.5 * a.dt * (r1[c] + a.r2[f][c]);
    }
}

__global__ __launch_bounds__(256) void k_qavg(const double *a, const double *b, double *out, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < count; c += stride)
        out[c] = 0.5 * (a[c] + b[c]);
}

struct ProjArgs {
    Dims d;
    double dx, dy, dt;
    const double *dz;
    double *ru, *rv, *rw;
    double2 *Z;
    double *cp, *phi, *pa;
    const double2 *twx, *twy;
    int lgx, lgy, cols;  // log2 nx, log2 ny, x-columns per block of the y transform
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Radix-2 Stockham passes over `cols` interleaved lines of length N = 2^lg
// held in LDS (element j of line q at j * cols + q), ping-ponging between a
// and b.  Pass s combines pairs of the 2^s-point transforms of the previous
// pass: with k = j mod 2^s, v0 = x[j], v1 = x[j + N/2] w^(k N / 2^(s+1)) go
// to positions 2 (j - k) + k and that plus 2^s as v0 + v1 and v0 - v1.
// tw[t] = exp(-2 pi i t / N); the inverse uses the conjugates.  Returns the
// buffer that holds the result.
__device__ double2 *fft_lds(double2 *a, double2 *b, int lg, int cols, const double2 *tw, bool inverse)
{
    const int half = (1 << lg) >> 1;
    for (int s = 0; s < lg; ++s) {
        const int ns = 1 << s;
        for (int t = threadIdx.x; t < half * cols; t += blockDim.x) {
            const int q = t % cols, j = t / cols;
            const int k = j & (ns - 1);
            double2 w = tw[k << (lg - 1 - s)];
            if (inverse) w.y = -w.y;
            const double2 v0 = a[j * cols + q];
            const double2 v1 = cmul(a[(j + half) * cols + q], w);
            const int o = ((j - k) << 1) + k;
            b[o * cols + q] = make_double2(v0.x + v1.x, v0.y + v1.y);
            b[(o + ns) * cols + q] = make_double2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
        double2 *tmp = a;
        a = b;
        b = tmp;
    }
    return a;
}

// one block per x-line (k, j): divergence, then its transform in x
__global__ __launch_bounds__(256) void k_div_fftx(ProjArgs a)
{
    extern __shared__ double2 lds[];
    const Dims &d = a.d;
    const int nx = d.nx, row = blockIdx.x, k = row / d.ny, j = row - k * d.ny;
    const int base = row * nx, jn = j + 1 == d.ny ? 0 : j + 1, bn = (k * d.ny + jn) * nx;
    double2 *A = lds, *B = lds + nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const int c = base + i, ie = i + 1 == nx ? 0 : i + 1;
        const double D = (a.ru[base + ie] - a.ru[c]) / a.dx + (a.rv[bn + i] - a.rv[c]) / a.dy +
                         (a.rw[c + d.nxy] - a.rw[c]) / a.dz[k];
        A[i] = make_double2(D, 0.0);
    }
    __syncthreads();
    const double2 *r = fft_lds(A, B, a.lgx, 1, a.twx, false);
    const int nh = nx / 2 + 1;
    for (int m = threadIdx.x; m < nh; m += blockDim.x) a.Z[row * nh + m] = r[m];
}

// one block per (level, group of `cols` adjacent x-wavenumbers): transform in
// y (the last group of a level may be partly past nh: zeros, not stored)
__global__ __launch_bounds__(256) void k_ffty(ProjArgs a, int inverse)
{
    extern __shared__ double2 lds[];
    const Dims &d = a.d;
    const int nh = d.nx / 2 + 1, cols = a.cols, ny = d.ny, groups = (nh + cols - 1) / cols;
    const int k = blockIdx.x / groups, m0 = (blockIdx.x - k * groups) * cols;
    double2 *A = lds, *B = lds + ny * cols;
    double2 *Z = a.Z + (size_t)k * ny * nh + m0;
    for (int t = threadIdx.x; t < ny * cols; t += blockDim.x) {
        const int q = t % cols;
        A[t] = m0 + q < nh ? Z[(t / cols) * nh + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const double2 *r = fft_lds(A, B, a.lgy, cols, a.twy, inverse != 0);
    for (int t = threadIdx.x; t < ny * cols; t += blockDim.x) {
        const int q = t % cols;
        if (m0 + q < nh) Z[(t / cols) * nh + q] = r[t];
    }
}

// one thread per horizontal wavenumber (m, l): the z operator
// a_k phi_{k-1} + b_k phi_k + c_k phi_{k+1} with a_k = 1/(dz_k dzc_k),
// c_k = 1/(dz_k dzc_{k+1}) (dzc: distance between centres; no flux through
// the lids) and b_k = -a_k - c_k - 4 sin^2(pi m/nx)/dx^2 - 4 sin^2(pi l/ny)/dy^2,
// solved by the Thomas algorithm; mode (0, 0) takes the gauge phi_0 = 0.
__global__ __launch_bounds__(64) void k_poisson_z(ProjArgs a)
{
    const Dims &d = a.d;
    const int nh = d.nx / 2 + 1;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nh * d.ny) return;
    const int l = q / nh, m = q - l * nh, nz = d.nz, P = nh * d.ny;
    const double *dz = a.dz;
    const double sx = sin(0.5 * kTwoPi * m / d.nx), sy = sin(0.5 * kTwoPi * l / d.ny);
    const double lam = -4.0 * sx * sx / (a.dx * a.dx) - 4.0 * sy * sy / (a.dy * a.dy);
    double2 *Z = a.Z + q;
    double *cp = a.cp + q;
    double cpm = 0.0;
    double2 dpm = make_double2(0.0, 0.0);
    // Both sweeps walk the column in chunks of kB levels; the values of the
    // next chunk are read before the current one is stored, so their loads are
    // in flight while it is eliminated (a load issued after a store to the same
    // array would wait for it).
    constexpr int kB = 8;
    double2 zb[kB], zn[kB];
#pragma unroll
    for (int t = 0; t < kB; ++t) zb[t] = t < nz ? Z[(size_t)t * P] : make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < nz; k0 += kB) {
#pragma unroll
        for (int t = 0; t < kB; ++t) zn[t] = k0 + kB + t < nz ? Z[(size_t)(k0 + kB + t) * P] : make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            const int k = k0 + t;
            if (k >= nz) break;
            const double ak = k > 0 ? 1.0 / (dz[k] * 0.5 * (dz[k - 1] + dz[k])) : 0.0;
            const double ck = k < nz - 1 ? 1.0 / (dz[k] * 0.5 * (dz[k] + dz[k + 1])) : 0.0;
            double bk = -ak - ck + lam, cc = ck;
            double2 r = zb[t];
            if (q == 0 && k == 0) {
                bk = 1.0;
                cc = 0.0;
                r = make_double2(0.0, 0.0);
            }
            double cpk;
            double2 dp;
            if (k == 0) {
                cpk = cc / bk;
                dp = make_double2(r.x / bk, r.y / bk);
            } else {
                const double den = bk - ak * cpm;
                cpk = cc / den;
                dp = make_double2((r.x - ak * dpm.x) / den, (r.y - ak * dpm.y) / den);
            }
            cp[(size_t)k * P] = cpk;
            Z[(size_t)k * P] = dp;
            cpm = cpk;
            dpm = dp;
        }
#pragma unroll
        for (int t = 0; t < kB; ++t) zb[t] = zn[t];
    }
    // back substitution from level nz - 2 down
    double2 x = dpm;
    double cb[kB], cn[kB];
    auto load_down = [&](double2 (&zv)[kB], double (&cv)[kB], int ktop) {
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            const int k = ktop - t;
            zv[t] = k >= 0 ? Z[(size_t)k * P] : make_double2(0.0, 0.0);
            cv[t] = k >= 0 ? cp[(size_t)k * P] : 0.0;
        }
    };
    load_down(zb, cb, nz - 2);
    for (int k1 = nz - 2; k1 >= 0; k1 -= kB) {
        load_down(zn, cn, k1 - kB);
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            const int k = k1 - t;
            if (k < 0) break;
            x = make_double2(zb[t].x - cb[t] * x.x, zb[t].y - cb[t] * x.y);
            Z[(size_t)k * P] = x;
        }
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            zb[t] = zn[t];
            cb[t] = cn[t];
        }
    }
}

// one block per x-line: inverse transform in x and the 1/(nx ny) of the
// inverse transform; phi is real
__global__ __launch_bounds__(256) void k_ifftx(ProjArgs a)
{
    extern __shared__ double2 lds[];
    const Dims &d = a.d;
    const int nx = d.nx, base = blockIdx.x * nx, nh = nx / 2 + 1;
    double2 *A = lds, *B = lds + nx;
    // the line from its half spectrum: X(nx - m) = conj(X(m))
    for (int m = threadIdx.x; m < nh; m += blockDim.x) {
        const double2 z = a.Z[blockIdx.x * nh + m];
        A[m] = z;
        if (m > 0 && m < nx - m) A[nx - m] = make_double2(z.x, -z.y);
    }
    __syncthreads();
    const double2 *r = fft_lds(A, B, a.lgx, 1, a.twx, true);
    const double s = (double)d.nx * d.ny;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) a.phi[base + i] = r[i].x / s;
}

// (rho0 u)^new = (rho0 u)^* - grad phi on every face; p' += phi / dt
__global__ __launch_bounds__(256) void k_project(ProjArgs a)
{
    const Dims &d = a.d;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.n) return;
    const int k = c / d.nxy, r = c - k * d.nxy, j = r / d.nx, i = r - j * d.nx;
    const int cw = c + (i == 0 ? d.nx - 1 : -1), cs = c + (j == 0 ? (d.ny - 1) * d.nx : -d.nx);
    const double p = a.phi[c];
    a.ru[c] -= (p - a.phi[cw]) / a.dx;
    a.rv[c] -= (p - a.phi[cs]) / a.dy;
    if (k > 0) a.rw[c] -= (p - a.phi[c - d.nxy]) / (0.5 * (a.dz[k - 1] + a.dz[k]));
    a.pa[c] += p / a.dt;
}

int grid_for(int64_t count)
{
    int64_t b = (count + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

int anel_ffty_cols(int nx, int ny)
{
    const int nh = nx / 2 + 1;
    int c = 8;
    while (c > 1 && (c > nh || c * ny > 2048)) c >>= 1;
    return c;
}

hipError_t launch_ssp_update(erf_ctx *cx, int stage, const void *const Sn[5], const void *const R1[5],
                             const void *const R2[5], void *const out[5], double dt)
{
    SspArgs a{};
    a.n = cx->d.n;
    a.nw = cx->d.nw;
    a.dt = dt;
    for (int f = 0; f < 4; ++f) {
        a.sn[f] = (const double *)Sn[f + 1];
        a.r1[f] = (const double *)R1[f + 1];
        a.r2[f] = R2 ? (const double *)R2[f + 1] : nullptr;
        a.out[f] = (double *)out[f + 1];
    }
    dim3 grd(grid_for(a.nw), 4);
    timing_start(cx, K_SSP);
    if (stage == 1)
        hipLaunchKernelGGL(k_ssp_update<1>, grd, dim3(256), 0, cx->stream, a);
    else
        hipLaunchKernelGGL(k_ssp_update<2>, grd, dim3(256), 0, cx->stream, a);
    timing_stop(cx, K_SSP);
    return hipGetLastError();
}

hipError_t launch_qavg(erf_ctx *cx, const void *a, const void *b, void *out, int64_t count)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_qavg, dim3(grid_for(count)), dim3(256), 0, cx->stream, (const double *)a,
                       (const double *)b, (double *)out, count);
    return hipGetLastError();
}

hipError_t launch_project(erf_ctx *cx, void *ru, void *rv, void *rw, double dt)
{
    const Dims &d = cx->d;
    ProjArgs a{};
    a.d = d;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.dt = dt;
    a.dz = cx->base.dz;
    a.ru = (double *)ru;
    a.rv = (double *)rv;
    a.rw = (double *)rw;
    a.Z = cx->an.Z;
    a.cp = cx->an.cp;
    a.phi = cx->an.phi;
    a.pa = cx->an.pa;
    a.twx = cx->an.twx;
    a.twy = cx->an.twy;
    a.lgx = cx->an.lgx;
    a.lgy = cx->an.lgy;
    a.cols = anel_ffty_cols(d.nx, d.ny);
    const int tx = d.nx / 2 < 64 ? 64 : (d.nx / 2 > 256 ? 256 : d.nx / 2);
    const size_t ldsx = 2 * (size_t)d.nx * sizeof(double2), ldsy = 2 * (size_t)d.ny * a.cols * sizeof(double2);
    const int nh = d.nx / 2 + 1;
    const int rows = d.ny * d.nz, ygroups = d.nz * ((nh + a.cols - 1) / a.cols);
    timing_start(cx, K_DIVFFTX);
    hipLaunchKernelGGL(k_div_fftx, dim3(rows), dim3(tx), ldsx, cx->stream, a);
    timing_stop(cx, K_DIVFFTX);
    timing_start(cx, K_FFTY);
    hipLaunchKernelGGL(k_ffty, dim3(ygroups), dim3(256), ldsy, cx->stream, a, 0);
    timing_stop(cx, K_FFTY);
    timing_start(cx, K_POISSON);
    // 64-lane blocks: one column per lane and a few tens of thousands of
    // columns, spread over every compute unit
    hipLaunchKernelGGL(k_poisson_z, dim3((nh * d.ny + 63) / 64), dim3(64), 0, cx->stream, a);
    timing_stop(cx, K_POISSON);
    timing_start(cx, K_FFTY);
    hipLaunchKernelGGL(k_ffty, dim3(ygroups), dim3(256), ldsy, cx->stream, a, 1);
    timing_stop(cx, K_FFTY);
    timing_start(cx, K_IFFTX);
    hipLaunchKernelGGL(k_ifftx, dim3(rows), dim3(tx), ldsx, cx->stream, a);
    timing_stop(cx, K_IFFTX);
    timing_start(cx, K_PROJECT);
    hipLaunchKernelGGL(k_project, dim3((d.n + 255) / 256), dim3(256), 0, cx->stream, a);
    timing_stop(cx, K_PROJECT);
    return hipGetLastError();
}

}  // namespace erfk
