// scalars.hip -- advected scalars after the acoustic substeps (Sec. 3.1):
//   (rho q)^new = (rho q)^n - dts * div(F q^t),  q^t = (rho q)^t / rho^t,
// F the stage-averaged momenta.  Face values of q^t come from the interpolants
// of Sec. 3.6 or from WENO5-JS (Jiang & Shu 1996, cited in Sec. 3.6), upwinded
// by the sign of F.  Stored and computed as T: double, or float for the FP32
// path (the bulk stencil arithmetic of the mixed-precision mode).
#include "erf_internal.h"

namespace erfk {
namespace {

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

template <typename T>
struct ScalArgs {
    Dims d;
    int nq, oh, ov, weno;
    double idx, idy, dts;
    const double *idz, *rho0;
    const T *rqn, *rho_t, *rq_t, *Fu, *Fv, *Fw;
    T *q, *out;
    // the Deardorff closure: the source of rho e (scalar 0), added times dts
    // and the result clipped at zero (null otherwise)
    const T *src;
};

// q^t = (rho q)^t / rho^t; one thread per cell for every scalar (rho read once)
template <typename T>
__device__ __forceinline__ void k_mixing_ratio_body(ScalArgs<T> a, VBlock vb)
{
    const int c = vb.x * blockDim.x + threadIdx.x;
    if (c >= a.d.n) return;
    // full rho^t: stored (FP64) or base + perturbation (FP32 storage), in T
    const T r = kPert<T> ? (T)a.rho0[c / a.d.nxy] + a.rho_t[c] : a.rho_t[c];
    for (int s = 0; s < a.nq; ++s) {
        const size_t o = (size_t)s * a.d.n + c;
        a.q[o] = a.rq_t[o] / r;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_mixing_ratio(ScalArgs<T> a)
{
    k_mixing_ratio_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(256) void k_mixing_ratio_batch(const ScalArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_mixing_ratio_body<T>(args[m], vb);
}

// a / b for the WENO5 weights: the hardware reciprocal (1 ulp) in float, an
// IEEE division in double
template <typename R>
__device__ __forceinline__ R wdiv(R a, R b)
{
    if constexpr (std::is_same<R, float>::value)
        return a * __builtin_amdgcn_rcpf(b);
    else
        return a / b;
}

// a * b + c: one fused operation (one rounding) in float, the product and the
// sum as written (two roundings) in double
template <typename R>
__device__ __forceinline__ R mad(R a, R b, R c)
{
    if constexpr (std::is_same<R, float>::value)
        return __builtin_fmaf(a, b, c);
    else
        return a * b + c;
}

// WENO5-JS face value; v2 is the upwind cell, candidate stencils of three cells
// with values p_k, smoothness indicators beta_k and weights d_k / (eps +
// beta_k)^2, d = (0.1, 0.6, 0.3), normalised.  Written over one common
// denominator: the weights are multiplied by the product of the three (eps +
// beta)^2 and the 1/6 of the p_k moves into the final quotient, so a face
// takes one division instead of seven (wdiv); equal to the three-weight form
// up to rounding.  In float the product of two (eps + beta)^2 stays above 1e-24 and
// below 1e30 for the mixing ratios and stencil jumps of the workloads (times
// 256 with the float form's 4 beta and 4 eps: still below 3e32).
// The sums of products are written as mad chains: fused in float; in double
// the same operations and roundings as the sums written out (an addition's
// operands commute exactly, and x + (-a) b equals x - a b).
template <typename R>
__device__ __forceinline__ R weno5_face(R v0, R v1, R v2, R v3, R v4)
{
    if constexpr (std::is_same<R, float>::value) {
        // float: 4 beta_k = (13/3) s_k^2 + t_k^2 against 4 eps, and the weights
        // without the common factor 0.1: both scale every weight alike, which
        // the normalisation cancels (4 fewer operations per face)
        const float eps4 = 4.0e-6f;
        const float P0 = mad(11.0f, v2, mad(-7.0f, v1, 2.0f * v0));
        const float P1 = mad(2.0f, v3, mad(5.0f, v2, -v1));
        const float P2 = mad(5.0f, v3, 2.0f * v2) - v4;
        const float s0 = mad(-2.0f, v1, v0) + v2, t0 = mad(3.0f, v2, mad(-4.0f, v1, v0));
        const float s1 = mad(-2.0f, v2, v1) + v3, t1 = v1 - v3;
        const float s2 = mad(-2.0f, v3, v2) + v4, t2 = mad(-4.0f, v3, 3.0f * v2) + v4;
        const float b0 = mad(float(13.0 / 3.0) * s0, s0, t0 * t0);
        const float b1 = mad(float(13.0 / 3.0) * s1, s1, t1 * t1);
        const float b2 = mad(float(13.0 / 3.0) * s2, s2, t2 * t2);
        const float a0 = (eps4 + b0) * (eps4 + b0), a1 = (eps4 + b1) * (eps4 + b1), a2 = (eps4 + b2) * (eps4 + b2);
        const float w0 = a1 * a2, w1 = 6.0f * (a0 * a2), w2 = 3.0f * (a0 * a1);
        return wdiv(mad(w2, P2, mad(w1, P1, w0 * P0)), 6.0f * (w0 + w1 + w2));
    }
    const R eps = R(1.0e-6);
    const R P0 = mad(R(11), v2, mad(R(-7), v1, R(2) * v0));  // 2 v0 - 7 v1 + 11 v2
    const R P1 = mad(R(2), v3, mad(R(5), v2, -v1));           // -v1 + 5 v2 + 2 v3
    const R P2 = mad(R(5), v3, R(2) * v2) - v4;               // 2 v2 + 5 v3 - v4
    const R s0 = mad(R(-2), v1, v0) + v2, t0 = mad(R(3), v2, mad(R(-4), v1, v0));
    const R s1 = mad(R(-2), v2, v1) + v3, t1 = v1 - v3;
    const R s2 = mad(R(-2), v3, v2) + v4, t2 = mad(R(-4), v3, R(3) * v2) + v4;
    const R be0 = mad(R(13.0 / 12.0) * s0, s0, R(0.25) * t0 * t0);
    const R be1 = mad(R(13.0 / 12.0) * s1, s1, R(0.25) * t1 * t1);
    const R be2 = mad(R(13.0 / 12.0) * s2, s2, R(0.25) * t2 * t2);
    const R a0 = (eps + be0) * (eps + be0), a1 = (eps + be1) * (eps + be1), a2 = (eps + be2) * (eps + be2);
    const R w0 = R(0.1) * (a1 * a2), w1 = R(0.6) * (a0 * a2), w2 = R(0.3) * (a0 * a1);
    return wdiv(mad(w2, P2, mad(w1, P1, w0 * P0)), R(6) * (w0 + w1 + w2));
}

// Tiles of kSX x kSY cells per block of kSX x (kSY + 1) threads (one
// wavefront per row), one chunk of up to kLev levels of one scalar, marched
// upward level by level.  Per level the block stages the plane of q^t over the
// tile and a 3-cell halo in LDS (periodic wrap resolved once, at the staging),
// so the horizontal stencils read LDS instead of gathering from memory.  The
// threads of the first kSY rows evaluate the x- and y-face on the low side of
// their cells.  The last row evaluates the y-faces just past the tile, and its
// first kSY lanes the x-faces just past the tile, one per row.  The faces go
// through LDS to the cells on both sides, so each face is evaluated once; the
// tiles are 64 cells wide, so grids whose width is a multiple of 64 carry no
// idle columns.
// Vertically each owning thread keeps q of its column at k - 3 .. k + 3 in
// registers (one new load per level) and evaluates only the face above its
// cell; the face below is the one it evaluated one level earlier.  kWeno:
// WENO5-JS faces, else the interpolant of the run's order.  kNear: the domain
// is at least 3 cells wide and 3 levels high (selects instead of general
// wraps for the column window).
constexpr int kSX = 64, kSY = 15, kLev = 16;
constexpr int kHX = kSX + 7, kHY = kSY + 1 + 6;  // staged plane with halo
template <typename T, bool kWeno, bool kNear>
__device__ __forceinline__ void k_scalar_body(ScalArgs<T> a, VBlock vb)
{
    using R = T;  // arithmetic type
    __shared__ R qs[kHY][kHX];
    __shared__ R fxs[kSY][kSX + 1], fys[kSY + 1][kSX];
    const Dims &d = a.d;
    const int lane = threadIdx.x, row = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int nchunk = (nz + kLev - 1) / kLev;
    const int kc = vb.z % nchunk, s = vb.z / nchunk;
    const int k0 = kc * kLev, k1 = min(k0 + kLev, nz);
    const int x0 = vb.x * kSX, y0 = vb.y * kSY;
    // the thread's cell, wrapped periodically (the last row and the cells of a
    // partial tile may lie past the domain's end)
    const int iu = x0 + lane, ju = y0 + row;
    const bool own = row < kSY && iu < nx && ju < ny;
    // the faces it evaluates where a cell of the domain needs them: in the first
    // kSY rows the low x- and y-face of its cell; in the last row the y-face
    // past the tile and, in lane r < kSY, the x-face past the tile in row r
    const bool fx_need = row < kSY ? (iu <= nx && ju < ny) : (lane < kSY && x0 + kSX <= nx && y0 + lane < ny);
    const bool fy_need = iu < nx && ju <= ny;
    const int i = iu % nx, j = ju % ny;
    const int col = j * nx + i;
    // (last row) the cell whose low x-face is the one past the tile in row lane
    const int xe_col = ((y0 + lane) % ny) * nx + (x0 + kSX) % nx;
    const T *q = a.q + (size_t)s * d.n;
    auto reflc = [&](int kk) {
        if constexpr (!kNear) return refl_centre(kk, nz);
        const int r = kk < 0 ? -1 - kk : kk;
        return r >= nz ? 2 * nz - 1 - r : r;
    };
    // face value on the low (oo = 0) or high (oo = 1) side of a point,
    // upwinded by the sign sg of the flux through it
    auto face = [&](const R (&v)[7], int oo, R sg, int order) {
        const R qm3 = v[oo], qm2 = v[oo + 1], qm1 = v[oo + 2], q0 = v[oo + 3], qp1 = v[oo + 4], qp2 = v[oo + 5];
        if constexpr (kWeno) {
            const bool pos = sg >= R(0);
            return weno5_face<R>(pos ? qm3 : qp2, pos ? qm2 : qp1, pos ? qm1 : q0, pos ? q0 : qm1, pos ? qp1 : qm2);
        } else {
            return face_interp<R>(order, qm3, qm2, qm1, q0, qp1, qp2, sg);
        }
    };
    // staging: element e of the (kHY x kHX) plane is cell (x0 - 3 + e % kHX,
    // y0 - 3 + e / kHX), wrapped; the offsets within a plane do not depend on k
    const int nthr = blockDim.x * blockDim.y, tid = row * blockDim.x + lane;
    constexpr int kStage = (kHX * kHY + 1023) / 1024;
    int soff[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int e = tid + u * nthr;
        const int ex = e % kHX, ey = e / kHX;
        soff[u] = e < kHX * kHY ? wrap_idx(y0 - 3 + ey, ny) * nx + wrap_idx(x0 - 3 + ex, nx) : -1;
    }
    const R idx = (R)a.idx, idy = (R)a.idy, dts = (R)a.dts;
    // the column window q(k - 3 .. k + 3) and the face below the current level
    R qz[7];
    R fz_below = 0;
    if (own) {
#pragma unroll
        for (int t = 0; t < 7; ++t) qz[t] = q[col + reflc(k0 + t - 4) * P];  // levels k0 - 4 .. k0 + 2
        // the face below k0 (zero flux through the bottom lid)
        const R Fz0 = a.Fw[col + k0 * P];
        R qb[7];
#pragma unroll
        for (int t = 0; t < 7; ++t) qb[t] = qz[t];
        fz_below = k0 > 0 ? Fz0 * face(qb, 1, sign_of(Fz0), a.ov) : R(0);
    }
    // a level's memory reads (its plane elements, the own column's values and
    // the fluxes of the faces the thread evaluates), issued one level ahead:
    // those of level k+1 are in flight while level k is computed
    R sv[kStage], nrq = 0, nFz1 = 0, nqn = 0, nFx = 0, nFy = 0, nsrc = 0;
    auto load_level = [&](int k) {
        const int pl = k * P;
#pragma unroll
        for (int u = 0; u < kStage; ++u) sv[u] = soff[u] >= 0 ? q[pl + soff[u]] : R(0);
        if (own) {
            nrq = a.rqn[(size_t)s * d.n + pl + col];
            nFz1 = a.Fw[col + pl + P];
            nqn = q[col + reflc(k + 3) * P];
            if (s == 0 && a.src) nsrc = a.src[pl + col];
        }
        if (fx_need) nFx = a.Fu[pl + (row < kSY ? col : xe_col)];
        if (fy_need) nFy = a.Fv[pl + col];
    };
    load_level(k0);
    for (int k = k0; k < k1; ++k) {
        const int pl = k * P;
#pragma unroll
        for (int u = 0; u < kStage; ++u)
            if (soff[u] >= 0) (&qs[0][0])[tid + u * nthr] = sv[u];
        const R rq = nrq, Fz1 = nFz1, qn = nqn, Fx0 = nFx, Fy0 = nFy, srcv = nsrc;
        const size_t o = (size_t)s * d.n + pl + col;
        __syncthreads();
        if (k + 1 < k1) load_level(k + 1);
        R fx0 = 0, fy0 = 0;
        {
            // x: the low face of the cell, or (last row) the face past the tile
            // in row `lane`; y: the low face of the cell (past the tile in the
            // last row)
            const int xr = row < kSY ? row : lane, xl = row < kSY ? lane : kSX;
            if (fx_need) {
                R qx[7];
#pragma unroll
                for (int t = 0; t < 7; ++t) qx[t] = qs[xr + 3][xl + t];
                fx0 = Fx0 * face(qx, 0, sign_of(Fx0), a.oh);
            }
            if (fy_need) {
                R qy[7];
#pragma unroll
                for (int t = 0; t < 7; ++t) qy[t] = qs[row + t][lane + 3];
                fy0 = Fy0 * face(qy, 0, sign_of(Fy0), a.oh);
            }
            if (row < kSY)
                fxs[row][lane] = fx0;
            else if (lane < kSY)
                fxs[lane][kSX] = fx0;
            fys[row][lane] = fy0;
        }
        R fz1 = 0;
        if (own) {
            // the window moves up one level: q(k - 3 .. k + 3)
#pragma unroll
            for (int t = 0; t < 6; ++t) qz[t] = qz[t + 1];
            qz[6] = qn;
            fz1 = k < nz - 1 ? Fz1 * face(qz, 1, sign_of(Fz1), a.ov) : R(0);
        }
        __syncthreads();
        if (own) {
            const R fx1 = fxs[row][lane + 1], fy1 = fys[row + 1][lane];
            const R div = (fx1 - fx0) * idx + (fy1 - fy0) * idy + (fz1 - fz_below) * (R)a.idz[k];
            R v = rq - dts * div;
            if (s == 0 && a.src) {
                v = v + dts * srcv;
                v = v < R(0) ? R(0) : v;
            }
            // read by later launches only (and rqn[o], its only other use, was read before)
            st_stream(a.out + o, (T)v);
        }
        fz_below = fz1;
    }
}
template <typename T, bool kWeno, bool kNear>
__global__ __launch_bounds__(1024) void k_scalar(ScalArgs<T> a)
{
    k_scalar_body<T, kWeno, kNear>(a, hw_block());
}
template <typename T, bool kWeno, bool kNear>
__global__ __launch_bounds__(1024) void k_scalar_batch(const ScalArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_scalar_body<T, kWeno, kNear>(args[m], vb);
}

}  // namespace

namespace {
// Terrain (FP64 contexts, Sec. 3.4 and App. A): one thread per cell and
// scalar; the horizontal fluxes carry h_zeta of their face, Fw is the
// stage-averaged rho Omega, and the divergence is divided by the cell's h_zeta
struct TerScalArgs {
    Dims d;
    int nq, oh, ov, weno;
    double dx, dy, dts;
    const double *dz, *J, *JU, *JV;
    const double *rqn, *Fu, *Fv, *Fw, *q;
    double *out;
};

__device__ __forceinline__ double ter_face(const TerScalArgs &a, double F, double qm3, double qm2, double qm1,
                                           double q0, double qp1, double qp2, int order)
{
    const double sg = sign_of(F);
    if (a.weno) {
        const bool pos = F > 0.0;
        return F * weno5_face<double>(pos ? qm3 : qp2, pos ? qm2 : qp1, pos ? qm1 : q0, pos ? q0 : qm1,
                                      pos ? qp1 : qm2);
    }
    return F * face_interp<double>(order, qm3, qm2, qm1, q0, qp1, qp2, sg);
}

// blocks are tiles of 64 x 4 cells of one level (blockIdx.x over the tiles of
// a level, blockIdx.y the level, blockIdx.z the scalar), so that the rows a
// y-stencil reaches are shared within a block
__global__ __launch_bounds__(256) void k_ter_scalar(TerScalArgs a)
{
    const Dims &d = a.d;
    const int ntx = (d.nx + 63) >> 6;
    const int ty = blockIdx.x / ntx, tx = blockIdx.x - ty * ntx;
    const int i = (tx << 6) + (threadIdx.x & 63), j = (ty << 2) + (threadIdx.x >> 6), k = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int c = (k * d.ny + j) * d.nx + i;
    const int s = blockIdx.z;
    const double *q = a.q + (size_t)s * d.n;
    const auto at = [&](int ii, int jj, int kk) {
        return q[(refl_centre(kk, d.nz) * d.ny + wrap_idx(jj, d.ny)) * d.nx + wrap_idx(ii, d.nx)];
    };
    const auto cc = [&](int ii, int jj) { return (k * d.ny + wrap_idx(jj, d.ny)) * d.nx + wrap_idx(ii, d.nx); };
    double f[6];
    for (int side = 0; side < 2; ++side) {
        const int ci = cc(i + side, j), cj = cc(i, j + side);
        f[side] = ter_face(a, a.Fu[ci], at(i + side - 3, j, k), at(i + side - 2, j, k), at(i + side - 1, j, k),
                           at(i + side, j, k), at(i + side + 1, j, k), at(i + side + 2, j, k), a.oh);
        f[2 + side] = ter_face(a, a.Fv[cj], at(i, j + side - 3, k), at(i, j + side - 2, k), at(i, j + side - 1, k),
                               at(i, j + side, k), at(i, j + side + 1, k), at(i, j + side + 2, k), a.oh);
        const int kf = k + side;
        f[4 + side] = (kf == 0 || kf == d.nz)
                          ? 0.0
                          : ter_face(a, a.Fw[c + side * d.nxy], at(i, j, kf - 3), at(i, j, kf - 2), at(i, j, kf - 1),
                                     at(i, j, kf), at(i, j, kf + 1), at(i, j, kf + 2), a.ov);
    }
    const double div = ((a.JU[cc(i + 1, j)] * f[1] - a.JU[c] * f[0]) / a.dx +
                        (a.JV[cc(i, j + 1)] * f[3] - a.JV[c] * f[2]) / a.dy + (f[5] - f[4]) / a.dz[k]) /
                       a.J[c];
    const size_t o = (size_t)s * d.n + c;
    a.out[o] = a.rqn[o] - a.dts * div;
}

template <typename T>
hipError_t scalar_t(erf_ctx *cx, const void *rqn, const void *rho_t, const void *rq_t, const void *Fu,
                    const void *Fv, const void *Fw, double dts, void *rq_out)
{
    const Dims &d = cx->d;
    ScalArgs<T> a{};
    a.d = d;
    a.nq = cx->prm.n_scalars;
    a.oh = cx->prm.adv_order_h;
    a.ov = cx->prm.adv_order_v;
    a.weno = cx->prm.scalar_scheme == ERF_SCALAR_WENO5;
    a.idx = 1.0 / cx->grid.dx;
    a.idy = 1.0 / cx->grid.dy;
    a.dts = dts;
    a.idz = cx->base.idz();
    a.rho0 = cx->base.rho0;
    a.rqn = (const T *)rqn;
    a.rho_t = (const T *)rho_t;
    a.rq_t = (const T *)rq_t;
    a.Fu = (const T *)Fu;
    a.Fv = (const T *)Fv;
    a.Fw = (const T *)Fw;
    a.q = (T *)cx->ws.q;
    a.out = (T *)rq_out;
    a.src = cx->prm.sgs == ERF_SGS_DEARDORFF ? (const T *)cx->ws.esrc : nullptr;
    if (a.nq <= 0) return hipSuccess;
    timing_start(cx, K_MIXRATIO);
    run<ScalArgs<T>, k_mixing_ratio<T>, k_mixing_ratio_batch<T>>(cx, dim3((d.n + 255) / 256), dim3(256), 0, a);
    timing_stop(cx, K_MIXRATIO);
    if constexpr (std::is_same<T, double>::value) {
        if (cx->ter.on) {
            TerScalArgs t{};
            t.d = d;
            t.nq = a.nq, t.oh = a.oh, t.ov = a.ov, t.weno = a.weno;
            t.dx = cx->grid.dx, t.dy = cx->grid.dy, t.dts = dts;
            t.dz = cx->base.dz, t.J = cx->ter.J, t.JU = cx->ter.JU, t.JV = cx->ter.JV;
            t.rqn = a.rqn, t.Fu = a.Fu, t.Fv = a.Fv, t.Fw = a.Fw, t.q = a.q, t.out = a.out;
            timing_start(cx, K_SCALAR);
            k_ter_scalar<<<dim3(((d.nx + 63) / 64) * ((d.ny + 3) / 4), d.nz, a.nq), 256, 0, cx->stream>>>(t);
            timing_stop(cx, K_SCALAR);
            return hipGetLastError();
        }
    }
    const int nchunk = (d.nz + kLev - 1) / kLev;
    dim3 blk(kSX, kSY + 1, 1), grd((d.nx + kSX - 1) / kSX, (d.ny + kSY - 1) / kSY, nchunk * a.nq);
    const bool near = d.nx >= 3 && d.ny >= 3 && d.nz >= 3;
    timing_start(cx, K_SCALAR);
    if (a.weno && near)
        run<ScalArgs<T>, k_scalar<T, true, true>, k_scalar_batch<T, true, true>>(cx, grd, blk, 0, a);
    else if (a.weno)
        run<ScalArgs<T>, k_scalar<T, true, false>, k_scalar_batch<T, true, false>>(cx, grd, blk, 0, a);
    else if (near)
        run<ScalArgs<T>, k_scalar<T, false, true>, k_scalar_batch<T, false, true>>(cx, grd, blk, 0, a);
    else
        run<ScalArgs<T>, k_scalar<T, false, false>, k_scalar_batch<T, false, false>>(cx, grd, blk, 0, a);
    timing_stop(cx, K_SCALAR);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_scalar_advance(erf_ctx *cx, const void *rqn, const void *rho_t, const void *rq_t,
                                 const void *Fu, const void *Fv, const void *Fw, double dts, void *rq_out)
{
    if (cx->prm.precision == ERF_FP32_MIXED) return scalar_t<float>(cx, rqn, rho_t, rq_t, Fu, Fv, Fw, dts, rq_out);
    return scalar_t<double>(cx, rqn, rho_t, rq_t, Fu, Fv, Fw, dts, rq_out);
}

}  // namespace erfk
