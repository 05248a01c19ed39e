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

// WENO5-JS face value; v2 is the upwind cell, candidate stencils of three cells
// with values p_k, smoothness indicators beta_k and weights d_k / (eps +
// beta_k)^2, d = (0.1, 0.6, 0.3), normalised.  Written over one common
// denominator: the weights are multiplied by the product of the three (eps +
// beta)^2 and the 1/6 of the p_k moves into the final quotient, so a face
// takes one division instead of seven (wdiv); equal to the three-weight form
// up to rounding.  In float the product of two (eps + beta)^2 stays above 1e-24 and
// below 1e30 for the mixing ratios and stencil jumps of the workloads.
template <typename R>
__device__ __forceinline__ R weno5_face(R v0, R v1, R v2, R v3, R v4)
{
    const R eps = R(1.0e-6);
    const R P0 = R(2) * v0 - R(7) * v1 + R(11) * v2;
    const R P1 = -v1 + R(5) * v2 + R(2) * v3;
    const R P2 = R(2) * v2 + R(5) * v3 - v4;
    const R s0 = v0 - R(2) * v1 + v2, t0 = v0 - R(4) * v1 + R(3) * v2;
    const R s1 = v1 - R(2) * v2 + v3, t1 = v1 - v3;
    const R s2 = v2 - R(2) * v3 + v4, t2 = R(3) * v2 - R(4) * v3 + v4;
    const R be0 = R(13.0 / 12.0) * s0 * s0 + R(0.25) * t0 * t0;
    const R be1 = R(13.0 / 12.0) * s1 * s1 + R(0.25) * t1 * t1;
    const R be2 = R(13.0 / 12.0) * s2 * s2 + R(0.25) * t2 * t2;
    const R a0 = (eps + be0) * (eps + be0), a1 = (eps + be1) * (eps + be1), a2 = (eps + be2) * (eps + be2);
    const R w0 = R(0.1) * (a1 * a2), w1 = R(0.6) * (a0 * a2), w2 = R(0.3) * (a0 * a1);
    return wdiv(w0 * P0 + w1 * P1 + w2 * P2, R(6) * (w0 + w1 + w2));
}

// Tiles of kSX x kSY cells per block of (kSX + 1) x (kSY + 1) threads, one
// chunk of up to kLev levels of one scalar, marched upward level by level.
// Per level the block stages the plane of q^t over the tile and a 3-cell halo
// in LDS (periodic wrap resolved once, at the staging), so the horizontal
// stencils read LDS instead of gathering from memory.  Every thread evaluates
// the x- and y-face on the low side of its cell; the last lane and the last
// row of threads hold the cells just past the tile and only lend those faces,
// through LDS, to their neighbours, so each interior face is evaluated once.
// Vertically each owning thread keeps q of its column at k - 3 .. k + 3 in
// registers (one new load per level) and evaluates only the face above its
// cell; the face below is the one it evaluated one level earlier.  kWeno:
// WENO5-JS faces, else the interpolant of the run's order.  kNear: the domain
// is at least 3 cells wide and 3 levels high (selects instead of general
// wraps for the column window).
constexpr int kSX = 63, kSY = 15, kLev = 16;
constexpr int kHX = kSX + 1 + 6, kHY = kSY + 1 + 6;  // staged plane with halo
template <typename T, bool kWeno, bool kNear>
__device__ __forceinline__ void k_scalar_body(ScalArgs<T> a, VBlock vb)
{
    using R = T;  // arithmetic type
    __shared__ R qs[kHY][kHX];
    __shared__ R fxs[kSY + 1][kSX + 1], fys[kSY + 1][kSX + 1];
    const Dims &d = a.d;
    const int lane = threadIdx.x, row = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int nchunk = (nz + kLev - 1) / kLev;
    const int kc = vb.z % nchunk, s = vb.z / nchunk;
    const int k0 = kc * kLev, k1 = min(k0 + kLev, nz);
    const int x0 = vb.x * kSX, y0 = vb.y * kSY;
    // the thread's cell, wrapped periodically (the lending lane and row may lie
    // past the domain's end); threads beyond them only stage and wait
    const int iu = x0 + lane, ju = y0 + row;
    const bool lend = iu <= nx && ju <= ny;
    const bool own = lane < kSX && row < kSY && iu < nx && ju < ny;
    const int i = iu % nx, j = ju % ny;
    const int col = j * nx + i;
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
    for (int k = k0; k < k1; ++k) {
        const int pl = k * P;
#pragma unroll
        for (int u = 0; u < kStage; ++u)
            if (soff[u] >= 0) (&qs[0][0])[tid + u * nthr] = q[pl + soff[u]];
        R rq = 0, Fz1 = 0, qn = 0;
        const size_t o = (size_t)s * d.n + pl + col;
        if (own) {
            // loads of this level issued before the barrier
            rq = a.rqn[o];
            Fz1 = a.Fw[col + pl + P];
            qn = q[col + reflc(k + 3) * P];
        }
        __syncthreads();
        R fx0 = 0, fy0 = 0;
        if (lend) {
            R qx[7], qy[7];
#pragma unroll
            for (int t = 0; t < 7; ++t) {
                qx[t] = qs[row + 3][lane + t];
                qy[t] = qs[row + t][lane + 3];
            }
            const R Fx0 = a.Fu[pl + col], Fy0 = a.Fv[pl + col];
            fx0 = Fx0 * face(qx, 0, sign_of(Fx0), a.oh);
            fy0 = Fy0 * face(qy, 0, sign_of(Fy0), a.oh);
            if (lane <= kSX && row <= kSY) {
                fxs[row][lane] = fx0;
                fys[row][lane] = fy0;
            }
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
                v = v + dts * (R)a.src[pl + col];
                v = v < R(0) ? R(0) : v;
            }
            // read by later launches only (and rqn[o], its only other use, is read above)
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
    const int nchunk = (d.nz + kLev - 1) / kLev;
    dim3 blk(kSX + 1, kSY + 1, 1), grd((d.nx + kSX - 1) / kSX, (d.ny + kSY - 1) / kSY, nchunk * a.nq);
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
