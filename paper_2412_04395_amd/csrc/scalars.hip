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
};

// q^t = (rho q)^t / rho^t; one thread per cell for every scalar (rho read once)
template <typename T>
__global__ __launch_bounds__(256) void k_mixing_ratio(ScalArgs<T> a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.d.n) return;
    // full rho^t: stored (FP64) or base + perturbation (FP32 storage), in T
    const T r = kPert<T> ? (T)a.rho0[c / a.d.nxy] + a.rho_t[c] : a.rho_t[c];
    for (int s = 0; s < a.nq; ++s) {
        const size_t o = (size_t)s * a.d.n + c;
        a.q[o] = a.rq_t[o] / r;
    }
}

// WENO5-JS face value; v2 is the upwind cell, candidate stencils of three cells
// with values p_k, smoothness indicators beta_k and weights d_k / (eps +
// beta_k)^2, d = (0.1, 0.6, 0.3), normalised.  Written over one common
// denominator: the weights are multiplied by the product of the three (eps +
// beta)^2 and the 1/6 of the p_k moves into the final quotient, so a face
// takes one division instead of seven; equal to the three-weight form up to
// rounding.  In float the product of two (eps + beta)^2 stays above 1e-24 and
// below 1e30 for the mixing ratios and stencil jumps of the workloads.
template <typename R>
__device__ __forceinline__ R weno5_face(R v0, R v1, R v2, R v3, R v4)
{
    const R eps = R(1.0e-6);
    const R P0 = R(2) * v0 - R(7) * v1 + R(11) * v2;  // 6 p0
    const R P1 = -v1 + R(5) * v2 + R(2) * v3;         // 6 p1
    const R P2 = R(2) * v2 + R(5) * v3 - v4;          // 6 p2
    const R s0 = v0 - R(2) * v1 + v2, t0 = v0 - R(4) * v1 + R(3) * v2;
    const R s1 = v1 - R(2) * v2 + v3, t1 = v1 - v3;
    const R s2 = v2 - R(2) * v3 + v4, t2 = R(3) * v2 - R(4) * v3 + v4;
    const R be0 = R(13.0 / 12.0) * s0 * s0 + R(0.25) * t0 * t0;
    const R be1 = R(13.0 / 12.0) * s1 * s1 + R(0.25) * t1 * t1;
    const R be2 = R(13.0 / 12.0) * s2 * s2 + R(0.25) * t2 * t2;
    const R a0 = (eps + be0) * (eps + be0), a1 = (eps + be1) * (eps + be1), a2 = (eps + be2) * (eps + be2);
    const R w0 = R(0.1) * (a1 * a2), w1 = R(0.6) * (a0 * a2), w2 = R(0.3) * (a0 * a1);
    return (w0 * P0 + w1 * P1 + w2 * P2) / (R(6) * (w0 + w1 + w2));
}

// Tiles of kSX x kSY cells per block of (kSX + 1) x (kSY + 1) threads, one
// level of one scalar.  Every thread evaluates the x- and y-face on the low
// side of its cell; the last lane and the last row of threads hold the cells
// just past the tile and only lend those faces, through LDS, to their
// neighbours, so each interior face is evaluated once instead of twice.  The
// z-faces (both, per cell) are evaluated by the tile's own cells.  kWeno:
// WENO5-JS faces, else the interpolant of the run's order.  kNear: the domain
// is at least 3 cells wide and 3 levels high, so that the periodic wrap and
// the lid reflection of any stencil offset are selects.  Every load first, the
// lid fluxes masked by a 0/1 product, the upwind candidate stencil picked by
// selects and evaluated once: with a branch between them (or one per sign,
// which diverges) the compiler issues the loads in small dependent groups.
constexpr int kSX = 63, kSY = 15;
template <typename T, bool kWeno, bool kNear>
__global__ __launch_bounds__(1024) void k_scalar(ScalArgs<T> a)
{
    using R = T;  // arithmetic type
    __shared__ R fxs[kSY + 1][kSX + 1], fys[kSY + 1][kSX + 1];
    const Dims &d = a.d;
    const int lane = threadIdx.x, row = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int k = blockIdx.z % nz, s = blockIdx.z / nz;
    // the thread's cell, wrapped periodically (the lending lane and row may lie
    // past the domain's end); threads beyond them have nothing to do but the barrier
    const int iu = blockIdx.x * kSX + lane, ju = blockIdx.y * kSY + row;
    const bool lend = iu <= nx && ju <= ny;
    const bool own = lane < kSX && row < kSY && iu < nx && ju < ny;
    const int i = iu % nx, j = ju % ny;
    const int c = cidx(d, i, j, k);
    const T *q = a.q + (size_t)s * d.n;
    auto wrap = [&](int v, int n) { return kNear ? v + (v < 0 ? n : 0) - (v >= n ? n : 0) : wrap_idx(v, n); };
    auto reflc = [&](int kk) {
        if constexpr (!kNear) return refl_centre(kk, nz);
        const int r = kk < 0 ? -1 - kk : kk;
        return r >= nz ? 2 * nz - 1 - r : r;
    };
    // face value on the low (oo = 0) or high (oo = 1) side of the cell,
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
    // q at offsets -3..3 in x and y (the low faces use -3..2)
    R qx[7], qy[7];
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        qx[t] = q[c + (wrap(i + t - 3, nx) - i)];
        qy[t] = q[c + (wrap(j + t - 3, ny) - j) * nx];
    }
    const R Fx0 = a.Fu[c], Fy0 = a.Fv[c];
    const R fx0 = Fx0 * face(qx, 0, sign_of(Fx0), a.oh), fy0 = Fy0 * face(qy, 0, sign_of(Fy0), a.oh);
    fxs[row][lane] = fx0;
    fys[row][lane] = fy0;
    R fz0 = 0, fz1 = 0, rq = 0;
    const size_t o = (size_t)s * d.n + c;
    if (row < kSY) {  // the tile's rows: their z-faces (the lending row has none to give)
        R qz[7];
#pragma unroll
        for (int t = 0; t < 7; ++t) qz[t] = q[c + (reflc(k + t - 3) - k) * P];
        const R Fz0 = a.Fw[c], Fz1 = a.Fw[c + P];
        const R not_bot = (R)(k > 0), not_top = (R)(k < nz - 1);
        rq = a.rqn[o];
        fz0 = Fz0 * face(qz, 0, sign_of(Fz0), a.ov) * not_bot;
        fz1 = Fz1 * face(qz, 1, sign_of(Fz1), a.ov) * not_top;
    }
    __syncthreads();
    if (!own || !lend) return;
    const R fx1 = fxs[row][lane + 1], fy1 = fys[row + 1][lane];
    const R div = (fx1 - fx0) * (R)a.idx + (fy1 - fy0) * (R)a.idy + (fz1 - fz0) * (R)a.idz[k];
    // read by later launches only (and rqn[o], its only other use, is read above)
    st_stream(a.out + o, (T)(rq - (R)a.dts * div));
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
    if (a.nq <= 0) return hipSuccess;
    timing_start(cx, K_MIXRATIO);
    hipLaunchKernelGGL(k_mixing_ratio<T>, dim3((d.n + 255) / 256), dim3(256), 0, cx->stream, a);
    timing_stop(cx, K_MIXRATIO);
    dim3 blk(kSX + 1, kSY + 1, 1), grd((d.nx + kSX - 1) / kSX, (d.ny + kSY - 1) / kSY, d.nz * a.nq);
    const bool near = d.nx >= 3 && d.ny >= 3 && d.nz >= 3;
    timing_start(cx, K_SCALAR);
    if (a.weno && near)
        hipLaunchKernelGGL((k_scalar<T, true, true>), grd, blk, 0, cx->stream, a);
    else if (a.weno)
        hipLaunchKernelGGL((k_scalar<T, true, false>), grd, blk, 0, cx->stream, a);
    else if (near)
        hipLaunchKernelGGL((k_scalar<T, false, true>), grd, blk, 0, cx->stream, a);
    else
        hipLaunchKernelGGL((k_scalar<T, false, false>), grd, blk, 0, cx->stream, a);
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
