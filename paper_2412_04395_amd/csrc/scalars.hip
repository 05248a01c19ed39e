// scalars.hip -- advected scalars after the acoustic substeps (Sec. 3.1):
//   (rho q)^new = (rho q)^n - dts * div(F q^t),  q^t = (rho q)^t / rho^t,
// F the stage-averaged momenta.  Face values of q^t come from the interpolants
// of Sec. 3.6 or from WENO5-JS (Jiang & Shu 1996, cited in Sec. 3.6), upwinded
// by the sign of F.  Stored as T (double or float); arithmetic in double.
#include "erf_internal.h"

namespace erfk {
namespace {

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

template <typename T>
struct ScalArgs {
    Dims d;
    int nq, oh, ov, weno;
    double dx, dy, dts;
    const double *dz, *rho0;
    const T *rqn, *rho_t, *rq_t, *Fu, *Fv, *Fw;
    T *q, *out;
};

template <typename T>
__global__ __launch_bounds__(256) void k_mixing_ratio(ScalArgs<T> a)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int total = a.nq * a.d.n;
    if (c >= total) return;
    const int cc = c % a.d.n;
    a.q[c] = (double)a.rq_t[c] / full_of(a.rho_t, cc, a.rho0[cc / a.d.nxy]);
}

// WENO5-JS face value; v2 is the upwind cell, candidate stencils of three cells
__device__ __forceinline__ double weno5_face(double v0, double v1, double v2, double v3, double v4)
{
    const double eps = 1.0e-6;
    double p0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) / 6.0;
    double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) / 6.0;
    double p2 = (2.0 * v2 + 5.0 * v3 - v4) / 6.0;
    double s0 = v0 - 2.0 * v1 + v2, t0 = v0 - 4.0 * v1 + 3.0 * v2;
    double s1 = v1 - 2.0 * v2 + v3, t1 = v1 - v3;
    double s2 = v2 - 2.0 * v3 + v4, t2 = 3.0 * v2 - 4.0 * v3 + v4;
    double be0 = 13.0 / 12.0 * s0 * s0 + 0.25 * t0 * t0;
    double be1 = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;
    double be2 = 13.0 / 12.0 * s2 * s2 + 0.25 * t2 * t2;
    double w0 = 0.1 / ((eps + be0) * (eps + be0));
    double w1 = 0.6 / ((eps + be1) * (eps + be1));
    double w2 = 0.3 / ((eps + be2) * (eps + be2));
    return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

template <typename T>
__device__ __forceinline__ double face_value(const ScalArgs<T> &a, int order, double qm3, double qm2, double qm1,
                                             double q0, double qp1, double qp2, double s)
{
    if (a.weno) {
        return s >= 0.0 ? weno5_face(qm3, qm2, qm1, q0, qp1) : weno5_face(qp2, qp1, q0, qm1, qm2);
    }
    return face_interp(order, qm3, qm2, qm1, q0, qp1, qp2, s);
}

template <typename T>
__global__ __launch_bounds__(256) void k_scalar(ScalArgs<T> a)
{
    const Dims &d = a.d;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int kq = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const int k = kq % d.nz, s = kq / d.nz;
    const int c = cidx(d, i, j, k);
    const T *q = a.q + (size_t)s * d.n;
    auto qx = [&](int ii) { return (double)q[cidx(d, wrap_idx(ii, d.nx), j, k)]; };
    auto qy = [&](int jj) { return (double)q[cidx(d, i, wrap_idx(jj, d.ny), k)]; };
    auto qz = [&](int kk) { return (double)q[cidx(d, i, j, refl_centre(kk, d.nz))]; };
    double Fx0 = a.Fu[c], Fx1 = a.Fu[cidx(d, wrap_idx(i + 1, d.nx), j, k)];
    double Fy0 = a.Fv[c], Fy1 = a.Fv[cidx(d, i, wrap_idx(j + 1, d.ny), k)];
    double Fz0 = a.Fw[c], Fz1 = a.Fw[c + d.nxy];
    double fx0 = Fx0 * face_value(a, a.oh, qx(i - 3), qx(i - 2), qx(i - 1), qx(i), qx(i + 1), qx(i + 2), sign_of(Fx0));
    double fx1 = Fx1 * face_value(a, a.oh, qx(i - 2), qx(i - 1), qx(i), qx(i + 1), qx(i + 2), qx(i + 3), sign_of(Fx1));
    double fy0 = Fy0 * face_value(a, a.oh, qy(j - 3), qy(j - 2), qy(j - 1), qy(j), qy(j + 1), qy(j + 2), sign_of(Fy0));
    double fy1 = Fy1 * face_value(a, a.oh, qy(j - 2), qy(j - 1), qy(j), qy(j + 1), qy(j + 2), qy(j + 3), sign_of(Fy1));
    double fz0 = (k == 0) ? 0.0
                          : Fz0 * face_value(a, a.ov, qz(k - 3), qz(k - 2), qz(k - 1), qz(k), qz(k + 1), qz(k + 2), sign_of(Fz0));
    double fz1 = (k == d.nz - 1) ? 0.0
                                 : Fz1 * face_value(a, a.ov, qz(k - 2), qz(k - 1), qz(k), qz(k + 1), qz(k + 2), qz(k + 3), sign_of(Fz1));
    double div = (fx1 - fx0) / a.dx + (fy1 - fy0) / a.dy + (fz1 - fz0) / a.dz[k];
    size_t o = (size_t)s * d.n + c;
    a.out[o] = (double)a.rqn[o] - a.dts * div;
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
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.dts = dts;
    a.dz = cx->base.dz;
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
    int total = a.nq * d.n;
    timing_start(cx, K_MIXRATIO);
    hipLaunchKernelGGL(k_mixing_ratio<T>, dim3((total + 255) / 256), dim3(256), 0, cx->stream, a);
    timing_stop(cx, K_MIXRATIO);
    dim3 blk(64, 4, 1), grd((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz * a.nq);
    timing_start(cx, K_SCALAR); hipLaunchKernelGGL(k_scalar<T>, grd, blk, 0, cx->stream, a); timing_stop(cx, K_SCALAR);
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
