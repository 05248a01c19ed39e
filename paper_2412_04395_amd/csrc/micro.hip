// micro.hip -- Kessler warm-rain microphysics (Sec. 2.4: the scheme of Kessler
// 1969 in the form of Klemp & Wilhelmson 1978) applied after a dynamics step,
// on rho q_v, rho q_c, rho q_r (scalars 0, 1, 2 of a moist context) and rho
// theta (latent heat).  Per step and column: sedimentation of rain (flux form,
// upwind from above, sub-stepped at a fall Courant number of at most 0.8; the
// flux through the ground accumulates as precipitation), then per cell
// autoconversion and accretion, evaporation of rain into subsaturated air, and
// the saturation adjustment of cloud water (Newton on q_v - d = q_vs(T + L d /
// c_p, p), six steps from d = 0, clamped to [-q_c, q_v]), all at the pressure
// of the step's start.  Constants: L = 2.5e6 J/kg; saturation pressure of
// Bolton (1980); autoconversion 1e-3 1/s above 1e-3 kg/kg; accretion 2.2 q_c
// q_r^0.875 1/s; rain evaporation and fall speed in the Klemp-Wilhelmson form
// (densities in g/cm^3, pressure in hPa).
//
// One thread per column (the sedimentation is a column recurrence); the work
// is a few transcendental functions per cell, done in FP64 for both storages
// (the FP32 path stores rho and rho theta as perturbations; increments are
// added to what is stored, so a cell where nothing happens keeps its values).
#include "erf_internal.h"

namespace erfk {
namespace {

constexpr double kLv = 2.5e6;

template <typename T>
struct MicroArgs {
    Dims d;
    double dt;
    const double *dz, *rho0, *Theta0;
    T *rho, *rt, *rq;
    double *precip;  // [ny][nx] accumulated rain at the ground [kg/m^2] (may be null)
};

__device__ __forceinline__ double esat(double T) { return 611.2 * exp(17.67 * (T - 273.15) / (T - 29.65)); }
__device__ __forceinline__ double qvsat(double T, double p)
{
    const double e = esat(T);
    return (kRd / kRv) * e / (p - e);
}
// d q_vs / dT at fixed pressure
__device__ __forceinline__ double dqvsat(double T, double p)
{
    const double e = esat(T);
    const double dlne = 17.67 * (273.15 - 29.65) / ((T - 29.65) * (T - 29.65));
    return (kRd / kRv) * p * e * dlne / ((p - e) * (p - e));
}
__device__ __forceinline__ double fall_speed(double rho, double rqr, double rho_s)
{
    const double g = 1e-3 * rqr;  // rho q_r in g/cm^3
    return g > 0.0 ? 36.34 * pow(g, 0.1364) * sqrt(rho_s / rho) : 0.0;
}

template <typename T>
__device__ __forceinline__ void k_kessler_body(MicroArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    const int col = vb.x * blockDim.x + threadIdx.x;
    if (col >= d.nxy) return;
    const int P = d.nxy, nz = d.nz, n = d.n;
    const double rho_s = a.rho0[0];  // the fall speed's reference density (lowest level)
    T *rqv = a.rq, *rqc = a.rq + n, *rqr = a.rq + 2 * n;
    auto rho_at = [&](int k) { return full_of(a.rho, col + k * P, a.rho0[k]); };
    // 1. sedimentation of rain
    double cmax = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double v = fall_speed(rho_at(k), (double)rqr[col + k * P], rho_s);
        cmax = fmax(cmax, v * a.dt / a.dz[k]);
    }
    int nsub = (int)ceil(cmax / 0.8);
    if (nsub < 1) nsub = 1;
    const double dts = a.dt / nsub;
    for (int s = 0; s < nsub; ++s) {
        // the flux leaving cell k downward is (rho q_r)_k V_k; k ascends, so
        // the cell above still holds its value from the start of the sub-step
        double m = rqr[col], fout = m * fall_speed(rho_at(0), m, rho_s);
        const double out0 = fout;
        for (int k = 0; k < nz; ++k) {
            const int c = col + k * P;
            double fin = 0.0, mu = 0.0;
            if (k + 1 < nz) {
                mu = rqr[c + P];
                fin = mu * fall_speed(rho_at(k + 1), mu, rho_s);
            }
            rqr[c] = (T)(m + dts * (fin - fout) / a.dz[k]);
            m = mu;
            fout = fin;
        }
        if (a.precip) a.precip[col] += dts * out0;
    }
    // 2-4. the cell processes
    for (int k = 0; k < nz; ++k) {
        const int c = col + k * P;
        const double rho = rho_at(k), Th = full_of(a.rt, c, a.Theta0[k]);
        const double qv = (double)rqv[c] / rho, qc0 = (double)rqc[c] / rho, qr0 = (double)rqr[c] / rho;
        const double pi = pow(kRd * (Th * (1.0 + kEpsV * qv)) / kP00, kGamma - 1.0);
        const double p = kP00 * pow(pi, kCp / kRd);
        double Tk = (Th / rho) * pi;
        // autoconversion and accretion
        const double au = qc0 > 1e-3 ? 1e-3 * (qc0 - 1e-3) : 0.0;
        const double ac = qr0 > 0.0 ? 2.2 * qc0 * pow(qr0, 0.875) : 0.0;
        double prod = a.dt * (au + ac);
        if (prod > qc0) prod = qc0;
        const double qc = qc0 - prod, qr = qr0 + prod;
        // evaporation of rain into subsaturated air
        double qvn = qv, ev = 0.0;
        const double qvs = qvsat(Tk, p);
        if (qr > 0.0 && qv < qvs) {
            const double rg = 1e-3 * rho, rqg = rg * qr;
            const double cv = 1.6 + 124.9 * pow(rqg, 0.2046);
            const double er = (1.0 - qv / qvs) * cv * pow(rqg, 0.525) / (rg * (5.4e5 + 2.55e6 / (1e-2 * p * qvs)));
            ev = a.dt * er;
            if (ev > qr) ev = qr;
            if (ev > qvs - qv) ev = qvs - qv;
            qvn = qv + ev;
            Tk -= kLv * ev / kCp;
        }
        // saturation adjustment of cloud water
        double dd = 0.0;
        if (!(qc <= 0.0 && qvn <= qvsat(Tk, p))) {
            for (int it = 0; it < 6; ++it) {
                const double Tn = Tk + kLv * dd / kCp;
                const double f = qvn - dd - qvsat(Tn, p);
                const double df = -1.0 - dqvsat(Tn, p) * kLv / kCp;
                dd = dd - f / df;
            }
            if (dd < -qc) dd = -qc;
            if (dd > qvn) dd = qvn;
        }
        // increments of the three processes
        rqv[c] = (T)((double)rqv[c] + rho * (ev - dd));
        rqc[c] = (T)((double)rqc[c] + rho * (dd - prod));
        rqr[c] = (T)((double)rqr[c] + rho * (prod - ev));
        a.rt[c] = (T)((double)a.rt[c] + rho * kLv * (dd - ev) / (kCp * pi));
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_kessler(MicroArgs<T> a)
{
    k_kessler_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(64) void k_kessler_batch(const MicroArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_kessler_body<T>(args[m], vb);
}

template <typename T>
hipError_t kessler_t(erf_ctx *cx, void *rho, void *rt, void *rq, double dt, double *precip)
{
    MicroArgs<T> a{};
    a.d = cx->d;
    a.dt = dt;
    a.dz = cx->base.dz;
    a.rho0 = cx->base.rho0;
    a.Theta0 = cx->base.Theta0;
    a.rho = (T *)rho;
    a.rt = (T *)rt;
    a.rq = (T *)rq;
    a.precip = precip;
    // 64-thread blocks: columns are few (nx ny), so more, smaller blocks
    // spread them over the compute units
    timing_start(cx, K_KESSLER);
    run<MicroArgs<T>, k_kessler<T>, k_kessler_batch<T>>(cx, dim3((cx->d.nxy + 63) / 64), dim3(64), 0, a);
    timing_stop(cx, K_KESSLER);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_kessler(erf_ctx *cx, void *rho, void *rt, void *rq, double dt, double *precip)
{
    if (cx->prm.precision == ERF_FP32_MIXED) return kessler_t<float>(cx, rho, rt, rq, dt, precip);
    return kessler_t<double>(cx, rho, rt, rq, dt, precip);
}

}  // namespace erfk
