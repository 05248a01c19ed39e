// erf_internal.h -- shared declarations of the liberf.so translation units.
//
// Device-side conventions: fields are SoA, x fastest, no halo; periodic wrap in
// x and y and the reflection ghosts at the lids are resolved by index
// arithmetic inside the kernels.  Kernels take a Dims by value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/erf.h"

namespace erfk {

// Dry-air constants.  The paper prints P00 and gamma = c_p / (c_p - R_d)
// (Sec. 2.1); R_d and c_p are the usual dry-air values.
constexpr double kRd = 287.0;
constexpr double kCp = 1004.5;
constexpr double kCv = kCp - kRd;
constexpr double kGamma = kCp / (kCp - kRd);
constexpr double kP00 = 1.0e5;

struct Dims {
    int nx, ny, nz;
    int nxy;  // nx * ny, one horizontal plane
    int n;    // cells
    int nw;   // z-face values, nxy * (nz + 1)
};

// ---------------------------------------------------------------------------
// index helpers (device)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_idx(int i, int n)
{
    if (i < 0) {
        i += n;
        if (i < 0) i = ((i % n) + n) % n;
    } else if (i >= n) {
        i -= n;
        if (i >= n) i %= n;
    }
    return i;
}

// even reflection of a centre index about the lids (k = -1 -> 0, nz -> nz-1)
__device__ __forceinline__ int refl_centre(int k, int nz)
{
    if (k >= 0 && k < nz) return k;
    int p = 2 * nz;
    k = ((k % p) + p) % p;
    return k >= nz ? p - 1 - k : k;
}

// odd reflection of a z-face index: returns the face index in [0, nz] and the
// sign to apply (w_{-m} = -w_m, w_{nz+m} = -w_{nz-m})
__device__ __forceinline__ int refl_face(int k, int nz, double &sgn)
{
    sgn = 1.0;
    if (k >= 0 && k <= nz) return k;
    int p = 2 * nz;
    k = ((k % p) + p) % p;
    if (k > nz) {
        sgn = -1.0;
        k = p - k;
    }
    return k;
}

__device__ __forceinline__ double sign_of(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Interpolated face value q_{m-1/2} (Sec. 3.6) from q[0..5] = q_{m-3..m+2};
// s is the sign of the normal momentum at the face.
__device__ __forceinline__ double face_interp(int order, double qm3, double qm2, double qm1,
                                              double q0, double qp1, double qp2, double s)
{
    if (order == 2) return 0.5 * (q0 + qm1);
    if (order == 3 || order == 4) {
        double c4 = 7.0 / 12.0 * (q0 + qm1) - 1.0 / 12.0 * (qp1 + qm2);
        if (order == 4) return c4;
        return c4 + s / 12.0 * ((qp1 - qm2) - 3.0 * (q0 - qm1));
    }
    double c6 = 37.0 / 60.0 * (q0 + qm1) - 2.0 / 15.0 * (qp1 + qm2) + 1.0 / 60.0 * (qp2 + qm3);
    if (order == 6) return c6;
    return c6 - s / 60.0 * ((qp2 - qm3) - 5.0 * (qp1 - qm2) + 10.0 * (q0 - qm1));
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Workspace {
    // stage states S*, S** (5 fields + scalars each)
    double *sa[6] = {};
    double *sb[6] = {};
    // slow tendencies
    double *R[5] = {};
    // stage-frozen fields at centres: theta, p', pi, velocities, mu_t
    double *th = nullptr, *pp = nullptr, *pit = nullptr;
    double *u = nullptr, *v = nullptr, *w = nullptr, *mut = nullptr;
    // stresses tau_11, tau_22, tau_33 (centres), tau_12 (xy-edges), tau_13,
    // tau_23 (z-face edges) and the heat diffusivity (centres)
    double *tau[6] = {};
    double *kap = nullptr;
    // substep perturbations: Theta'' (three time levels), rho'', U'' and V''
    // (double-buffered), W''
    double *t2[3] = {};
    double *u2[2] = {}, *v2[2] = {};
    double *r2 = nullptr, *w2 = nullptr;
    // running sums of the substep momenta (stage-averaged fluxes at the end)
    double *su = nullptr, *sv = nullptr, *sw = nullptr;
    // per-stage tridiagonal coefficients on z-faces
    double *ca = nullptr, *cb = nullptr, *cc = nullptr;  // a_k / den_k, 1 / den_k, c'_k (Thomas)
    double *cC = nullptr;                                // buoyancy coefficient of the W'' rows
    // mixing ratios q^t of the scalars, stage-averaged momenta of rk3_step
    double *q = nullptr;
    double *fu = nullptr, *fv = nullptr, *fw = nullptr;
    // diagnostics partial sums
    double *diag = nullptr;
};

struct Base {
    double *rho0 = nullptr, *theta0 = nullptr, *Theta0 = nullptr, *p0 = nullptr, *pi0 = nullptr;
    // device: dz [nz], centre heights [nz], 1/dz [nz] and the reciprocal
    // centre-to-centre distances across the z-faces, 2/(dz_{k-1} + dz_k) [nz + 1]
    // (zero on the lids), in one buffer
    double *dz = nullptr;
    const double *zc() const { return dz + nz; }
    const double *idz() const { return dz + 2 * nz; }
    const double *idzf() const { return dz + 3 * nz; }
    int nz = 0;
};

}  // namespace erfk

struct erf_ctx {
    erf_grid grid{};
    erf_params prm{};
    erfk::Dims d{};
    hipStream_t stream = nullptr;
    double *dz_host = nullptr;
    erfk::Base base;
    erfk::Workspace ws;
    bool have_base = false;
    erf_status sticky = ERF_OK;
    std::string err;
    int64_t ws_bytes = 0;
    int device = 0;
    void *arena = nullptr;  // the single device allocation behind the workspace
    // kernel timing (erf_timing_begin / erf_timing_end)
    int timed_kernel = -1;
    int timed_count = 0;
    std::vector<hipEvent_t> timing_events;  // start, stop pairs
};

namespace erfk {

// kernel ids for the timing instrumentation
enum KernelId { K_PREP, K_MUT, K_STRESS, K_RHS, K_STAGE_INIT, K_COEF, K_SUBSTEP, K_FINALIZE, K_MIXRATIO, K_SCALAR, K_COUNT };
inline const char *kernel_name(int id)
{
    static const char *names[K_COUNT] = {"prep", "mut", "stress", "rhs", "stage_init", "coef", "substep",
                                         "finalize", "mixing_ratio", "scalar"};
    return (id >= 0 && id < K_COUNT) ? names[id] : "";
}
// bracket a launch with events when its kernel is being timed
inline void timing_start(erf_ctx *c, int id)
{
    if (c->timed_kernel == id && 2 * c->timed_count + 1 < (int)c->timing_events.size())
        (void)hipEventRecord(c->timing_events[2 * c->timed_count], c->stream);
}
inline void timing_stop(erf_ctx *c, int id)
{
    if (c->timed_kernel == id && 2 * c->timed_count + 1 < (int)c->timing_events.size()) {
        (void)hipEventRecord(c->timing_events[2 * c->timed_count + 1], c->stream);
        ++c->timed_count;
    }
}

// ---------------------------------------------------------------------------
// launchers (host), one translation unit each
// ---------------------------------------------------------------------------
// rhs.hip
hipError_t launch_slow_rhs(erf_ctx *c, const double *rho, const double *rt, const double *ru,
                           const double *rv, const double *rw, double *Rr, double *Rt, double *Ru,
                           double *Rv, double *Rw);
// acoustic.hip
hipError_t launch_acoustic_stage(erf_ctx *c, const double *const Sn[5], const double *const St[5],
                                 const double *const Rt[5], int n_sub, double dtau,
                                 double *const Sout[5], double *Fu, double *Fv, double *Fw);
// scalars.hip
hipError_t launch_scalar_advance(erf_ctx *c, const double *rqn, const double *rho_t,
                                 const double *rq_t, const double *Fu, const double *Fv,
                                 const double *Fw, double dts, double *rq_out);
// diag.hip
size_t diag_slots_needed();
hipError_t launch_diagnostics(erf_ctx *c, const double *rho, const double *rt, const double *ru,
                              const double *rv, const double *rw, const double *rq, double *host_out);

}  // namespace erfk
