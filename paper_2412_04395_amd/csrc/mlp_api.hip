// mlp_api.hip -- C-ABI of the learned subgrid closure (include/erf_mlp.h):
// closure state allocation, weights, training and data-preparation calls.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/erf_mlp.h"
#include "erf_internal.h"

using namespace erfk;

namespace {

erf_status fail(erf_ctx *c, erf_status s, const char *msg)
{
    c->err = msg;
    if (s == ERF_E_HIP) c->sticky = ERF_E_HIP;
    return s;
}

erf_status hip_fail(erf_ctx *c, hipError_t e, const char *where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return fail(c, ERF_E_HIP, buf);
}

#define CHECK_CTX(c)                                   \
    do {                                               \
        if (!(c)) return ERF_E_ARG;                    \
        if ((c)->sticky != ERF_OK) return (c)->sticky; \
    } while (0)

size_t al(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t al_c(size_t x) { return (x + 255) & ~size_t(255); }

// one allocation for parameters, Adam moments, gradient, packed operands,
// biases, statistics, fallback counter and loss slot
erf_status ensure_state(erf_ctx *c)
{
    MlpState &m = c->mlp;
    if (m.alloc) return ERF_OK;
    const size_t P = kMlpParams * sizeof(float);
    const size_t sizes[] = {P, P, P, P, 22 * 64 * 16, 208 * sizeof(float), kMlpNorm * sizeof(double),
                            closure_count_slots() * sizeof(unsigned long long), sizeof(double),
                            train_weight_shorts() * sizeof(unsigned short)};
    size_t total = 0;
    for (size_t s : sizes) total += al(s);
    hipError_t e = hipMalloc(&m.alloc, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        m.alloc = nullptr;
        return fail(c, ERF_E_NOMEM, "closure state allocation failed");
    }
    char *p = (char *)m.alloc;
    void **dst[] = {(void **)&m.master, (void **)&m.adam_m, (void **)&m.adam_v, (void **)&m.grad, &m.wpk,
                    (void **)&m.bias, (void **)&m.norm, (void **)&m.fallbacks, (void **)&m.loss, (void **)&m.tw};
    for (int i = 0; i < 10; ++i) {
        *dst[i] = p;
        p += al(sizes[i]);
    }
    e = hipMemsetAsync(m.alloc, 0, total, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "clearing the closure state");
    e = mlp_train_prepare();
    if (e != hipSuccess) return hip_fail(c, e, "training kernel attributes");
    double nrm[kMlpNorm];
    for (int i = 0; i < kMlpNorm; ++i) nrm[i] = (i >= kMlpIn && i < 2 * kMlpIn) || i >= 2 * kMlpIn + kMlpOut ? 1.0 : 0.0;
    e = hipMemcpyAsync(m.norm, nrm, sizeof nrm, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "initialising the closure statistics");
    return ERF_OK;
}

erf_status ensure_train(erf_ctx *c, int64_t n)
{
    MlpState &m = c->mlp;
    if (m.talloc && m.cap >= n) return ERF_OK;
    if (m.talloc) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(m.talloc);
        m.talloc = nullptr;
        m.cap = 0;
    }
    const size_t b = al(train_part_floats(n) * sizeof(float)), d = al(train_part_doubles(n) * sizeof(double));
    hipError_t e = hipMalloc(&m.talloc, b + d);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        m.talloc = nullptr;
        return fail(c, ERF_E_NOMEM, "training buffers allocation failed");
    }
    m.tpart = (float *)m.talloc;
    m.tdpart = (double *)((char *)m.talloc + b);
    m.cap = n;
    return ERF_OK;
}

bool state5(const erf_state *S) { return S && S->rho && S->rhotheta && S->rhou && S->rhov && S->rhow; }

// ---------------------------------------------------------------------------
// fixed training scratch of erf_mlp_loss_grad_noalloc
// ---------------------------------------------------------------------------
// Partial sums of the fused training pass (FP32 weight gradients and FP64 bias
// and loss sums per block) for a batch of at most ERF_MLP_NOALLOC_MAX_BATCH
// samples, each region 256-byte aligned: one block per 64 samples up to 256
// blocks (8192 samples: 128 blocks), 9609 floats and 256 doubles each
// (checked against the library's sizing functions at the first call).
constexpr int64_t kNaMax = ERF_MLP_NOALLOC_MAX_BATCH;
constexpr int64_t kNaBlocks = (kNaMax + 63) / 64 < 256 ? (kNaMax + 63) / 64 : 256;
constexpr size_t kNaPart = (size_t)kNaBlocks * 9609 * sizeof(float);
constexpr size_t kNaDbl = (size_t)kNaBlocks * 256 * sizeof(double);
constexpr size_t kNaBytes = al_c(kNaPart) + al_c(kNaDbl);
}  // namespace

// One copy per GPU, held from the library's load until the process ends.  In
// host code `scratch` is a host-side stand-in: its device address comes from
// hipGetSymbolAddress, per device (na_scratch).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex na_mutex;
void *na_ptr[kNaMaxDevices] = {};

// The device address of `scratch` on the context's GPU, looked up once per
// device with that device current.
erf_status na_scratch(erf_ctx *c, char **out)
{
    const int dev = c->device;
    if (dev < 0 || dev >= kNaMaxDevices) return fail(c, ERF_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        if (train_part_floats(kNaMax) * sizeof(float) > kNaPart || train_part_doubles(kNaMax) * sizeof(double) > kNaDbl)
            return fail(c, ERF_E_UNSUPPORTED, "training scratch smaller than the maximum batch needs");
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "locating the training scratch");
        }
        na_ptr[dev] = p;
    }
    *out = (char *)na_ptr[dev];
    return ERF_OK;
}

}  // namespace

extern "C" {

erf_status erf_mlp_set_weights(erf_ctx *c, const float *params, const double *norm)
{
    CHECK_CTX(c);
    if (!params) return fail(c, ERF_E_ARG, "params is NULL");
    if (norm)
        for (int i = 0; i < kMlpNorm; ++i) {
            const bool sd = (i >= kMlpIn && i < 2 * kMlpIn) || i >= 2 * kMlpIn + kMlpOut;
            if (!(norm[i] == norm[i]) || (sd && !(norm[i] > 0.0)))
                return fail(c, ERF_E_ARG, "norm: means must be numbers and deviations positive");
        }
    erf_status s = ensure_state(c);
    if (s != ERF_OK) return s;
    MlpState &m = c->mlp;
    hipError_t e = hipMemcpyAsync(m.master, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && norm)
        e = hipMemcpyAsync(m.norm, norm, kMlpNorm * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m.adam_m, 0, kMlpParams * sizeof(float), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m.adam_v, 0, kMlpParams * sizeof(float), c->stream);
    if (e == hipSuccess) e = mlp_pack(c);
    // the host arrays may be reused by the caller as soon as this returns
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "setting the closure weights");
    m.step = 0;
    m.have_weights = true;
    return ERF_OK;
}

erf_status erf_mlp_get_weights(erf_ctx *c, float *params, double *norm)
{
    CHECK_CTX(c);
    MlpState &m = c->mlp;
    if (!m.have_weights) return fail(c, ERF_E_STATE, "no closure weights set");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && params) e = hipMemcpy(params, m.master, kMlpParams * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && norm) e = hipMemcpy(norm, m.norm, kMlpNorm * sizeof(double), hipMemcpyDeviceToHost);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "reading the closure weights");
}

erf_status erf_mlp_forward(erf_ctx *c, const float *x, int64_t n, float *y)
{
    CHECK_CTX(c);
    if (!c->mlp.have_weights) return fail(c, ERF_E_STATE, "no closure weights set");
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, ERF_E_ARG, "x, y and n >= 0 required");
    if (n == 0) return ERF_OK;
    hipError_t e = launch_mlp_forward(c, x, n, y);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "closure network launch");
}

erf_status erf_mlp_features(erf_ctx *c, const erf_state *S, double *feat)
{
    CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!state5(S) || !feat) return fail(c, ERF_E_ARG, "null pointer");
    // the inputs are gradients along the flat grid's axes
    if (c->ter.on) return fail(c, ERF_E_UNSUPPORTED, "closure inputs are not provided over terrain");
    const void *s5[5] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow};
    hipError_t e = launch_prep(c, s5);
    if (e == hipSuccess) e = launch_features(c, feat);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "closure inputs launch");
}

erf_status erf_box_filter(erf_ctx *c, const erf_state *S, int32_t r, double Cs, double Pr_t, erf_state *coarse,
                          double *targets)
{
    CHECK_CTX(c);
    if (!c->have_base) return fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!state5(S) || !state5(coarse) || !targets) return fail(c, ERF_E_ARG, "null pointer");
    if (c->ter.on) return fail(c, ERF_E_UNSUPPORTED, "the box filter is not provided over terrain");
    if (r < 1 || c->d.nx % r || c->d.ny % r || c->d.nz % r)
        return fail(c, ERF_E_SHAPE, "nx, ny and nz must be multiples of r");
    if (Cs < 0.0 || (Cs > 0.0 && !(Pr_t > 0.0))) return fail(c, ERF_E_ARG, "Cs >= 0 and Pr_t > 0 required");
    const void *s5[5] = {S->rho, S->rhotheta, S->rhou, S->rhov, S->rhow};
    double *c5[5] = {(double *)coarse->rho, (double *)coarse->rhotheta, (double *)coarse->rhou,
                     (double *)coarse->rhov, (double *)coarse->rhow};
    hipError_t e = launch_prep(c, s5);
    if (e == hipSuccess) e = launch_box_filter(c, s5, r, Cs, Pr_t, c5, targets);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "box filter launch");
}

erf_status erf_mlp_fit_norm(erf_ctx *c, const double *feat, const double *targets, int64_t n)
{
    CHECK_CTX(c);
    if (!feat || !targets || n < 1) return fail(c, ERF_E_ARG, "feat, targets and n >= 1 required");
    erf_status s = ensure_state(c);
    if (s != ERF_OK) return s;
    void *part = nullptr;
    hipError_t e = hipMalloc(&part, stat_partials(n) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, ERF_E_NOMEM, "statistics partials allocation failed");
    }
    double *nrm = c->mlp.norm;
    e = launch_col_stats(c, feat, n, kMlpIn, nrm, nrm + kMlpIn, (double *)part);
    if (e == hipSuccess)
        e = launch_col_stats(c, targets, n, kMlpOut, nrm + 2 * kMlpIn, nrm + 2 * kMlpIn + kMlpOut, (double *)part);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    (void)hipFree(part);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "training statistics");
}

erf_status erf_mlp_standardize(erf_ctx *c, const double *feat, const double *targets, int64_t n, float *x, float *t)
{
    CHECK_CTX(c);
    if (n < 0 || (n > 0 && (!feat || !x))) return fail(c, ERF_E_ARG, "feat, x and n >= 0 required");
    erf_status s = ensure_state(c);
    if (s != ERF_OK) return s;
    if (n == 0) return ERF_OK;
    const double *nrm = c->mlp.norm;
    hipError_t e = launch_standardize(c, feat, n, kMlpIn, nrm, nrm + kMlpIn, x);
    if (e == hipSuccess && targets && t)
        e = launch_standardize(c, targets, n, kMlpOut, nrm + 2 * kMlpIn, nrm + 2 * kMlpIn + kMlpOut, t);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "standardisation launch");
}

erf_status erf_mlp_loss_grad(erf_ctx *c, const float *x, const float *t, int64_t n, float *grad, double *loss)
{
    CHECK_CTX(c);
    if (!c->mlp.have_weights) return fail(c, ERF_E_STATE, "no closure weights set");
    if (!x || !t || !grad || n < 1) return fail(c, ERF_E_ARG, "x, t, grad and n >= 1 required");
    if (n > ((int64_t)1 << 31) / 64) return fail(c, ERF_E_ARG, "batch too large");
    erf_status s = ensure_train(c, n);
    if (s != ERF_OK) return s;
    MlpState &m = c->mlp;
    hipError_t e = launch_loss_grad(c, x, t, n, grad, m.loss, m.tpart, m.tdpart);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, c->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && loss) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "closure gradient");
}

erf_status erf_mlp_loss_grad_noalloc(erf_ctx *c, const float *x, const float *t, int64_t n, float *grad,
                                     double *loss_dev)
{
    CHECK_CTX(c);
    if (!c->mlp.have_weights) return fail(c, ERF_E_STATE, "no closure weights set");
    if (!x || !t || !grad || n < 1) return fail(c, ERF_E_ARG, "x, t, grad and n >= 1 required");
    if (n > kNaMax) return fail(c, ERF_E_ARG, "batch larger than ERF_MLP_NOALLOC_MAX_BATCH");
    char *p = nullptr;
    erf_status s = na_scratch(c, &p);
    if (s != ERF_OK) return s;
    // the same kernels as erf_mlp_loss_grad (the same blocks for the same n)
    // on slices of the fixed scratch; nothing in it has to start at zero
    // (every partial is written before it is read)
    float *part = (float *)p;
    double *dpart = (double *)(p + al_c(kNaPart));
    hipError_t e = launch_loss_grad(c, x, t, n, grad, loss_dev ? loss_dev : c->mlp.loss, part, dpart);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "closure gradient (fixed scratch)");
}

erf_status erf_mlp_train_step(erf_ctx *c, const float *x, const float *t, int64_t n, double lr, double *loss)
{
    CHECK_CTX(c);
    if (!(lr > 0.0)) return fail(c, ERF_E_ARG, "lr > 0 required");
    erf_status s = erf_mlp_loss_grad(c, x, t, n, c->mlp.grad, nullptr);
    if (s != ERF_OK) return s;
    hipError_t e = launch_adam(c, lr, ++c->mlp.step);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, c->mlp.loss, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && loss) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? ERF_OK : hip_fail(c, e, "closure training step");
}

erf_status erf_mlp_fallback_count(erf_ctx *c, int64_t *count)
{
    CHECK_CTX(c);
    if (!count) return fail(c, ERF_E_ARG, "count is NULL");
    if (!c->mlp.alloc) {
        *count = 0;
        return ERF_OK;
    }
    std::vector<unsigned long long> v(closure_count_slots());
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(v.data(), c->mlp.fallbacks, v.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "reading the fallback count");
    unsigned long long sum = 0;
    for (unsigned long long x : v) sum += x;
    *count = (int64_t)sum;
    return ERF_OK;
}

}  // extern "C"
