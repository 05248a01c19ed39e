// mlp.hip -- learned subgrid closure: a 10 -> 64 -> 64 -> 64 -> 9 ReLU network
// that maps the resolved velocity-gradient tensor and dtheta/dz at a cell
// centre to the kinematic subgrid stresses tau_ij and heat fluxes q_j, used in
// place of the Smagorinsky stresses of Sec. 2.3 (the paper names learned
// surrogates only as future work, Sec. 6).
//
// Matrix products run on the CDNA matrix cores: v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation).  The network is evaluated in the
// transposed form H^T = W^T X^T: hidden units are the MFMA rows, cells the
// columns, so a layer's FP32 result (lane l: cell l%16, units 4*(l/16)+r of
// each 16-unit tile) is already in the place of the next layer's B operand,
// with the K index permuted: K-step s, lane group g, slot i stands for input
// unit 32s + 4g + i (i < 4) or 32s + 16 + 4g + i - 4 (i >= 4).  The weights are
// packed once into A operands with the same permutation, so no value crosses
// lanes between layers.
//
// Everything around the products (closure inputs, de-standardisation, the
// Smagorinsky fallback, the stress divergence) is FP64, like the rest of the
// slow right-hand side.
#include <cmath>

#include "erf_internal.h"

namespace erfk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two floats -> packed bfloat16, round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned int pack2(float a, float b)
{
    bf16x2 v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(unsigned int, v);
}
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// order this wave's LDS writes before its later LDS reads (the rows a wave
// exchanges through LDS belong to that wave alone)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// K-step operand from two 16-unit tiles: ReLU, then BF16
__device__ __forceinline__ bf16x8 relu_pack(floatx4 lo, floatx4 hi)
{
    u32x4 v;
    v.x = pack2(fmaxf(lo[0], 0.f), fmaxf(lo[1], 0.f));
    v.y = pack2(fmaxf(lo[2], 0.f), fmaxf(lo[3], 0.f));
    v.z = pack2(fmaxf(hi[0], 0.f), fmaxf(hi[1], 0.f));
    v.w = pack2(fmaxf(hi[2], 0.f), fmaxf(hi[3], 0.f));
    return as_bf16x8(v);
}

// the input unit that K-step s, lane group g, slot i of a hidden layer stands for
__device__ __forceinline__ int perm_unit(int s, int g, int i) { return 32 * s + (i < 4 ? 4 * g + i : 16 + 4 * g + i - 4); }

// ---------------------------------------------------------------------------
// weight packing: master FP32 parameters -> 22 A operands x 64 lanes (BF16)
// ---------------------------------------------------------------------------
// operands 0..3: layer 1 tiles; 4..11: layer 2 (tile t, K-step s at 4 + 2t + s);
// 12..19: layer 3; 20..21: layer 4 (K-steps 0, 1).  Biases: float[208] =
// b1, b2, b3, b4 padded to 16.
__global__ __launch_bounds__(64) void k_mlp_pack(const float *__restrict__ P, u32x4 *__restrict__ wpk,
                                                 float *__restrict__ bias)
{
    const int o = blockIdx.x, l = threadIdx.x, g = l >> 4, r = l & 15;
    float v[8];
    for (int i = 0; i < 8; ++i) {
        float x = 0.f;
        if (o < 4) {
            const int f = 8 * g + i, unit = 16 * o + r;
            x = f < kMlpIn ? P[kMlpW1 + f * kMlpH + unit] : 0.f;
        } else if (o < 20) {
            const int base = o < 12 ? kMlpW2 : kMlpW3, q = (o - 4) & 7, t = q >> 1, s = q & 1;
            x = P[base + perm_unit(s, g, i) * kMlpH + 16 * t + r];
        } else {
            const int s = o - 20;
            x = r < kMlpOut ? P[kMlpW4 + perm_unit(s, g, i) * kMlpOut + r] : 0.f;
        }
        v[i] = x;
    }
    u32x4 w;
    w.x = pack2(v[0], v[1]);
    w.y = pack2(v[2], v[3]);
    w.z = pack2(v[4], v[5]);
    w.w = pack2(v[6], v[7]);
    wpk[o * 64 + l] = w;
    if (o == 0) {
        for (int u = l; u < 208; u += 64) {
            float b;
            if (u < 64) b = P[kMlpB1 + u];
            else if (u < 128) b = P[kMlpB2 + u - 64];
            else if (u < 192) b = P[kMlpB3 + u - 128];
            else b = (u - 192) < kMlpOut ? P[kMlpB4 + u - 192] : 0.f;
            bias[u] = b;
        }
    }
}

// ---------------------------------------------------------------------------
// the network on 64 samples of one wave
// ---------------------------------------------------------------------------
// xs: 64 rows of 16 BF16 inputs (10 used) as two u32x4 each; ys: 64 rows of 12
// floats (9 used).  The 22 packed operands and the biases sit in LDS, shared by
// the block's wavefronts (registers stay free for more wavefronts per SIMD).
struct WaveWeights {
    const u32x4 *w;  // LDS, [22][64]
    int lane;
    __device__ __forceinline__ bf16x8 operator[](int o) const { return as_bf16x8(w[o * 64 + lane]); }
};

// the block copies the packed operands and biases into LDS
__device__ __forceinline__ void stage_weights(u32x4 *wl, float *bias, const u32x4 *__restrict__ wpk,
                                              const float *__restrict__ biasg)
{
    for (int u = threadIdx.x; u < 22 * 64; u += blockDim.x) wl[u] = wpk[u];
    for (int u = threadIdx.x; u < 208; u += blockDim.x) bias[u] = biasg[u];
}

__device__ __forceinline__ floatx4 bias4(const float *b, int g)
{
    floatx4 c;
    c[0] = b[4 * g];
    c[1] = b[4 * g + 1];
    c[2] = b[4 * g + 2];
    c[3] = b[4 * g + 3];
    return c;
}

__device__ __forceinline__ floatx4 mlp16(const WaveWeights &W, const float *bias, bf16x8 x, int g)
{
    floatx4 h[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h[t] = mfma(W[t], x, bias4(bias + 16 * t, g));
    bf16x8 b0 = relu_pack(h[0], h[1]), b1 = relu_pack(h[2], h[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) h[t] = mfma(W[5 + 2 * t], b1, mfma(W[4 + 2 * t], b0, bias4(bias + 64 + 16 * t, g)));
    b0 = relu_pack(h[0], h[1]);
    b1 = relu_pack(h[2], h[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        h[t] = mfma(W[13 + 2 * t], b1, mfma(W[12 + 2 * t], b0, bias4(bias + 128 + 16 * t, g)));
    b0 = relu_pack(h[0], h[1]);
    b1 = relu_pack(h[2], h[3]);
    return mfma(W[21], b1, mfma(W[20], b0, bias4(bias + 192, g)));
}

// Two 16-sample groups at once: every weight operand read from LDS serves
// both groups' products (half the LDS weight traffic of one group at a time),
// and the two groups' products are independent, so they fill each other's
// pipeline gaps.  Each group's arithmetic is exactly mlp16's.
__device__ __forceinline__ void mlp32(const WaveWeights &W, const float *bias, bf16x8 x0, bf16x8 x1, int g,
                                      floatx4 &y0, floatx4 &y1)
{
    floatx4 h[4], k[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bf16x8 w = W[t];
        const floatx4 c = bias4(bias + 16 * t, g);
        h[t] = mfma(w, x0, c);
        k[t] = mfma(w, x1, c);
    }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int ob = 4 + 8 * layer, bb = 64 + 64 * layer;
        const bf16x8 a0 = relu_pack(h[0], h[1]), a1 = relu_pack(h[2], h[3]);
        const bf16x8 c0 = relu_pack(k[0], k[1]), c1 = relu_pack(k[2], k[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const floatx4 c = bias4(bias + bb + 16 * t, g);
            const bf16x8 w0 = W[ob + 2 * t];
            h[t] = mfma(w0, a0, c);
            k[t] = mfma(w0, c0, c);
            const bf16x8 w1 = W[ob + 2 * t + 1];
            h[t] = mfma(w1, a1, h[t]);
            k[t] = mfma(w1, c1, k[t]);
        }
    }
    const bf16x8 a0 = relu_pack(h[0], h[1]), a1 = relu_pack(h[2], h[3]);
    const bf16x8 c0 = relu_pack(k[0], k[1]), c1 = relu_pack(k[2], k[3]);
    const floatx4 c = bias4(bias + 192, g);
    const bf16x8 w0 = W[20], w1 = W[21];
    y0 = mfma(w1, a1, mfma(w0, a0, c));
    y1 = mfma(w1, c1, mfma(w0, c0, c));
}

// xs/ys are this wave's LDS rows; the caller synchronises around the call
__device__ __forceinline__ void mlp64(const WaveWeights &W, const float *bias, const u32x4 *xs, float *ys, int lane)
{
    const int g = lane >> 4, col = lane & 15;
#pragma unroll
    for (int q = 0; q < 4; q += 2) {
        const int row0 = 16 * q + col, row1 = row0 + 16;
        const u32x4 zero = {0u, 0u, 0u, 0u};
        const bf16x8 x0 = as_bf16x8(g < 2 ? xs[2 * row0 + g] : zero);
        const bf16x8 x1 = as_bf16x8(g < 2 ? xs[2 * row1 + g] : zero);
        // an index the compiler cannot prove equal across pairs: every operand
        // is read from LDS right before its two products instead of being held
        // in 88 registers for the whole loop
        int ln = W.lane;
        asm volatile("" : "+v"(ln));
        floatx4 y0, y1;
        mlp32(WaveWeights{W.w, ln}, bias, x0, x1, g, y0, y1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (4 * g + r < kMlpOut) {
                ys[row0 * 12 + 4 * g + r] = y0[r];
                ys[row1 * 12 + 4 * g + r] = y1[r];
            }
    }
}

// standardised inputs x[10] -> LDS row (BF16, zero padded)
__device__ __forceinline__ void store_inputs(u32x4 *xs, int lane, const float x[10])
{
    u32x4 a, b;
    a.x = pack2(x[0], x[1]);
    a.y = pack2(x[2], x[3]);
    a.z = pack2(x[4], x[5]);
    a.w = pack2(x[6], x[7]);
    b.x = pack2(x[8], x[9]);
    b.y = 0u;
    b.z = 0u;
    b.w = 0u;
    xs[2 * lane] = a;
    xs[2 * lane + 1] = b;
}

// ---------------------------------------------------------------------------
// closure inputs at a cell centre (FP64)
// ---------------------------------------------------------------------------
template <typename T>
struct ClosureIn {
    Dims d;
    double idx, idy;
    const double *idz, *idzf, *theta0;
    const T *u, *v, *w, *th;
};

template <typename T>
__device__ __forceinline__ double theta_full(const ClosureIn<T> &a, int c, int k)
{
    return kPert<T> ? (double)a.th[c] + a.theta0[k] : (double)a.th[c];
}

// du/dx, du/dy, du/dz, dv/dx, dv/dy, dv/dz, dw/dx, dw/dy, dw/dz, dtheta/dz:
// diagonal terms across the cell, off-diagonal ones as the mean of the four
// edge differences around the centre (zero on lid edges for du/dz, dv/dz,
// dw/dx, dw/dy), dtheta/dz as the mean of the two face differences (zero
// through the lids); also the centred horizontal theta gradients.
// Branch-free, so that all ~40 loads can be in flight together: periodic
// neighbours by selects, vertical neighbours clamped to the column; the lid
// terms vanish because 2/(dz_{k-1} + dz_k) is stored as zero on both lids and w
// is zero on the lid faces.
template <typename T>
__device__ void closure_inputs(const ClosureIn<T> &a, int i, int j, int k, double f[10], double &dthx, double &dthy)
{
    const Dims &d = a.d;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.nxy;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int rj = j * nx, rjm = (j == 0 ? ny - 1 : j - 1) * nx, rjp = (j == ny - 1 ? 0 : j + 1) * nx;
    const int lk = k * P, lkm = (k > 0 ? k - 1 : 0) * P, lkp = (k < nz - 1 ? k + 1 : nz - 1) * P;
    const int kp1 = k + 1;  // the face above
    auto U = [&](int ii, int r, int l) { return (double)a.u[l + r + ii]; };
    auto V = [&](int ii, int r, int l) { return (double)a.v[l + r + ii]; };
    auto Wf = [&](int ii, int r, int l) { return (double)a.w[l + r + ii]; };
    const double gz0 = a.idzf[k], gz1 = a.idzf[kp1];  // zero on the lids
    const double th0k = kPert<T> ? a.theta0[k] : 0.0;
    const double th0m = kPert<T> ? a.theta0[k > 0 ? k - 1 : 0] : 0.0;
    const double th0p = kPert<T> ? a.theta0[k < nz - 1 ? k + 1 : nz - 1] : 0.0;
    auto TH = [&](int ii, int r, int l, double t0) { return (double)a.th[l + r + ii] + t0; };
    // u on the x-faces i, i+1 of rows j-1, j, j+1 and levels k-1, k, k+1
    const double u_c = U(i, rj, lk), u_e = U(ip, rj, lk);
    const double u_s = U(i, rjm, lk), u_se = U(ip, rjm, lk), u_n = U(i, rjp, lk), u_ne = U(ip, rjp, lk);
    const double u_b = U(i, rj, lkm), u_be = U(ip, rj, lkm), u_t = U(i, rj, lkp), u_te = U(ip, rj, lkp);
    // v on the y-faces j, j+1 of columns i-1, i, i+1 and levels k-1, k, k+1
    const double v_c = V(i, rj, lk), v_n = V(i, rjp, lk);
    const double v_w = V(im, rj, lk), v_e = V(ip, rj, lk), v_nw = V(im, rjp, lk), v_ne = V(ip, rjp, lk);
    const double v_b = V(i, rj, lkm), v_bn = V(i, rjp, lkm), v_t = V(i, rj, lkp), v_tn = V(i, rjp, lkp);
    // w on the z-faces k, k+1 of the column and its four neighbours
    const int lk1 = kp1 * P;
    const double w_c = Wf(i, rj, lk), w_u = Wf(i, rj, lk1);
    const double w_w = Wf(im, rj, lk), w_e = Wf(ip, rj, lk), w_wu = Wf(im, rj, lk1), w_eu = Wf(ip, rj, lk1);
    const double w_s = Wf(i, rjm, lk), w_n = Wf(i, rjp, lk), w_su = Wf(i, rjm, lk1), w_nu = Wf(i, rjp, lk1);
    // theta at the centre, below, above and at the four horizontal neighbours
    const double t_c = TH(i, rj, lk, th0k), t_b = TH(i, rj, lkm, th0m), t_t = TH(i, rj, lkp, th0p);
    const double t_w = TH(im, rj, lk, th0k), t_e = TH(ip, rj, lk, th0k), t_s = TH(i, rjm, lk, th0k),
                 t_n = TH(i, rjp, lk, th0k);

    f[0] = (u_e - u_c) * a.idx;
    f[4] = (v_n - v_c) * a.idy;
    f[8] = (w_u - w_c) * a.idz[k];
    f[1] = 0.25 * (((u_c - u_s) + (u_e - u_se)) + ((u_n - u_c) + (u_ne - u_e))) * a.idy;
    f[3] = 0.25 * (((v_c - v_w) + (v_e - v_c)) + ((v_n - v_nw) + (v_ne - v_n))) * a.idx;
    f[2] = 0.25 * (((u_c - u_b) * gz0 + (u_e - u_be) * gz0) + ((u_t - u_c) * gz1 + (u_te - u_e) * gz1));
    f[5] = 0.25 * (((v_c - v_b) * gz0 + (v_n - v_bn) * gz0) + ((v_t - v_c) * gz1 + (v_tn - v_n) * gz1));
    f[6] = 0.25 * (((w_c - w_w) + (w_e - w_c)) + ((w_u - w_wu) + (w_eu - w_u))) * a.idx;
    f[7] = 0.25 * (((w_c - w_s) + (w_n - w_c)) + ((w_u - w_su) + (w_nu - w_u))) * a.idy;
    f[9] = 0.5 * ((t_c - t_b) * gz0 + (t_t - t_c) * gz1);
    dthx = 0.5 * (t_e - t_w) * a.idx;
    dthy = 0.5 * (t_n - t_s) * a.idy;
}

// Smagorinsky stresses and heat fluxes at a centre from the closure inputs:
// tau = -2 nu_t (S - tr S / 3), q = -(nu_t / Pr_t) grad theta; returns the
// dissipation nu_t |S|^2.
__device__ __forceinline__ double centre_smag(const double f[10], double dthx, double dthy, double cd, double Pr_t,
                                              double t[9])
{
    const double s11 = f[0], s22 = f[4], s33 = f[8];
    const double s12 = 0.5 * (f[1] + f[3]), s13 = 0.5 * (f[2] + f[6]), s23 = 0.5 * (f[5] + f[7]);
    const double ss = 2.0 * (s11 * s11 + s22 * s22 + s33 * s33) + 4.0 * (s12 * s12 + s13 * s13 + s23 * s23);
    const double nut = cd * cd * sqrt(ss);
    const double dd = (s11 + s22 + s33) / 3.0;
    t[0] = -2.0 * nut * (s11 - dd);
    t[1] = -2.0 * nut * (s22 - dd);
    t[2] = -2.0 * nut * (s33 - dd);
    t[3] = -2.0 * nut * s12;
    t[4] = -2.0 * nut * s13;
    t[5] = -2.0 * nut * s23;
    t[6] = -(nut / Pr_t) * dthx;
    t[7] = -(nut / Pr_t) * dthy;
    t[8] = -(nut / Pr_t) * f[9];
    return nut * ss;
}

// ---------------------------------------------------------------------------
// closure: inputs -> network -> stresses rho tau, rho q at centres
// ---------------------------------------------------------------------------
template <typename T>
struct ClosureArgs {
    ClosureIn<T> in;
    double iPr_t;
    const double *cs2, *rho0, *norm;  // cs2: (Cs Delta_k)^2 per level; norm: mean_x, std_x, mean_y, std_y
    const T *rho;
    const u32x4 *wpk;
    const float *bias;
    T *out[9];
    unsigned long long *fallbacks;  // one running count per workgroup slot
};

constexpr int kClosureBlock = 512;  // 8 wavefronts
constexpr int kClosureMaxBlocks = 512;

// One wave takes 64 consecutive cells at a time (a persistent loop over the
// grid): inputs in FP64 into LDS as BF16, the network on four groups of 16,
// then per cell the de-standardised stresses, the fallback test and rho tau.
template <typename T>
__device__ __forceinline__ void k_mlp_closure_body(ClosureArgs<T> a, VBlock vb)
{
    __shared__ u32x4 wl[22 * 64];
    __shared__ u32x4 xs_all[kClosureBlock / 64][128];
    __shared__ float ys_all[kClosureBlock / 64][64 * 12];
    __shared__ float bias[208];
    __shared__ double nrm[38];  // mean_x, 1 / std_x, mean_y, std_y
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    stage_weights(wl, bias, a.wpk, a.bias);
    for (int u = threadIdx.x; u < 38; u += kClosureBlock)
        nrm[u] = (u >= 10 && u < 20) ? 1.0 / a.norm[u] : a.norm[u];
    const WaveWeights W{wl, lane};
    u32x4 *xs = xs_all[wave];
    float *ys = ys_all[wave];
    const Dims &d = a.in.d;
    __syncthreads();
    const int64_t stride = (int64_t)vb.gx * kClosureBlock;
    unsigned int nfb = 0;  // fallback cells of this wavefront
    for (int64_t base = (int64_t)vb.x * kClosureBlock + wave * 64; base < d.n; base += stride) {
        const int c = (int)base + lane;
        const bool valid = c < d.n;
        double f[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, dthx = 0.0, dthy = 0.0, r = 0.0;
        int k = 0;
        if (valid) {
            k = c / d.nxy;
            const int rem = c - k * d.nxy, j = rem / d.nx, i = rem - j * d.nx;
            closure_inputs(a.in, i, j, k, f, dthx, dthy);
            r = full_of(a.rho, c, a.rho0[k]);  // with the gather: no second round trip after the network
        }
        float x[10];
#pragma unroll
        for (int o = 0; o < 10; ++o) x[o] = valid ? (float)((f[o] - nrm[o]) * nrm[10 + o]) : 0.f;
        store_inputs(xs, lane, x);
        wave_sync();
        mlp64(W, bias, xs, ys, lane);
        wave_sync();
        bool fb = false;
        if (valid) {
            double t[9];
            bool finite = true;
#pragma unroll
            for (int o = 0; o < 9; ++o) {
                t[o] = (double)ys[lane * 12 + o] * nrm[29 + o] + nrm[20 + o];
                finite = finite && isfinite(t[o]);
            }
            const double s11 = f[0], s22 = f[4], s33 = f[8];
            const double s12 = 0.5 * (f[1] + f[3]), s13 = 0.5 * (f[2] + f[6]), s23 = 0.5 * (f[5] + f[7]);
            const double ss = 2.0 * (s11 * s11 + s22 * s22 + s33 * s33) + 4.0 * (s12 * s12 + s13 * s13 + s23 * s23);
            const double nut = a.cs2[k] * sqrt(ss);
            // energy transfer to the subgrid scales, -tau:S, against the
            // Smagorinsky dissipation nu_t |S|^2
            const double pi = -(t[0] * s11 + t[1] * s22 + t[2] * s33 + 2.0 * (t[3] * s12 + t[4] * s13 + t[5] * s23));
            if (!finite || pi < -2.0 * (nut * ss)) {
                fb = true;
                const double dd = (s11 + s22 + s33) / 3.0;
                t[0] = -2.0 * nut * (s11 - dd);
                t[1] = -2.0 * nut * (s22 - dd);
                t[2] = -2.0 * nut * (s33 - dd);
                t[3] = -2.0 * nut * s12;
                t[4] = -2.0 * nut * s13;
                t[5] = -2.0 * nut * s23;
                t[6] = -(nut * a.iPr_t) * dthx;
                t[7] = -(nut * a.iPr_t) * dthy;
                t[8] = -(nut * a.iPr_t) * f[9];
            }
            // read by the divergence kernel only: streaming stores
#pragma unroll
            for (int o = 0; o < 9; ++o) st_stream(a.out[o] + c, (T)(r * t[o]));
        }
        nfb += (unsigned int)__popcll(__ballot(fb));
        // the next chunk rewrites this wave's rows only after it read them
        wave_sync();
    }
    // the block's count goes to its own slot: no atomics (a single counter
    // updated by every wavefront costs more than the network itself)
    __shared__ unsigned int wcount[kClosureBlock / 64];
    if (lane == 0) wcount[wave] = nfb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < kClosureBlock / 64; ++w) sum += wcount[w];
        a.fallbacks[vb.x] += sum;
    }
}
template <typename T>
__global__ __launch_bounds__(kClosureBlock, 4) void k_mlp_closure(ClosureArgs<T> a)
{
    k_mlp_closure_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(kClosureBlock, 4) void k_mlp_closure_batch(const ClosureArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_mlp_closure_body<T>(args[m], vb);
}

// ---------------------------------------------------------------------------
// divergence of the closure stresses onto the slow tendencies
// ---------------------------------------------------------------------------
template <typename T>
struct DivArgs {
    Dims d;
    int ntx, nty;
    double idx, idy;
    const double *idz, *idzf;
    const T *s[9];
    T *Rt, *Ru, *Rv, *Rw;
};

// tau_12 on xy-edges, tau_13 / tau_23 on the z-face edges (zero on the lids)
// and the heat fluxes on faces are 4-cell and 2-cell means of the centre values.
// Every load first (periodic neighbours by selects, levels clamped into the
// column, the lid terms masked by a 0/1 product rather than a conditional),
// then the arithmetic, then the stores: with a store or a branch between them
// the compiler splits the loads into dependent groups.  The tendencies are
// read by later launches only: streaming stores.
template <typename T>
__device__ __forceinline__ void k_mlp_div_body(DivArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    const TileIdx tc = tile_cell(vb, a.ntx, a.nty);
    const int i = tc.i, j = tc.j, k = tc.k;
    if (i >= d.nx || j >= d.ny) return;
    const int nz = d.nz, nx = d.nx, P = d.nxy;
    const int xm = (i == 0 ? nx - 1 : i - 1) - i, xp = (i == nx - 1 ? 0 : i + 1) - i;
    const int ym = ((j == 0 ? d.ny - 1 : j - 1) - j) * nx, yp = ((j == d.ny - 1 ? 0 : j + 1) - j) * nx;
    const int dn = k > 0 ? P : 0, up = k < nz - 1 ? P : 0;  // the levels below, above (clamped)
    const double not_bot = (double)(k > 0), not_top = (double)(k < nz - 1);
    const int c = cidx(d, i, j, k);
    auto L = [&](int o, int cc) { return (double)a.s[o][cc]; };
    // tau_11, tau_22, tau_33 at the centres
    const double s0c = L(0, c), s0w = L(0, c + xm), s1c = L(1, c), s1s = L(1, c + ym);
    const double s2c = L(2, c), s2b = L(2, c - dn);
    // S_12 at the four centres around an edge, for the edges (i, j), (i, j+1), (i+1, j)
    const double a_ws = L(3, c + xm + ym), a_s = L(3, c + ym), a_w = L(3, c + xm), a_c = L(3, c);
    const double a_wn = L(3, c + xm + yp), a_n = L(3, c + yp), a_es = L(3, c + xp + ym), a_e = L(3, c + xp);
    // S_13 around the edges of face k (x: i, i+1) and face k+1 (x: i)
    const double b_wb = L(4, c + xm - dn), b_b = L(4, c - dn), b_w = L(4, c + xm), b_c = L(4, c);
    const double b_wu = L(4, c + xm + up), b_u = L(4, c + up), b_eb = L(4, c + xp - dn), b_e = L(4, c + xp);
    // S_23 likewise with y
    const double g_sb = L(5, c + ym - dn), g_b = L(5, c - dn), g_s = L(5, c + ym), g_c = L(5, c);
    const double g_su = L(5, c + ym + up), g_u = L(5, c + up), g_nb = L(5, c + yp - dn), g_n = L(5, c + yp);
    // heat fluxes at the centres
    const double h6w = L(6, c + xm), h6c = L(6, c), h6e = L(6, c + xp);
    const double h7s = L(7, c + ym), h7c = L(7, c), h7n = L(7, c + yp);
    const double h8b = L(8, c - dn), h8c = L(8, c), h8u = L(8, c + up);
    const double Ru = a.Ru[c], Rv = a.Rv[c], Rw = a.Rw[c], Rt = a.Rt[c];

    const double idz = a.idz[k];
    const double e12 = 0.25 * (a_ws + a_s + a_w + a_c);    // edge (i, j)
    const double e12n = 0.25 * (a_w + a_c + a_wn + a_n);   // edge (i, j+1)
    const double e12e = 0.25 * (a_s + a_es + a_c + a_e);   // edge (i+1, j)
    const double e13 = 0.25 * (b_wb + b_b + b_w + b_c) * not_bot;   // face k
    const double e13u = 0.25 * (b_w + b_c + b_wu + b_u) * not_top;  // face k+1
    const double e13e = 0.25 * (b_b + b_eb + b_c + b_e) * not_bot;  // face k, i+1
    const double e23 = 0.25 * (g_sb + g_b + g_s + g_c) * not_bot;
    const double e23u = 0.25 * (g_s + g_c + g_su + g_u) * not_top;
    const double e23n = 0.25 * (g_b + g_nb + g_c + g_n) * not_bot;
    const double du = (s0c - s0w) * a.idx + (e12n - e12) * a.idy + (e13u - e13) * idz;
    const double dv = (e12e - e12) * a.idx + (s1c - s1s) * a.idy + (e23u - e23) * idz;
    const double dw = (e13e - e13) * a.idx + (e23n - e23) * a.idy + (s2c - s2b) * a.idzf[k];
    const double hx0 = 0.5 * (h6w + h6c), hx1 = 0.5 * (h6c + h6e);
    const double hy0 = 0.5 * (h7s + h7c), hy1 = 0.5 * (h7c + h7n);
    const double hz0 = 0.5 * (h8b + h8c) * not_bot, hz1 = 0.5 * (h8c + h8u) * not_top;
    st_stream(a.Ru + c, (T)(Ru - du));
    st_stream(a.Rv + c, (T)(Rv - dv));
    if (k > 0) st_stream(a.Rw + c, (T)(Rw - dw));  // the bottom lid face keeps its tendency
    st_stream(a.Rt + c, (T)(Rt - ((hx1 - hx0) * a.idx + (hy1 - hy0) * a.idy + (hz1 - hz0) * idz)));
}
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_div(DivArgs<T> a)
{
    k_mlp_div_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_div_batch(const DivArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_mlp_div_body<T>(args[m], vb);
}

// ---------------------------------------------------------------------------
// the network alone: standardised x[n][10] -> y[n][9]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 3) void k_mlp_forward(const float *__restrict__ X, int64_t n,
                                                     const u32x4 *__restrict__ wpk, const float *__restrict__ biasg,
                                                     float *__restrict__ Y)
{
    __shared__ u32x4 wl[22 * 64];
    __shared__ u32x4 xs_all[4][128];
    __shared__ float ys_all[4][64 * 12];
    __shared__ float bias[208];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    stage_weights(wl, bias, wpk, biasg);
    const WaveWeights W{wl, lane};
    u32x4 *xs = xs_all[wave];
    float *ys = ys_all[wave];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t base = (int64_t)blockIdx.x * 256 + wave * 64; base < n; base += stride) {
        const int64_t s = base + lane;
        const bool valid = s < n;
        float x[10];
#pragma unroll
        for (int o = 0; o < 10; ++o) x[o] = valid ? X[s * 10 + o] : 0.f;
        store_inputs(xs, lane, x);
        wave_sync();
        mlp64(W, bias, xs, ys, lane);
        wave_sync();
        if (valid)
#pragma unroll
            for (int o = 0; o < 9; ++o) Y[s * 9 + o] = ys[lane * 12 + o];
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// closure inputs of every cell (training data), FP64
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_features(ClosureIn<T> a, double *__restrict__ feat)
{
    const Dims &d = a.d;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.n) return;
    const int k = c / d.nxy, rem = c - k * d.nxy, j = rem / d.nx, i = rem - j * d.nx;
    double f[10], dthx, dthy;
    closure_inputs(a, i, j, k, f, dthx, dthy);
    for (int o = 0; o < 10; ++o) feat[(int64_t)c * 10 + o] = f[o];
}

// ---------------------------------------------------------------------------
// box filter of a fine state onto the r-coarsened grid, with SGS targets
// ---------------------------------------------------------------------------
template <typename T>
struct BoxArgs {
    ClosureIn<T> in;
    int r;
    Dims cd;  // coarse dims
    double dx, dy, Cs, Pr_t;
    const double *dz, *rho0, *Theta0;
    const T *rho, *rt, *ru, *rv, *rw;
    double *crho, *crt, *cru, *crv, *crw, *targets;
};

template <typename T>
__global__ __launch_bounds__(256) void k_box_filter(BoxArgs<T> a)
{
    const Dims &cd = a.cd, &d = a.in.d;
    const int cc = blockIdx.x * blockDim.x + threadIdx.x;
    if (cc >= cd.n) return;
    const int K = cc / cd.nxy, rem = cc - K * cd.nxy, J = rem / cd.nx, I = rem - J * cd.nx;
    const int r = a.r;
    double mr = 0, mt = 0, su[3] = {0, 0, 0}, sth = 0, suu[6] = {0, 0, 0, 0, 0, 0}, sut[3] = {0, 0, 0};
    double ssg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int kk = 0; kk < r; ++kk)
        for (int jj = 0; jj < r; ++jj)
            for (int ii = 0; ii < r; ++ii) {
                const int i = I * r + ii, j = J * r + jj, k = K * r + kk;
                const int c = cidx(d, i, j, k);
                mr += full_of(a.rho, c, a.rho0[k]);
                mt += full_of(a.rt, c, a.Theta0[k]);
                const double uc = 0.5 * ((double)a.in.u[c] + (double)a.in.u[cidx(d, wrap_idx(i + 1, d.nx), j, k)]);
                const double vc = 0.5 * ((double)a.in.v[c] + (double)a.in.v[cidx(d, i, wrap_idx(j + 1, d.ny), k)]);
                const double wc = 0.5 * ((double)a.in.w[c] + (double)a.in.w[c + d.nxy]);
                const double t = theta_full(a.in, c, k);
                su[0] += uc;
                su[1] += vc;
                su[2] += wc;
                sth += t;
                suu[0] += uc * uc;
                suu[1] += vc * vc;
                suu[2] += wc * wc;
                suu[3] += uc * vc;
                suu[4] += uc * wc;
                suu[5] += vc * wc;
                sut[0] += uc * t;
                sut[1] += vc * t;
                sut[2] += wc * t;
                if (a.Cs > 0.0) {
                    double f[10], dthx, dthy, ts[9];
                    closure_inputs(a.in, i, j, k, f, dthx, dthy);
                    centre_smag(f, dthx, dthy, a.Cs * cbrt(a.dx * a.dy * a.dz[k]), a.Pr_t, ts);
                    for (int o = 0; o < 9; ++o) ssg[o] += ts[o];
                }
            }
    const double r3 = (double)r * r * r, r2 = (double)r * r;
    a.crho[cc] = mr / r3;
    a.crt[cc] = mt / r3;
    const double m0 = su[0] / r3, m1 = su[1] / r3, m2 = su[2] / r3, mth = sth / r3;
    double *tg = a.targets + (int64_t)cc * 9;
    tg[0] = suu[0] / r3 - m0 * m0 + ssg[0] / r3;
    tg[1] = suu[1] / r3 - m1 * m1 + ssg[1] / r3;
    tg[2] = suu[2] / r3 - m2 * m2 + ssg[2] / r3;
    tg[3] = suu[3] / r3 - m0 * m1 + ssg[3] / r3;
    tg[4] = suu[4] / r3 - m0 * m2 + ssg[4] / r3;
    tg[5] = suu[5] / r3 - m1 * m2 + ssg[5] / r3;
    tg[6] = sut[0] / r3 - m0 * mth + ssg[6] / r3;
    tg[7] = sut[1] / r3 - m1 * mth + ssg[7] / r3;
    tg[8] = sut[2] / r3 - m2 * mth + ssg[8] / r3;
    double fu = 0, fv = 0, fw = 0;
    for (int p = 0; p < r; ++p)
        for (int q = 0; q < r; ++q) {
            fu += (double)a.ru[cidx(d, I * r, J * r + p, K * r + q)];
            fv += (double)a.rv[cidx(d, I * r + p, J * r, K * r + q)];
            fw += (double)a.rw[cidx(d, I * r + p, J * r + q, K * r)];
        }
    a.cru[cc] = fu / r2;
    a.crv[cc] = fv / r2;
    a.crw[cc] = K == 0 ? 0.0 : fw / r2;
    if (K == cd.nz - 1) a.crw[cc + cd.nxy] = 0.0;
}

// ---------------------------------------------------------------------------
// statistics and standardisation of training data
// ---------------------------------------------------------------------------
constexpr int kStatRows = 1024;  // rows per partial block

// partial column sums of (x - shift)^p, p = 1 or 2, over kStatRows rows
__global__ __launch_bounds__(64) void k_col_moments(const double *__restrict__ X, int64_t n, int ncol,
                                                    const double *__restrict__ shift, int power,
                                                    double *__restrict__ part)
{
    const int col = threadIdx.x;
    if (col >= ncol) return;
    const int64_t r0 = (int64_t)blockIdx.x * kStatRows, r1 = r0 + kStatRows < n ? r0 + kStatRows : n;
    const double s0 = shift ? shift[col] : 0.0;
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double v = X[r * ncol + col] - s0;
        acc += power == 1 ? v : v * v;
    }
    part[(int64_t)blockIdx.x * ncol + col] = acc;
}

// out[col] = sum of the partials in block order / n (square root for p = 2)
__global__ __launch_bounds__(64) void k_col_finish(const double *__restrict__ part, int nblk, int ncol, int64_t n,
                                                   int take_sqrt, double *__restrict__ out)
{
    const int col = threadIdx.x;
    if (col >= ncol) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(int64_t)b * ncol + col];
    double v = acc / (double)n;
    if (take_sqrt) {
        v = sqrt(v);
        if (!(v > 0.0)) v = 1.0;  // a constant column keeps unit scale
    }
    out[col] = v;
}

__global__ __launch_bounds__(256) void k_standardize(const double *__restrict__ X, int64_t n, int ncol,
                                                     const double *__restrict__ mean, const double *__restrict__ sd,
                                                     float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ncol) return;
    const int col = (int)(e % ncol);
    out[e] = (float)((X[e] - mean[col]) / sd[col]);
}

// ---------------------------------------------------------------------------
// training: one fused pass per chunk of 64 samples (forward, loss, backward and
// the weight-gradient products), BF16 MFMA operands with FP32 accumulation,
// FP64 loss and bias sums; per-block partials reduced in a fixed order
// ---------------------------------------------------------------------------
// The BF16 rounding points are those of the layer-by-layer products: every
// matrix operand (inputs, post-ReLU activations, the output error and the
// back-propagated errors, the weights) is rounded to BF16 from its FP32 value;
// biases, ReLU, the masks and dY = 2 (Y - T)/(9 n) are FP32 (dY formed in FP64).
//
// Each wavefront takes 16 samples of the block's chunk: the layer products run
// as C[sample][unit] = sum_k A[sample][k] B[k][unit] on the 16 x 16 x 32 BF16
// matrix instruction, with the activations and errors in LDS twice, sample-major
// (A operands of the next product) and unit-major (K = samples for the weight
// gradients).  After a block barrier the four wavefronts share the 40 weight-
// gradient tiles (10 each, accumulated in registers over all of the block's
// chunks): dW = H_in^T D over the chunk's 64 samples.
constexpr int kTrainChunk = 64;
constexpr int kTrainMaxBlocks = 256;
constexpr int kTrainDbl = 256;  // per block: b1, b2, b3 (64 each), b4 (9), loss at 208
// training weight operands (BF16 bits), row-major with 16-byte aligned rows:
// WT* forward (row = output unit, column = input), WN* backward (row = input
// unit, column = output unit); padding zero
constexpr int kTW1 = 0, kTW2 = kTW1 + 64 * 32, kTW3 = kTW2 + 64 * 64, kTW4 = kTW3 + 64 * 64;
constexpr int kTN4 = kTW4 + 16 * 64, kTN3 = kTN4 + 64 * 32, kTN2 = kTN3 + 64 * 64, kTWords = kTN2 + 64 * 64;
// LDS (bytes): weights, biases, per-wavefront sample-major arrays, block unit-major arrays
constexpr int kSU_X = 0, kSU_H1 = kSU_X + 16 * 32, kSU_H2 = kSU_H1 + 16 * 64, kSU_H3 = kSU_H2 + 16 * 64;
constexpr int kSU_DY = kSU_H3 + 16 * 64, kSU_D3 = kSU_DY + 16 * 32, kSU_D2 = kSU_D3 + 16 * 64, kSU_Words = kSU_D2 + 16 * 64;
constexpr int kUS_X = 0, kUS_H1 = kUS_X + 16 * 64, kUS_H2 = kUS_H1 + 64 * 64, kUS_H3 = kUS_H2 + 64 * 64;
constexpr int kUS_D1 = kUS_H3 + 64 * 64, kUS_D2 = kUS_D1 + 64 * 64, kUS_D3 = kUS_D2 + 64 * 64;
constexpr int kUS_DY = kUS_D3 + 64 * 64, kUS_Words = kUS_DY + 16 * 64;
constexpr int kL_W = 0, kL_B = kL_W + kTWords * 2, kL_SU = kL_B + 208 * 4, kL_US = kL_SU + 4 * kSU_Words * 2;
constexpr int kL_Total = kL_US + kUS_Words * 2;
static_assert(kL_SU % 16 == 0 && kL_US % 16 == 0 && kL_Total <= 160 * 1024, "training LDS layout");
static_assert(4 * 4 * 13 * 16 * 8 + 256 * 8 <= kUS_Words * 2, "bias reduction fits the unit-major area");

__device__ __forceinline__ unsigned short bf(float v) { return (unsigned short)(pack2(v, 0.f) & 0xffffu); }
__device__ __forceinline__ bf16x8 ld8(const unsigned short *p) { return as_bf16x8(*(const u32x4 *)p); }

// packed training operands from the FP32 master parameters
__global__ __launch_bounds__(256) void k_train_pack(const float *__restrict__ P, unsigned short *__restrict__ tw)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kTWords) return;
    float v = 0.f;
    if (e < kTW2) {
        const int o = (e - kTW1) / 32, i = (e - kTW1) % 32;
        if (i < kMlpIn) v = P[kMlpW1 + i * kMlpH + o];
    } else if (e < kTW3) {
        const int o = (e - kTW2) / 64, i = (e - kTW2) % 64;
        v = P[kMlpW2 + i * kMlpH + o];
    } else if (e < kTW4) {
        const int o = (e - kTW3) / 64, i = (e - kTW3) % 64;
        v = P[kMlpW3 + i * kMlpH + o];
    } else if (e < kTN4) {
        const int o = (e - kTW4) / 64, i = (e - kTW4) % 64;
        if (o < kMlpOut) v = P[kMlpW4 + i * kMlpOut + o];
    } else if (e < kTN3) {
        const int i = (e - kTN4) / 32, o = (e - kTN4) % 32;
        if (o < kMlpOut) v = P[kMlpW4 + i * kMlpOut + o];
    } else if (e < kTN2) {
        const int i = (e - kTN3) / 64, o = (e - kTN3) % 64;
        v = P[kMlpW3 + i * kMlpH + o];
    } else {
        const int i = (e - kTN2) / 64, o = (e - kTN2) % 64;
        v = P[kMlpW2 + i * kMlpH + o];
    }
    tw[e] = bf(v);
}

struct TrainArgs {
    const float *X, *T;
    int64_t n;
    int chunks;
    const unsigned short *tw;
    const float *P;
    float *part;    // [blocks][kMlpParams] weight-gradient partials (bias slots unused)
    double *dpart;  // [blocks][kTrainDbl] bias-gradient and loss partials
    double scale;   // 2 / (9 n)
};

// one product tile's result (lane: samples 4g + r, unit u) into both LDS
// layouts, as BF16; su is the wavefront's sample-major array (row length su_len;
// null: not stored), us the block's unit-major one (64 samples per row, the
// wavefront's 16 at s0)
__device__ __forceinline__ void put_tile(unsigned short *su, int su_len, unsigned short *us, int s0, int g, int u,
                                         const float v[4])
{
    if (su)
#pragma unroll
        for (int r = 0; r < 4; ++r) su[(4 * g + r) * su_len + u] = bf(v[r]);
    uint2 w;
    w.x = pack2(v[0], v[1]);
    w.y = pack2(v[2], v[3]);
    *(uint2 *)(us + u * 64 + s0 + 4 * g) = w;
}

__global__ __launch_bounds__(256, 1) void k_mlp_train(TrainArgs a)
{
    extern __shared__ __align__(16) unsigned char sm[];
    unsigned short *W = (unsigned short *)(sm + kL_W);
    float *bias = (float *)(sm + kL_B);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
    unsigned short *SU = (unsigned short *)(sm + kL_SU) + wave * kSU_Words;
    unsigned short *US = (unsigned short *)(sm + kL_US);
    const int s0 = wave * 16;  // the wavefront's samples within the chunk
    for (int e = tid; e < kTWords / 8; e += 256) ((u32x4 *)W)[e] = ((const u32x4 *)a.tw)[e];
    for (int e = tid; e < 208; e += 256) {
        float b = 0.f;
        if (e < 64) b = a.P[kMlpB1 + e];
        else if (e < 128) b = a.P[kMlpB2 + e - 64];
        else if (e < 192) b = a.P[kMlpB3 + e - 128];
        else if (e - 192 < kMlpOut) b = a.P[kMlpB4 + e - 192];
        bias[e] = b;
    }
    // the activation arrays start at zero: their padding (inputs 10..31,
    // outputs 9..31) is never written
    for (int e = tid; e < (4 * kSU_Words + kUS_Words) / 8; e += 256) ((u32x4 *)(sm + kL_SU))[e] = u32x4{0u, 0u, 0u, 0u};
    __syncthreads();

    const floatx4 z4 = {0.f, 0.f, 0.f, 0.f};
    floatx4 acc[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = z4;
    double db[13];
#pragma unroll
    for (int j = 0; j < 13; ++j) db[j] = 0.0;
    double sq = 0.0;

    for (int ch = blockIdx.x; ch < a.chunks; ch += gridDim.x) {
        const int64_t sb = (int64_t)ch * kTrainChunk + s0;
        // inputs of the wavefront's 16 samples (zero past n)
        for (int e = lane; e < 16 * kMlpIn; e += 64) {
            const int sl = e / kMlpIn, k = e - sl * kMlpIn;
            const int64_t s = sb + sl;
            const unsigned short b = bf(s < a.n ? a.X[s * kMlpIn + k] : 0.f);
            SU[kSU_X + sl * 32 + k] = b;
            US[kUS_X + k * 64 + s0 + sl] = b;
        }
        wave_sync();
        unsigned mask[3] = {0u, 0u, 0u};
        // hidden layers: H = ReLU(A W + b)
        auto hidden = [&](int L, const unsigned short *Ain, int alen, int ksteps, int wofs, unsigned short *su_out,
                          unsigned short *us_out) {
            bf16x8 A[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (s < ksteps) A[s] = ld8(Ain + col * alen + 32 * s + 8 * g);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int u = 16 * nt + col;
                floatx4 c = z4;
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    if (s < ksteps) c = mfma(A[s], ld8(W + wofs + u * (32 * ksteps) + 32 * s + 8 * g), c);
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = fmaxf(c[r] + bias[64 * L + u], 0.f);
                    if (v[r] > 0.f) mask[L] |= 1u << (4 * nt + r);
                }
                put_tile(su_out, 64, us_out, s0, g, u, v);
            }
            wave_sync();
        };
        hidden(0, SU + kSU_X, 32, 1, kTW1, SU + kSU_H1, US + kUS_H1);
        hidden(1, SU + kSU_H1, 64, 2, kTW2, SU + kSU_H2, US + kUS_H2);
        hidden(2, SU + kSU_H2, 64, 2, kTW3, SU + kSU_H3, US + kUS_H3);
        // output layer, loss and dY = 2 (Y - T)/(9 n)
        {
            floatx4 c = z4;
#pragma unroll
            for (int s = 0; s < 2; ++s)
                c = mfma(ld8(SU + kSU_H3 + col * 64 + 32 * s + 8 * g), ld8(W + kTW4 + col * 64 + 32 * s + 8 * g), c);
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t s = sb + 4 * g + r;
                v[r] = 0.f;
                if (col < kMlpOut && s < a.n) {
                    const float y = c[r] + bias[192 + col];
                    const double err = (double)y - (double)a.T[s * kMlpOut + col];
                    sq += err * err;
                    v[r] = (float)(a.scale * err);
                    db[0] += (double)v[r];
                }
            }
            // sample-major rows of 32 outputs (16..31 stay zero)
            put_tile(SU + kSU_DY, 32, US + kUS_DY, s0, g, col, v);
            wave_sync();
        }
        // errors back through the layers: D = (D_next W_next^T) * [H > 0]
        auto back = [&](int L, const unsigned short *Din, int dlen, int ksteps, int wofs, int slot,
                        unsigned short *su_out, unsigned short *us_out) {
            bf16x8 A[2];
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (s < ksteps) A[s] = ld8(Din + col * dlen + 32 * s + 8 * g);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int u = 16 * nt + col;
                floatx4 c = z4;
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    if (s < ksteps) c = mfma(A[s], ld8(W + wofs + u * (32 * ksteps) + 32 * s + 8 * g), c);
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = (mask[L] >> (4 * nt + r)) & 1u ? c[r] : 0.f;
                    db[slot + nt] += (double)v[r];
                }
                put_tile(su_out, 64, us_out, s0, g, u, v);  // (no sample-major copy of D1: nothing reads it)
            }
            wave_sync();
        };
        back(2, SU + kSU_DY, 32, 1, kTN4, 1, SU + kSU_D3, US + kUS_D3);
        back(1, SU + kSU_D3, 64, 2, kTN3, 5, SU + kSU_D2, US + kUS_D2);
        back(0, SU + kSU_D2, 64, 2, kTN2, 9, nullptr, US + kUS_D1);
        __syncthreads();
        // weight gradients over the chunk's 64 samples: tile q = wave + 4 j of
        // dW4 (4 tiles), dW3 (16), dW2 (16), dW1 (4)
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int q = wave + 4 * j;
            int mt, nt, ain, bin;
            if (q < 4) { mt = q; nt = 0; ain = kUS_H3; bin = kUS_DY; }
            else if (q < 20) { mt = (q - 4) >> 2; nt = (q - 4) & 3; ain = kUS_H2; bin = kUS_D3; }
            else if (q < 36) { mt = (q - 20) >> 2; nt = (q - 20) & 3; ain = kUS_H1; bin = kUS_D2; }
            else { mt = 0; nt = q - 36; ain = kUS_X; bin = kUS_D1; }
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                acc[j] = mfma(ld8(US + ain + (16 * mt + col) * 64 + 32 * ks + 8 * g),
                              ld8(US + bin + (16 * nt + col) * 64 + 32 * ks + 8 * g), acc[j]);
        }
        __syncthreads();
    }

    // weight-gradient partials (lane: input unit 16 mt + 4 g + r, output 16 nt + col)
    float *part = a.part + (size_t)blockIdx.x * kMlpParams;
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const int q = wave + 4 * j;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int idx = -1;
            if (q < 4) {
                const int in = 16 * q + 4 * g + r;
                if (col < kMlpOut) idx = kMlpW4 + in * kMlpOut + col;
            } else if (q < 20) {
                const int in = 16 * ((q - 4) >> 2) + 4 * g + r, out = 16 * ((q - 4) & 3) + col;
                idx = kMlpW3 + in * kMlpH + out;
            } else if (q < 36) {
                const int in = 16 * ((q - 20) >> 2) + 4 * g + r, out = 16 * ((q - 20) & 3) + col;
                idx = kMlpW2 + in * kMlpH + out;
            } else {
                const int in = 4 * g + r, out = 16 * (q - 36) + col;
                if (in < kMlpIn) idx = kMlpW1 + in * kMlpH + out;
            }
            if (idx >= 0) part[idx] = acc[j][r];
        }
    }
    // bias and loss partials: the 16 lane groups of the block combined in LDS
    // in a fixed order (the unit-major area is free after the last barrier)
    double *red = (double *)(sm + kL_US);
#pragma unroll
    for (int j = 0; j < 13; ++j) red[((wave * 4 + g) * 13 + j) * 16 + col] = db[j];
    double *lred = red + 4 * 4 * 13 * 16;
    lred[tid] = sq;
    __syncthreads();
    if (tid < 208) {
        int slot, c;
        if (tid < 64) { slot = 9 + tid / 16; c = tid % 16; }
        else if (tid < 128) { slot = 5 + (tid - 64) / 16; c = (tid - 64) % 16; }
        else if (tid < 192) { slot = 1 + (tid - 128) / 16; c = (tid - 128) % 16; }
        else { slot = 0; c = tid - 192; }
        double s = 0.0;
        for (int wg = 0; wg < 16; ++wg) s += red[(wg * 13 + slot) * 16 + c];
        a.dpart[(size_t)blockIdx.x * kTrainDbl + tid] = s;
    }
    if (tid == 255) {
        double s = 0.0;
        for (int l = 0; l < 256; ++l) s += lred[l];
        a.dpart[(size_t)blockIdx.x * kTrainDbl + 208] = s;
    }
}

// G[p] and the loss from the block partials, FP64 sums in a fixed order: a
// workgroup of 256 covers 64 parameters (lane = parameter); wavefront w sums
// the blocks b = w mod 4 in eight interleaved chains (eight loads in flight),
// the chains and the wavefronts combined in fixed order
__global__ __launch_bounds__(256) void k_train_reduce(const float *__restrict__ part, const double *__restrict__ dpart,
                                                      int nblk, int64_t n, float *__restrict__ G, double *__restrict__ loss)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (p < kMlpParams + 1) {
        // p == kMlpParams: the loss
        int bi = -1;
        if (p == kMlpParams) bi = 208;
        else if (p >= kMlpB1 && p < kMlpB1 + kMlpH) bi = p - kMlpB1;
        else if (p >= kMlpB2 && p < kMlpB2 + kMlpH) bi = 64 + p - kMlpB2;
        else if (p >= kMlpB3 && p < kMlpB3 + kMlpH) bi = 128 + p - kMlpB3;
        else if (p >= kMlpB4) bi = 192 + p - kMlpB4;
        double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = w;
        for (; b + 28 < nblk; b += 32) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int bb = b + 4 * u;
                c[u] += bi >= 0 ? dpart[(size_t)bb * kTrainDbl + bi] : (double)part[(size_t)bb * kMlpParams + p];
            }
        }
        for (int u = 0; b < nblk; b += 4, ++u)
            c[u & 7] += bi >= 0 ? dpart[(size_t)b * kTrainDbl + bi] : (double)part[(size_t)b * kMlpParams + p];
        s = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && p < kMlpParams + 1) {
        const double v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        if (p < kMlpParams)
            G[p] = (float)v;
        else
            *loss = v / ((double)n * 9.0);
    }
}

// Adam (Kingma & Ba) with bias correction; FP32 storage, FP64 arithmetic
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, const float *__restrict__ G,
                                              float *__restrict__ Mo, float *__restrict__ Vo, int np, double lr,
                                              double b1, double b2, double eps, double c1, double c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= np) return;
    const double g = G[e];
    const double m = b1 * (double)Mo[e] + (1.0 - b1) * g;
    const double v = b2 * (double)Vo[e] + (1.0 - b2) * g * g;
    Mo[e] = (float)m;
    Vo[e] = (float)v;
    P[e] = (float)((double)P[e] - lr * (m / c1) / (sqrt(v / c2) + eps));
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
template <typename T>
ClosureIn<T> closure_in(erf_ctx *cx)
{
    ClosureIn<T> in{};
    in.d = cx->d;
    in.idx = 1.0 / cx->grid.dx;
    in.idy = 1.0 / cx->grid.dy;
    in.idz = cx->base.idz();
    in.idzf = cx->base.idzf();
    in.theta0 = cx->base.theta0;
    in.u = (const T *)cx->ws.u;
    in.v = (const T *)cx->ws.v;
    in.w = (const T *)cx->ws.w;
    in.th = (const T *)cx->ws.th;
    return in;
}

int grid_for(int64_t items, int per_block, int cap)
{
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

template <typename T>
hipError_t closure_t(erf_ctx *cx, const void *rho, void *const R[5])
{
    MlpState &m = cx->mlp;
    ClosureArgs<T> a{};
    a.in = closure_in<T>(cx);
    a.iPr_t = 1.0 / cx->prm.Pr_t;
    a.cs2 = cx->base.cs2();
    a.rho0 = cx->base.rho0;
    a.norm = m.norm;
    a.rho = (const T *)rho;
    a.wpk = (const u32x4 *)m.wpk;
    a.bias = m.bias;
    for (int o = 0; o < 9; ++o) a.out[o] = (T *)cx->ws.sg[o];
    a.fallbacks = m.fallbacks;
    const Dims &d = cx->d;
    timing_start(cx, K_MLP);
    run<ClosureArgs<T>, k_mlp_closure<T>, k_mlp_closure_batch<T>>(
        cx, dim3(grid_for(d.n, kClosureBlock, kClosureMaxBlocks)), dim3(kClosureBlock), 0, a);
    timing_stop(cx, K_MLP);
    DivArgs<T> v{};
    v.d = d;
    v.idx = 1.0 / cx->grid.dx;
    v.idy = 1.0 / cx->grid.dy;
    v.idz = cx->base.idz();
    v.idzf = cx->base.idzf();
    for (int o = 0; o < 9; ++o) v.s[o] = (const T *)cx->ws.sg[o];
    v.Rt = (T *)R[1];
    v.Ru = (T *)R[2];
    v.Rv = (T *)R[3];
    v.Rw = (T *)R[4];
    const int tx = tile_width(d.nx, d.ny, 256), ty = 256 / tx;
    v.ntx = (d.nx + tx - 1) / tx;
    v.nty = (d.ny + ty - 1) / ty;
    timing_start(cx, K_MLP_DIV);
    run<DivArgs<T>, k_mlp_div<T>, k_mlp_div_batch<T>>(cx, dim3(v.ntx * v.nty * d.nz), dim3(tx, ty, 1), 0, v);
    timing_stop(cx, K_MLP_DIV);
    return hipGetLastError();
}

template <typename T>
hipError_t features_t(erf_ctx *cx, double *feat)
{
    hipLaunchKernelGGL(k_features<T>, dim3(grid_for(cx->d.n, 256, 1 << 30)), dim3(256), 0, cx->stream,
                       closure_in<T>(cx), feat);
    return hipGetLastError();
}

template <typename T>
hipError_t box_filter_t(erf_ctx *cx, const void *const S[5], int r, double Cs, double Pr_t, double *const C[5],
                        double *targets)
{
    BoxArgs<T> a{};
    a.in = closure_in<T>(cx);
    a.r = r;
    a.cd.nx = cx->d.nx / r;
    a.cd.ny = cx->d.ny / r;
    a.cd.nz = cx->d.nz / r;
    a.cd.nxy = a.cd.nx * a.cd.ny;
    a.cd.n = a.cd.nxy * a.cd.nz;
    a.cd.nw = a.cd.nxy * (a.cd.nz + 1);
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.Cs = Cs;
    a.Pr_t = Pr_t;
    a.dz = cx->base.dz;
    a.rho0 = cx->base.rho0;
    a.Theta0 = cx->base.Theta0;
    a.rho = (const T *)S[0];
    a.rt = (const T *)S[1];
    a.ru = (const T *)S[2];
    a.rv = (const T *)S[3];
    a.rw = (const T *)S[4];
    a.crho = C[0];
    a.crt = C[1];
    a.cru = C[2];
    a.crv = C[3];
    a.crw = C[4];
    a.targets = targets;
    hipLaunchKernelGGL(k_box_filter<T>, dim3(grid_for(a.cd.n, 256, 1 << 30)), dim3(256), 0, cx->stream, a);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t mlp_pack(erf_ctx *cx)
{
    MlpState &m = cx->mlp;
    hipLaunchKernelGGL(k_mlp_pack, dim3(22), dim3(64), 0, cx->stream, m.master, (u32x4 *)m.wpk, m.bias);
    return hipGetLastError();
}

hipError_t launch_mlp_closure(erf_ctx *cx, const void *rho, void *const R[5])
{
    if (cx->prm.precision == ERF_FP32_MIXED) return closure_t<float>(cx, rho, R);
    return closure_t<double>(cx, rho, R);
}

hipError_t launch_mlp_forward(erf_ctx *cx, const float *x, int64_t n, float *y)
{
    MlpState &m = cx->mlp;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(n, 256, 1024)), dim3(256), 0, cx->stream, x, n,
                       (const u32x4 *)m.wpk, (const float *)m.bias, y);
    return hipGetLastError();
}

hipError_t launch_features(erf_ctx *cx, double *feat)
{
    if (cx->prm.precision == ERF_FP32_MIXED) return features_t<float>(cx, feat);
    return features_t<double>(cx, feat);
}

hipError_t launch_box_filter(erf_ctx *cx, const void *const S[5], int r, double Cs, double Pr_t,
                             double *const C[5], double *targets)
{
    if (cx->prm.precision == ERF_FP32_MIXED) return box_filter_t<float>(cx, S, r, Cs, Pr_t, C, targets);
    return box_filter_t<double>(cx, S, r, Cs, Pr_t, C, targets);
}

int closure_count_slots() { return kClosureMaxBlocks; }

size_t stat_partials(int64_t n) { return (size_t)((n + kStatRows - 1) / kStatRows) * 16; }

hipError_t launch_col_stats(erf_ctx *cx, const double *X, int64_t n, int ncol, double *mean, double *sd,
                            double *part)
{
    const int nblk = (int)((n + kStatRows - 1) / kStatRows);
    hipLaunchKernelGGL(k_col_moments, dim3(nblk), dim3(64), 0, cx->stream, X, n, ncol, (const double *)nullptr, 1, part);
    hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(64), 0, cx->stream, (const double *)part, nblk, ncol, n, 0, mean);
    hipLaunchKernelGGL(k_col_moments, dim3(nblk), dim3(64), 0, cx->stream, X, n, ncol, (const double *)mean, 2, part);
    hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(64), 0, cx->stream, (const double *)part, nblk, ncol, n, 1, sd);
    return hipGetLastError();
}

hipError_t launch_standardize(erf_ctx *cx, const double *X, int64_t n, int ncol, const double *mean,
                              const double *sd, float *out)
{
    hipLaunchKernelGGL(k_standardize, dim3(grid_for(n * ncol, 256, 1 << 30)), dim3(256), 0, cx->stream, X, n, ncol,
                       mean, sd, out);
    return hipGetLastError();
}

int train_blocks(int64_t n)
{
    const int64_t chunks = (n + kTrainChunk - 1) / kTrainChunk;
    return (int)(chunks < kTrainMaxBlocks ? (chunks > 0 ? chunks : 1) : kTrainMaxBlocks);
}
size_t train_part_floats(int64_t n) { return (size_t)train_blocks(n) * kMlpParams; }
size_t train_part_doubles(int64_t n) { return (size_t)train_blocks(n) * kTrainDbl; }
size_t train_weight_shorts() { return kTWords; }

hipError_t mlp_train_prepare()
{
    return hipFuncSetAttribute((const void *)k_mlp_train, hipFuncAttributeMaxDynamicSharedMemorySize, kL_Total);
}

hipError_t launch_loss_grad(erf_ctx *cx, const float *X, const float *Tt, int64_t n, float *G, double *loss_dev,
                            float *part, double *dpart)
{
    MlpState &m = cx->mlp;
    hipLaunchKernelGGL(k_train_pack, dim3((kTWords + 255) / 256), dim3(256), 0, cx->stream, (const float *)m.master,
                       m.tw);
    TrainArgs a{};
    a.X = X;
    a.T = Tt;
    a.n = n;
    a.chunks = (int)((n + kTrainChunk - 1) / kTrainChunk);
    a.tw = m.tw;
    a.P = m.master;
    a.part = part;
    a.dpart = dpart;
    a.scale = 2.0 / ((double)n * 9.0);
    const int nblk = train_blocks(n);
    hipLaunchKernelGGL(k_mlp_train, dim3(nblk), dim3(256), kL_Total, cx->stream, a);
    hipLaunchKernelGGL(k_train_reduce, dim3((kMlpParams + 1 + 63) / 64), dim3(256), 0, cx->stream,
                       (const float *)part, (const double *)dpart, nblk, n, G, loss_dev);
    return hipGetLastError();
}

hipError_t launch_adam(erf_ctx *cx, double lr, int64_t step)
{
    MlpState &m = cx->mlp;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, cx->stream, m.master,
                       (const float *)m.grad, m.adam_m, m.adam_v, kMlpParams, lr, b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_pack(cx);
}

}  // namespace erfk
