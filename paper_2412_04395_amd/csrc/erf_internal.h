// erf_internal.h -- shared declarations of the liberf.so translation units.
//
// Device-side conventions: fields are SoA, x fastest, no halo; periodic wrap in
// x and y and the reflection ghosts at the lids are resolved by index
// arithmetic inside the kernels.  Kernels take a Dims by value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
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
// gas constant of water vapour (usual value); water vapour enters the equation
// of state through the factor 1 + (R_v / R_d) q_v on rho theta (Sec. 2.1)
constexpr double kRv = 461.6;
constexpr double kEpsV = kRv / kRd;

// learned closure: 10 -> 64 -> 64 -> 64 -> 9, parameters W1[10][64], b1,
// W2[64][64], b2, W3[64][64], b3, W4[64][9], b4 (row = input unit)
constexpr int kMlpIn = 10, kMlpH = 64, kMlpOut = 9;
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpIn * kMlpH, kMlpW2 = kMlpB1 + kMlpH;
constexpr int kMlpB2 = kMlpW2 + kMlpH * kMlpH, kMlpW3 = kMlpB2 + kMlpH, kMlpB3 = kMlpW3 + kMlpH * kMlpH;
constexpr int kMlpW4 = kMlpB3 + kMlpH, kMlpB4 = kMlpW4 + kMlpH * kMlpOut, kMlpParams = kMlpB4 + kMlpOut;
constexpr int kMlpNorm = 2 * kMlpIn + 2 * kMlpOut;
static_assert(kMlpParams == 9609, "parameter layout");

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

// Workgroups go to the 8 XCDs of the chip round-robin by linear id.  This maps
// the linear id b of a grid of n workgroups to a position such that every XCD
// receives one contiguous range of positions, so neighbouring tiles (and
// their stencil halos) share one L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int x = b % 8, m = b / 8, q = n / 8, r = n % 8;
    return x * q + (x < r ? x : r) + m;
}

// Cell (i, j, k) of a flattened 64 x 4 x 1 tiling launched as a 1-D grid of
// ntx * nty * nlev workgroups.  Every XCD takes one slab of tile rows (an
// eighth of a level) across all levels, level by level, so that the y-stencil
// neighbours of a tile share its L2 and the tiles of neighbouring levels are
// resident at the same time, as in the plain order.  (Measured on the slow-RHS
// kernels: 1.5-7 % faster than the plain order, which is itself 5-7 % faster
// than an order in which each XCD owns a contiguous range of whole levels.)
// Streaming accesses: loads of values that no other lane or workgroup of the
// launch reads, and stores of results read only by a later launch, carry the
// nontemporal hint, so that they do not push stencil neighbours out of the
// caches (measured: the fused acoustic substep 375 -> 342 us per launch at
// 256 x 256 x 128 in FP64).
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// block geometry: the hardware's, or one context's share of a batched launch
// ---------------------------------------------------------------------------
// Kernel bodies read their block index and grid size from a VBlock.  A plain
// launch passes the hardware values; a batched launch (one launch running one
// kernel for the contexts of an ensemble) gives every context a contiguous
// range of blocks and passes each block its index within its context's own
// grid, so the body runs exactly as in the context's own launch.
struct VBlock {
    int x, y, z;     // block index in the context's grid
    int gx, gy, gz;  // the context's grid
};
__device__ __forceinline__ VBlock hw_block()
{
    return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}

// Block ranges of a batched launch (device arrays): context m owns launch
// blocks [first[m], first[m + 1]); its own grid is grid[3m .. 3m + 2].  Ranges
// start on multiples of 8 (each XCD then sees every context's blocks in the
// round-robin order of a plain launch); blocks past a context's own grid are
// padding and exit at once.
struct BatchMap {
    const int *first;
    const int *grid;
    int n;
};
__device__ __forceinline__ bool batch_block(const BatchMap &bm, int &m, VBlock &vb)
{
    const int b = blockIdx.x;
    int lo = 0, hi = bm.n - 1;  // the last m with first[m] <= b (uniform: scalar loads)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bm.first[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    m = lo;
    const int gx = bm.grid[3 * m], gy = bm.grid[3 * m + 1], gz = bm.grid[3 * m + 2];
    const int l = b - bm.first[m];
    if (l >= gx * gy * gz) return false;
    vb = {l % gx, (l / gx) % gy, l / (gx * gy), gx, gy, gz};
    return true;
}

struct TileIdx {
    int i, j, k;
};
__device__ __forceinline__ TileIdx tile_cell(VBlock vb, int ntx, int nty)
{
    const int nrow = ntx * nty, b = vb.x;
    int t = b;
    if (nrow % 8 == 0) {
        const int rows = nrow / 8, x = b % 8, m = b / 8;
        t = (m / rows) * nrow + x * rows + m % rows;
    }
    const int bx = t % ntx, r = t / ntx, by = r % nty, bz = r / nty;
    return {bx * (int)blockDim.x + (int)threadIdx.x, by * (int)blockDim.y + (int)threadIdx.y, bz};
}

// Width of a workgroup's tile row for tiles of `lanes` cells in an nx x ny
// plane: of 64, 32 and 16, the one that pads the plane least (a 96-wide grid
// in rows of 64 would leave a third of its lanes idle); on a tie the widest,
// whose rows are the longest contiguous segments.
inline int tile_width(int nx, int ny, int lanes)
{
    int best = 64;
    long best_cells = -1;
    for (int tx = 64; tx >= 16; tx /= 2) {
        const int ty = lanes / tx;
        const long cells = (long)((nx + tx - 1) / tx) * tx * ((ny + ty - 1) / ty) * ty;
        if (best_cells < 0 || cells < best_cells) {
            best = tx;
            best_cells = cells;
        }
    }
    return best;
}

template <typename R>
__device__ __forceinline__ R sign_of(R x)
{
    return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

// Storage conventions.  FP64 storage holds full rho and rho*theta; FP32
// storage holds their perturbations about the base state.  These return the
// full value and the perturbation of element c on level k, in double.
template <typename T>
inline constexpr bool kPert = std::is_same<T, float>::value;

template <typename T>
__device__ __forceinline__ double full_of(const T *f, int c, double base)
{
    if constexpr (kPert<T>)
        return base + (double)f[c];
    else
        return f[c];
}
template <typename T>
__device__ __forceinline__ double pert_of(const T *f, int c, double base)
{
    if constexpr (kPert<T>)
        return (double)f[c];
    else
        return f[c] - base;
}

// The same in the storage type T itself (the arithmetic type of the FP32
// path, double for the FP64 path): the base value rounded to T.
template <typename T>
__device__ __forceinline__ T full_in(const T *f, int c, double base)
{
    if constexpr (kPert<T>)
        return (T)base + f[c];
    else
        return f[c];
}
template <typename T>
__device__ __forceinline__ T pert_in(const T *f, int c, double base)
{
    if constexpr (kPert<T>)
        return f[c];
    else
        return f[c] - base;
}

// Interpolated face value q_{m-1/2} (Sec. 3.6) from q[0..5] = q_{m-3..m+2};
// s is the sign of the normal momentum at the face (-1, 0 or 1, so that
// s * (1/12) and s * (1/60) equal s / 12 and s / 60 exactly).  R is the
// arithmetic type (the coefficients rounded to it).
template <typename R>
__device__ __forceinline__ R face_interp(int order, R qm3, R qm2, R qm1, R q0, R qp1, R qp2, R s)
{
    if (order == 2) return R(0.5) * (q0 + qm1);
    if (order == 3 || order == 4) {
        R c4 = R(7.0 / 12.0) * (q0 + qm1) - R(1.0 / 12.0) * (qp1 + qm2);
        if (order == 4) return c4;
        return c4 + s * R(1.0 / 12.0) * ((qp1 - qm2) - R(3) * (q0 - qm1));
    }
    R c6 = R(37.0 / 60.0) * (q0 + qm1) - R(2.0 / 15.0) * (qp1 + qm2) + R(1.0 / 60.0) * (qp2 + qm3);
    if (order == 6) return c6;
    return c6 - s * R(1.0 / 60.0) * ((qp2 - qm3) - R(5) * (qp1 - qm2) + R(10) * (q0 - qm1));
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// Bulk fields are stored in the context's precision (double for ERF_FP64,
// float for ERF_FP32_MIXED) and kept as untyped pointers here; the tridiagonal
// factors and the reduction partials are always double.
struct Workspace {
    // stage states S*, S** (5 fields + scalars each)
    void *sa[6] = {};
    void *sb[6] = {};
    // slow tendencies
    void *R[5] = {};
    // stage fields at centres / faces: theta (theta - theta0 in FP32 storage),
    // p', Exner, velocities, mu_t
    void *th = nullptr, *pp = nullptr, *pit = nullptr;
    void *u = nullptr, *v = nullptr, *w = nullptr, *mut = nullptr;
    // stresses tau_11, tau_22, tau_33 (centres), tau_12 (xy-edges), tau_13,
    // tau_23 (z-face edges) and the heat diffusivity (centres)
    void *tau[6] = {};
    void *kap = nullptr;
    // substep perturbations: Theta'' (three time levels), rho'', U'' and V''
    // (double-buffered), W''
    void *t2[3] = {};
    void *u2[2] = {}, *v2[2] = {};
    void *r2 = nullptr, *w2 = nullptr;
    // running sums of the substep momenta (stage-averaged fluxes at the end)
    void *su = nullptr, *sv = nullptr, *sw = nullptr;
    // per-stage tridiagonal rows on z-faces: buoyancy coefficient (bulk
    // precision) and the Thomas pivots 1 / den_k (double)
    void *cC = nullptr;
    double *cb = nullptr;
    // mixing ratios q^t of the scalars, stage-averaged momenta of rk3_step
    void *q = nullptr;
    void *fu = nullptr, *fv = nullptr, *fw = nullptr;
    // diagnostics partial sums
    double *diag = nullptr;
    // moist contexts only: 1 + q_v + q_c and the total-density departure
    // rho (1 + q_v + q_c + q_r) - rho0 (1 + qv0) of the slow right-hand side;
    // the moist Exner function pi^t and rho_d / rho_m = 1/(1 + q_v + q_c + q_r)
    // of the stage state (the acoustic coefficients)
    void *qf = nullptr, *bm = nullptr, *pex = nullptr, *rdm = nullptr;
    // rain accumulated at the ground by the microphysics [kg/m^2], [ny][nx]
    double *precip = nullptr;
    // Deardorff closure: the source of rho e at the latest right-hand side's
    // state (centres); surface layer: tau_13, tau_23 per column ([2][ny][nx])
    void *esrc = nullptr, *most = nullptr;
    // learned closure: rho tau_11, 22, 33, 12, 13, 23 and rho q_1, 2, 3 at
    // centres (allocated for the learned closure only)
    void *sg[9] = {};
};

// Anelastic contexts only (FP64): the perturbation pressure the projections
// accumulate (lagged into the next right-hand side), the spectral work array of
// the Poisson solve, the Thomas factors c'_k of its z solves, the potential
// phi = dt psi, and the twiddle factors exp(-2 pi i t / N), t < N/2, of the x
// and y transforms.
struct Anel {
    double *pa = nullptr;
    double2 *Z = nullptr;
    double *cp = nullptr, *phi = nullptr;
    double2 *twx = nullptr, *twy = nullptr;
    int lgx = 0, lgy = 0;  // log2 nx, log2 ny
};

// Learned-closure state: FP32 master parameters with Adam moments, the BF16
// operands packed for the matrix cores, biases, input/output statistics, the
// running count of cells that fell back to Smagorinsky, and training buffers.
struct MlpState {
    void *alloc = nullptr;
    float *master = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    void *wpk = nullptr;            // 22 operands x 64 lanes x 16 bytes
    unsigned short *tw = nullptr;   // BF16 operands of the training pass
    float *bias = nullptr;          // b1, b2, b3, b4 padded to 16: 208
    double *norm = nullptr;         // mean_x[10], std_x[10], mean_y[9], std_y[9]
    unsigned long long *fallbacks = nullptr;  // per-workgroup running counts
    double *loss = nullptr;
    bool have_weights = false;
    int64_t step = 0;
    // training partials, grown on demand
    void *talloc = nullptr;
    int64_t cap = 0;
    float *tpart = nullptr;
    double *tdpart = nullptr;
};

struct Base {
    double *rho0 = nullptr, *theta0 = nullptr, *Theta0 = nullptr, *p0 = nullptr, *pi0 = nullptr;
    // base-state vapour qv0 and total density rho0 (1 + qv0) [nz] (zero and
    // rho0 for a dry context)
    double *qv0 = nullptr, *rho0t = nullptr;
    // device: dz [nz], centre heights [nz], 1/dz [nz], the reciprocal
    // centre-to-centre distances across the z-faces, 2/(dz_{k-1} + dz_k) [nz + 1]
    // (zero on the lids), and the squared Smagorinsky length (Cs Delta_k)^2 with
    // Delta_k = (dx dy dz_k)^(1/3) [nz], in one buffer
    double *dz = nullptr;
    const double *zc() const { return dz + nz; }
    const double *idz() const { return dz + 2 * nz; }
    const double *idzf() const { return dz + 3 * nz; }
    const double *cs2() const { return dz + 4 * nz + 1; }
    int nz = 0;
};

// Terrain-following coordinates (FP64 contexts): the geometry, the base state
// per cell and the work arrays of the terrain kernels, in one allocation.
struct Terrain {
    bool on = false;
    double beta = 1.0;
    // s_k = (1 - zeta_k / z_t)^beta [nz + 1]; the mean of each cell's four
    // corner heights [ny][nx]; physical cell heights [n]
    double *s = nullptr, *hb = nullptr, *Hc = nullptr;
    // base state per cell [n]
    double *rho0 = nullptr, *theta0 = nullptr, *Theta0 = nullptr, *p0 = nullptr, *pi0 = nullptr;
    // rho Omega on z-faces [nw]; theta^t [n]; the substeps' rho'' before the
    // implicit part [n]; Thomas factors c', d' on z-faces [nw]
    double *om = nullptr, *tht = nullptr, *rh = nullptr, *cp = nullptr, *dp = nullptr;
    // h_zeta = Hc / dz_k per cell [n]; the metric part M of Omega'' of the old
    // and new horizontal momenta on z-faces [nw]
    double *J = nullptr, *mo = nullptr, *mn = nullptr;
    // face metrics: h_zeta on x- and y-faces, h_xi on x-faces, h_eta on
    // y-faces [n each]; h_xi and h_eta on z-faces [nw each]
    double *JU = nullptr, *JV = nullptr, *hxU = nullptr, *heV = nullptr, *hxW = nullptr, *heW = nullptr;
    // physical distance of the centres above and below each cell [n]
    double *dzc = nullptr;
    void *mem = nullptr;
    std::vector<double> Hc_host, zc_host;  // for erf_terrain_heights
};

}  // namespace erfk

namespace erfk {
// A kernel launch recorded instead of enqueued (for a batched ensemble step):
// the batched instance of the kernel, the context's own grid and block, the
// dynamic LDS, and the bytes of the argument structure.
using BatchFn = hipError_t (*)(const void *args, BatchMap map, int blocks, dim3 block, size_t lds, hipStream_t st,
                               bool prepare);
struct LaunchRec {
    BatchFn fn;
    dim3 grid, block;
    size_t lds;
    std::vector<unsigned char> args;
};
struct Recorder {
    std::vector<LaunchRec> recs;
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
    erfk::MlpState mlp;
    erfk::Anel an;
    bool have_base = false;
    erf_status sticky = ERF_OK;
    std::string err;
    int64_t ws_bytes = 0;
    int device = 0;
    void *arena = nullptr;  // the single device allocation behind the workspace
    // acoustic substep launch shape chosen by erf_autotune (0: the default rule)
    int tune_levels = 0, tune_rows = 0;
    // while set, launches are recorded here instead of enqueued (the batched
    // ensemble step records each member's step once, then replays batches)
    erfk::Recorder *rec = nullptr;
    // a member of an ensemble: its slow right-hand side keeps the single-level
    // tendency kernel (the z-marching one is not used inside ensemble graphs)
    bool member = false;
    // terrain-following coordinates (erf_set_terrain)
    erfk::Terrain ter;
    // kernel timing (erf_timing_begin / erf_timing_end)
    int timed_kernel = -1;
    int timed_count = 0;
    std::vector<hipEvent_t> timing_events;  // start, stop pairs
};

namespace erfk {

// kernel ids for the timing instrumentation
enum KernelId { K_PREP, K_MUT, K_STRESS, K_RHS, K_STAGE_INIT, K_COEF, K_SUBSTEP, K_FINALIZE, K_MIXRATIO, K_SCALAR,
                K_MLP, K_MLP_DIV, K_KESSLER, K_SSP, K_DIVFFTX, K_FFTY, K_POISSON, K_IFFTX, K_PROJECT, K_MOST,
                K_TKE, K_TER_RHS, K_TER_UV, K_TER_COL, K_TER_M, K_TER_HAT, K_COUNT };
inline const char *kernel_name(int id)
{
    static const char *names[K_COUNT] = {"prep", "mut", "stress", "rhs", "stage_init", "coef", "substep",
                                         "finalize", "mixing_ratio", "scalar", "mlp", "mlp_div", "kessler",
                                         "ssp_update", "div_fftx", "ffty", "poisson_z", "ifftx", "project",
                                         "most", "tke", "ter_rhs", "ter_uv", "ter_tri", "ter_m", "ter_hat"};
    return (id >= 0 && id < K_COUNT) ? names[id] : "";
}
// The batched instance KB of a kernel, launched over the block ranges of map
// (prepare: only allow its dynamic LDS, before a graph capture).
template <typename Args, void (*KB)(const Args *, BatchMap)>
hipError_t batch_launch(const void *args, BatchMap map, int blocks, dim3 block, size_t lds, hipStream_t st,
                        bool prepare)
{
    if (prepare)
        return lds > 65536 ? hipFuncSetAttribute((const void *)KB, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                           : hipSuccess;
    const Args *ap = (const Args *)args;
    void *argv[] = {(void *)&ap, (void *)&map};
    return hipLaunchKernel((const void *)KB, dim3(blocks), block, argv, lds, st);
}
// record one launch of a recording context
template <typename Args>
void record(erf_ctx *c, BatchFn fn, dim3 grid, dim3 block, size_t lds, const Args &a)
{
    LaunchRec r{fn, grid, block, lds, {}};
    r.args.assign((const unsigned char *)&a, (const unsigned char *)&a + sizeof(Args));
    c->rec->recs.push_back(std::move(r));
}
// Enqueue kernel K on the context's stream, or, while the context records,
// record the launch with KB, K's batched instance.
template <typename Args, void (*K)(Args), void (*KB)(const Args *, BatchMap)>
void run(erf_ctx *c, dim3 grid, dim3 block, size_t lds, const Args &a)
{
    if (c->rec) {
        record(c, &batch_launch<Args, KB>, grid, block, lds, a);
        return;
    }
    void *argv[] = {(void *)&a};
    (void)hipLaunchKernel((const void *)K, grid, block, argv, lds, c->stream);
}

// bracket a launch with events when its kernel is being timed
inline void timing_start(erf_ctx *c, int id)
{
    if (c->rec) return;
    if (c->timed_kernel == id && 2 * c->timed_count + 1 < (int)c->timing_events.size())
        (void)hipEventRecord(c->timing_events[2 * c->timed_count], c->stream);
}
inline void timing_stop(erf_ctx *c, int id)
{
    if (c->rec) return;
    if (c->timed_kernel == id && 2 * c->timed_count + 1 < (int)c->timing_events.size()) {
        (void)hipEventRecord(c->timing_events[2 * c->timed_count + 1], c->stream);
        ++c->timed_count;
    }
}

// ---------------------------------------------------------------------------
// launchers (host), one translation unit each
// ---------------------------------------------------------------------------
// rhs.hip
// rq: the state's scalars (read by moist contexts only; may be NULL otherwise)
hipError_t launch_slow_rhs(erf_ctx *c, const void *const S[5], const void *rq, void *const R[5]);
// primitive fields of S (theta, p', u, v, w) into the workspace only
hipError_t launch_prep(erf_ctx *c, const void *const S[5]);
// acoustic.hip
// rq_t: the stage state's scalars (read by moist contexts only)
hipError_t launch_acoustic_stage(erf_ctx *c, const void *const Sn[5], const void *const St[5], const void *rq_t,
                                 const void *const Rt[5], int n_sub, double dtau, void *const Sout[5],
                                 void *Fu, void *Fv, void *Fw);
// scalars.hip
hipError_t launch_scalar_advance(erf_ctx *c, const void *rqn, const void *rho_t, const void *rq_t,
                                 const void *Fu, const void *Fv, const void *Fw, double dts, void *rq_out);
// mlp.hip
hipError_t mlp_pack(erf_ctx *c);
hipError_t launch_mlp_closure(erf_ctx *c, const void *rho, void *const R[5]);
int closure_count_slots();
hipError_t launch_mlp_forward(erf_ctx *c, const float *x, int64_t n, float *y);
hipError_t launch_features(erf_ctx *c, double *feat);
hipError_t launch_box_filter(erf_ctx *c, const void *const S[5], int r, double Cs, double Pr_t,
                             double *const C[5], double *targets);
size_t stat_partials(int64_t n);
hipError_t launch_col_stats(erf_ctx *c, const double *X, int64_t n, int ncol, double *mean, double *sd,
                            double *part);
hipError_t launch_standardize(erf_ctx *c, const double *X, int64_t n, int ncol, const double *mean,
                              const double *sd, float *out);
// fused training pass: blocks for a batch of n samples (a function of n only,
// so that every caller of the same n gets the same partial sums), its FP32
// and FP64 partial space, and the packed BF16 weight operands (MlpState::tw)
int train_blocks(int64_t n);
size_t train_part_floats(int64_t n);
size_t train_part_doubles(int64_t n);
size_t train_weight_shorts();
// allow the training kernel its LDS (once per device, before any capture)
hipError_t mlp_train_prepare();
// loss and gradient of n samples; part and dpart hold train_part_floats(n)
// and train_part_doubles(n) values, every one written before it is read
hipError_t launch_loss_grad(erf_ctx *c, const float *X, const float *T, int64_t n, float *G, double *loss_dev,
                            float *part, double *dpart);
hipError_t launch_adam(erf_ctx *c, double lr, int64_t step);
// micro.hip: Kessler microphysics over dt on S (rho, rho theta, rho q);
// precip (may be null) accumulates the rain reaching the ground
hipError_t launch_kessler(erf_ctx *c, void *rho, void *rt, void *rq, double dt, double *precip);
// anelastic.hip (FP64 contexts): stage 1 out = Sn + dt R1, stage 2 out = Sn +
// dt (R1 + R2) / 2 for rho theta and the face momenta (out may alias Sn);
// out_q = (a + b) / 2 over count values; the projection of the face momenta
// ru, rv, rw in place, adding psi = phi / dt to the context's pressure
hipError_t launch_ssp_update(erf_ctx *c, int stage, const void *const Sn[5], const void *const R1[5],
                             const void *const R2[5], void *const out[5], double dt);
hipError_t launch_qavg(erf_ctx *c, const void *a, const void *b, void *out, int64_t count);
hipError_t launch_project(erf_ctx *c, void *ru, void *rv, void *rw, double dt);
// x-lines per block of the y transform for an ny-point transform
int anel_ffty_cols(int nx, int ny);
// terrain.hip (FP64 contexts with terrain): the slow right-hand side and one
// RK stage of acoustic substeps with the metric terms
hipError_t launch_terrain_rhs(erf_ctx *c, const void *const S[5], void *const R[5]);
// (Fu, Fv, Fw: the stage-averaged fluxes for scalars, rho Omega vertically; null: none)
hipError_t launch_terrain_stage(erf_ctx *c, const void *const Sn[5], const void *const St[5],
                                const void *const Rt[5], int n_sub, double dtau, void *const Sout[5],
                                void *Fu, void *Fv, void *Fw);
// diag.hip
size_t diag_slots_needed();
hipError_t launch_diagnostics(erf_ctx *c, const void *const S[6], double *host_out);

}  // namespace erfk
