// acoustic.hip -- one RK stage of semi-implicit acoustic substepping (App. C of
// the ERF paper, Sec. 3.1).  Bulk fields are stored as T (double, or float with
// rho and rho*theta as perturbations about the base state).  The explicit
// horizontal part of a substep (U'', V'' and the horizontal divergences of
// Theta'' and rho'') is computed in T; the frozen coefficients, the right-hand
// sides of the vertical W'' rows, their factors, the Thomas sweeps and the
// implicit finish of Theta'' and rho'' are always double.
//
// Kernels of one stage:
//   k_stage_init  S'' = S^n - S^t, frozen theta^t and Exner pi^t, zero sums
//                 (moist: the pressure-gradient factor, the moist Exner
//                 function and rho_d / rho_m of the stage state)
//                 (a stage that starts from S^t = S^n with a single substep,
//                 the first of RK3, has S'' = 0 exactly: its stage init and
//                 substep are instances that neither write nor read the zeros)
//   k_coef        per column: the tridiagonal rows of the implicit W'' equation
//                 (they depend only on S^t and dtau) factorised once per stage;
//                 only the pivots 1/den_k are kept, the off-diagonals are
//                 recomputed by the substep from values it loads anyway
//   k_substep     one launch per substep, everything of the substep fused:
//                 U'', V'' forward step with the forward-predicted Theta''
//                 (divergence damping); explicit parts of Theta'', rho'';
//                 right-hand sides of the W'' rows; Thomas solve; update.
//   k_finalize    S_out = S^t + S'', stage-averaged momenta
//
// k_substep layout.  A block owns a tile of 64 columns (TX x TY, TX*TY = 64,
// one lane per column) and all nz levels.  Its KG wavefronts split the levels
// into chunks of L consecutive levels; the explicit work is parallel over
// levels and keeps the per-level results (That in LDS up to 8 levels per
// wavefront, Rhat in registers; theta^t on faces is recomputed from the cache
// where needed).  The W'' right-hand sides go to LDS; the two Thomas sweeps (LU
// factors frozen per stage) run as chunked linear recurrences, each wavefront
// on its own rows with one short carry chain between chunks; every wavefront
// then finishes its levels.  Neighbour columns'
// U'', V'' on the tile's far faces are recomputed by the lane that needs them
// (U'', V'' are double-buffered so no lane reads a value another block has
// already overwritten).  Blocks are remapped so that the tiles one XCD
// processes form a contiguous band of the domain and tile halos hit its L2.
#include "erf_internal.h"


namespace erfk {
namespace {

constexpr int kLanes = 64;  // columns per tile (one wavefront)

__device__ __forceinline__ int cidx(const Dims &d, int i, int j, int k) { return (k * d.ny + j) * d.nx + i; }

template <typename T>
struct StageArgs {
    Dims d;
    double dx, dy;
    const double *dz, *idz, *idzf;
    double g, b1, b2, bd, dtau;
    const double *rho0, *pi0, *Theta0;
    // moist: base-state vapour and total density rho0 (1 + qv0); the stage
    // state's rho q_v, rho q_c, rho q_r (n apart)
    const double *qv0, *rho0t;
    const T *t_q;
    // S^n, S^t, R^t
    const T *n_r, *n_t, *n_u, *n_v, *n_w;
    const T *t_r, *t_t, *t_u, *t_v, *t_w;
    const T *R_r, *R_t, *R_u, *R_v, *R_w;
    // frozen fields: theta^t and the pressure-gradient factor pi^t (moist: pi^t
    // (1 + R_v/R_d q_v)/(1 + q_v + q_c)); moist also the Exner function pi^t and
    // rho_d / rho_m, read by k_coef for the buoyancy coefficient
    T *tht, *pit, *pex, *rdm;
    // perturbations (Theta'' three levels, U'' and V'' double-buffered) and sums
    T *T2cur, *T2prv, *T2nxt, *r2, *u2in, *u2out, *v2in, *v2out, *w2, *su, *sv, *sw;
    int sums;
    // coefficients on z-faces: C_k (bulk precision) and the Thomas pivots
    // m_k = 1 / den_k (double)
    T *cC;
    double *cm;
    // tiles
    int TX, TY, ntx, nty;
    // stage end S^t + S'' (written by the last substep when no flux sums are kept)
    T *o_r, *o_t, *o_u, *o_v, *o_w;
};

template <typename T, bool kZero, bool kMoist>
__device__ __forceinline__ void k_stage_init_body(StageArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    int i = vb.x * blockDim.x + threadIdx.x;
    int j = vb.y * blockDim.y + threadIdx.y;
    int k = vb.z;  // 0..nz (the extra plane handles the top z-face)
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    // every value is read and written once: streaming accesses throughout
    if constexpr (kZero) {
        // S'' = 0: only the lid faces of W'' are stored (no substep writes them)
        if (k == 0 || k == d.nz) st_stream(a.w2 + c, (T)0);
    } else {
        st_stream(a.w2 + c, (T)((double)ld_stream(a.n_w + c) - (double)ld_stream(a.t_w + c)));
    }
    if (a.sums) st_stream(a.sw + c, (T)0);
    if (k == d.nz) return;
    const double T0 = a.Theta0[k];
    const T tt = ld_stream(a.t_t + c), tr = ld_stream(a.t_r + c);
    const double Tt = kPert<T> ? T0 + (double)tt : (double)tt;
    const double rt = kPert<T> ? a.rho0[k] + (double)tr : (double)tr;
    st_stream(a.tht + c, (T)(Tt / rt));
    if constexpr (kMoist) {
        // Moist: the Exner function of Theta (1 + eps q_v) (Sec. 2.1), from the
        // perturbation X/X0 - 1 about the moist base state in FP32 storage; the
        // horizontal pressure gradient and A use gamma R_d pi^t (1 + eps q_v) /
        // (1 + q_v + q_c), the exact dp/dTheta over the moisture factor of the
        // momentum equation
        const double qv = (double)ld_stream(a.t_q + c) / rt, qc = (double)ld_stream(a.t_q + c + d.n) / rt;
        const double qr = (double)ld_stream(a.t_q + c + 2 * d.n) / rt;
        const double fv = 1.0 + kEpsV * qv;
        double pex;
        if constexpr (kPert<T>) {
            const double qv0 = a.qv0[k];
            const double x = ((double)tt * fv + kEpsV * T0 * (qv - qv0)) / (T0 * (1.0 + kEpsV * qv0));
            pex = a.pi0[k] * exp((kGamma - 1.0) * log1p(x));
        } else {
            pex = pow(kRd * (Tt * fv) / kP00, kGamma - 1.0);
        }
        st_stream(a.pit + c, (T)(pex * (fv / (1.0 + qv + qc))));
        st_stream(a.pex + c, (T)pex);
        st_stream(a.rdm + c, (T)(1.0 / (1.0 + qv + qc + qr)));
    } else {
        // Exner function of the stage state: (R_d Theta / P00)^(gamma - 1); from
        // the perturbation in FP32 storage, pi0 (1 + Theta'/Theta0)^(gamma - 1)
        if constexpr (kPert<T>)
            st_stream(a.pit + c, (T)(a.pi0[k] * exp((kGamma - 1.0) * log1p((double)tt / T0))));
        else
            st_stream(a.pit + c, (T)pow(kRd * Tt / kP00, kGamma - 1.0));
    }
    if constexpr (!kZero) {
        st_stream(a.T2cur + c, (T)((double)ld_stream(a.n_t + c) - (double)tt));
        st_stream(a.r2 + c, (T)((double)ld_stream(a.n_r + c) - (double)tr));
        st_stream(a.u2in + c, (T)((double)ld_stream(a.n_u + c) - (double)ld_stream(a.t_u + c)));
        st_stream(a.v2in + c, (T)((double)ld_stream(a.n_v + c) - (double)ld_stream(a.t_v + c)));
    }
    if (a.sums) {
        st_stream(a.su + c, (T)0);
        st_stream(a.sv + c, (T)0);
    }
}
template <typename T, bool kZero, bool kMoist>
__global__ __launch_bounds__(256) void k_stage_init(StageArgs<T> a)
{
    k_stage_init_body<T, kZero, kMoist>(a, hw_block());
}
template <typename T, bool kZero, bool kMoist>
__global__ __launch_bounds__(256) void k_stage_init_batch(const StageArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_stage_init_body<T, kZero, kMoist>(args[m], vb);
}

// Off-diagonal entries of the W'' row on face k (1 <= k <= nz - 1): lo
// multiplies W''_{k-1}, up multiplies W''_{k+1}.  A = gamma R_d pi^t and C on
// face k; tfm, tfp = theta^t on faces k - 1 and k + 1 (zero on the lids);
// 1/dz of the levels below and above the face and 2/(dz_{k-1} + dz_k); D =
// (dtau b2)^2.  k_coef and the substep evaluate the rows with this one
// function on the same inputs, so the substep's alpha_k = lo_k m_k and c'_k =
// up_k m_k are bitwise those of the factorisation.
__device__ __forceinline__ void w_row_offdiag(double D, double g, double A, double C, double tfm, double tfp,
                                              double idzm, double idzk, double idzf, int k, int nz, double &lo,
                                              double &up)
{
    lo = (k == 1) ? 0.0 : -D * (A * tfm * idzm * idzf + 0.5 * C * tfm * idzm - 0.5 * g * idzm);
    up = (k == nz - 1) ? 0.0 : -D * (A * tfp * idzk * idzf - 0.5 * C * tfp * idzk + 0.5 * g * idzk);
}

// Tridiagonal rows for W'' at interior faces k = 1..nz-1.  Substituting
// Theta''_new = That - dtau b2 delta_z(W theta_f)/dz and rho''_new = Rhat -
// dtau b2 delta_z(W)/dz into the W'' equation of App. C couples W_{k-1}, W_k,
// W_{k+1} with coefficients of the frozen state only.  Factorised here (Thomas,
// no pivoting; the rows are diagonally dominant).  C enters the rows as
// stored (rounded to the bulk type), as the substep reads it.  kMoist: C from
// the moist Exner function, the base state's total density and the face mean
// of rho_d / rho_m (App. C with the moist equation of state).
template <typename T, bool kMoist>
__device__ __forceinline__ void k_coef_body(StageArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    int i = vb.x * blockDim.x + threadIdx.x;
    int j = vb.y * blockDim.y + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int col = j * d.nx + i, nxy = d.nxy, nz = d.nz;
    const double D = a.dtau * a.dtau * a.b2 * a.b2, g = a.g;
    // The elimination is serial in k, but its inputs are not: they are loaded
    // for kChunk levels at a time (levels clamped into the column, unused
    // values at the lids), so that a column waits for one memory round trip
    // per chunk rather than one per level.
    constexpr int kChunk = 8;
    auto lev = [&](int k) { return col + min(max(k, 0), nz - 1) * nxy; };
    double cprev = 0.0;
    for (int k0 = 1; k0 < nz; k0 += kChunk) {
        double P[kChunk + 1], TT[kChunk + 1], H[kChunk + 3];
        double PX[kMoist ? kChunk + 1 : 1], RD[kMoist ? kChunk + 1 : 1];
#pragma unroll
        for (int q = 0; q <= kChunk; ++q) {
            P[q] = a.pit[lev(k0 - 1 + q)];      // pressure-gradient factor (dry: Exner) at level k0 - 1 + q
            TT[q] = a.t_t[lev(k0 - 1 + q)];     // rho theta (stored form)
            if constexpr (kMoist) {
                PX[q] = a.pex[lev(k0 - 1 + q)];  // moist Exner function
                RD[q] = a.rdm[lev(k0 - 1 + q)];  // rho_d / rho_m
            }
        }
#pragma unroll
        for (int q = 0; q < kChunk + 3; ++q) H[q] = a.tht[lev(k0 - 2 + q)];  // theta at k0 - 2 + q
        // theta on face m (between levels m - 1 and m); zero on the lids
        auto tface = [&](int m, int q) { return (m <= 0 || m >= nz) ? 0.0 : 0.5 * (H[q] + H[q + 1]); };
#pragma unroll
        for (int l = 0; l < kChunk; ++l) {
            const int k = k0 + l;
            if (k >= nz) break;
            const int c = col + k * nxy;
            double pif = 0.5 * (P[l] + P[l + 1]);
            double A = kGamma * kRd * pif;
            const double Tm = kPert<T> ? a.Theta0[k - 1] + TT[l] : TT[l];
            const double Tk = kPert<T> ? a.Theta0[k] + TT[l + 1] : TT[l + 1];
            T Cst;
            if constexpr (kMoist) {
                const double pxf = 0.5 * (PX[l] + PX[l + 1]);
                Cst = (T)(g * 0.5 * (a.rho0t[k - 1] + a.rho0t[k]) * (kRd / kCv) *
                          (pxf / (0.5 * (a.pi0[k - 1] + a.pi0[k]))) / (0.5 * (Tm + Tk)) * (0.5 * (RD[l] + RD[l + 1])));
            } else {
                Cst = (T)(g * 0.5 * (a.rho0[k - 1] + a.rho0[k]) * (kRd / kCv) *
                          (pif / (0.5 * (a.pi0[k - 1] + a.pi0[k]))) / (0.5 * (Tm + Tk)));
            }
            const double C = Cst;
            const double idzm = a.idz[k - 1], idz = a.idz[k], idzf = a.idzf[k];
            const double tfm = tface(k - 1, l), tf = tface(k, l + 1), tfp = tface(k + 1, l + 2);
            double lo, up;
            w_row_offdiag(D, g, A, C, tfm, tfp, idzm, idz, idzf, k, nz, lo, up);
            double di = 1.0 + D * (A * tf * (idz + idzm) * idzf + 0.5 * C * tf * (idzm - idz) - 0.5 * g * (idzm - idz));
            double den = (k == 1) ? di : di - lo * cprev;
            double m = 1.0 / den;
            st_stream(a.cm + c, m);
            st_stream(a.cC + c, Cst);
            cprev = up * m;
        }
    }
}
template <typename T, bool kMoist>
__global__ __launch_bounds__(256) void k_coef(StageArgs<T> a)
{
    k_coef_body<T, kMoist>(a, hw_block());
}
template <typename T, bool kMoist>
__global__ __launch_bounds__(256) void k_coef_batch(const StageArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_coef_body<T, kMoist>(args[m], vb);
}

// Phase 1 of a substep on one wavefront's levels of one column: U'', V'' with
// the forward-predicted Theta'', the explicit parts of Theta'' (in LDS, thl,
// up to 8 levels per wavefront; else in th) and rho'' (rh), and the
// right-hand sides of the W'' rows (rbuf; chunk-end e, f in bnd).  Keeping few
// values live across the level loop leaves registers for more loads in
// flight.  The pointers are restrict: the arrays
// written here (U'', V'' of the next level, their sums) are never read here,
// so the loads of later levels may be issued ahead of earlier stores.  kZero:
// S'' is zero on entry (Theta'', U'', V'', rho'', W'' are not read; the same
// arithmetic runs on zeros, so the results are those of reading them).
template <typename T, int kLevels, bool kLast, bool kZero, bool kSums>
__device__ __forceinline__ void substep_explicit(
    const T *__restrict__ t_u, const T *__restrict__ t_v, const T *__restrict__ T2cur, const T *__restrict__ T2prv, const T *__restrict__ pit, const T *__restrict__ tht,
    const T *__restrict__ u2in, const T *__restrict__ v2in, const T *__restrict__ R_u, const T *__restrict__ R_v,
    const T *__restrict__ R_t, const T *__restrict__ R_r, const T *__restrict__ R_w, const T *__restrict__ w2,
    const T *__restrict__ r2, const T *__restrict__ cC, const double *__restrict__ idz_t,
    const double *__restrict__ idzf_t, T *__restrict__ u2out, T *__restrict__ v2out, T *__restrict__ su,
    T *__restrict__ sv, int sums, double *rbuf, double *bnd, bool act, int col, int nxy, int nz, int k0, int g,
    int lane, int o_e, int o_w, int o_n, int o_s, double dt, double b1, double b2, double gr, double bd,
    double gRd, double idx, double idy, double D, double (&th)[kLevels], double *thl, double (&rh)[kLevels],
    double (&lo)[kLevels <= 8 ? kLevels : 1], double (&up)[kLevels <= 8 ? kLevels : 1], double &e_first,
    double &f_first)
{
    using R = T;  // arithmetic type of the explicit horizontal part
    // an S'' value on entry
    auto in = [&](const T *__restrict__ p, int i) -> R {
        if constexpr (kZero)
            return R(0);
        else
            return p[i];
    };
    const R dtR = (R)dt, gRdR = (R)gRd, idxR = (R)idx, idyR = (R)idy, bdR = (R)bd, h = R(0.5);
    if (act && k0 < nz) {
        double e_prev = 0.0, f_prev = 0.0, tf_prev = 0.0;
        double pi_below = (k0 > 0) ? pit[col + (k0 - 1) * nxy] : 0.0;
        double th_below = (k0 > 0) ? tht[col + (k0 - 1) * nxy] : 0.0;
        double w_lo = in(w2, col + k0 * nxy);
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            const int k = k0 + l;
            if (k < nz) {
                const int c = col + k * nxy;
                // the running flux sums (kSums: scalars are transported), read
                // with this level's other loads and written at its end
                double su0 = 0.0, sv0 = 0.0;
                if constexpr (kSums) {
                    su0 = su[c];
                    sv0 = sv[c];
                }
                // forward-predicted Theta'' at the centre and its four neighbours
                const R Tc = in(T2cur, c);
                const R ttc = Tc + bdR * (Tc - in(T2prv, c));
                const R Tw = in(T2cur, c + o_w), Te = in(T2cur, c + o_e), Ts = in(T2cur, c + o_s),
                        Tn = in(T2cur, c + o_n);
                const R ttw = Tw + bdR * (Tw - in(T2prv, c + o_w));
                const R tte = Te + bdR * (Te - in(T2prv, c + o_e));
                const R tts = Ts + bdR * (Ts - in(T2prv, c + o_s));
                const R ttn = Tn + bdR * (Tn - in(T2prv, c + o_n));
                const R pc = pit[c], pw = pit[c + o_w], pe = pit[c + o_e], ps = pit[c + o_s], pn = pit[c + o_n];
                // U'' on this column's x-face and on the next one, V'' likewise
                const R Uw = in(u2in, c) + dtR * (-gRdR * (h * (pw + pc)) * (ttc - ttw) * idxR + R_u[c]);
                const R Ue = in(u2in, c + o_e) + dtR * (-gRdR * (h * (pc + pe)) * (tte - ttc) * idxR + R_u[c + o_e]);
                const R Vs = in(v2in, c) + dtR * (-gRdR * (h * (ps + pc)) * (ttc - tts) * idyR + R_v[c]);
                const R Vn = in(v2in, c + o_n) + dtR * (-gRdR * (h * (pc + pn)) * (ttn - ttc) * idyR + R_v[c + o_n]);
                if constexpr (kLast) {
                    // the stage's last substep writes S^t + S'' (u2out, v2out
                    // point to the stage-end momenta; S'' rounded as if stored)
                    st_stream(u2out + c, (T)((double)ld_stream(t_u + c) + (double)(T)Uw));
                    st_stream(v2out + c, (T)((double)ld_stream(t_v + c) + (double)(T)Vs));
                } else {
                    st_stream(u2out + c, (T)Uw);
                    st_stream(v2out + c, (T)Vs);
                }
                // explicit parts of Theta'' and rho'': horizontal divergences in
                // the arithmetic type, the vertical terms in double
                const R thcR = tht[c];
                const R thx0 = h * ((R)tht[c + o_w] + thcR), thx1 = h * (thcR + (R)tht[c + o_e]);
                const R thy0 = h * ((R)tht[c + o_s] + thcR), thy1 = h * (thcR + (R)tht[c + o_n]);
                const double hdiv_t = (Ue * thx1 - Uw * thx0) * idxR + (Vn * thy1 - Vs * thy0) * idyR;
                const double hdiv_r = (Ue - Uw) * idxR + (Vn - Vs) * idyR;
                const double thc = thcR;
                // the level above, clamped at the lid (its value unused there)
                const double th_above = tht[c + (k < nz - 1 ? nxy : 0)];
                const double tfk = (k == 0) ? 0.0 : 0.5 * (th_below + thc);
                const double tfk1 = (k == nz - 1) ? 0.0 : 0.5 * (thc + th_above);
                const double w_hi = in(w2, c + nxy);
                const double idzk = idz_t[k];
                // values read by this lane only: streaming loads
                const double r2c = kZero ? 0.0 : (double)ld_stream(r2 + c);
                const double Rt = ld_stream(R_t + c), Rr = ld_stream(R_r + c);
                const double that = Tc + dt * (-hdiv_t - b1 * (w_hi * tfk1 - w_lo * tfk) * idzk + Rt);
                const double rhat = r2c + dt * (-hdiv_r - b1 * (w_hi - w_lo) * idzk + Rr);
                const double e = b1 * Tc + b2 * that, f = b1 * r2c + b2 * rhat;
                if (l == 0) {
                    e_first = e;
                    f_first = f;
                } else {
                    // right-hand side of the W'' row on face k
                    const double idzf = idzf_t[k];
                    const double A = gRd * (0.5 * (pi_below + pc));
                    const double C = ld_stream(cC + c);
                    rbuf[k * kLanes + lane] = w_lo + dt * (-A * (e - e_prev) * idzf + 0.5 * C * (e + e_prev) -
                                                           0.5 * gr * (f + f_prev) + ld_stream(R_w + c));
                    // the row's off-diagonals (up to 8 levels: kept for the sweeps)
                    if constexpr (kLevels <= 8)
                        w_row_offdiag(D, gr, A, C, tf_prev, tfk1, idz_t[k - 1], idzk, idzf, k, nz, lo[l], up[l]);
                }
                if constexpr (kLevels <= 8)
                    thl[k * kLanes + lane] = that;
                else
                    th[l] = that;
                rh[l] = rhat;
                e_prev = e;
                f_prev = f;
                pi_below = pc;
                th_below = thc;
                tf_prev = tfk;
                w_lo = w_hi;
                if (l == kLevels - 1 || k == nz - 1) {
                    bnd[(g * 2 + 0) * kLanes + lane] = e;
                    bnd[(g * 2 + 1) * kLanes + lane] = f;
                }
                if constexpr (kSums) {
                    su[c] = (T)(su0 + Uw);
                    sv[c] = (T)(sv0 + Vs);
                }
            }
        }
    }
}

// One fused acoustic substep.  blockDim = (64, KG), kLevels levels per
// wavefront; dynamic LDS holds the (nz + 1) x 64 solve buffer and the
// chunk-boundary values.
template <typename T, int kLevels, bool kLast, bool kZero, bool kSums>
__device__ __forceinline__ void k_substep_body(StageArgs<T> a, VBlock vb)
{
    extern __shared__ double lds[];
    const Dims &d = a.d;
    const int nz = d.nz, nxy = d.nxy;
    // blockDim.x is one wavefront, so the level chunk g is uniform per
    // wavefront: said so to the compiler, level indices live in scalar
    // registers and per-level tables (1/dz) are read with scalar loads
    const int lane = threadIdx.x, g = __builtin_amdgcn_readfirstlane(threadIdx.y);
    double *rbuf = lds;                     // [(nz + 1) * 64]
    double *bnd = lds + (nz + 1) * kLanes;  // [KG][2][64]
    double *thl = bnd + 2 * blockDim.y * kLanes;  // [nz][64] when kLevels <= 8

    const int tile = xcd_remap(vb.x, vb.gx);
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int i = tx * a.TX + lane % a.TX, j = ty * a.TY + lane / a.TX;
    const bool act = (i < d.nx) && (j < d.ny);
    const int ic = act ? i : 0, jc = act ? j : 0;
    const int col = jc * d.nx + ic;
    const int o_e = wrap_idx(ic + 1, d.nx) - ic, o_w = wrap_idx(ic - 1, d.nx) - ic;
    const int o_n = (wrap_idx(jc + 1, d.ny) - jc) * d.nx, o_s = (wrap_idx(jc - 1, d.ny) - jc) * d.nx;
    const double dt = a.dtau, b1 = a.b1, b2 = a.b2, gr = a.g, bd = a.bd;
    const double gRd = kGamma * kRd;
    const double idx = 1.0 / a.dx, idy = 1.0 / a.dy;

    const double D = dt * dt * b2 * b2;  // as in k_coef
    const int k0 = g * kLevels;
    double th[kLevels], rh[kLevels];
    double e_first = 0.0, f_first = 0.0;
    // Up to 8 levels per wavefront the rows' off-diagonals come out of phase 1
    // in registers and the pivots are loaded together, levels clamped into
    // the column so that no branch separates the loads: the sweeps then wait
    // on LDS only instead of one global round trip per level.  With 16 levels
    // the rows are evaluated where used, from loads of the frozen fields.
    constexpr bool kPre = kLevels <= 8;
    constexpr int kP = kPre ? kLevels : 1;
    double flo[kP], fup[kP], fcm[kP];

    // the off-diagonals of the row on face k (1 <= k <= nz - 1) from the
    // frozen fields, as phase 1 and k_coef evaluate them
    auto row_at = [&](int k, double &lo, double &up) {
        const int c = col + k * nxy;
        const double A = gRd * (0.5 * (a.pit[c - nxy] + a.pit[c]));
        const double C = a.cC[c];
        const double thm2 = a.tht[col + max(k - 2, 0) * nxy], thm = a.tht[c - nxy], thk = a.tht[c];
        const double thp = a.tht[col + min(k + 1, nz - 1) * nxy];
        const double tfm = (k - 1 <= 0) ? 0.0 : 0.5 * (thm2 + thm);
        const double tfp = (k + 1 >= nz) ? 0.0 : 0.5 * (thk + thp);
        w_row_offdiag(D, gr, A, C, tfm, tfp, a.idz[k - 1], a.idz[k], a.idzf[k], k, nz, lo, up);
    };

    // ---------------- phase 1: explicit work, W'' right-hand sides ----------
    substep_explicit<T, kLevels, kLast, kZero, kSums>(a.t_u, a.t_v, a.T2cur, a.T2prv, a.pit, a.tht, a.u2in, a.v2in, a.R_u, a.R_v, a.R_t, a.R_r, a.R_w,
                                 a.w2, a.r2, a.cC, a.idz, a.idzf, a.u2out, a.v2out, a.su, a.sv, a.sums, rbuf, bnd,
                                 act, col, nxy, nz, k0, g, lane, o_e, o_w, o_n, o_s, dt, b1, b2, gr, bd, gRd, idx,
                                 idy, D, th, thl, rh, flo, fup, e_first, f_first);
    if constexpr (kPre) {
#pragma unroll
        for (int l = 0; l < kLevels; ++l) fcm[l] = ld_stream(a.cm + col + min(k0 + l, nz - 1) * nxy);
    }
    __syncthreads();
    // row k0 of every chunk but the first needs the last level of the chunk below
    if (act && k0 < nz && g > 0) {
        const int k = k0, c = col + k * nxy;
        const double e_prev = bnd[((g - 1) * 2 + 0) * kLanes + lane];
        const double f_prev = bnd[((g - 1) * 2 + 1) * kLanes + lane];
        const double idzf = a.idzf[k];
        const double A = gRd * (0.5 * (a.pit[c - nxy] + a.pit[c]));
        const double C = a.cC[c];
        const double w0 = kZero ? 0.0 : (double)a.w2[c];
        rbuf[k * kLanes + lane] = w0 + dt * (-A * (e_first - e_prev) * idzf + 0.5 * C * (e_first + e_prev) -
                                                  0.5 * gr * (f_first + f_prev) + a.R_w[c]);
        if constexpr (kPre) row_at(k, flo[0], fup[0]);
    }
    __syncthreads();

    // ---------------- phase 2: the Thomas sweeps as chunked recurrences -----
    // Forward: d_k = r_k m_k - alpha_k d_{k-1}; backward: x_k = d_k - c'_k x_{k+1}.
    // Both are first-order linear recurrences with frozen coefficients, so each
    // wavefront runs them over its own rows from a zero carry, keeping the
    // carry multipliers (products of -alpha, resp. -c'); one wavefront then
    // chains the chunk ends, and every wavefront adds carry x multiplier.
    // Rows of chunk g: faces k0..k0+L-1 (face 0, the lid, is not a row).
    double *carry = bnd;  // reuses the boundary area: [KG][2][64]
    double mult[kLevels];
    const int rlo = k0 > 0 ? k0 : 1;
    const int rhi = (k0 + kLevels < nz ? k0 + kLevels : nz) - 1;  // last row of the chunk
    if (act && rlo <= rhi) {
        double dl = 0.0, pm = 1.0;
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            const int k = k0 + l;
            if (k >= rlo && k <= rhi) {
                const int c = col + k * nxy;
                double lo = 0.0, up = 0.0, m;
                if constexpr (kPre) {
                    lo = flo[l];
                    m = fcm[l];
                } else {
                    row_at(k, lo, up);
                    m = a.cm[c];
                }
                const double al = lo * m;  // alpha_k = a_k / den_k
                dl = rbuf[k * kLanes + lane] * m - al * dl;
                pm = -al * pm;
                rbuf[k * kLanes + lane] = dl;
                mult[l] = pm;
            }
        }
        carry[(g * 2 + 0) * kLanes + lane] = dl;  // local d at the chunk's last row
        carry[(g * 2 + 1) * kLanes + lane] = pm;  // its carry multiplier
    }
    __syncthreads();
    const int KG = blockDim.y;
    if (g == 0 && act) {
        double D = 0.0;
        for (int q = 0; q < KG; ++q) {
            if (q * kLevels >= nz) break;
            D = carry[(q * 2 + 0) * kLanes + lane] + carry[(q * 2 + 1) * kLanes + lane] * D;
            carry[(q * 2 + 0) * kLanes + lane] = D;  // true d at the end of chunk q
        }
    }
    __syncthreads();
    if (act && rlo <= rhi) {
        const double Dprev = g > 0 ? carry[((g - 1) * 2 + 0) * kLanes + lane] : 0.0;
        double xl = 0.0, qm = 1.0;
#pragma unroll
        for (int l = kLevels - 1; l >= 0; --l) {
            const int k = k0 + l;
            if (k >= rlo && k <= rhi) {
                const double dk = rbuf[k * kLanes + lane] + mult[l] * Dprev;
                double cp;  // c'_k = c_k / den_k
                if constexpr (kPre) {
                    cp = fup[l] * fcm[l];
                } else {
                    double lo, up;
                    row_at(k, lo, up);
                    cp = up * a.cm[col + k * nxy];
                }
                xl = dk - cp * xl;
                qm = -cp * qm;
                rbuf[k * kLanes + lane] = xl;
                mult[l] = qm;
            }
        }
    }
    // theta^t of the levels k0 - 1 .. k0 + kLevels (clamped) for phase 3, in
    // flight while the chunk ends are chained
    double thv[kP + 2];
    if constexpr (kPre) {
#pragma unroll
        for (int l = 0; l < kLevels + 2; ++l) thv[l] = a.tht[col + min(max(k0 + l - 1, 0), nz - 1) * nxy];
    }
    __syncthreads();
    if (act && rlo <= rhi) {
        carry[(g * 2 + 0) * kLanes + lane] = rbuf[rlo * kLanes + lane];  // local x at the first row
        carry[(g * 2 + 1) * kLanes + lane] = (g == 0) ? mult[1] : mult[0];  // rlo - k0 is 1 or 0
    }
    __syncthreads();
    if (g == 0 && act) {
        double X = 0.0;  // x above the last chunk: the lid
        for (int q = KG - 1; q >= 0; --q) {
            if (q * kLevels >= nz) continue;
            X = carry[(q * 2 + 0) * kLanes + lane] + carry[(q * 2 + 1) * kLanes + lane] * X;
            carry[(q * 2 + 0) * kLanes + lane] = X;  // true x at the first row of chunk q
        }
    }
    __syncthreads();

    // ---------------- phase 3: implicit parts of Theta'', rho''; W'' -------
    if (act && k0 < nz) {
        const double Xnext = (k0 + kLevels < nz) ? carry[((g + 1) * 2 + 0) * kLanes + lane] : 0.0;
        double wk1 = Xnext;  // W on the face above the current level
#pragma unroll
        for (int l = kLevels - 1; l >= 0; --l) {
            const int k = k0 + l;
            if (k < nz) {
                const int c = col + k * nxy;
                const double wk = (k >= rlo && k <= rhi) ? rbuf[k * kLanes + lane] + mult[l] * Xnext : 0.0;
                // theta^t on the faces below and above
                const int p = kPre ? l : 0;
                const double thc = kPre ? thv[p + 1] : (double)a.tht[c];
                const double tfl = (k == 0) ? 0.0 : 0.5 * ((kPre ? thv[p] : (double)a.tht[c - nxy]) + thc);
                const double tf1 = (k == nz - 1) ? 0.0 : 0.5 * (thc + (kPre ? thv[p + 2] : (double)a.tht[c + nxy]));
                const double idzk = a.idz[k];
                const double thk = (kLevels <= 8) ? thl[k * kLanes + lane] : th[l];
                const double Tn = thk - dt * b2 * (wk1 * tf1 - wk * tfl) * idzk;
                const double rn = rh[l] - dt * b2 * (wk1 - wk) * idzk;
                if constexpr (kLast) {
                    // stage end S^t + S'' in place of S'' (S'' rounded to the
                    // storage type first, as if it had been stored); the lid
                    // faces keep W^t + W'' as they are
                    st_stream(a.o_t + c, (T)((double)ld_stream(a.t_t + c) + (double)(T)Tn));
                    st_stream(a.o_r + c, (T)((double)ld_stream(a.t_r + c) + (double)(T)rn));
                    const int cw = k >= 1 ? c : col;  // face k, or the bottom lid
                    const T wlid_lo = kZero ? (T)0 : a.w2[cw];
                    st_stream(a.o_w + cw, (T)((double)ld_stream(a.t_w + cw) + (double)(k >= 1 ? (T)wk : wlid_lo)));
                    if (k == nz - 1) {
                        const int ct = col + nz * nxy;
                        const T wlid_hi = kZero ? (T)0 : a.w2[ct];
                        st_stream(a.o_w + ct, (T)((double)ld_stream(a.t_w + ct) + (double)wlid_hi));
                    }
                } else {
                    st_stream(a.T2nxt + c, (T)Tn);
                    st_stream(a.r2 + c, (T)rn);
                    if (k >= 1) {
                        st_stream(a.w2 + c, (T)wk);
                        if constexpr (kSums) a.sw[c] += wk;
                    }
                }
                wk1 = wk;
            }
        }
    }
}
template <typename T, int kLevels, bool kLast, bool kZero, bool kSums>
__global__ __launch_bounds__(1024) void k_substep(StageArgs<T> a)
{
    k_substep_body<T, kLevels, kLast, kZero, kSums>(a, hw_block());
}
template <typename T, int kLevels, bool kLast, bool kZero, bool kSums>
__global__ __launch_bounds__(1024) void k_substep_batch(const StageArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_substep_body<T, kLevels, kLast, kZero, kSums>(args[m], vb);
}

template <typename T>
struct FinArgs {
    Dims d;
    int n_sub;
    double b1;
    const T *t_r, *t_t, *t_u, *t_v, *t_w, *n_w;
    const T *T2, *r2, *u2, *v2, *w2, *su, *sv, *sw;
    T *o_r, *o_t, *o_u, *o_v, *o_w, *Fu, *Fv, *Fw;
};

// S_out = S^t + S''; stage-averaged momenta.  The W-sum accumulated only the
// new W'' of each substep; the beta-weighted average over substeps is
// b1 W''_0 + W''_1 + ... + W''_{N-1} + b2 W''_N = sum_{s=1..N} W''_s + b1 (W''_0 - W''_N).
// In both storages S^t and S'' are added as stored: full + perturbation in FP64,
// perturbation about the base state + perturbation in FP32.
template <typename T>
__device__ __forceinline__ void k_finalize_body(FinArgs<T> a, VBlock vb)
{
    const Dims &d = a.d;
    int i = vb.x * blockDim.x + threadIdx.x;
    int j = vb.y * blockDim.y + threadIdx.y;
    int k = vb.z;
    if (i >= d.nx || j >= d.ny) return;
    int c = cidx(d, i, j, k);
    // every value is read and written once: streaming accesses throughout
    double inv = 1.0 / a.n_sub;
    double wt = ld_stream(a.t_w + c), wN = ld_stream(a.w2 + c);
    if (a.Fw) {
        double w0 = (double)ld_stream(a.n_w + c) - wt;
        st_stream(a.Fw + c, (T)(wt + ((double)ld_stream(a.sw + c) + a.b1 * (w0 - wN)) * inv));
    }
    st_stream(a.o_w + c, (T)(wt + wN));
    if (k == d.nz) return;
    st_stream(a.o_r + c, (T)((double)ld_stream(a.t_r + c) + (double)ld_stream(a.r2 + c)));
    st_stream(a.o_t + c, (T)((double)ld_stream(a.t_t + c) + (double)ld_stream(a.T2 + c)));
    double ut = ld_stream(a.t_u + c), vt = ld_stream(a.t_v + c);
    st_stream(a.o_u + c, (T)(ut + (double)ld_stream(a.u2 + c)));
    st_stream(a.o_v + c, (T)(vt + (double)ld_stream(a.v2 + c)));
    if (a.Fu) st_stream(a.Fu + c, (T)(ut + (double)ld_stream(a.su + c) * inv));
    if (a.Fv) st_stream(a.Fv + c, (T)(vt + (double)ld_stream(a.sv + c) * inv));
}
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(FinArgs<T> a)
{
    k_finalize_body<T>(a, hw_block());
}
template <typename T>
__global__ __launch_bounds__(256) void k_finalize_batch(const FinArgs<T> *args, BatchMap bm)
{
    int m;
    VBlock vb;
    if (batch_block(bm, m, vb)) k_finalize_body<T>(args[m], vb);
}

}  // namespace

namespace {
// one substep launch: the instance for the level count, the stage end, a zero
// S'' on entry and the flux sums (never together with the stage end: the sums
// keep a separate finalize)
template <typename T, int L, bool kLast, bool kZero, bool kSums>
void substep_one(erf_ctx *cx, dim3 grid, dim3 block, size_t lds, const StageArgs<T> &a)
{
    run<StageArgs<T>, k_substep<T, L, kLast, kZero, kSums>, k_substep_batch<T, L, kLast, kZero, kSums>>(cx, grid, block,
                                                                                                       lds, a);
}
template <typename T, int L>
void launch_substep(erf_ctx *cx, bool last, bool zero, bool sums, dim3 grid, dim3 block, size_t lds,
                    const StageArgs<T> &a)
{
    if (last && zero)
        substep_one<T, L, true, true, false>(cx, grid, block, lds, a);
    else if (last)
        substep_one<T, L, true, false, false>(cx, grid, block, lds, a);
    else if (sums && zero)
        substep_one<T, L, false, true, true>(cx, grid, block, lds, a);
    else if (sums)
        substep_one<T, L, false, false, true>(cx, grid, block, lds, a);
    else if (zero)
        substep_one<T, L, false, true, false>(cx, grid, block, lds, a);
    else
        substep_one<T, L, false, false, false>(cx, grid, block, lds, a);
}

template <typename T, int L>
hipError_t allow_lds(size_t lds)
{
    const void *fn[6] = {(const void *)k_substep<T, L, false, false, false>,
                         (const void *)k_substep<T, L, true, false, false>,
                         (const void *)k_substep<T, L, false, true, false>,
                         (const void *)k_substep<T, L, true, true, false>,
                         (const void *)k_substep<T, L, false, false, true>,
                         (const void *)k_substep<T, L, false, true, true>};
    for (const void *f : fn) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t acoustic_t(erf_ctx *cx, const void *const Sn_[5], const void *const St_[5], const void *rq_t,
                      const void *const Rt_[5], int n_sub, double dtau, void *const Sout_[5], T *Fu, T *Fv, T *Fw)
{
    const T *Sn[5], *St[5], *Rt[5];
    T *Sout[5];
    for (int f = 0; f < 5; ++f) {
        Sn[f] = (const T *)Sn_[f];
        St[f] = (const T *)St_[f];
        Rt[f] = (const T *)Rt_[f];
        Sout[f] = (T *)Sout_[f];
    }
    const Dims &d = cx->d;
    Workspace &w = cx->ws;
    StageArgs<T> a{};
    a.d = d;
    a.dx = cx->grid.dx;
    a.dy = cx->grid.dy;
    a.dz = cx->base.dz;
    a.idz = cx->base.idz();
    a.idzf = cx->base.idzf();
    a.g = cx->prm.grav;
    a.b1 = 0.5 * (1.0 - cx->prm.beta_s);
    a.b2 = 0.5 * (1.0 + cx->prm.beta_s);
    a.dtau = dtau;
    a.rho0 = cx->base.rho0;
    a.pi0 = cx->base.pi0;
    a.Theta0 = cx->base.Theta0;
    a.qv0 = cx->base.qv0;
    a.rho0t = cx->base.rho0t;
    const bool moist = cx->prm.moist != 0;
    if (moist && !rq_t) return hipErrorInvalidValue;
    a.t_q = (const T *)rq_t;
    a.pex = (T *)w.pex;
    a.rdm = (T *)w.rdm;
    a.n_r = Sn[0]; a.n_t = Sn[1]; a.n_u = Sn[2]; a.n_v = Sn[3]; a.n_w = Sn[4];
    a.t_r = St[0]; a.t_t = St[1]; a.t_u = St[2]; a.t_v = St[3]; a.t_w = St[4];
    a.R_r = Rt[0]; a.R_t = Rt[1]; a.R_u = Rt[2]; a.R_v = Rt[3]; a.R_w = Rt[4];
    a.tht = (T *)w.th;
    a.pit = (T *)w.pit;
    a.r2 = (T *)w.r2;
    a.w2 = (T *)w.w2;
    a.su = (T *)w.su;
    a.sv = (T *)w.sv;
    a.sw = (T *)w.sw;
    a.sums = (Fu || Fv || Fw) ? 1 : 0;
    a.cm = w.cb;
    a.cC = (T *)w.cC;
    // tile shape: 64 columns as one row of 64 (measured 1.3 % faster than
    // 16 x 4 at 256 x 256) unless rows of 32 or 16 pad the grid less
    a.TY = kLanes / tile_width(d.nx, d.ny, kLanes);
    if (cx->tune_rows > 0) a.TY = cx->tune_rows;  // erf_autotune's choice
    a.TX = kLanes / a.TY;
    a.ntx = (d.nx + a.TX - 1) / a.TX;
    a.nty = (d.ny + a.TY - 1) / a.TY;
    // 8 levels per wavefront up to nz = 128 (registers without spills), 16 above
    const int L = cx->tune_levels > 0 ? cx->tune_levels : (d.nz <= 128 ? 8 : 16);
    const int KG = (d.nz + L - 1) / L;
    if (KG > 16) return hipErrorInvalidValue;  // nz <= 256
    const size_t lds = sizeof(double) * ((size_t)(d.nz + 1) * kLanes + 2 * (size_t)KG * kLanes +
                                         (L == 8 ? (size_t)d.nz * kLanes : 0));
    // without flux sums the last substep also writes the stage end S^t + S''
    // (no separate finalize pass over the five fields)
    const bool fuse_end = !a.sums;
    a.o_r = Sout[0]; a.o_t = Sout[1]; a.o_u = Sout[2]; a.o_v = Sout[3]; a.o_w = Sout[4];
    // S^t = S^n and one substep (the first RK3 stage): S'' = 0 throughout the
    // stage init and the substep's inputs, neither stored nor read
    bool zero = n_sub == 1;
    for (int f = 0; f < 5; ++f) zero = zero && Sn[f] == St[f];

    int t_cur = 0, t_prv = 2, u_in = 0;  // Theta'' rotates over 3 buffers, U'' and V'' over 2
    T *t2[3] = {(T *)w.t2[0], (T *)w.t2[1], (T *)w.t2[2]};
    T *u2[2] = {(T *)w.u2[0], (T *)w.u2[1]}, *v2[2] = {(T *)w.v2[0], (T *)w.v2[1]};
    a.T2cur = t2[0];
    a.u2in = u2[0];
    a.v2in = v2[0];

    if (lds > 64 * 1024) {
        const hipError_t e = L == 8 ? allow_lds<T, 8>(lds) : allow_lds<T, 16>(lds);
        if (e != hipSuccess) return e;
    }
    dim3 blk(64, 4, 1);
    dim3 g3w((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz + 1);
    dim3 g2((d.nx + 63) / 64, (d.ny + 3) / 4, 1);
    timing_start(cx, K_STAGE_INIT);
    if (zero && moist)
        run<StageArgs<T>, k_stage_init<T, true, true>, k_stage_init_batch<T, true, true>>(cx, g3w, blk, 0, a);
    else if (zero)
        run<StageArgs<T>, k_stage_init<T, true, false>, k_stage_init_batch<T, true, false>>(cx, g3w, blk, 0, a);
    else if (moist)
        run<StageArgs<T>, k_stage_init<T, false, true>, k_stage_init_batch<T, false, true>>(cx, g3w, blk, 0, a);
    else
        run<StageArgs<T>, k_stage_init<T, false, false>, k_stage_init_batch<T, false, false>>(cx, g3w, blk, 0, a);
    timing_stop(cx, K_STAGE_INIT);
    timing_start(cx, K_COEF);
    if (moist)
        run<StageArgs<T>, k_coef<T, true>, k_coef_batch<T, true>>(cx, g2, blk, 0, a);
    else
        run<StageArgs<T>, k_coef<T, false>, k_coef_batch<T, false>>(cx, g2, blk, 0, a);
    timing_stop(cx, K_COEF);
    for (int s = 0; s < n_sub; ++s) {
        const int t_nxt = 3 - t_cur - t_prv;
        a.T2cur = t2[t_cur];
        a.T2prv = (s == 0) ? t2[t_cur] : t2[t_prv];
        a.T2nxt = t2[t_nxt];
        a.u2in = u2[u_in];
        a.u2out = u2[u_in ^ 1];
        a.v2in = v2[u_in];
        a.v2out = v2[u_in ^ 1];
        a.bd = (s == 0) ? 0.0 : cx->prm.beta_d;
        const bool last = fuse_end && s == n_sub - 1;
        if (last) {
            a.u2out = Sout[2];
            a.v2out = Sout[3];
        }
        const dim3 grid(a.ntx * a.nty), block(kLanes, KG);
        timing_start(cx, K_SUBSTEP);
        if (L == 8)
            launch_substep<T, 8>(cx, last, zero && s == 0, a.sums != 0, grid, block, lds, a);
        else
            launch_substep<T, 16>(cx, last, zero && s == 0, a.sums != 0, grid, block, lds, a);
        timing_stop(cx, K_SUBSTEP);
        t_prv = t_cur;
        t_cur = t_nxt;
        u_in ^= 1;
    }
    if (fuse_end) return hipGetLastError();
    FinArgs<T> f{};
    f.d = d;
    f.n_sub = n_sub;
    f.b1 = a.b1;
    f.t_r = St[0]; f.t_t = St[1]; f.t_u = St[2]; f.t_v = St[3]; f.t_w = St[4]; f.n_w = Sn[4];
    f.T2 = t2[t_cur]; f.r2 = (T *)w.r2; f.u2 = u2[u_in]; f.v2 = v2[u_in]; f.w2 = (T *)w.w2;
    f.su = (T *)w.su; f.sv = (T *)w.sv; f.sw = (T *)w.sw;
    f.o_r = Sout[0]; f.o_t = Sout[1]; f.o_u = Sout[2]; f.o_v = Sout[3]; f.o_w = Sout[4];
    f.Fu = Fu; f.Fv = Fv; f.Fw = Fw;
    timing_start(cx, K_FINALIZE);
    run<FinArgs<T>, k_finalize<T>, k_finalize_batch<T>>(cx, g3w, blk, 0, f);
    timing_stop(cx, K_FINALIZE);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_acoustic_stage(erf_ctx *cx, const void *const Sn[5], const void *const St[5], const void *rq_t,
                                 const void *const Rt[5], int n_sub, double dtau, void *const Sout[5],
                                 void *Fu, void *Fv, void *Fw)
{
    if (cx->prm.precision == ERF_FP32_MIXED)
        return acoustic_t<float>(cx, Sn, St, rq_t, Rt, n_sub, dtau, Sout, (float *)Fu, (float *)Fv, (float *)Fw);
    return acoustic_t<double>(cx, Sn, St, rq_t, Rt, n_sub, dtau, Sout, (double *)Fu, (double *)Fv, (double *)Fw);
}

}  // namespace erfk
