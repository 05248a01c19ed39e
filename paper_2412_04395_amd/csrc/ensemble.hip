// ensemble.hip -- batched RK3 steps of independent members (include/erf_ensemble.h):
// one HIP graph per ensemble step, members spread over forked branch streams.
// Batched mode (the default): every member's step is recorded once, launch by
// launch, and on each branch the k-th launches of its members that run the
// same kernel instance with the same block shape become one launch over a
// (member, block) work list.  Unbatched mode: the members' own launches.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/erf_ensemble.h"
#include "erf_internal.h"

struct erf_ens {
    std::vector<erf_ctx *> members;
    std::vector<int> branch_of;  // member -> branch
    hipStream_t user = nullptr;  // ordering stream given at creation
    hipStream_t main = nullptr;  // capture origin and graph launch stream
    hipStream_t branch[ERF_ENSEMBLE_MAX_BRANCHES] = {};
    hipEvent_t fork = nullptr, done = nullptr, join[ERF_ENSEMBLE_MAX_BRANCHES] = {};
    int n_branches = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<erf_state> captured;  // state pointers the graph was captured with
    erf_status sticky = ERF_OK;
    std::string err;
    // batched mode: the launch list of the captured step and the device buffer
    // holding its argument structures and block maps
    int batched = 1;
    struct Batch {
        erfk::BatchFn fn;
        dim3 block;
        size_t lds;
        int n, blocks;
        size_t args_off, map_off;
        int branch;
    };
    std::vector<Batch> plan;
    void *plan_dev = nullptr;
    size_t plan_cap = 0;
};

namespace {

erf_status efail(erf_ens *e, erf_status s, const std::string &msg)
{
    e->err = msg;
    if (s == ERF_E_HIP) e->sticky = ERF_E_HIP;
    return s;
}

erf_status ehip(erf_ens *e, hipError_t h, const char *where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(h));
    return efail(e, ERF_E_HIP, buf);
}

void drop_graph(erf_ens *e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
    e->captured.clear();
}

// members by decreasing cell count, each to the least loaded branch
void assign(erf_ens *e)
{
    const int n = (int)e->members.size();
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return e->members[a]->d.n > e->members[b]->d.n; });
    std::vector<int64_t> load(e->n_branches, 0);
    e->branch_of.assign(n, 0);
    for (int m : order) {
        int best = 0;
        for (int b = 1; b < e->n_branches; ++b)
            if (load[b] < load[best]) best = b;
        e->branch_of[m] = best;
        load[best] += e->members[m]->d.n;
    }
}

bool same_states(const std::vector<erf_state> &a, const erf_state *b, size_t n)
{
    if (a.size() != n) return false;
    return std::memcmp(a.data(), b, n * sizeof(erf_state)) == 0;
}

// Record every member's step, group the k-th launches of the members by
// kernel instance, block shape and LDS, and upload the argument structures and
// block maps of the resulting batched launches.
erf_status build_plan(erf_ens *e, const erf_state *states)
{
    const int n = (int)e->members.size();
    std::vector<erfk::Recorder> rec(n);
    size_t maxlen = 0;
    for (int m = 0; m < n; ++m) {
        erf_state s = states[m];
        e->members[m]->rec = &rec[m];
        const erf_status st = erf_rk3_step(e->members[m], &s);
        e->members[m]->rec = nullptr;
        if (st != ERF_OK) return efail(e, st, std::string("member ") + std::to_string(m) + ": " +
                                                  erf_last_error(e->members[m]));
        maxlen = std::max(maxlen, rec[m].recs.size());
    }
    std::vector<unsigned char> hb;
    auto align = [&](size_t a) { hb.resize((hb.size() + a - 1) / a * a); };
    e->plan.clear();
    std::vector<char> used(n);
    for (int br = 0; br < e->n_branches; ++br)
    for (size_t p = 0; p < maxlen; ++p) {
        // members of other branches count as used: batches stay within a branch
        for (int m = 0; m < n; ++m) used[m] = e->branch_of[m] != br;
        for (int m = 0; m < n; ++m) {
            if (used[m] || p >= rec[m].recs.size()) continue;
            const erfk::LaunchRec &r0 = rec[m].recs[p];
            std::vector<int> grp;
            for (int q = m; q < n; ++q) {
                if (used[q] || p >= rec[q].recs.size()) continue;
                const erfk::LaunchRec &r = rec[q].recs[p];
                if (r.fn == r0.fn && r.block.x == r0.block.x && r.block.y == r0.block.y &&
                    r.block.z == r0.block.z && r.lds == r0.lds && r.args.size() == r0.args.size()) {
                    grp.push_back(q);
                    used[q] = 1;
                }
            }
            erf_ens::Batch b{r0.fn, r0.block, r0.lds, (int)grp.size(), 0, 0, 0, br};
            align(256);
            b.args_off = hb.size();
            for (int q : grp) hb.insert(hb.end(), rec[q].recs[p].args.begin(), rec[q].recs[p].args.end());
            align(256);
            b.map_off = hb.size();
            std::vector<int> first(grp.size() + 1), grid(3 * grp.size());
            int64_t tot = 0;
            for (size_t g = 0; g < grp.size(); ++g) {
                const erfk::LaunchRec &r = rec[grp[g]].recs[p];
                first[g] = (int)tot;
                grid[3 * g] = (int)r.grid.x;
                grid[3 * g + 1] = (int)r.grid.y;
                grid[3 * g + 2] = (int)r.grid.z;
                const int64_t nb = (int64_t)r.grid.x * r.grid.y * r.grid.z;
                tot += (nb + 7) / 8 * 8;  // each range starts on a multiple of 8
            }
            if (tot >= ((int64_t)1 << 31)) return efail(e, ERF_E_SHAPE, "batched launch too large");
            first[grp.size()] = (int)tot;
            b.blocks = (int)tot;
            const unsigned char *pf = (const unsigned char *)first.data(), *pg = (const unsigned char *)grid.data();
            hb.insert(hb.end(), pf, pf + first.size() * sizeof(int));
            hb.insert(hb.end(), pg, pg + grid.size() * sizeof(int));
            e->plan.push_back(b);
        }
    }
    hipError_t h = hipSuccess;
    if (hb.size() > e->plan_cap) {
        // a buffer an earlier graph still reads is freed only once that graph is done
        h = hipStreamSynchronize(e->main);
        if (h == hipSuccess && e->plan_dev) h = hipFree(e->plan_dev);
        e->plan_dev = nullptr;
        e->plan_cap = 0;
        if (h == hipSuccess) h = hipMalloc(&e->plan_dev, hb.size());
        if (h != hipSuccess) {
            (void)hipGetLastError();
            e->plan_dev = nullptr;
            return efail(e, ERF_E_NOMEM, "ensemble launch list allocation failed");
        }
        e->plan_cap = hb.size();
    } else {
        h = hipStreamSynchronize(e->main);
    }
    if (h == hipSuccess && !hb.empty()) h = hipMemcpy(e->plan_dev, hb.data(), hb.size(), hipMemcpyHostToDevice);
    for (const erf_ens::Batch &b : e->plan)
        if (h == hipSuccess) h = b.fn(nullptr, erfk::BatchMap{}, 0, b.block, b.lds, nullptr, true);
    return h == hipSuccess ? ERF_OK : ehip(e, h, "uploading the ensemble launch list");
}

erf_status capture_batched(erf_ens *e, const erf_state *states)
{
    drop_graph(e);
    erf_status st = build_plan(e, states);
    if (st != ERF_OK) return st;
    hipError_t h = hipStreamBeginCapture(e->main, hipStreamCaptureModeThreadLocal);
    if (h != hipSuccess) return ehip(e, h, "begin capture");
    char *base = (char *)e->plan_dev;
    // each branch's batched launches on its own stream, forked from and joined
    // back to the capture stream
    h = hipEventRecord(e->fork, e->main);
    for (int b = 0; h == hipSuccess && b < e->n_branches; ++b) h = hipStreamWaitEvent(e->branch[b], e->fork, 0);
    for (const erf_ens::Batch &b : e->plan) {
        if (h != hipSuccess) break;
        const int *first = (const int *)(base + b.map_off);
        erfk::BatchMap map{first, first + b.n + 1, b.n};
        h = b.fn(base + b.args_off, map, b.blocks, b.block, b.lds, e->branch[b.branch], false);
    }
    for (int b = 0; h == hipSuccess && b < e->n_branches; ++b) {
        h = hipEventRecord(e->join[b], e->branch[b]);
        if (h == hipSuccess) h = hipStreamWaitEvent(e->main, e->join[b], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t he = hipStreamEndCapture(e->main, &g);
    if (h != hipSuccess || he != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ehip(e, h != hipSuccess ? h : he, "capturing the batched ensemble step");
    }
    e->graph = g;
    h = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
    if (h != hipSuccess) {
        e->exec = nullptr;
        drop_graph(e);
        return ehip(e, h, "instantiating the batched ensemble graph");
    }
    e->captured.assign(states, states + e->members.size());
    return ERF_OK;
}

erf_status capture(erf_ens *e, const erf_state *states)
{
    if (e->batched) return capture_batched(e, states);
    drop_graph(e);
    const int n = (int)e->members.size();
    hipError_t h = hipStreamBeginCapture(e->main, hipStreamCaptureModeThreadLocal);
    if (h != hipSuccess) return ehip(e, h, "begin capture");
    erf_status st = ERF_OK;
    h = hipEventRecord(e->fork, e->main);
    for (int b = 0; h == hipSuccess && b < e->n_branches; ++b) h = hipStreamWaitEvent(e->branch[b], e->fork, 0);
    // members in branch order so that each branch's work is enqueued together;
    // a member's context enqueues on its branch stream only while capturing
    for (int b = 0; h == hipSuccess && st == ERF_OK && b < e->n_branches; ++b)
        for (int m = 0; m < n && st == ERF_OK; ++m)
            if (e->branch_of[m] == b) {
                erf_state s = states[m];
                e->members[m]->stream = e->branch[b];
                st = erf_rk3_step(e->members[m], &s);
                e->members[m]->stream = e->user;
                if (st != ERF_OK) e->err = std::string("member ") + std::to_string(m) + ": " + erf_last_error(e->members[m]);
            }
    for (int b = 0; h == hipSuccess && st == ERF_OK && b < e->n_branches; ++b) {
        h = hipEventRecord(e->join[b], e->branch[b]);
        if (h == hipSuccess) h = hipStreamWaitEvent(e->main, e->join[b], 0);
    }
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(e->main, &g);
    if (st != ERF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (h != hipSuccess || he != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return ehip(e, h != hipSuccess ? h : he, "capturing the ensemble step");
    }
    e->graph = g;
    h = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
    if (h != hipSuccess) {
        e->exec = nullptr;
        drop_graph(e);
        return ehip(e, h, "instantiating the ensemble graph");
    }
    e->captured.assign(states, states + n);
    return ERF_OK;
}

}  // namespace

extern "C" {

erf_status erf_ensemble_create(int32_t n, const erf_grid *grids, const erf_params *params, void *hip_stream,
                               erf_ens **out)
{
    if (!out || !grids || !params || n < 1) return ERF_E_ARG;
    *out = nullptr;
    erf_ens *e = new (std::nothrow) erf_ens();
    if (!e) return ERF_E_NOMEM;
    e->user = (hipStream_t)hip_stream;
    hipError_t h = hipStreamCreateWithFlags(&e->main, hipStreamNonBlocking);
    for (int b = 0; h == hipSuccess && b < ERF_ENSEMBLE_MAX_BRANCHES; ++b)
        h = hipStreamCreateWithFlags(&e->branch[b], hipStreamNonBlocking);
    if (h == hipSuccess) h = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming);
    if (h == hipSuccess) h = hipEventCreateWithFlags(&e->done, hipEventDisableTiming);
    for (int b = 0; h == hipSuccess && b < ERF_ENSEMBLE_MAX_BRANCHES; ++b)
        h = hipEventCreateWithFlags(&e->join[b], hipEventDisableTiming);
    if (h != hipSuccess) {
        (void)hipGetLastError();
        erf_ensemble_destroy(e);
        return ERF_E_HIP;
    }
    for (int m = 0; m < n; ++m) {
        erf_ctx *c = nullptr;
        erf_status s = erf_create(&grids[m], &params[m], e->user, &c);
        if (s != ERF_OK) {
            erf_ensemble_destroy(e);
            return s;
        }
        c->member = true;
        e->members.push_back(c);
    }
    e->n_branches = std::min(n, 4);
    assign(e);
    *out = e;
    return ERF_OK;
}

void erf_ensemble_destroy(erf_ens *e)
{
    if (!e) return;
    if (e->main) (void)hipStreamSynchronize(e->main);
    drop_graph(e);
    for (erf_ctx *c : e->members) erf_destroy(c);
    for (int b = 0; b < ERF_ENSEMBLE_MAX_BRANCHES; ++b) {
        if (e->branch[b]) (void)hipStreamDestroy(e->branch[b]);
        if (e->join[b]) (void)hipEventDestroy(e->join[b]);
    }
    if (e->fork) (void)hipEventDestroy(e->fork);
    if (e->done) (void)hipEventDestroy(e->done);
    if (e->main) (void)hipStreamDestroy(e->main);
    if (e->plan_dev) (void)hipFree(e->plan_dev);
    delete e;
}

const char *erf_ensemble_last_error(const erf_ens *e) { return e ? e->err.c_str() : "null ensemble"; }

erf_ctx *erf_ensemble_member(erf_ens *e, int32_t m)
{
    if (!e || m < 0 || m >= (int32_t)e->members.size()) return nullptr;
    return e->members[m];
}

erf_status erf_ensemble_set_branches(erf_ens *e, int32_t nb)
{
    if (!e) return ERF_E_ARG;
    if (e->sticky != ERF_OK) return e->sticky;
    if (nb < 1 || nb > ERF_ENSEMBLE_MAX_BRANCHES) return efail(e, ERF_E_ARG, "branches must be 1..16");
    // graph launches already enqueued finish before the branches are reassigned
    hipError_t h = hipStreamSynchronize(e->main);
    if (h != hipSuccess) return ehip(e, h, "draining the ensemble stream");
    drop_graph(e);
    e->n_branches = std::min<int>(nb, (int)e->members.size());
    assign(e);
    return ERF_OK;
}

int32_t erf_ensemble_branches(const erf_ens *e) { return e ? e->n_branches : 0; }

erf_status erf_ensemble_set_batched(erf_ens *e, int32_t on)
{
    if (!e) return ERF_E_ARG;
    if (e->sticky != ERF_OK) return e->sticky;
    if (on != 0 && on != 1) return efail(e, ERF_E_ARG, "batched must be 0 or 1");
    hipError_t h = hipStreamSynchronize(e->main);
    if (h != hipSuccess) return ehip(e, h, "draining the ensemble stream");
    drop_graph(e);
    e->batched = on;
    return ERF_OK;
}

int32_t erf_ensemble_batched(const erf_ens *e) { return e ? e->batched : 0; }

erf_status erf_ensemble_rk3_step(erf_ens *e, const erf_state *states)
{
    if (!e || !states) return e ? efail(e, ERF_E_ARG, "states is NULL") : ERF_E_ARG;
    if (e->sticky != ERF_OK) return e->sticky;
    const size_t n = e->members.size();
    if (!e->exec || !same_states(e->captured, states, n)) {
        erf_status s = capture(e, states);
        if (s != ERF_OK) return s;
    }
    // order: user stream -> graph -> user stream
    hipError_t h = hipEventRecord(e->done, e->user);
    if (h == hipSuccess) h = hipStreamWaitEvent(e->main, e->done, 0);
    if (h == hipSuccess) h = hipGraphLaunch(e->exec, e->main);
    if (h == hipSuccess) h = hipEventRecord(e->done, e->main);
    if (h == hipSuccess) h = hipStreamWaitEvent(e->user, e->done, 0);
    return h == hipSuccess ? ERF_OK : ehip(e, h, "launching the ensemble step");
}

erf_status erf_ensemble_autotune(erf_ens *e, const erf_state *states, int32_t trials, int32_t *best_branches,
                                 double *best_ms)
{
    if (!e || !states || trials < 1) return e ? efail(e, ERF_E_ARG, "states and trials >= 1 required") : ERF_E_ARG;
    if (e->sticky != ERF_OK) return e->sticky;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t h = hipEventCreate(&t0);
    if (h == hipSuccess) h = hipEventCreate(&t1);
    if (h != hipSuccess) return ehip(e, h, "timing events");
    int best = e->n_branches, best_batched = e->batched;
    double best_t = 1e300;
    erf_status st = ERF_OK;
    // batched and unbatched launches, each on 1, 2, 4, 8, 16 branch streams
    const int cands[] = {1, 2, 4, 8, 16};
    for (int bat = 1; bat >= 0 && st == ERF_OK; --bat)
    for (int nb : cands) {
        if (nb > (int)e->members.size() && nb > 1) break;
        if ((st = erf_ensemble_set_batched(e, bat)) != ERF_OK) break;
        if ((st = erf_ensemble_set_branches(e, nb)) != ERF_OK) break;
        if ((st = erf_ensemble_rk3_step(e, states)) != ERF_OK) break;  // capture + warm-up
        h = hipEventRecord(t0, e->main);
        for (int t = 0; h == hipSuccess && t < trials; ++t) h = hipGraphLaunch(e->exec, e->main);
        if (h == hipSuccess) h = hipEventRecord(t1, e->main);
        if (h == hipSuccess) h = hipEventSynchronize(t1);
        float ms = 0.f;
        if (h == hipSuccess) h = hipEventElapsedTime(&ms, t0, t1);
        if (h != hipSuccess) {
            st = ehip(e, h, "timing the ensemble step");
            break;
        }
        if (ms / trials < best_t) {
            best_t = ms / trials;
            best = nb;
            best_batched = bat;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != ERF_OK) return st;
    if ((st = erf_ensemble_set_batched(e, best_batched)) != ERF_OK) return st;
    if ((st = erf_ensemble_set_branches(e, best)) != ERF_OK) return st;
    if (best_branches) *best_branches = e->n_branches;
    if (best_ms) *best_ms = best_t;
    return ERF_OK;
}

}  // extern "C"
