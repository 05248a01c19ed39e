// tune.hip -- field layout queries and the launch-shape autotuner of the
// acoustic substep (include/erf.h: erf_layout, erf_autotune).
#include <cstdio>
#include <cstring>

#include "erf_internal.h"

namespace {

erf_status tune_fail(erf_ctx *c, erf_status s, const char *msg)
{
    c->err = msg;
    if (s == ERF_E_HIP) c->sticky = ERF_E_HIP;
    return s;
}

// the shapes erf_create accepts, as far as the layout depends on them
erf_status check_sizes(const erf_grid *g, const erf_params *p)
{
    if (g->nx < 1 || g->ny < 1 || g->nz < 2 || g->nz > 256) return ERF_E_SHAPE;
    const int64_t nw = (int64_t)g->nx * g->ny * (g->nz + 1);
    if (nw * (p->n_scalars > 1 ? p->n_scalars : 1) >= ((int64_t)1 << 31)) return ERF_E_SHAPE;
    if (p->precision != ERF_FP64 && p->precision != ERF_FP32_MIXED) return ERF_E_ARG;
    if (p->n_scalars < 0 || p->n_scalars > 8) return ERF_E_ARG;
    // anelastic contexts: the projection's transform lengths
    auto pow2 = [](int v) { return v >= 1 && v <= 2048 && (v & (v - 1)) == 0; };
    if (p->anelastic == 1 && (!pow2(g->nx) || !pow2(g->ny))) return ERF_E_SHAPE;
    return ERF_OK;
}

bool shape_valid(int nz, int levels, int rows)
{
    const bool lv = (levels == 8 && nz <= 128) || (levels == 16 && nz <= 256);
    return lv && (rows == 1 || rows == 2 || rows == 4);
}

// the cache key of a context: grid size and precision
void cache_key(const erf_ctx *c, char *buf, size_t n)
{
    std::snprintf(buf, n, "substep %d %d %d %d", c->d.nx, c->d.ny, c->d.nz, c->prm.precision);
}

// last line of the cache file that matches the key and holds a valid shape
bool cache_lookup(const erf_ctx *c, const char *path, int &levels, int &rows, double &ms)
{
    std::FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char key[96], line[256];
    cache_key(c, key, sizeof key);
    const size_t kl = std::strlen(key);
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key, kl) != 0 || line[kl] != ' ') continue;
        int L = 0, r = 0;
        double t = 0.0;
        if (std::sscanf(line + kl, "%d %d %lf", &L, &r, &t) == 3 && shape_valid(c->d.nz, L, r)) {
            levels = L;
            rows = r;
            ms = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

}  // namespace

extern "C" {

erf_status erf_layout(const erf_grid *grid, const erf_params *params, int32_t field, erf_field_layout *out)
{
    if (!grid || !params || !out) return ERF_E_ARG;
    if (field < ERF_FIELD_RHO || field > ERF_FIELD_RHOQ) return ERF_E_ARG;
    const erf_status s = check_sizes(grid, params);
    if (s != ERF_OK) return s;
    erf_field_layout L{};
    L.nx = grid->nx;
    L.ny = grid->ny;
    L.nz = field == ERF_FIELD_RHOW ? grid->nz + 1 : grid->nz;
    L.components = field == ERF_FIELD_RHOQ ? params->n_scalars : 1;
    L.stride_y = grid->nx;
    L.stride_z = (int64_t)grid->nx * grid->ny;
    L.stride_c = L.stride_z * L.nz;
    L.count = L.stride_c * L.components;
    L.elem_bytes = params->precision == ERF_FP64 ? 8 : 4;
    L.bytes = L.count * L.elem_bytes;
    L.perturbation =
        (params->precision == ERF_FP32_MIXED && (field == ERF_FIELD_RHO || field == ERF_FIELD_RHOTHETA)) ? 1 : 0;
    *out = L;
    return ERF_OK;
}

erf_status erf_autotune(erf_ctx *c, erf_state *S, int32_t trials, const char *cache_path, erf_tuning *out)
{
    if (!c) return ERF_E_ARG;
    if (c->sticky != ERF_OK) return c->sticky;
    if (c->prm.anelastic) return tune_fail(c, ERF_E_UNSUPPORTED, "an anelastic context has no acoustic substeps");
    if (c->ter.on) return tune_fail(c, ERF_E_UNSUPPORTED, "the terrain substeps have no tunable launch shape");
    if (!c->have_base) return tune_fail(c, ERF_E_STATE, "erf_init_base_state must come first");
    if (!S || !S->rho || !S->rhotheta || !S->rhou || !S->rhov || !S->rhow || (c->prm.n_scalars > 0 && !S->rhoq))
        return tune_fail(c, ERF_E_ARG, "null field pointer");
    if (trials < 1) return tune_fail(c, ERF_E_ARG, "trials must be >= 1");
    erf_tuning res{};
    int levels = 0, rows = 0;
    double ms = 0.0;
    if (cache_path && cache_lookup(c, cache_path, levels, rows, ms)) {
        c->tune_levels = levels;
        c->tune_rows = rows;
        res = {levels, rows, ms, 1};
        if (out) *out = res;
        return ERF_OK;
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t h = hipEventCreate(&t0);
    if (h == hipSuccess) h = hipEventCreate(&t1);
    if (h != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return tune_fail(c, ERF_E_HIP, "timing events");
    }
    const int old_levels = c->tune_levels, old_rows = c->tune_rows;
    double best = 1e300;
    int best_levels = 0, best_rows = 0;
    erf_status st = ERF_OK;
    const int cand_levels[2] = {8, 16}, cand_rows[3] = {1, 2, 4};
    for (int li = 0; li < 2 && st == ERF_OK; ++li)
        for (int ri = 0; ri < 3 && st == ERF_OK; ++ri) {
            if (!shape_valid(c->d.nz, cand_levels[li], cand_rows[ri])) continue;
            c->tune_levels = cand_levels[li];
            c->tune_rows = cand_rows[ri];
            if ((st = erf_rk3_step(c, S)) != ERF_OK) break;  // untimed: first use of the shape
            h = hipEventRecord(t0, c->stream);
            for (int t = 0; t < trials && st == ERF_OK && h == hipSuccess; ++t) st = erf_rk3_step(c, S);
            if (st != ERF_OK) break;
            if (h == hipSuccess) h = hipEventRecord(t1, c->stream);
            if (h == hipSuccess) h = hipEventSynchronize(t1);
            float e = 0.f;
            if (h == hipSuccess) h = hipEventElapsedTime(&e, t0, t1);
            if (h != hipSuccess) {
                st = tune_fail(c, ERF_E_HIP, "timing the substep shapes");
                break;
            }
            if (e / trials < best) {
                best = e / trials;
                best_levels = cand_levels[li];
                best_rows = cand_rows[ri];
            }
        }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != ERF_OK || best_levels == 0) {
        c->tune_levels = old_levels;
        c->tune_rows = old_rows;
        return st != ERF_OK ? st : tune_fail(c, ERF_E_ARG, "no launch shape fits this grid");
    }
    c->tune_levels = best_levels;
    c->tune_rows = best_rows;
    res = {best_levels, best_rows, best, 0};
    if (out) *out = res;
    if (cache_path) {
        std::FILE *f = std::fopen(cache_path, "a");
        if (!f) return tune_fail(c, ERF_E_ARG, "cannot write the autotune cache file");
        char key[96];
        cache_key(c, key, sizeof key);
        std::fprintf(f, "%s %d %d %.6f\n", key, best_levels, best_rows, best);
        std::fclose(f);
    }
    return ERF_OK;
}

}  // extern "C"
