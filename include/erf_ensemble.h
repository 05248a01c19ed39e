/*
 * erf_ensemble.h -- batched RK3 steps of many independent members (contexts of
 * erf.h, each with its own grid, parameters and workspace) on one GPU.
 *
 * An ensemble step is defined as every member taking one erf_rk3_step (Sec.
 * 3.1, 3.3) from its own state; members never exchange data, so a batched step
 * is bitwise identical to stepping the members one after another.
 *
 * Execution: the whole ensemble step is captured once into a HIP graph; each
 * later step is one graph launch.  The graph is captured again when the state
 * pointers, the mode or the branch layout change.  The members are spread over
 * up to 16 internal streams (branches, default priority) that fork from and
 * join back to the ensemble's launch stream, assigned by decreasing cell
 * count, each to the branch with the fewest cells so far, so that different
 * kernels of different members run side by side.  Within a branch:
 *  - batched mode (the default): each member's step is recorded launch by
 *    launch (without running it); the k-th launches of the branch's members
 *    that run the same kernel instance with the same block shape become one
 *    launch whose blocks are a (member, tile) work list, each block running
 *    exactly the member's own block of that kernel.  A step of 48
 *    boundary-layer members on one branch is about 70 launches instead of
 *    about 3,000;
 *  - unbatched mode: the members' own launches, one after another.
 * Both give results bitwise identical to stepping the members one by one.
 *
 * Ordering: erf_ensemble_rk3_step orders itself after the work already
 * enqueued on the stream given to erf_ensemble_create, and later work on that
 * stream after the step.  Returns without waiting, like erf_rk3_step.
 */
#ifndef ERF_ENSEMBLE_H
#define ERF_ENSEMBLE_H

#include "erf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct erf_ens erf_ens;

#define ERF_ENSEMBLE_MAX_BRANCHES 16

/* Create n >= 1 members from grids[n] and params[n] (each as erf_create; the
 * members' workspaces are allocated here).  hip_stream: the stream the
 * ensemble's steps are ordered with (NULL: the default stream).  Starts with
 * min(n, 4) branches. */
erf_status erf_ensemble_create(int32_t n, const erf_grid *grids, const erf_params *params, void *hip_stream,
                               erf_ens **out);
void erf_ensemble_destroy(erf_ens *ens);
const char *erf_ensemble_last_error(const erf_ens *ens);

/* Member m's context (owned by the ensemble, valid until erf_ensemble_destroy):
 * for erf_init_base_state, erf_mlp_set_weights, erf_diagnostics and single
 * calls, which it enqueues on the ensemble's stream, ordered with the steps.
 * NULL for m out of range. */
erf_ctx *erf_ensemble_member(erf_ens *ens, int32_t m);

/* Use n_branches in 1..ERF_ENSEMBLE_MAX_BRANCHES concurrent branches (fewer if
 * there are fewer members).  Drops the captured graph. */
erf_status erf_ensemble_set_branches(erf_ens *ens, int32_t n_branches);
int32_t erf_ensemble_branches(const erf_ens *ens);

/* batched = 1: batched mode (the default); 0: unbatched.  Waits for the
 * steps already enqueued and drops the captured graph.  ERF_E_ARG otherwise.
 * The batched launch list and its argument structures live in one device
 * buffer of the ensemble (allocated at capture, tens of KB per member). */
erf_status erf_ensemble_set_batched(erf_ens *ens, int32_t batched);
int32_t erf_ensemble_batched(const erf_ens *ens);

/* One RK3 step of every member: states[m] holds member m's state (device, its
 * context's layout), advanced in place.  Every member needs its base state
 * (and closure weights if it uses the learned closure) before the first step. */
erf_status erf_ensemble_rk3_step(erf_ens *ens, const erf_state *states);

/* Time `trials` graph launches for each mode (batched, then unbatched) and
 * each branch count 1, 2, 4, 8, 16 (up to the member count) after one untimed
 * launch each, keep the fastest and report it (best_branches, best_ms = average
 * ms per ensemble step; either may be NULL; erf_ensemble_batched tells the
 * mode).  The states advance by every step taken.  Synchronous. */
erf_status erf_ensemble_autotune(erf_ens *ens, const erf_state *states, int32_t trials, int32_t *best_branches,
                                 double *best_ms);

#ifdef __cplusplus
}
#endif
#endif /* ERF_ENSEMBLE_H */
