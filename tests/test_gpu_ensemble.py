"""Ensemble batching (include/erf_ensemble.h) on the GPU.

Members are independent contexts and both modes run each member's own kernel
bodies on forked branch streams (batched mode: the k-th launches of a branch's
members fused into one launch over a (member, block) work list; unbatched: the
members' own launches), so an ensemble step must equal stepping the members one
after another bitwise, whatever the mode, the branch layout, the graph
re-captures and the autotuner's trials.  One FP64 member is also checked against the
oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _members():
    """Six uneven members: precisions, closures and shapes mixed."""
    base = dict(dx=40.0, dy=40.0, dt=0.4, n_substeps=8, adv_order_h=5, adv_order_v=5, Cs=0.1,
                f_cor=1e-4, Ug=10.0)
    shapes = [(24, 20, 16), (32, 16, 12), (40, 24, 16), (16, 16, 20), (48, 8, 10), (20, 28, 14)]
    cfgs = []
    for m, (nx, ny, nz) in enumerate(shapes):
        cfgs.append(W.small(name=f"ens_{m}", nx=nx, ny=ny, nz=nz, dz=W.uniform_dz(nz, 40.0), seed=70 + m,
                            sgs=m % 3, prec="fp32" if m % 2 else "fp64", surf_heat_flux=0.05 * (m + 1), **base))
    return cfgs


def _weights(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(9609)
    for off, fi, fo in ((0, 10, 64), (704, 64, 64), (4864, 64, 64), (9024, 64, 9)):
        p[off:off + fi * fo] = rng.normal(0, np.sqrt(2.0 / fi), fi * fo)
    nrm = np.concatenate([np.zeros(10), np.full(9, 1e-2), [1e-3], np.zeros(9), np.full(9, 1e-4)])
    return p.astype(np.float32), nrm


def _setup(solver, cfg):
    th0, qv0 = W.theta_sounding(cfg), W.qv0_of(cfg)
    b = solver.init_base_state(th0, qv0=qv0)
    if cfg.sgs == 2:
        solver.mlp_set_weights(*_weights(cfg.seed))
    return solver.from_full(W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"], qv0))


def _sequential(cfgs, steps):
    from paper_2412_04395_amd import erf
    out = []
    for c in cfgs:
        s = erf.Solver(c)
        S = _setup(s, c)
        for _ in range(steps):
            s.rk3_step(S)
        out.append(s.to_numpy(S))
        s.close()
    return out


def _same(a, b):
    return all(np.array_equal(x[f], y[f]) for x, y in zip(a, b) for f in ("rho", "rt", "ru", "rv", "rw", "rq"))


@pytest.mark.parametrize("batched,branches", [(1, 1), (1, 3), (0, 1), (0, 3), (0, 6)])
def test_batched_step_equals_sequential_bitwise(batched, branches):
    from paper_2412_04395_amd import erf
    cfgs = _members()
    ens = erf.Ensemble(cfgs)
    assert ens.batched  # the default
    ens.set_batched(bool(batched))
    ens.set_branches(branches)
    states = [_setup(s, c) for s, c in zip(ens.members, cfgs)]
    for _ in range(3):
        ens.rk3_step(states)
    got = [m.to_numpy(S) for m, S in zip(ens.members, states)]
    ref = _sequential(cfgs, 3)
    mode = f"{'batched' if ens.batched else 'unbatched'}, {ens.branches} branches"
    _say(f"ensemble, {mode}: bitwise equal {_same(got, ref)}")
    assert _same(got, ref)
    for m, S in zip(ens.members, states):
        assert m.diagnostics(S)["nonfinite"] == 0
    ens.close()


def test_batched_with_scalars_and_moisture():
    """Members that transport scalars (WENO5 and an interpolant, FP32 and FP64,
    moist, one with Kessler microphysics) beside plain ones: the batched
    mixing-ratio, scalar, finalize, moist and microphysics launches give the
    sequential result bitwise."""
    from paper_2412_04395_amd import erf
    base = dict(dx=250.0, dy=250.0, dt=2.0, n_substeps=8, adv_order_h=3, adv_order_v=3)
    cfgs = [W.small(name="deep_small", nx=36, ny=20, nz=14, dz=W.stretched_dz(14, 50.0, 500.0, 4000.0), seed=81,
                    n_scalars=3, scalar_scheme=1, moist=1, microphysics=1, prec="fp32", **base),
            W.small(name="deep_small", nx=24, ny=30, nz=12, dz=W.uniform_dz(12, 200.0), seed=82, n_scalars=3,
                    scalar_scheme=0, prec="fp64", **base),
            W.small(name="deep_small", nx=40, ny=16, nz=14, dz=W.stretched_dz(14, 50.0, 500.0, 4000.0), seed=83,
                    n_scalars=3, scalar_scheme=1, moist=1, prec="fp64", **base),
            W.small(name="bubble_small", nx=28, ny=20, nz=16, seed=84, prec="fp32")]
    ens = erf.Ensemble(cfgs)
    states = [_setup(s, c) for s, c in zip(ens.members, cfgs)]
    for _ in range(2):
        ens.rk3_step(states)
    got = [m.to_numpy(S) for m, S in zip(ens.members, states)]
    assert _same(got, _sequential(cfgs, 2))
    ens.close()


def test_recapture_on_new_state_buffers():
    from paper_2412_04395_amd import erf
    cfgs = _members()[:3]
    ens = erf.Ensemble(cfgs)
    A = [_setup(s, c) for s, c in zip(ens.members, cfgs)]
    B = [{k: v.clone() for k, v in S.items()} for S in A]
    ens.rk3_step(A)          # graph for A
    ens.rk3_step(B)          # new buffers: captured again
    ens.rk3_step(B)
    ens.rk3_step(A)          # and back
    a = [m.to_numpy(S) for m, S in zip(ens.members, A)]
    b = [m.to_numpy(S) for m, S in zip(ens.members, B)]
    assert _same(a, _sequential(cfgs, 2)) and _same(b, _sequential(cfgs, 2))
    ens.close()


def test_autotune_keeps_results_bitwise():
    from paper_2412_04395_amd import erf
    cfgs = _members()
    ens = erf.Ensemble(cfgs)
    states = [_setup(s, c) for s, c in zip(ens.members, cfgs)]
    trials = 2
    nb, ms = ens.autotune(states, trials)
    # one capture step and `trials` timed steps per candidate: batched and
    # unbatched, each on 1, 2, 4 branches (6 members: 8 and 16 skipped)
    steps = 2 * 3 * (1 + trials)
    _say(f"autotune: {'batched' if ens.batched else 'unbatched'}, {nb} branches, {ms:.3f} ms per ensemble step, "
         f"{steps} steps")
    assert nb in (1, 2, 4) and ms > 0 and ens.branches == nb
    got = [m.to_numpy(S) for m, S in zip(ens.members, states)]
    assert _same(got, _sequential(cfgs, steps))
    ens.close()


def test_member_matches_oracle():
    from paper_2412_04395_amd import erf
    cfgs = _members()
    c = cfgs[0]  # FP64, no closure
    ens = erf.Ensemble(cfgs[:2])
    states = [_setup(s, cc) for s, cc in zip(ens.members, cfgs[:2])]
    for _ in range(2):
        ens.rk3_step(states)
    got = ens.members[0].to_numpy(states[0])
    o = oracle.Oracle(c)
    th0 = W.theta_sounding(c)
    b = o.init_base_state(th0, c.p_surface)
    S = W.initial_state(c, b["rho0"], th0, b["p0"], b["pi0"])
    S = {k: np.ascontiguousarray(v) for k, v in S.items()}
    for _ in range(2):
        o.rk3_step(S)
    rho0 = b["rho0"][:, None, None]
    e_rho = np.abs(got["rho"] - S["rho"]).max() / np.abs(S["rho"] - rho0).max()
    mom = max(np.abs(S[f]).max() for f in ("ru", "rv", "rw"))
    e_mom = max(np.abs(got[f] - S[f]).max() for f in ("ru", "rv", "rw")) / mom
    _say(f"ensemble member vs oracle: rho' {e_rho:.1e}, momentum {e_mom:.1e}")
    assert e_rho <= 1e-11 and e_mom <= 1e-12
    ens.close()
