"""erf_autotune: the launch shape of the acoustic substep, timed or read from a
cache file, through the C-ABI.

The row shape of a workgroup's 64 columns only decides which lane handles which
column, so every row shape gives bitwise the same step.  The level count per
wavefront changes how the tridiagonal sweeps are chunked, so it changes the
rounding only; each shape is also compared with the FP64 oracle at the bound of
the RK3 parity tests (5 steps, 1e-12).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu

# 70 x 20 columns: every row shape has partial tiles; 40 levels: 5 chunks of 8
# or 3 of 16, the last one partial
CFG = dict(name="cbl_small", nx=70, ny=20, nz=40, dx=20.0, dy=20.0, dz=W.uniform_dz(40, 10.0), dt=0.1,
           adv_order_h=5, adv_order_v=5, sgs=1, Cs=0.1, f_cor=1e-4, Ug=10.0, Vg=1.0, surf_heat_flux=0.2)
# 64 x 8 columns: every row shape fills its tiles exactly (no idle lanes, no
# partial tile at the domain's end)
CFG_FULL = dict(CFG, nx=64, ny=8, nz=24, dz=W.uniform_dz(24, 10.0))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(cfg):
    from paper_2412_04395_amd import erf
    s = erf.Solver(cfg)
    th0 = W.theta_sounding(cfg)
    b = s.init_base_state(th0)
    return s, th0, b


def _force(s, S, cfg, path, levels, rows):
    """Apply a shape through a one-line cache file (no timing involved)."""
    prec = 0 if cfg.prec == "fp64" else 1
    with open(path, "w") as f:
        f.write(f"substep {cfg.nx} {cfg.ny} {cfg.nz} {prec} {levels} {rows} 1.0\n")
    t = s.autotune(S, trials=1, cache_path=str(path))
    assert t["from_cache"] == 1 and (t["levels_per_wave"], t["tile_rows"]) == (levels, rows)


def _pert(S, b):
    out = dict(S)
    out["rho"] = S["rho"] - b["rho0"][:, None, None]
    out["rt"] = S["rt"] - (b["rho0"] * b["theta0"])[:, None, None]
    return out


def test_autotune_times_then_reads_its_cache(tmp_path):
    cfg = W.small(**CFG)
    _say("autotune timing + cache", cfg.nx, cfg.ny, cfg.nz)
    s, th0, b = _solver(cfg)
    S = s.to_device(W.initial_state(cfg, b["rho0"], th0))
    path = tmp_path / "tune.txt"
    t = s.autotune(S, trials=1, cache_path=str(path))
    assert t["from_cache"] == 0 and t["ms_per_step"] > 0
    assert t["levels_per_wave"] in (8, 16) and t["tile_rows"] in (1, 2, 4)
    line = open(path).read().split()
    assert line[:5] == ["substep", "70", "20", "40", "0"]
    assert (int(line[5]), int(line[6])) == (t["levels_per_wave"], t["tile_rows"])
    # a second context reads the choice without timing; a later line wins
    s2, _, _ = _solver(cfg)
    S2 = s2.to_device(W.initial_state(cfg, b["rho0"], th0))
    t2 = s2.autotune(S2, trials=1, cache_path=str(path))
    assert t2["from_cache"] == 1
    assert (t2["levels_per_wave"], t2["tile_rows"]) == (t["levels_per_wave"], t["tile_rows"])
    with open(path, "a") as f:
        f.write("substep 70 20 40 0 16 4 0.5\nsubstep 70 20 40 1 8 2 0.5\nsubstep 70 20 40 0 8 3 0.1\n")
    t3 = s2.autotune(S2, trials=1, cache_path=str(path))
    # the FP32 line is another key and the row count 3 is not a shape: skipped
    assert (t3["levels_per_wave"], t3["tile_rows"], t3["from_cache"]) == (16, 4, 1)
    np.testing.assert_equal(np.isfinite(s2.to_numpy(S2)["rw"]).all(), True)


def test_autotune_rejects_bad_arguments(tmp_path):
    from paper_2412_04395_amd import erf
    cfg = W.small(**CFG)
    s, th0, b = _solver(cfg)
    S = s.to_device(W.initial_state(cfg, b["rho0"], th0))
    with pytest.raises(erf.ErfError) as e:
        s.autotune(S, trials=0)
    assert e.value.status == erf.ERF_E_ARG
    # an unwritable cache path: the choice is still made and applied
    with pytest.raises(erf.ErfError) as e:
        s.autotune(S, trials=1, cache_path=str(tmp_path / "no_such_dir" / "tune.txt"))
    assert e.value.status == erf.ERF_E_ARG
    S0 = s.to_numpy(S)
    s.rk3_step(S)
    assert np.isfinite(s.to_numpy(S)["ru"]).all() and not np.array_equal(s.to_numpy(S)["ru"], S0["ru"])


@pytest.mark.parametrize("grid", ["ragged", "full"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_shape_gives_the_same_step(tmp_path, prec, grid):
    cfg = W.small(**(CFG if grid == "ragged" else CFG_FULL), prec=prec)
    _say("shapes", prec, grid, cfg.nx, cfg.ny, cfg.nz)
    s, th0, b = _solver(cfg)
    S0 = W.initial_state(cfg, b["rho0"], th0)
    out = {}
    for levels in (8, 16):
        for rows in (1, 2, 4):
            S = s.to_device(S0)
            _force(s, S, cfg, tmp_path / f"t{levels}{rows}.txt", levels, rows)
            for _ in range(5):
                s.rk3_step(S)
            out[(levels, rows)] = s.to_numpy(S)
    for levels in (8, 16):
        for rows in (2, 4):
            for f in out[(levels, 1)]:
                assert np.array_equal(out[(levels, rows)][f], out[(levels, 1)][f]), (prec, levels, rows, f)
    if prec == "fp64":
        o = oracle.Oracle(cfg)
        bo = o.init_base_state(th0, cfg.p_surface)
        S = {f: v.copy() for f, v in S0.items()}
        for _ in range(5):
            o.rk3_step(S)
        ref = _pert(S, bo)
        for levels in (8, 16):
            got = _pert(out[(levels, 1)], b)
            mom = max(np.max(np.abs(ref[f])) for f in ("ru", "rv", "rw"))
            for f in ("rho", "rt", "ru", "rv", "rw"):
                # momentum components against the largest one, as in the parity tests
                scale = mom if f in ("ru", "rv", "rw") else np.max(np.abs(ref[f]))
                floor = 4.0 * np.spacing(np.max(np.abs(S[f]))) / scale if f in ("rho", "rt") else 0.0
                err = np.max(np.abs(got[f] - ref[f])) / scale
                _say(f"levels {levels} {f}: {err:.2e}")
                assert err <= max(1e-12, floor), (levels, f, err)
