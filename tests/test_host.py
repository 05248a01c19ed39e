"""Host-side logic on the CPU: the benchmark's contract, the workload recipes
and the analysis of the closure-training script (no GPU needed)."""
import subprocess
import sys
import os

import numpy as np
import pytest

from paper_2412_04395_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_constants():
    sys.path.insert(0, ROOT)
    import bench
    # multiply-adds of 10 -> 64 -> 64 -> 64 -> 9, two flops each
    assert bench.MLP_FLOP_PER_CELL == 18816
    # substep: 19 bulk values and the FP64 Thomas pivots per cell
    assert bench._kernel_bytes("substep", 1, "fp64") == 20 * 8
    assert bench._kernel_bytes("substep", 1, "fp32") == 19 * 4 + 1 * 8
    # whole step of the 14-substep boundary layer: 22 substeps of 20 values,
    # 5 more in each stage's last, 48 + 17 + 5 per stage (slow right-hand side,
    # stage init, coefficients); the first stage, with S'' = 0 on entry, moves
    # 13 + 6 values fewer.  In FP64 the stress pass evaluates mu_t itself: the
    # slow right-hand side is then 10 + 11 + 21 = 42 values, not 10 + 5 + 12 + 21
    cfg = bench._cfg("cbl")
    bulk, f64 = bench._step_values(cfg)
    assert bulk + f64 == 22 * 20 + 3 * 5 + 3 * (42 + 17 + 5) - 19
    assert sum(bench._step_values(cfg.replace(prec="fp32"))) == 22 * 20 + 3 * 5 + 3 * (48 + 17 + 5) - 19
    assert bench._one_pass_values(cfg) == 13 * 5 + 6 + 22 * (3 * 5 + 3)
    # the deep workload (3 WENO5 tracers, 13 substeps, no SGS): prep 3 x 10,
    # tendencies 3 x 14, stage init 3 x 17 - 13, coefficients 3 x 5, substeps
    # 13 x 20 - 6, finalize 3 x 15, flux sums 13 x 6 + 3 x 3 + 3 x 7, mixing
    # ratios 3 x 7 and the scalar update 3 x 12; moist dynamics add 3 x 14
    # (species in and two moist fields out of the primitives pass and of the
    # stage init, each read back by the next kernel)
    deep = W.deep()
    assert sum(bench._step_values(deep)) == 30 + 42 + 38 + 15 + 254 + 45 + 108 + 21 + 36 + 42
    assert sum(bench._step_values(deep.replace(moist=0))) == 30 + 42 + 38 + 15 + 254 + 45 + 108 + 21 + 36


def test_ensemble_recipe():
    cfgs = W.ensemble()
    assert len(cfgs) == 48
    assert sum(c.cells for c in cfgs) == 82_837_504
    qs = np.array([c.surf_heat_flux for c in cfgs])
    assert qs.min() >= 0.05 and qs.max() <= 0.3 and len(set(qs)) == 48
    assert [c.sgs for c in cfgs[:4]] == [1, 2, 1, 2]
    assert [c.seed for c in cfgs[:2]] == [5000, 5001]
    assert all(c.prec == "fp32" and c.dx == 40.0 for c in cfgs)


@pytest.mark.parametrize("make", [W.les_mlp, W.les_fine])
def test_closure_workloads_acoustic_courant(make):
    """Horizontal acoustic Courant number c dtau / dx = 0.43 with c = 347 m/s."""
    c = make()
    cr = 347.0 * (c.dt / c.n_substeps) / c.dx
    assert abs(cr - 0.43) < 0.01
    fine, coarse = W.les_fine(), W.les_mlp()
    assert fine.dx * 4 == coarse.dx and fine.nz // 4 * coarse.dz[0] == fine.nz * fine.dz[0]


def test_profiles_closed_forms():
    """k(z) and the heat flux of a state whose centre velocities and theta are
    known plane waves: <u'u'> = a^2/2 for a cos wave, <w'theta'> = a b / 2."""
    from paper_2412_04395_amd import closure_training as CT
    nz, ny, nx = 4, 8, 16
    x = np.arange(nx)
    kx = 2 * np.pi / nx
    a, b = 2.0, 0.5
    # face velocities whose two-point centre means are a cos(kx (i + 1/2))
    uf = a * np.cos(kx * x) / np.cos(kx / 2)
    rho = np.ones((nz, ny, nx))
    S = {"rho": rho, "ru": np.broadcast_to(uf, (nz, ny, nx)).copy(), "rv": np.zeros((nz, ny, nx)),
         "rw": np.zeros((nz + 1, ny, nx)), "rt": 300.0 + np.zeros((nz, ny, nx))}
    k, flux = CT.profiles(S, np.zeros((nz, ny, nx)))
    assert np.allclose(k, 0.25 * a * a, rtol=1e-12)
    assert np.allclose(flux, 0.0, atol=1e-12)
    # w on faces constant in z (interior): centre w = w0 cos; theta' = b cos
    wf = np.zeros((nz + 1, ny, nx))
    wf[1:-1] = a * np.cos(kx * (x + 0.5))
    S["ru"][:] = 0.0
    S["rw"] = wf
    S["rt"] = 300.0 + b * np.broadcast_to(np.cos(kx * (x + 0.5)), (nz, ny, nx))
    q3 = np.full((nz, ny, nx), 0.01)
    k, flux = CT.profiles(S, q3)
    centre_w = np.array([0.5, 1.0, 1.0, 0.5]) * a   # lid faces carry w = 0
    assert np.allclose(flux, centre_w * b / 2 + 0.01, rtol=1e-12)
    assert np.allclose(k, centre_w ** 2 / 4, rtol=1e-12)


def test_smagorinsky_heat_flux_closed_form():
    """Uniform shear du/dz = g and dtheta/dz = s: nu_t = (Cs Delta)^2 g and
    q_3 = -(nu_t / Pr_t) s."""
    from paper_2412_04395_amd import closure_training as CT
    cfg = W.les_mlp(nx=4, ny=4, nz=4, dz=W.uniform_dz(4, 40.0))
    g, s = 0.02, 0.003
    feat = np.zeros((cfg.cells, 10))
    feat[:, 2] = g
    feat[:, 9] = s
    q3 = CT.smagorinsky_q3(feat, cfg)
    delta = (cfg.dx * cfg.dy * cfg.dz[0]) ** (1 / 3)
    assert np.allclose(q3, -((cfg.Cs * delta) ** 2 * g / cfg.Pr_t) * s, rtol=1e-12)
