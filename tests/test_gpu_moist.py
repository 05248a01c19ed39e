"""Moist dynamics of the HIP path (through the C-ABI) against the FP64 oracle:
the equation of state with water vapour (Sec. 2.1), the 1/(1 + q_v + q_c)
factor on the pressure gradient and the buoyancy of the total density
(eq. mom), the moist base state, and the moist acoustic coefficients of App. C.

Error measures and tolerances as in test_gpu_parity.py: 1e-13 for one call
(FP64), 1e-12 after a few RK3 steps, 1e-5 of each field's scale for the FP32
storage on FP32-representable inputs.  Two exact properties are checked bit
for bit: a moist context given no water reproduces the dry context, and the
host base state with vapour is the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu

CALL_TOL = 1e-13
STEPS_TOL = 1e-12
TOL32 = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _moist(**kw):
    """A small moist column set: stretched levels, three water species by
    WENO5, 3rd-order momentum, the deep workload's time step and substeps."""
    base = dict(name="deep_small", nx=40, ny=19, nz=14, n_scalars=3, scalar_scheme=1, adv_order_h=3,
                adv_order_v=3, dt=2.0, n_substeps=8, moist=1, dx=250.0, dy=250.0,
                dz=W.stretched_dz(14, 50.0, 500.0, 4000.0), seed=31)
    base.update(kw)
    return W.small(**base)


def _sides(cfg):
    """Oracle (FP64) and library context for cfg, each with its own moist base
    state; the two are bitwise equal."""
    from paper_2412_04395_amd import erf
    cfg64 = cfg.replace(prec="fp64")
    qv0 = W.qv0_of(cfg)
    o = oracle.Oracle(cfg64)
    th0 = W.theta_sounding(cfg64)
    bo = o.init_base_state(th0, cfg64.p_surface, qv0)
    s = erf.Solver(cfg)
    bs = s.init_base_state(th0, qv0=qv0)
    for k in ("rho0", "p0", "pi0"):
        assert np.array_equal(bo[k], bs[k]), k
    return o, s, th0, bo, qv0


def _rough(cfg, b, th0, qv0, seed):
    """The workload's initial state with seeded momenta, density and water
    perturbations, so that every moist term is active."""
    S = W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"], qv0)
    shp = S["rho"].shape
    S["ru"] = S["ru"] + S["rho"] * W.uniform_noise(seed + 11, shp, 2.0)
    S["rv"] = S["rv"] + S["rho"] * W.uniform_noise(seed + 12, shp, 2.0)
    rw = W.uniform_noise(seed + 13, S["rw"].shape, 1.0)
    rw[0] = 0.0
    rw[-1] = 0.0
    S["rw"] = rw
    S["rho"] = S["rho"] * (1.0 + W.uniform_noise(seed + 14, shp, 1e-3))
    S["rq"] = S["rq"] * (1.0 + W.uniform_noise(seed + 15, S["rq"].shape, 0.2))
    return {f: np.ascontiguousarray(v) for f, v in S.items()}


def _round32(S, b):
    """The FP64 state that the FP32 storage represents exactly."""
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    out = {"rho": rho0 + (S["rho"] - rho0).astype(np.float32).astype(np.float64),
           "rt": T0 + (S["rt"] - T0).astype(np.float32).astype(np.float64)}
    for f in ("ru", "rv", "rw", "rq"):
        out[f] = S[f].astype(np.float32).astype(np.float64)
    return {k: np.ascontiguousarray(v) for k, v in out.items()}


def _rel(a, b):
    d = np.max(np.abs(a - b)) if a.size else 0.0
    m = np.max(np.abs(b)) if b.size else 0.0
    return d / m if m > 0 else d


def _errs(got, ref, b, fields=("rho", "rt", "ru", "rv", "rw")):
    """Relative errors: rho and rho theta as perturbations about the base state,
    the momenta against the largest momentum component."""
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    e = {}
    if "rho" in fields:
        e["rho"] = _rel(got["rho"] - rho0, ref["rho"] - rho0)
    if "rt" in fields:
        e["rt"] = _rel(got["rt"] - T0, ref["rt"] - T0)
    mom = [f for f in ("ru", "rv", "rw") if f in fields]
    scale = max(np.max(np.abs(ref[f])) for f in mom) if mom else 0.0
    for f in mom:
        e[f] = np.max(np.abs(got[f] - ref[f])) / scale
    return e


MOIST_CASES = {
    # the deep workload's schemes on stretched levels (3rd-order instance)
    "o33": dict(),
    # constant viscosity, 5th-order momentum: the general moist instance
    "o53_visc": dict(adv_order_h=5, adv_order_v=5, nu_m=40.0),
    # narrower than the stencil in x: the general wrap path
    "narrow": dict(nx=2, ny=9),
    # 40 levels in two chunks of the z-marching FP64 tendency kernel, with
    # viscous stresses: the second chunk starts from the moist values below it
    "tall_visc": dict(nx=20, ny=9, nz=40, dz=W.stretched_dz(40, 50.0, 500.0, 8000.0), nu_m=40.0),
}


@pytest.mark.parametrize("case", sorted(MOIST_CASES))
def test_moist_slow_rhs_parity(case):
    cfg = _moist(**MOIST_CASES[case])
    _say("moist slow_rhs", case, cfg.nx, cfg.ny, cfg.nz)
    o, s, th0, b, qv0 = _sides(cfg)
    S = _rough(cfg, b, th0, qv0, 100)
    R_ref = o.slow_rhs(S)
    R = s.to_numpy(s.slow_rhs(s.to_device(S)))
    e = {f: _rel(R[f], R_ref[f]) for f in ("rho", "rt")}
    scale = max(np.max(np.abs(R_ref[f])) for f in ("ru", "rv", "rw"))
    for f in ("ru", "rv", "rw"):
        e[f] = np.max(np.abs(R[f] - R_ref[f])) / scale
    _say(f"moist slow_rhs[{case}]", {f: f"{v:.2e}" for f, v in e.items()})
    for f, v in e.items():
        assert v <= CALL_TOL, (f, v)


@pytest.mark.parametrize("nsub,zero", [(1, True), (1, False), (4, False)])
def test_moist_acoustic_substeps_parity(nsub, zero):
    cfg = _moist()
    _say("moist acoustic", nsub, zero)
    o, s, th0, b, qv0 = _sides(cfg)
    St = _rough(cfg, b, th0, qv0, 200)
    Sn = St if zero else _rough(cfg, b, th0, qv0, 300)
    Rt = o.slow_rhs(St)
    dtau = cfg.dt / cfg.n_substeps if nsub > 1 else cfg.dt / 3.0
    out_ref, F_ref = o.acoustic_substeps(Sn, St, Rt, nsub, dtau)
    Std = s.to_device(St)
    Snd = Std if zero else s.to_device(Sn)
    out, F = s.acoustic_substeps(Snd, Std, s.to_device(Rt), nsub, dtau)
    out, F = s.to_numpy(out), s.to_numpy(F)
    e = _errs(out, out_ref, b)
    for name, a, r in zip(("Fu", "Fv", "Fw"), (F["ru"], F["rv"], F["rw"]), F_ref):
        e[name] = _rel(a, r)
    _say(f"moist acoustic[{nsub},{zero}]", {f: f"{v:.2e}" for f, v in e.items()})
    for f, v in e.items():
        assert v <= CALL_TOL, (f, v)


def test_moist_rk3_parity():
    cfg = _moist()
    _say("moist rk3 x5")
    o, s, th0, b, qv0 = _sides(cfg)
    S = W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"], qv0)
    S["ru"] = S["ru"] + 5.0 * S["rho"]
    Sg = s.to_device(S)
    for _ in range(5):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    e = _errs(got, S, b)
    for q in range(3):
        e[f"rq{q}"] = _rel(got["rq"][q], S["rq"][q])
    _say("moist rk3 x5", {f: f"{v:.2e}" for f, v in e.items()})
    for f, v in e.items():
        assert v <= STEPS_TOL, (f, v)
    dg, do = s.diagnostics(Sg), o.diagnostics(S)
    assert abs(dg["mass"] / do["mass"] - 1) < 1e-14
    for q in range(3):
        assert abs(dg["scalar_mass"][q] / do["scalar_mass"][q] - 1) < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_moist_without_water_is_the_dry_context_bitwise(prec):
    """moist = 1 with zero water and qv0 = 0 against moist = 0 on the same
    state: every moist factor is exactly 1 and every added term exactly 0, so
    two RK3 steps agree bit for bit."""
    from paper_2412_04395_amd import erf
    cfg = _moist(prec=prec)
    dry = cfg.replace(moist=0)
    th0 = W.theta_sounding(cfg)
    sm, sd = erf.Solver(cfg), erf.Solver(dry)
    bm = sm.init_base_state(th0, qv0=np.zeros(cfg.nz))
    bd = sd.init_base_state(th0)
    for k in ("rho0", "p0", "pi0"):
        assert np.array_equal(bm[k], bd[k]), k
    S = W.initial_state(dry, bd["rho0"], th0, bd["p0"], bd["pi0"])
    S["ru"] = S["ru"] + 4.0 * S["rho"]
    S["rq"][:] = 0.0
    Sm, Sd = sm.from_full(S), sd.from_full(S)
    for _ in range(2):
        sm.rk3_step(Sm)
        sd.rk3_step(Sd)
    a, c = sm.to_numpy(Sm), sd.to_numpy(Sd)
    for f in ("rho", "rt", "ru", "rv", "rw", "rq"):
        assert np.array_equal(a[f], c[f]), f
    _say("moist without water == dry", prec)


def test_moist_rest_state_stays_at_rest():
    """rho = rho0, Theta = rho0 theta0, rho q_v = rho0 q_v0 without wind or
    condensate is the moist base state itself: 20 RK3 steps keep w at the
    rounding level of q_v = (rho0 q_v0) / rho0, as on the oracle."""
    cfg = _moist()
    o, s, th0, b, qv0 = _sides(cfg)
    S = o.zeros_state()
    S["rho"][:] = b["rho0"][:, None, None]
    S["rt"][:] = (b["rho0"] * th0)[:, None, None]
    S["rq"][0] = (b["rho0"] * qv0)[:, None, None]
    Sg = s.to_device(S)
    for _ in range(20):
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    wmax = np.max(np.abs(got["rw"]))
    _say("moist rest state: max |rho w| after 20 steps", f"{wmax:.2e}")
    assert wmax < 1e-10
    assert np.max(np.abs(got["rho"] - b["rho0"][:, None, None])) < 1e-12


def test_moist_fp32_rk3_against_fp64():
    """Four FP32 RK3 steps of the moist case against the FP64 oracle from the
    FP32-rounded initial state (nx = 130: two x-tiles of the scalar kernel and
    a tail), each field to 1e-5 of its scale."""
    cfg = _moist(nx=130, ny=17, prec="fp32", seed=33)
    _say("moist fp32 rk3 x4")
    o, s, th0, b, qv0 = _sides(cfg)
    S = W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"], qv0)
    S["ru"] = S["ru"] + 5.0 * S["rho"]
    S = _round32(S, b)
    Sg = s.from_full(S)
    for _ in range(4):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_full(Sg)
    e = _errs(got, S, b)
    for q in range(3):
        e[f"rq{q}"] = _rel(got["rq"][q], S["rq"][q])
    _say("moist fp32 rk3 x4", {f: f"{v:.2e}" for f, v in e.items()})
    for f, v in e.items():
        assert v <= TOL32, (f, v)


def test_moist_fp32_slow_rhs_and_stage():
    """One FP32 slow right-hand side and one stage of four substeps on
    FP32-representable moist inputs, against the FP64 oracle."""
    cfg = _moist(prec="fp32", seed=35)
    o, s, th0, b, qv0 = _sides(cfg)
    St = _round32(_rough(cfg, b, th0, qv0, 400), b)
    Sn = _round32(_rough(cfg, b, th0, qv0, 500), b)
    R_ref = o.slow_rhs(St)
    R = s.to_numpy(s.slow_rhs(s.from_full(St)))
    e = {f"R{f}": _rel(R[f], R_ref[f]) for f in ("rho", "rt")}
    scale = max(np.max(np.abs(R_ref[f])) for f in ("ru", "rv", "rw"))
    for f in ("ru", "rv", "rw"):
        e[f"R{f}"] = np.max(np.abs(R[f] - R_ref[f])) / scale
    R32 = {f: R_ref[f].astype(np.float32).astype(np.float64) for f in ("rho", "rt", "ru", "rv", "rw")}
    R32["rq"] = np.zeros((3, cfg.nz, cfg.ny, cfg.nx))
    dtau = cfg.dt / cfg.n_substeps
    out_ref, _ = o.acoustic_substeps(Sn, St, R32, 4, dtau)
    Rd = s.to_device(R32)
    out, _ = s.acoustic_substeps(s.from_full(Sn), s.from_full(St), Rd, 4, dtau)
    e.update(_errs(s.to_full(out), out_ref, b))
    _say("moist fp32 per call", {f: f"{v:.2e}" for f, v in e.items()})
    for f, v in e.items():
        assert v <= TOL32, (f, v)
