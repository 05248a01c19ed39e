"""FP32 path against FP64 on the large workloads, beside an FP64 twin.

    python -m paper_2412_04395_amd.precision_study --out FILE.json [--workloads cbl,deep,member] [--minutes 60]

For each workload three runs start from the same initial state (the seeded
state rounded through the FP32 storage, so that the FP32 run starts exactly
where the FP64 runs do):
  fp64  the FP64 path;
  twin  the FP64 path with rho*theta multiplied by 1 + 2^-52 (one unit in the
        last place of most values) everywhere at the start;
  fp32  the FP32 path (FP32 storage and bulk arithmetic, FP64 column solve and
        sums).
Pointwise differences in a turbulent flow grow chaotically whatever the
precision, so the FP32 error is only meaningful beside the twin's: at every
report time the file holds max |theta' difference| [K], max |u|, |v|, |w|
differences [m/s] (face velocities), the mixing ratios' max differences for
workloads with scalars, and the largest difference of the plane-averaged
theta and u profiles, for fp32 - fp64 and twin - fp64.  Runs on the GPU
through liberf.so; prints a progress line at every report time.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import erf
from . import workloads as W


def _log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


WORKLOADS = {
    # the boundary-layer LES (stable variant, 14 substeps), 256 x 256 x 128
    "cbl": lambda: W.cbl(n_substeps=14, name="cbl@stable_ns14"),
    # the moist deep atmosphere, 512 x 512 x 80, WENO5 water species
    "deep": lambda: W.deep(),
    # one 128 x 128 x 64 member of the ensemble recipe (40 m, Smagorinsky)
    "member": lambda: W.ensemble()[16].replace(sgs=1),
}


def _velocities(S, b):
    rho = S["rho"]
    u = S["ru"] / (0.5 * (rho + np.roll(rho, 1, axis=2)))
    v = S["rv"] / (0.5 * (rho + np.roll(rho, 1, axis=1)))
    w = np.zeros_like(S["rw"])
    w[1:-1] = S["rw"][1:-1] / (0.5 * (rho[1:] + rho[:-1]))
    theta = S["rt"] / rho - b["theta0"][:, None, None]
    return theta, u, v, w


def _compare(A, B, b, nq):
    ta, ua, va, wa = _velocities(A, b)
    tb, ub, vb, wb = _velocities(B, b)
    out = {"theta_K": float(np.abs(ta - tb).max()), "u_m_s": float(np.abs(ua - ub).max()),
           "v_m_s": float(np.abs(va - vb).max()), "w_m_s": float(np.abs(wa - wb).max()),
           "mean_theta_profile_K": float(np.abs(ta.mean(axis=(1, 2)) - tb.mean(axis=(1, 2))).max()),
           "mean_u_profile_m_s": float(np.abs(ua.mean(axis=(1, 2)) - ub.mean(axis=(1, 2))).max())}
    if nq:
        qa, qb = A["rq"] / A["rho"][None], B["rq"] / B["rho"][None]
        out["q_max"] = [float(np.abs(qa[s] - qb[s]).max()) for s in range(nq)]
    return out


def study(name: str, minutes: float, reports: int) -> dict:
    import torch
    cfg32 = WORKLOADS[name]().replace(prec="fp32")
    cfg64 = cfg32.replace(prec="fp64")
    th0, qv0 = W.theta_sounding(cfg64), W.qv0_of(cfg64)
    runs = {}
    for tag, cfg in (("fp64", cfg64), ("twin", cfg64), ("fp32", cfg32)):
        s = erf.Solver(cfg)
        b = s.init_base_state(th0, qv0=qv0)
        runs[tag] = [s, b]
    b = runs["fp64"][1]
    S0 = W.initial_state(cfg64, b["rho0"], th0, b["p0"], b["pi0"], qv0)
    # the state the FP32 storage represents exactly
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    S0["rho"] = rho0 + (S0["rho"] - rho0).astype(np.float32).astype(np.float64)
    S0["rt"] = T0 + (S0["rt"] - T0).astype(np.float32).astype(np.float64)
    for f in ("ru", "rv", "rw", "rq"):
        S0[f] = S0[f].astype(np.float32).astype(np.float64)
    twin = dict(S0)
    twin["rt"] = S0["rt"] * (1.0 + 2.0 ** -52)
    states = {"fp64": runs["fp64"][0].from_full(S0), "twin": runs["twin"][0].from_full(twin),
              "fp32": runs["fp32"][0].from_full(S0)}
    steps = int(round(minutes * 60.0 / cfg64.dt))
    every = max(1, steps // reports)
    series = []
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        for tag in ("fp64", "twin", "fp32"):
            s = runs[tag][0]
            for _ in range(n):
                s.rk3_step(states[tag])
        torch.cuda.synchronize()
        done += n
        full = {tag: runs[tag][0].to_full(states[tag]) for tag in states}
        row = {"t_s": done * cfg64.dt, "fp32_minus_fp64": _compare(full["fp32"], full["fp64"], b, cfg64.n_scalars),
               "twin_minus_fp64": _compare(full["twin"], full["fp64"], b, cfg64.n_scalars),
               "max_w_m_s": float(runs["fp64"][0].diagnostics(states["fp64"], allow_nonfinite=True)["max_w"])}
        series.append(row)
        _log(f"{name}: t = {row['t_s']:.0f} s, fp32 theta' {row['fp32_minus_fp64']['theta_K']:.2e} K, "
             f"w {row['fp32_minus_fp64']['w_m_s']:.2e}; twin theta' {row['twin_minus_fp64']['theta_K']:.2e} K, "
             f"w {row['twin_minus_fp64']['w_m_s']:.2e} ({time.time() - t0:.0f} s)")
    for tag in runs:
        runs[tag][0].close()
    del states
    torch.cuda.empty_cache()
    return {"workload": cfg64.name, "grid": [cfg64.nx, cfg64.ny, cfg64.nz], "dt_s": cfg64.dt,
            "n_substeps": cfg64.n_substeps, "steps": steps, "series": series}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--workloads", default="cbl,deep,member")
    ap.add_argument("--minutes", type=float, default=60.0, help="simulated minutes per workload")
    ap.add_argument("--reports", type=int, default=6)
    a = ap.parse_args(argv)
    res = {"definition": "max abs differences of theta - theta0 [K] and of the face velocities [m/s] against the "
                         "FP64 run; twin = FP64 from rho*theta (1 + 2^-52)", "workloads": []}
    for name in a.workloads.split(","):
        res["workloads"].append(study(name, a.minutes, a.reports))
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
    _log(f"written {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
