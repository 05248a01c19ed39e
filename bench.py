"""Benchmark: cell-updates/s of one RK3 step (with all acoustic substeps) of the
compressible dynamical core on one MI355X, through the C-ABI of liberf.so.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
    (NAME: cbl (default), cbl_as_stated, cbl_fp32, bubble2d; ensemble and
    closure_training run that leg alone)

Prints ONE JSON line.  The workload is the 3-D dry convective boundary layer
LES, 256 x 256 x 128 cells, FP64 (5th-order upwind advection, Smagorinsky,
Coriolis with geostrophic wind, surface heat flux), with seeded synthetic
initial data.  As specified (dt = 0.5 s, 6 substeps) the horizontal acoustic
substep is unstable at 20 m spacing and the run diverges in its first step;
the headline therefore uses the stable variant with 14 substeps per step, and
the as-specified variant is timed beside it (values do not change the
arithmetic performed).

``value`` is whole-job throughput with inputs resident in HBM; the roofline
object refers to the kernel with the largest share of the step time, whose
average launch duration is measured with HIP events recorded by the library on
its own stream during the timed steps.  ``cpu_baseline`` times the FP64 CPU
oracle (a reported baseline, never the target) on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2412_04395_amd import workloads as W  # noqa: E402

METRIC = "cell-updates/s per RK3 step (incl. acoustic substeps), % HBM roofline, FP64 vs FP32"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, vendor figure
# multiply-adds of one evaluation of the 10 -> 64 -> 64 -> 64 -> 9 closure network
MLP_FLOP_PER_CELL = 2 * (10 * 64 + 64 * 64 + 64 * 64 + 64 * 9)

# Compulsory (algorithmic) values moved per cell by one launch of each kernel:
# every distinct input field read once and every output written once.
# (bulk values, FP64 values): bulk fields are stored in the run's precision
# (8 B in FP64, 4 B in FP32); the tridiagonal pivots are always FP64.
# 'sgs' = 1 adds the fields only viscous runs touch.
KERNEL_VALUES = {
    # rho, U, V, W, theta, p', u, v, w read (+ 6 stresses and the diffusivity); 5 tendencies written
    "rhs": lambda sgs: (9 + 7 * sgs + 5, 0),
    # rho, Theta, U, V, W read; theta, p', u, v, w written
    "prep": lambda sgs: (5 + 5, 0),
    # rho, u, v, w read; mu_t written
    "mut": lambda sgs: (4 + 1, 0),
    # u, v, w, rho, mu_t read; 6 stresses and the diffusivity written
    "stress": lambda sgs: (5 + 7, 0),
    # FP64 outside the Deardorff closure: mu_t evaluated in the stress pass
    # itself (u, v, w, rho read; 6 stresses and the diffusivity written), no
    # separate mu_t pass
    "stress_fused": lambda sgs: (4 + 7, 0),
    # one fused substep: Theta'' (two levels), U'', V'', rho'', W'', the five
    # tendencies, theta^t, Exner and the buoyancy coefficient read, the Thomas
    # pivots read; Theta'', U'', V'', rho'', W'' written
    "substep": lambda sgs: (14 + 5, 1),
    # (the last substep of a stage, without scalars, also reads S^t and writes
    # S_out in place of S'': 5 more bulk values; see _substep_value_adjust)
    # S^n, S^t read; theta^t, Exner, Theta'', rho'', U'', V'', W'' written
    "stage_init": lambda sgs: (10 + 7, 0),
    # Exner, theta^t, Theta^t read; buoyancy coefficient and the pivots written
    "coef": lambda sgs: (3 + 1, 1),
    # S^t and S'' read; S_out written
    "finalize": lambda sgs: (10 + 5, 0),
    # Deardorff closure: rho e, rho, mu_t and the local source read; the source written
    "tke": lambda sgs: (4 + 1, 0),
}
# Advected scalars (nq of them), per cell of one launch: the mixing ratios
# q^t = (rho q)^t / rho^t (rho q and rho read, q written); the scalar update
# (q, the three averaged momenta and (rho q)^n read, (rho q)^new written).
SCALAR_VALUES = {"mixing_ratio": lambda nq: (2 * nq + 1, 0), "scalar": lambda nq: (3 * nq + 3, 0)}
# Kessler microphysics once per step: rho, rho theta and the three species read,
# rho theta and the species written (the fall of rain re-reads its column)
MICRO_VALUES = {"kessler": lambda nq: (5 + 4, 0)}
# The first RK3 stage starts from S^t = S^n with one substep, so S'' = 0 on
# entry: its stage init moves only Theta^t, rho^t in and theta^t, Exner out
# (13 bulk values fewer) and its substep reads none of the 6 S'' inputs
# (Theta'' twice, U'', V'', rho'', W'').
ZERO_START_SAVED = {"stage_init": 13, "substep": 6}
# Anelastic step (SSP-RK2 with two projections), per cell of one launch, all
# FP64: the stage update reads S^n, R1 (and R2) for rho theta and the three
# momenta and writes four fields (12 values in stage 1, 16 in stage 2: 14 on
# average); the projection's divergence and x transform read three momenta
# and write a complex value of the half spectrum (nx/2 + 1 of nx per line);
# each y transform reads and writes a complex value of it; the z solve reads
# and writes the complex value twice and writes and reads the Thomas factor;
# the inverse x transform reads a complex value and writes phi; the
# correction reads three momenta, phi, the pressure and writes the momenta
# and the pressure.  h = (nx/2 + 1)/nx.
def anel_values(nx: int) -> dict:
    h = (nx // 2 + 1) / nx
    return {"ssp_update": 14, "div_fftx": 3 + 2 * h, "ffty": 4 * h, "poisson_z": 10 * h, "ifftx": 2 * h + 1,
            "project": 9}


ANEL_KERNELS = ("prep", "mut", "stress", "rhs", "ssp_update", "div_fftx", "ffty", "poisson_z", "ifftx", "project")

# Moist dynamics, per stage: the primitives pass also reads rho q_v, rho q_c,
# rho q_r and writes 1 + q_v + q_c and the total-density departure, which the
# tendencies read; the stage init reads the three species and writes the moist
# Exner function and rho_d / rho_m, which the coefficients read.
MOIST_STAGE_VALUES = {"prep": 5, "rhs": 2, "stage_init": 5, "coef": 2}


def _stress_fused(cfg) -> bool:
    """FP64 runs with Smagorinsky evaluate mu_t inside the stress pass."""
    return cfg.prec == "fp64" and cfg.sgs == 1


def _kernel_bytes(kernel: str, sgs: int, prec: str) -> float:
    bulk, f64 = KERNEL_VALUES[kernel](sgs)
    return bulk * (8.0 if prec == "fp64" else 4.0) + f64 * 8.0


def _profiled_traffic(kernel: str, prec: str = "fp64"):
    """HBM bytes per launch of `kernel` in precision `prec` from the committed
    rocprofv3 counter summary under profiles/, if the kernel's source is
    unchanged since."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        fields = dict(re.findall(r"^\s+(kernel|precision|source|source_sha256|traffic_bytes_per_launch): (\S+)$",
                                 text, re.M))
        if fields.get("kernel") != kernel or fields.get("precision", "fp64") != prec or "source" not in fields:
            continue
        src = os.path.join(ROOT, fields["source"])
        if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == fields.get("source_sha256"):
            return float(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def _cfg(workload: str) -> W.Config:
    if workload == "cbl":
        return W.cbl(n_substeps=14, name="cbl@stable_ns14")
    if workload == "cbl_as_stated":
        return W.cbl(n_substeps=6, name="cbl@as_stated_ns6")
    if workload == "cbl_fp32":
        return W.cbl(n_substeps=14, name="cbl@stable_ns14", prec="fp32")
    if workload == "bubble2d":
        return W.bubble2d()
    raise SystemExit(f"unknown workload {workload}")


def _time_steps(s, S, steps: int, torch, kernel: str | None = None):
    if kernel:
        s.timing_begin(kernel, max_launches=64 * steps + 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.rk3_step(S)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = s.timing_end() if kernel else (0.0, 0)
    return el, kt


def run_gpu(cfg: W.Config, steps: int, warmup: int):
    import torch
    from paper_2412_04395_amd import erf

    s = erf.Solver(cfg)
    th0, qv0 = W.theta_sounding(cfg), W.qv0_of(cfg)
    b = s.init_base_state(th0, qv0=qv0)
    S = s.from_full(W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"], qv0))
    for _ in range(warmup):
        s.rk3_step(S)
    tune = s.autotune(S, trials=2, cache_path=_tune_cache())
    # find the kernel with the largest share of a step (one short timed step per kernel)
    shares = {}
    for k in (list(KERNEL_VALUES) + (list(SCALAR_VALUES) if cfg.n_scalars else []) +
              (list(MICRO_VALUES) if getattr(cfg, "microphysics", 0) else []) +
              (["tke"] if cfg.sgs == 3 else []) + (["most"] if getattr(cfg, "most_z0", 0.0) > 0 else [])):
        if (k == "mut" and not cfg.sgs) or k == "stress_fused":  # (an accounting entry, timed as "stress")
            continue
        _, (ms, n) = _time_steps(s, S, 1, torch, kernel=k)
        if n:
            shares[k] = (ms, n)
    dominant = max(shares, key=lambda k: shares[k][0])
    el, (kms, kn) = _time_steps(s, S, steps, torch, kernel=dominant)
    d = s.diagnostics(S, allow_nonfinite=True)
    s.close()
    d["substep_shape"] = {"levels_per_wave": tune["levels_per_wave"], "tile_rows": tune["tile_rows"],
                          "from_cache": bool(tune["from_cache"])}
    return el, dominant, kms, kn, shares, d


WEIGHTS = os.path.join(ROOT, "paper_2412_04395_amd", "data", "closure_les40m.npz")
# launch shapes of the acoustic substep chosen by erf_autotune on MI355X, one
# line per grid size and precision
TUNE_CACHE = os.path.join(ROOT, "paper_2412_04395_amd", "data", "substep_shapes.txt")
_tune_copy = None


def _tune_cache() -> str:
    """A private copy of the committed cache: its lines are read, and shapes
    tuned for grids it lacks are appended to the copy, not to the package."""
    global _tune_copy
    if _tune_copy is None:
        import shutil
        import tempfile
        import atexit
        fd, _tune_copy = tempfile.mkstemp(prefix="substep_shapes_", suffix=".txt")
        os.close(fd)
        atexit.register(lambda p=_tune_copy: os.path.exists(p) and os.remove(p))
        if os.path.exists(TUNE_CACHE):
            shutil.copyfile(TUNE_CACHE, _tune_copy)
    return _tune_copy


def closure_weights(solver, S, seed: int):
    """Trained closure weights if the package holds them, else He-initialised
    weights with input scales from S floored at physical values (1e-2 1/s,
    1e-3 K/m) and output scales of 1e-4 (the values do not change the work)."""
    if os.path.exists(WEIGHTS):
        z = np.load(WEIGHTS, allow_pickle=False)
        solver.mlp_set_weights(z["params"], z["norm"])
        return "trained"
    import torch
    from paper_2412_04395_amd import erf
    rng = np.random.default_rng(seed)
    p = np.zeros(erf.MLP_NPARAMS)
    for off, fan_in, fan_out in ((0, 10, 64), (704, 64, 64), (4864, 64, 64), (9024, 64, 9)):
        p[off:off + fan_in * fan_out] = rng.normal(0, np.sqrt(2.0 / fan_in), fan_in * fan_out)
    solver.mlp_set_weights(p.astype(np.float32))
    feat = solver.mlp_features(S)
    solver.mlp_fit_norm(feat, torch.zeros((feat.shape[0], 9), dtype=torch.float64, device=feat.device))
    del feat
    p32, nrm = solver.mlp_get_weights()
    nrm[10:19] = np.maximum(nrm[10:19], 1e-2)
    nrm[19] = max(nrm[19], 1e-3)
    nrm[29:] = 1e-4
    solver.mlp_set_weights(p32, nrm)
    return "he-initialised"


def run_closure(steps: int, warmup: int):
    """RK3 steps of the coarse LES with the learned closure (128x128x64, FP32):
    step throughput and the closure kernel's matrix-core roofline (weights as
    closure_weights gives them)."""
    import torch
    from paper_2412_04395_amd import erf

    cfg = W.les_mlp()
    s = erf.Solver(cfg)
    th0 = W.theta_sounding(cfg)
    b = s.init_base_state(th0)
    S = s.from_full(W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"]))
    weights = closure_weights(s, S, cfg.seed)
    for _ in range(warmup):
        s.rk3_step(S)
    tune = s.autotune(S, trials=2, cache_path=_tune_cache())
    shares = {}
    for k in ("mlp", "mlp_div", "rhs", "substep"):
        _, (ms, n) = _time_steps(s, S, 1, torch, kernel=k)
        shares[k] = round(ms, 4)
    fb0 = s.mlp_fallback_count()
    el, (kms, kn) = _time_steps(s, S, steps, torch, kernel="mlp")
    fb = s.mlp_fallback_count() - fb0
    d = s.diagnostics(S, allow_nonfinite=True)
    s.close()
    avg_ms = kms / max(kn, 1)
    flops = MLP_FLOP_PER_CELL * cfg.cells
    achieved = flops / (avg_ms * 1e-3) / 1e12
    return {"workload": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "precision": "FP32 storage, BF16 network",
            "weights": weights, "substep_shape": {"levels_per_wave": tune["levels_per_wave"],
                                                  "tile_rows": tune["tile_rows"],
                                                  "from_cache": bool(tune["from_cache"])},
            "value": cfg.cells * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
            "kernel_ms_per_step": shares, "fallback_fraction": fb / (3 * steps * cfg.cells),
            "final_diag": {"max_w": d["max_w"], "nonfinite": d["nonfinite"]},
            "roofline": {"bound": "mfma", "kernel": "mlp", "achieved": round(achieved, 2),
                         "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                         "traffic": None, "flop_per_launch": flops, "avg_launch_ms": round(avg_ms, 4),
                         "launches_timed": kn}}


# one training sample: the forward products (MLP_FLOP_PER_CELL), the weight
# gradients of all four layers (as many multiply-adds again) and the input
# gradients of layers 2-4 (64*64 + 64*64 + 64*9 multiply-adds)
TRAIN_FLOP_PER_SAMPLE = 2 * MLP_FLOP_PER_CELL + 2 * (64 * 64 + 64 * 64 + 64 * 9)


def run_training(steps: int, batches=(16384, 262144)):
    """Adam steps of the closure network (erf_mlp_train_step: BF16 MFMA forward
    and backward products, FP64 loss and column sums, Adam) on synthetic
    standardised samples; throughput against the BF16 matrix-core peak."""
    import torch
    from paper_2412_04395_amd import erf

    cfg = W.les_mlp(nx=16, ny=16, nz=8, dz=W.uniform_dz(8, 40.0))  # the context only holds the network
    s = erf.Solver(cfg)
    gen = torch.Generator(device="cuda").manual_seed(cfg.seed)
    p = np.random.default_rng(cfg.seed).normal(0.0, 0.1, erf.MLP_NPARAMS).astype(np.float32)
    s.mlp_set_weights(p)
    out = {}
    for b in batches:
        x = torch.randn((b, 10), generator=gen, device="cuda", dtype=torch.float32)
        t = torch.randn((b, 9), generator=gen, device="cuda", dtype=torch.float32)
        for _ in range(3):
            s.mlp_train_step(x, t, 1e-4, want_loss=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        for _ in range(steps):
            s.mlp_train_step(x, t, 1e-4, want_loss=False)
        e1.record(s.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        tflops = TRAIN_FLOP_PER_SAMPLE * b / (ms * 1e-3) / 1e12
        out[str(b)] = {"ms_per_step": round(ms, 4), "samples_per_s": b / (ms * 1e-3),
                       "achieved_tflops": round(tflops, 2), "frac_bf16_peak": round(tflops / BF16_PEAK_TFLOPS, 4)}
    s.close()
    return {"workload": "closure network training, synthetic standardised samples",
            "flop_per_sample": TRAIN_FLOP_PER_SAMPLE, "peak_tflops": BF16_PEAK_TFLOPS, "batches": out}


def _ensemble_leg(cfgs, steps: int, warmup: int):
    """Member steps one after another on one stream, then the ensemble's graph
    launches in the autotuned mode (batched or not, branch count)."""
    import torch
    from paper_2412_04395_amd import erf

    ens = erf.Ensemble(cfgs)
    states, weights = [], None
    for s, c in zip(ens.members, cfgs):
        th0 = W.theta_sounding(c)
        b = s.init_base_state(th0)
        S = s.from_full(W.initial_state(c, b["rho0"], th0, b["p0"], b["pi0"]))
        if c.sgs == 2:
            weights = closure_weights(s, S, c.seed)
        states.append(S)
    cells = sum(c.cells for c in cfgs)
    for _ in range(warmup):
        for s, S in zip(ens.members, states):
            s.rk3_step(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, S in zip(ens.members, states):
            s.rk3_step(S)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    nb, tune_ms = ens.autotune(states, trials=2)
    mode = f"{'batched' if ens.batched else 'unbatched'}, {nb} branches"
    for _ in range(warmup):
        ens.rk3_step(states)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ens.rk3_step(states)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bad = sum(s.diagnostics(S, allow_nonfinite=True)["nonfinite"] for s, S in zip(ens.members, states))
    ens.close()
    del states
    torch.cuda.empty_cache()
    return {"value": cells * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
            "mode": mode, "weights": weights,
            "sequential_ms_per_step": 1e3 * el_seq / steps, "speedup_vs_sequential": el_seq / el,
            "nonfinite": bad}, cells


def run_ensemble(steps: int, warmup: int, per_size: int = 16):
    """The 48-member ensemble (16 each of 96x96x64, 128x128x64, 192x192x96 at
    40 m, FP32 path, odd members on the learned closure) and the same 48 grids
    as FP64 members on Smagorinsky (the reference the FP32 + closure ensemble is
    compared with): member steps one after another on one stream against one
    graph launch per ensemble step in the autotuned mode."""
    cfgs = W.ensemble(per_size=per_size)
    out, cells = _ensemble_leg(cfgs, steps, warmup)
    ref, _ = _ensemble_leg([c.replace(prec="fp64", sgs=1) for c in cfgs], steps, warmup)
    out.update({"workload": f"ensemble of {len(cfgs)} boundary-layer members", "members": len(cfgs),
                "cells": cells, "precision": "FP32 storage and bulk arithmetic; odd members BF16 closure",
                "fp64_smagorinsky": {k: ref[k] for k in ("value", "ms_per_step", "mode", "sequential_ms_per_step",
                                                         "speedup_vs_sequential", "nonfinite")},
                "ratio_vs_fp64_smagorinsky": out["value"] / ref["value"]})
    return out


def _omp_threads(n=None):
    """The OpenMP runtime the oracle runs on (libgomp): its thread count, set
    to n first if given; None where the runtime cannot be reached."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def cpu_baseline(cfg: W.Config, target_s: float = 12.0, target_1core_s: float = 8.0):
    """FP64 oracle on a bounded sample: the same physics on a 64 x 64 column
    block of the workload (periodic), timed for whole RK3 steps on all the
    OpenMP threads of the host and again on one thread."""
    import oracle

    sample = cfg.replace(nx=64, ny=64, name=cfg.name)
    o = oracle.Oracle(sample)
    th0 = W.theta_sounding(sample)
    b = o.init_base_state(th0, sample.p_surface)
    S = W.initial_state(sample, b["rho0"], th0, b["p0"], b["pi0"])

    def timed(limit):
        steps, t0 = 0, time.perf_counter()
        while True:
            o.rk3_step(S)
            steps += 1
            el = time.perf_counter() - t0
            if el > limit or steps >= 60:
                return steps, el

    cores = _omp_threads() or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    steps, el = timed(target_s)
    out = {"value": sample.cells * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{sample.nx}x{sample.ny}x{sample.nz} block of the same workload, {steps} RK3 steps, "
                     f"{el:.1f} s"}
    if _omp_threads(1) == 1:
        s1, e1 = timed(target_1core_s)
        _omp_threads(cores)
        out["value_1core"] = sample.cells * s1 / e1
        out["sample_1core"] = f"the same block on one thread, {s1} RK3 steps, {e1:.1f} s"
    return out


def _step_values(cfg):
    """Algorithmic values per cell of one RK3 step, summed over the kernels that
    run in it: (values in the storage precision, FP64 values)."""
    sgs = 1 if cfg.sgs else 0
    ns = cfg.n_substeps
    counts = {"prep": 3, "rhs": 3, "mut": 3 * sgs, "stress": 3 * sgs, "stage_init": 3, "coef": 3,
              "substep": 1 + ns // 2 + ns, "finalize": 3 if cfg.n_scalars else 0}
    if _stress_fused(cfg):
        counts["mut"] = counts["stress"] = 0
        counts["stress_fused"] = 3
    bulk = f64 = 0
    for k, n in counts.items():
        b, f = KERNEL_VALUES[k](sgs)
        bulk += n * b - (ZERO_START_SAVED.get(k, 0) if n else 0)
        f64 += n * f
    if getattr(cfg, "moist", 0):
        bulk += 3 * sum(MOIST_STAGE_VALUES.values())
    if not cfg.n_scalars:
        bulk += 3 * 5  # the stage end written by the last substep of each stage
    if cfg.n_scalars:
        # flux sums for the scalar transport: read and written by every
        # substep, zeroed by each stage init; the finalize then also reads
        # them and W^n and writes the averaged momenta (22 values, not 15)
        bulk += 6 * counts["substep"] + 3 * 3 + 3 * (22 - 15)
        for f in SCALAR_VALUES.values():
            bulk += 3 * f(cfg.n_scalars)[0]
    return bulk, f64


def _one_pass_values(cfg) -> int:
    """Lower bound on values per cell of a step for a design that makes one
    grid pass per substep and per stage (3-D, F = 5 acoustic fields)."""
    F, ns, nq = 5, cfg.n_substeps, cfg.n_scalars
    chi = 1 if nq else 0
    return 13 * F + 6 + (1 + ns // 2 + ns) * (3 * F + 3 + 6 * chi) + 9 * nq + 12 * chi


def _copy_gbs() -> float:
    """Measured device-to-device copy rate (1 GiB each way), GB/s."""
    import torch
    src = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * 5 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def _step_roofline(cfg, ms_per_step: float, copy_gbs: float) -> dict:
    eb = 8.0 if cfg.prec == "fp64" else 4.0
    bulk, f64 = _step_values(cfg)
    design = (bulk * eb + f64 * 8.0) * cfg.cells
    bound = _one_pass_values(cfg) * eb * cfg.cells
    ach = design / (ms_per_step * 1e-3) / 1e9
    return {"design_values_per_cell": bulk + f64, "design_gb_per_step": round(design / 1e9, 3),
            "achieved_gbs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "one_pass_bound_values_per_cell": _one_pass_values(cfg),
            "one_pass_bound_frac": round(bound / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(ach / copy_gbs, 4)}


def run_scalars(steps: int, warmup: int) -> dict:
    """The 80-level deep-atmosphere workload: 512 x 512 x 80, FP32 storage, three
    tracers advected by WENO5 after every stage (the scalar-heavy case)."""
    cfg = W.deep()
    el, dom, kms, kn, shares, diag = run_gpu(cfg, steps, warmup)
    out = {"workload": "moist deep atmosphere 512x512x80, stretched dz, q_v, q_c, q_r by WENO5 and in the dynamics",
           "grid": [cfg.nx, cfg.ny, cfg.nz],
           "precision": "FP32 storage and bulk stencil arithmetic; FP64 base state, column solve and sums",
           "n_scalars": cfg.n_scalars,
           "n_substeps": cfg.n_substeps, "value": cfg.cells * steps / el, "unit": "cell-updates/s",
           "ms_per_step": 1e3 * el / steps, "substep_shape": diag["substep_shape"],
           "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares.items()},
           "nonfinite": diag["nonfinite"]}
    if "scalar" in shares:
        ms, n = shares["scalar"]
        us = 1e3 * ms / n
        byts = SCALAR_VALUES["scalar"](cfg.n_scalars)[0] * 4.0 * cfg.cells
        out["scalar_kernel"] = {"us_per_launch": round(us, 1), "algorithmic_bytes_per_launch": byts,
                                "achieved_gbs": round(byts / (us * 1e-6) / 1e9, 1),
                                "frac": round(byts / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    out["step_roofline"] = _step_roofline(cfg, 1e3 * el / steps, _copy_gbs())
    # the same workload with Kessler warm rain after every step
    cfg_k = cfg.replace(microphysics=1)
    el_k, _, _, _, shares_k, diag_k = run_gpu(cfg_k, steps, warmup)
    out["with_kessler"] = {"ms_per_step": 1e3 * el_k / steps, "value": cfg.cells * steps / el_k,
                           "kessler_ms_per_step": round(shares_k.get("kessler", (0.0, 0))[0], 4),
                           "nonfinite": diag_k["nonfinite"]}
    return out


def run_tke(steps: int, warmup: int) -> dict:
    """The 256 x 256 x 128 boundary layer with the Deardorff TKE closure and a
    Monin-Obukhov surface layer (FP64, 14 substeps)."""
    cfg = W.cbl_tke()
    el, dom, kms, kn, shares, diag = run_gpu(cfg, steps, warmup)
    return {"workload": "boundary-layer LES 256x256x128, Deardorff TKE closure, surface layer z0 = 0.1 m",
            "grid": [cfg.nx, cfg.ny, cfg.nz], "precision": "fp64", "n_substeps": cfg.n_substeps,
            "value": cfg.cells * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
            "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares.items()},
            "roofline": _roofline(cfg, dom, kms, kn),
            "final_diag": {"max_w": diag["max_w"], "nonfinite": diag["nonfinite"]}}


def run_anelastic(steps: int, warmup: int) -> dict:
    """The boundary-layer workload in the anelastic equation set: 256 x 256 x
    128, FP64, Smagorinsky, SSP-RK2 with a projection after each stage, the
    same dt."""
    import torch
    from paper_2412_04395_amd import erf

    cfg = W.cbl(anelastic=1, name="cbl_anelastic")
    s = erf.Solver(cfg)
    th0 = W.theta_sounding(cfg)
    b = s.init_base_state(th0)
    S = s.to_device(W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"]))
    s.project(S, cfg.dt)  # a divergence-free start
    for _ in range(warmup):
        s.ssprk2_step(S)

    def timed(n, kernel=None):
        if kernel:
            s.timing_begin(kernel, max_launches=16 * n + 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            s.ssprk2_step(S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return el, (s.timing_end() if kernel else (0.0, 0))

    shares = {}
    for k in ANEL_KERNELS:
        _, (ms, n) = timed(1, k)
        if n:
            shares[k] = (ms, n)
    dom = max(shares, key=lambda k: shares[k][0])
    el, (kms, kn) = timed(steps, dom)
    d = s.diagnostics(S, allow_nonfinite=True)
    s.close()
    avg_ms = kms / max(kn, 1)
    av = anel_values(cfg.nx)
    vals = av[dom] if dom in av else KERNEL_VALUES[dom](1)[0]
    byts = vals * 8.0 * cfg.cells
    gbs = byts / (avg_ms * 1e-3) / 1e9
    return {"workload": "boundary-layer LES 256x256x128 in the anelastic equation set (SSP-RK2, projections)",
            "grid": [cfg.nx, cfg.ny, cfg.nz], "precision": "fp64", "dt": cfg.dt,
            "value": cfg.cells * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
            "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares.items()},
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": byts,
                         "avg_launch_ms": round(avg_ms, 4), "launches_timed": kn},
            "final_diag": {"max_w": d["max_w"], "nonfinite": d["nonfinite"]}}


# terrain kernels: compulsory FP64 values per cell of one launch (reads +
# writes): the slow tendencies read rho, rho u, rho v, theta, u, v, w, p',
# rho Omega, the cell height and rho0 and write five tendencies; the U'', V''
# step reads Theta'' (two levels), pi^t, U'', V'', their tendencies and the
# cell height and writes U'', V''; the metric part of Omega'' reads U'', V''
# and writes one value per z-face; the explicit Theta'', rho'' read theta^t,
# U'', V'', W'', Theta'', rho'', two tendencies, h_zeta, the cell height and
# the old and new metric parts and write two; the column kernel reads the
# cell height, pi^t, rho0, pi0, rho theta^t, theta^t, Theta'' (current and
# explicit), rho'' (current and explicit), W'' and its tendency and writes
# W'', Theta'', rho''
TERRAIN_VALUES = {"ter_rhs": 16, "ter_uv": 10, "ter_m": 3, "ter_hat": 14, "ter_tri": 15}


def terrain_cpu_oracle(target_s: float = 8.0) -> dict:
    """FP64 oracle on a bounded sample of the terrain workload: a 64 x 64 column
    block of the same grid over the same hill (scaled to the block), timed for
    whole RK3 steps on all the host's OpenMP threads."""
    import oracle

    cfg = W.terrain_hill()
    sample = cfg.replace(nx=64, ny=64)
    h = W.agnesi_nodes(sample, 400.0, 2000.0 * 64 / cfg.nx)
    o = oracle.Oracle(sample)
    o.set_terrain(h, 1.0)
    Hc, zc = o.terrain_heights()
    th0 = W.stratified_theta(zc, 300.0, 0.01, sample.grav)
    ps = W.stratified_ground_pressure(W.cell_mean_nodes(h), 300.0, 0.01, sample.p_surface, sample.grav)
    b = o.init_base_state_columns(th0, ps)
    shp = b["rho0"].shape
    S = {"rho": b["rho0"].copy(), "rt": b["rho0"] * b["theta0"], "ru": b["rho0"] * 10.0, "rv": np.zeros(shp),
         "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": np.zeros((0,) + shp)}
    S = {k: np.ascontiguousarray(v) for k, v in S.items()}
    steps, t0 = 0, time.perf_counter()
    while True:
        o.rk3_step(S)
        steps += 1
        el = time.perf_counter() - t0
        if el > target_s or steps >= 40:
            break
    cores = _omp_threads() or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sample.cells * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample.nx}x{sample.ny}x{sample.nz} block of the terrain grid over a hill of the same "
                      f"height and shape, {steps} RK3 steps, {el:.1f} s"}


def run_terrain(steps: int, warmup: int, cpu: bool = True) -> dict:
    """Flow over a Witch of Agnesi hill in terrain-following coordinates (Sec.
    3.4, 4.3): 256 x 256 x 128, FP64, basic terrain following, 10 m/s across a
    400 m hill of 2 km half-width, constant N = 0.01 1/s, 6 substeps."""
    import torch
    from paper_2412_04395_amd import erf

    cfg = W.terrain_hill()
    h = W.agnesi_nodes(cfg, 400.0, 2000.0)
    s = erf.Solver(cfg)
    s.set_terrain(h, 1.0)
    Hc, zc = s.terrain_heights()
    th0 = W.stratified_theta(zc, 300.0, 0.01, cfg.grav)
    ps = W.stratified_ground_pressure(W.cell_mean_nodes(h), 300.0, 0.01, cfg.p_surface, cfg.grav)
    b = s.init_base_state_columns(th0, ps)
    shp = b["rho0"].shape
    S = s.to_device({"rho": b["rho0"], "rt": b["rho0"] * b["theta0"], "ru": b["rho0"] * 10.0,
                     "rv": np.zeros(shp), "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": np.zeros((0,) + shp)})
    del Hc, zc, th0, b
    for _ in range(warmup):
        s.rk3_step(S)
    shares = {}
    for k in TERRAIN_VALUES:
        _, (ms, n) = _time_steps(s, S, 1, torch, k)
        if n:
            shares[k] = (ms, n)
    dom = max(shares, key=lambda k: shares[k][0])
    el, (kms, kn) = _time_steps(s, S, steps, torch, dom)
    d = s.diagnostics(S, allow_nonfinite=True)
    s.close()
    del S
    # the same flow carrying three tracers by WENO5 (the scalar update over
    # terrain and the substeps' flux sums)
    cq = cfg.replace(n_scalars=3, scalar_scheme=1)
    sq = erf.Solver(cq)
    sq.set_terrain(h, 1.0)
    Hq, zq = sq.terrain_heights()
    bq = sq.init_base_state_columns(W.stratified_theta(zq, 300.0, 0.01, cq.grav), ps)
    rq = np.stack([bq["rho0"] * (1e-3 * (m + 1)) * (1.0 + W.uniform_noise(cq.seed + m, shp, 0.5)) for m in range(3)])
    Sq = sq.to_device({"rho": bq["rho0"], "rt": bq["rho0"] * bq["theta0"], "ru": bq["rho0"] * 10.0,
                       "rv": np.zeros(shp), "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": rq})
    del Hq, zq, rq
    for _ in range(warmup):
        sq.rk3_step(Sq)
    qshares = {}
    for k in ("mixing_ratio", "scalar"):
        _, (ms, n) = _time_steps(sq, Sq, 1, torch, k)
        qshares[k] = round(ms, 4)
    elq, _ = _time_steps(sq, Sq, steps, torch)
    sq.close()
    avg_ms = kms / max(kn, 1)
    byts = TERRAIN_VALUES[dom] * 8.0 * cfg.cells
    gbs = byts / (avg_ms * 1e-3) / 1e9
    return {"workload": "flow over a Witch of Agnesi hill (400 m, half-width 2 km), terrain-following "
                        "coordinates, 256x256x128, N = 0.01 1/s, 10 m/s",
            "grid": [cfg.nx, cfg.ny, cfg.nz], "precision": "fp64", "n_substeps": cfg.n_substeps,
            "value": cfg.cells * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
            "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares.items()},
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": byts,
                         "avg_launch_ms": round(avg_ms, 4), "launches_timed": kn},
            "final_diag": {"max_w": d["max_w"], "nonfinite": d["nonfinite"]},
            "with_scalars": {"n_scalars": 3, "scheme": "WENO5", "value": cq.cells * steps / elq,
                             "ms_per_step": 1e3 * elq / steps, "kernel_ms_per_step": qshares},
            **({"cpu_oracle": terrain_cpu_oracle()} if cpu else {})}


def _substep_value_adjust(cfg) -> float:
    """Bulk values per cell by which the average substep launch of a step
    differs from KERNEL_VALUES: +5 for the one per stage that writes the stage
    end (none with scalars, whose flux sums keep a separate finalize), -6 for
    the first stage's, which reads no S''."""
    ns = cfg.n_substeps
    n = 1 + ns // 2 + ns
    return ((0.0 if cfg.n_scalars else 3.0 * 5) - ZERO_START_SAVED["substep"]) / n


def _roofline(cfg, dom, kms, kn):
    if dom not in KERNEL_VALUES:
        return {"kernel": dom, "avg_launch_ms": round(kms / max(kn, 1), 4), "note": "no per-cell byte count"}
    sgs = 1 if cfg.sgs else 0
    avg_ms = kms / max(kn, 1)
    bytes_per_launch = _kernel_bytes(dom, sgs, cfg.prec) * cfg.cells
    if dom == "substep":  # averaged over the timed launches
        bytes_per_launch += _substep_value_adjust(cfg) * (8.0 if cfg.prec == "fp64" else 4.0) * cfg.cells
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic, tsrc = _profiled_traffic(dom, cfg.prec) if "stable" in cfg.name else (None, None)
    out = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": tsrc,
           "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": round(avg_ms, 4),
           "launches_timed": kn}
    if dom == "substep":
        # the streaming model's substep: F perturbations, F tendencies, two
        # coefficients and the previous Theta'' read, F perturbations written
        # (3F + 3 values, F = 5), plus 6 for the flux sums with scalars
        mv = 3 * 5 + 3 + (6 if cfg.n_scalars else 0)
        mb = mv * (8.0 if cfg.prec == "fp64" else 4.0) * cfg.cells
        out["model_values_per_cell"] = mv
        out["model_frac"] = round(mb / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cbl")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-as-stated", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-closure", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-training", action="store_true")
    ap.add_argument("--no-scalars", action="store_true")
    ap.add_argument("--no-anelastic", action="store_true")
    ap.add_argument("--no-tke", action="store_true")
    ap.add_argument("--no-terrain", action="store_true")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="first run one plain device copy of this many GiB (reference for HBM counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU layout is a design "
              f"of the library, not a measured path", file=sys.stderr)
        return 2
    rank = int(os.environ.get("RANK", "0"))

    if a.copy_gib > 0:
        import torch
        n = int(a.copy_gib * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # single legs, each printed as its own JSON object (for profiling them alone)
    if a.workload == "ensemble":
        print(json.dumps(run_ensemble(min(a.steps, 5), min(a.warmup, 1))), flush=True)
        return 0
    if a.workload == "anelastic":
        print(json.dumps(run_anelastic(a.steps, a.warmup)), flush=True)
        return 0
    if a.workload == "tke":
        print(json.dumps(run_tke(a.steps, a.warmup)), flush=True)
        return 0
    if a.workload == "terrain":
        print(json.dumps(run_terrain(a.steps, a.warmup, cpu=not a.no_cpu_baseline)), flush=True)
        return 0
    if a.workload == "closure_training":
        print(json.dumps(run_training(a.steps)), flush=True)
        return 0
    cfg = _cfg(a.workload)
    el, dom, kms, kn, shares, diag = run_gpu(cfg, a.steps, a.warmup)
    value = cfg.cells * a.steps / el
    roof = _roofline(cfg, dom, kms, kn)
    copy_gbs = _copy_gbs()
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if cfg.prec == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "cells": cfg.cells,
                   "dt": cfg.dt, "n_substeps": cfg.n_substeps, "adv_order": [cfg.adv_order_h, cfg.adv_order_v],
                   "sgs": "smagorinsky" if cfg.sgs else "none", "precision": cfg.prec,
                   "substep_shape": diag["substep_shape"]},
        "roofline": roof,
        # the whole step against HBM: the design's algorithmic bytes, the
        # one-pass lower bound, and the measured copy rate
        "step_roofline": _step_roofline(cfg, 1e3 * el / a.steps, copy_gbs),
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares.items()},
        "final_diag": {"max_w": diag["max_w"], "nonfinite": diag["nonfinite"]},
    }
    if a.workload == "cbl" and not a.no_as_stated:
        c2 = _cfg("cbl_as_stated")
        el2, *_ = run_gpu(c2, a.steps, a.warmup)
        out["as_stated"] = {"workload": c2.name, "value": c2.cells * a.steps / el2,
                            "ms_per_step": 1e3 * el2 / a.steps, "note": "diverges in the first step (acoustic "
                            "CFL); timed for throughput only"}
    if a.workload == "cbl" and not a.no_fp32:
        c3 = _cfg("cbl_fp32")
        el3, dom3, kms3, kn3, shares3, diag3 = run_gpu(c3, a.steps, a.warmup)
        out["fp32"] = {"workload": c3.name,
                       "precision": "FP32 storage and bulk stencil arithmetic; FP64 base state, column solve and sums",
                       "value": c3.cells * a.steps / el3, "ms_per_step": 1e3 * el3 / a.steps,
                       "speedup_vs_fp64": el / el3, "roofline": _roofline(c3, dom3, kms3, kn3),
                       "step_roofline": _step_roofline(c3, 1e3 * el3 / a.steps, copy_gbs),
                       "substep_shape": diag3["substep_shape"],
                       "kernel_ms_per_step": {k: round(v[0], 4) for k, v in shares3.items()}}
    if a.workload == "cbl" and not a.no_closure:
        out["closure"] = run_closure(a.steps, a.warmup)
    if a.workload == "cbl" and not a.no_training:
        out["training"] = run_training(a.steps)
    if a.workload == "cbl" and not a.no_scalars:
        out["scalars"] = run_scalars(min(a.steps, 10), min(a.warmup, 2))
    if a.workload == "cbl" and not a.no_tke:
        out["tke"] = run_tke(a.steps, a.warmup)
    if a.workload == "cbl" and not a.no_anelastic:
        out["anelastic"] = run_anelastic(a.steps, a.warmup)
    if a.workload == "cbl" and not a.no_terrain:
        out["terrain"] = run_terrain(a.steps, a.warmup, cpu=rank == 0 and not a.no_cpu_baseline)
    if a.workload == "cbl" and not a.no_ensemble:
        out["ensemble"] = run_ensemble(min(a.steps, 5), min(a.warmup, 1))
    if rank == 0 and not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    if rank == 0:
        print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
