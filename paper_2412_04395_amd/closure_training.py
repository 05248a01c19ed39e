"""Training data, training and an a-posteriori check of the learned subgrid
closure (include/erf_mlp.h), all on the GPU through liberf.so.

    python -m paper_2412_04395_amd.closure_training --out DIR [--spin STEPS] ...

Recipe
  1. Fine LES of the dry convective boundary layer at 10 m (workloads.les_fine:
     FP64, Smagorinsky), seeded; a spin-up, then snapshots at a fixed interval.
  2. Each snapshot is box-filtered by 4 onto the 40 m grid of
     workloads.les_mlp (erf_box_filter, the fine grid's own Smagorinsky
     stresses included in the targets); the closure inputs are those of the
     filtered state on the coarse grid (erf_mlp_features).
  3. Statistics of the training set (erf_mlp_fit_norm), standardisation
     (erf_mlp_standardize), Adam on random minibatches (erf_mlp_train_step);
     the loss of a second, held-out fine run is tracked.
  4. A-posteriori: coarse runs from the filtered held-out state, one with the
     network and one with Smagorinsky, against the filtered continuation of the
     fine run: plane-averaged resolved kinetic energy of the fluctuations,
     k(z) = (<u'u'> + <v'v'> + <w'w'>) / 2, and the total vertical heat flux
     <w'theta'> + <q_3>(z) (resolved plus subgrid), relative L2 errors over z.

Writes DIR/closure_les40m.npz (params float32[9609], norm float64[38]) and
DIR/closure_les40m.json (recipe, losses, a-posteriori errors).  Prints one
progress line at least every minute of GPU work.

    python -m paper_2412_04395_amd.closure_training --gain-fixture PATH

writes the reduced a-posteriori case that the GPU test of the closure's gain
runs: the held-out fine run (seed 44) after its spin-up, box-filtered onto the
coarse grid (the coarse initial state, as the FP32 perturbations the coarse
context stores), and the filtered continuation's k(z), heat-flux profiles and
1-D spectra of u and w at z_i / 2 (the reference the coarse runs are judged
against).  The reference is the dycore's own filtered fine FP64 run: the
method's judge of the closure, not a parity value.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import erf
from . import workloads as W

R_FILTER = 4


def _log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def coarse_config(fine: W.Config, sgs: int) -> W.Config:
    return W.les_mlp(nx=fine.nx // R_FILTER, ny=fine.ny // R_FILTER, nz=fine.nz // R_FILTER,
                     dz=W.uniform_dz(fine.nz // R_FILTER, fine.dz[0] * R_FILTER), sgs=sgs, Cs=fine.Cs,
                     Pr_t=fine.Pr_t, seed=fine.seed)


class Coarse:
    """A coarse FP32 context with its base state."""

    def __init__(self, cfg: W.Config):
        self.cfg = cfg
        self.s = erf.Solver(cfg)
        self.th0 = W.theta_sounding(cfg)
        self.b = self.s.init_base_state(self.th0)

    def load(self, Cst):
        """Device state of this context from a filtered full FP64 state."""
        S = {f: Cst[f].cpu().numpy() for f in ("rho", "rt", "ru", "rv", "rw")}
        S["rq"] = np.zeros((0,) + S["rho"].shape)
        return self.s.from_full(S)


# -- diagnostics on full FP64 host states -----------------------------------------
def _centre_fields(S):
    rho = S["rho"]
    u = S["ru"] / (0.5 * (rho + np.roll(rho, 1, axis=2)))
    v = S["rv"] / (0.5 * (rho + np.roll(rho, 1, axis=1)))
    w = np.zeros_like(S["rw"])
    w[1:-1] = S["rw"][1:-1] / (0.5 * (rho[1:] + rho[:-1]))
    uc = 0.5 * (u + np.roll(u, -1, axis=2))
    vc = 0.5 * (v + np.roll(v, -1, axis=1))
    wc = 0.5 * (w[:-1] + w[1:])
    return uc, vc, wc, S["rt"] / rho


def profiles(S, q3):
    """Plane-averaged resolved k(z) and total heat flux; q3: subgrid vertical
    heat flux per cell (nz, ny, nx)."""
    uc, vc, wc, th = _centre_fields(S)
    fl = lambda a: a - a.mean(axis=(1, 2), keepdims=True)
    k = 0.5 * ((fl(uc) ** 2).mean(axis=(1, 2)) + (fl(vc) ** 2).mean(axis=(1, 2)) + (fl(wc) ** 2).mean(axis=(1, 2)))
    flux = (fl(wc) * fl(th)).mean(axis=(1, 2)) + q3.mean(axis=(1, 2))
    return k, flux


def smagorinsky_q3(feat, cfg):
    f = feat
    s11, s22, s33 = f[:, 0], f[:, 4], f[:, 8]
    s12, s13, s23 = 0.5 * (f[:, 1] + f[:, 3]), 0.5 * (f[:, 2] + f[:, 6]), 0.5 * (f[:, 5] + f[:, 7])
    ss = 2 * (s11 ** 2 + s22 ** 2 + s33 ** 2) + 4 * (s12 ** 2 + s13 ** 2 + s23 ** 2)
    delta = (cfg.dx * cfg.dy * np.repeat(cfg.dz, cfg.nx * cfg.ny)) ** (1.0 / 3.0)
    nut = (cfg.Cs * delta) ** 2 * np.sqrt(ss)
    return (-(nut / cfg.Pr_t) * f[:, 9]).reshape(cfg.nz, cfg.ny, cfg.nx)


def network_q3(c: Coarse, S_dev, nrm):
    feat = c.s.mlp_features(S_dev)
    x, _ = c.s.mlp_standardize(feat)
    y = c.s.mlp_forward(x).cpu().double().numpy()
    return (y[:, 8] * nrm[37] + nrm[28]).reshape(c.cfg.nz, c.cfg.ny, c.cfg.nx)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


SPECTRUM_HEIGHT_M = 500.0  # z_i / 2 for the 1 km inversion of the sounding


def spectra(S, cfg):
    """1-D power spectra along x of the centre velocities u and w, averaged
    over y, at the level nearest z_i / 2: (E_u, E_w) for wavenumbers 1 .. nx/2."""
    uc, _, wc, _ = _centre_fields(S)
    k = int(np.argmin(np.abs(cfg.z_centres() - SPECTRUM_HEIGHT_M)))
    out = []
    for f in (uc[k], wc[k]):
        F = np.fft.rfft(f - f.mean(axis=1, keepdims=True), axis=1)
        out.append((np.abs(F[:, 1:cfg.nx // 2 + 1]) ** 2).mean(axis=0) / cfg.nx ** 2)
    return out


def _log_spectral_error(a, b):
    """rms of ln(a / b) over the wavenumbers 1 .. nx/4 (wavelengths of at least
    four coarse cells): above them the 4x box filter of the reference and the
    two-point centring of u (which removes the shortest wave exactly) shape
    both spectra more than the closure does"""
    m = len(b) // 2
    return float(np.sqrt(np.mean(np.log(np.maximum(a[:m], 1e-300) / np.maximum(b[:m], 1e-300)) ** 2)))


def a_posteriori(c: "Coarse", init_state, ref_profiles, steps_per_eval: int, evals: int, nrm=None, ref_spectra=None):
    """Run the coarse context c from init_state (device, its storage) and
    compare, after every steps_per_eval steps, its k(z) and total heat flux
    with ref_profiles[e] = (k, flux); with ref_spectra (E_u, E_w at the end)
    also the final 1-D spectra.  nrm: the network's statistics (closure runs).
    Returns the per-evaluation errors and their means over e >= 1."""
    S = init_state
    errs = []
    for e in range(evals + 1):
        if e > 0:
            for _ in range(steps_per_eval):
                c.s.rk3_step(S)
        full = c.s.to_full(S)
        if c.cfg.sgs == erf.ERF_SGS_MLP:
            q3 = network_q3(c, S, nrm)
        else:
            q3 = smagorinsky_q3(c.s.mlp_features(S).cpu().numpy(), c.cfg)
        k, flux = profiles(full, q3)
        errs.append({"tke": _rel_l2(k, ref_profiles[e][0]), "heat_flux": _rel_l2(flux, ref_profiles[e][1])})
    out = {"errors": errs, "mean_tke_error": float(np.mean([x["tke"] for x in errs[1:]])),
           "mean_heat_flux_error": float(np.mean([x["heat_flux"] for x in errs[1:]]))}
    out["nonfinite"] = c.s.diagnostics(S, allow_nonfinite=True)["nonfinite"]
    if ref_spectra is not None:
        eu, ew = spectra(c.s.to_full(S), c.cfg)
        out["spectrum_u_error"] = _log_spectral_error(eu, ref_spectra[0])
        out["spectrum_w_error"] = _log_spectral_error(ew, ref_spectra[1])
    return out


# -- fine runs ----------------------------------------------------------------------
def fine_run(cfg, spin, every, nsnap, on_snapshot):
    import torch
    s = erf.Solver(cfg)
    th0 = W.theta_sounding(cfg)
    b = s.init_base_state(th0)
    S = s.from_full(W.initial_state(cfg, b["rho0"], th0, b["p0"], b["pi0"]))
    t0 = time.time()
    for n in range(spin):
        s.rk3_step(S)
        if (n + 1) % 1000 == 0:
            torch.cuda.synchronize()
            _log(f"{cfg.name} seed {cfg.seed}: spin-up {n + 1}/{spin} steps, {time.time() - t0:.0f} s")
    for k in range(nsnap):
        on_snapshot(k, s, S)
        if k + 1 < nsnap:
            for n in range(every):
                s.rk3_step(S)
        torch.cuda.synchronize()
        _log(f"{cfg.name} seed {cfg.seed}: snapshot {k + 1}/{nsnap}, {time.time() - t0:.0f} s")
    d = s.diagnostics(S, allow_nonfinite=True)
    s.close()
    return d


def gain_fixture(path, spin=12000, every=1200, evals=5, nx=256, nz=128):
    """The reduced a-posteriori case of the module docstring, written to path
    (.npz): coarse initial state (float32 perturbations rho - rho0, rho theta -
    rho0 theta0, and the momenta), reference profiles k[evals + 1][nz_c],
    flux[evals + 1][nz_c] and final spectra E_u, E_w, and the recipe."""
    fine = W.les_fine(nx=nx, ny=nx, nz=nz, dz=W.uniform_dz(nz, 10.0), seed=44)
    cm = Coarse(coarse_config(fine, erf.ERF_SGS_SMAGORINSKY))
    ks, fluxes, keep = [], [], {}

    def snap(k, s, S):
        Cst, tg = s.box_filter(S, R_FILTER, Cs=fine.Cs, Pr_t=fine.Pr_t)
        full = {f: Cst[f].cpu().numpy() for f in ("rho", "rt", "ru", "rv", "rw")}
        q3 = tg[:, 8].cpu().numpy().reshape(cm.cfg.nz, cm.cfg.ny, cm.cfg.nx)
        kz, fl = profiles(full, q3)
        ks.append(kz)
        fluxes.append(fl)
        if k == 0:
            keep["init"] = full
        if k == evals:
            keep["spectra"] = spectra(full, cm.cfg)

    fine_run(fine, spin, every, evals + 1, snap)
    init = keep["init"]
    rho0 = cm.b["rho0"][:, None, None]
    T0 = (cm.b["rho0"] * cm.b["theta0"])[:, None, None]
    recipe = {"fine_grid": [fine.nx, fine.ny, fine.nz], "fine_dx_m": fine.dx, "fine_dt_s": fine.dt, "seed": fine.seed,
              "spin_up_s": spin * fine.dt, "eval_every_s": every * fine.dt, "evals": evals, "filter": R_FILTER,
              "coarse_grid": [cm.cfg.nx, cm.cfg.ny, cm.cfg.nz], "spectrum_height_m": SPECTRUM_HEIGHT_M}
    np.savez_compressed(path, rho_p=(init["rho"] - rho0).astype(np.float32),
                        rt_p=(init["rt"] - T0).astype(np.float32), ru=init["ru"].astype(np.float32),
                        rv=init["rv"].astype(np.float32), rw=init["rw"].astype(np.float32),
                        k_ref=np.array(ks), flux_ref=np.array(fluxes), spec_u_ref=keep["spectra"][0],
                        spec_w_ref=keep["spectra"][1], recipe=json.dumps(recipe))
    _log(f"gain fixture written to {path}")


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--gain-fixture", help="write the reduced a-posteriori case to this .npz and stop")
    ap.add_argument("--out")
    ap.add_argument("--spin", type=int, default=12000, help="fine spin-up steps (0.1 s each)")
    ap.add_argument("--every", type=int, default=600, help="fine steps between snapshots")
    ap.add_argument("--snaps", type=int, default=10, help="training snapshots")
    ap.add_argument("--eval-every", type=int, default=1200, help="fine steps between a-posteriori comparisons")
    ap.add_argument("--evals", type=int, default=5)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--nz", type=int, default=128)
    a = ap.parse_args(argv)
    if a.gain_fixture:
        gain_fixture(a.gain_fixture, spin=a.spin, every=a.eval_every, evals=a.evals, nx=a.nx, nz=a.nz)
        return 0
    if not a.out:
        ap.error("--out is required")
    os.makedirs(a.out, exist_ok=True)
    fine = W.les_fine(nx=a.nx, ny=a.nx, nz=a.nz, dz=W.uniform_dz(a.nz, 10.0), seed=41)
    held = fine.replace(seed=44)
    cmlp = Coarse(coarse_config(fine, erf.ERF_SGS_MLP))
    csmag = Coarse(coarse_config(fine, erf.ERF_SGS_SMAGORINSKY))
    feats, targs = [], []

    def collect(store):
        def f(k, s, S):
            Cst, tg = s.box_filter(S, R_FILTER, Cs=fine.Cs, Pr_t=fine.Pr_t)
            store[0].append(cmlp.s.mlp_features(cmlp.load(Cst)))
            store[1].append(tg)
        return f

    # 1-2. training data
    t_start = time.time()
    fine_run(fine, a.spin, a.every, a.snaps, collect((feats, targs)))
    X_raw, T_raw = torch.cat(feats), torch.cat(targs)
    # held-out run: validation data and the reference for the a-posteriori runs
    vfeats, vtargs, ref, init = [], [], [], {}

    def held_snap(k, s, S):
        Cst, tg = s.box_filter(S, R_FILTER, Cs=fine.Cs, Pr_t=fine.Pr_t)
        full = {f: Cst[f].cpu().numpy() for f in ("rho", "rt", "ru", "rv", "rw")}
        if k == 0:
            init["state"] = Cst
        q3 = tg[:, 8].cpu().numpy().reshape(cmlp.cfg.nz, cmlp.cfg.ny, cmlp.cfg.nx)
        ref.append(profiles(full, q3))
        vfeats.append(cmlp.s.mlp_features(cmlp.load(Cst)))
        vtargs.append(tg)

    fine_run(held, a.spin, a.eval_every, a.evals + 1, held_snap)
    Xv_raw, Tv_raw = torch.cat(vfeats), torch.cat(vtargs)
    _log(f"data: {X_raw.shape[0]} training and {Xv_raw.shape[0]} held-out samples, {time.time() - t_start:.0f} s")

    # 3. training
    s = cmlp.s
    rng = np.random.default_rng(fine.seed)
    p = np.zeros(erf.MLP_NPARAMS)
    for off, fi, fo in ((0, 10, 64), (704, 64, 64), (4864, 64, 64), (9024, 64, 9)):
        p[off:off + fi * fo] = rng.normal(0, np.sqrt(2.0 / fi), fi * fo)
    s.mlp_set_weights(p.astype(np.float32))
    s.mlp_fit_norm(X_raw, T_raw)
    X, T = s.mlp_standardize(X_raw, T_raw)
    Xv, Tv = s.mlp_standardize(Xv_raw, Tv_raw)
    n = X.shape[0]
    gen = torch.Generator(device=X.device)
    gen.manual_seed(fine.seed)
    history = []
    t0 = time.time()
    for it in range(a.train_steps):
        lr = a.lr * 0.5 ** (4 * it // a.train_steps)
        idx = torch.randint(0, n, (min(a.batch, n),), device=X.device, generator=gen)
        loss = s.mlp_train_step(X[idx].contiguous(), T[idx].contiguous(), lr, want_loss=(it % 250 == 0))
        if it % 250 == 0 or it == a.train_steps - 1:
            vloss, _ = s.mlp_loss_grad(Xv, Tv)
            tl, _ = s.mlp_loss_grad(X, T)
            history.append({"step": it, "train_loss": tl, "heldout_loss": vloss})
            _log(f"train step {it}: minibatch {loss}, train {tl:.4f}, held-out {vloss:.4f}, {time.time() - t0:.0f} s")
    params, nrm = s.mlp_get_weights()

    # 4. a-posteriori
    steps_per_eval = a.eval_every * fine.dt / cmlp.cfg.dt
    assert abs(steps_per_eval - round(steps_per_eval)) < 1e-9
    steps_per_eval = int(round(steps_per_eval))
    res = {}
    for name, c in (("network", cmlp), ("smagorinsky", csmag)):
        S = c.load(init["state"])
        fb0 = c.s.mlp_fallback_count() if c is cmlp else 0
        errs = []
        for e in range(a.evals + 1):
            if e > 0:
                for _ in range(steps_per_eval):
                    c.s.rk3_step(S)
            full = c.s.to_full(S)
            if c is cmlp:
                q3 = network_q3(c, S, nrm)
            else:
                q3 = smagorinsky_q3(c.s.mlp_features(S).cpu().numpy(), c.cfg)
            k, flux = profiles(full, q3)
            errs.append({"t_s": e * a.eval_every * fine.dt, "tke": _rel_l2(k, ref[e][0]),
                         "heat_flux": _rel_l2(flux, ref[e][1])})
        d = c.s.diagnostics(S, allow_nonfinite=True)
        cells = c.cfg.cells * 3 * steps_per_eval * a.evals
        res[name] = {"errors": errs, "mean_tke_error": float(np.mean([x["tke"] for x in errs[1:]])),
                     "mean_heat_flux_error": float(np.mean([x["heat_flux"] for x in errs[1:]])),
                     "nonfinite": d["nonfinite"],
                     "fallback_fraction": ((c.s.mlp_fallback_count() - fb0) / cells) if c is cmlp else None}
        _log(f"a-posteriori {name}: mean TKE error {res[name]['mean_tke_error']:.3f}, "
             f"heat flux error {res[name]['mean_heat_flux_error']:.3f}")
    report = {
        "fine": {"grid": [fine.nx, fine.ny, fine.nz], "dx_m": fine.dx, "dt_s": fine.dt, "n_substeps": fine.n_substeps,
                 "precision": fine.prec, "seeds": {"train": fine.seed, "heldout": held.seed},
                 "spin_up_s": a.spin * fine.dt, "snapshot_every_s": a.every * fine.dt, "snapshots": a.snaps},
        "coarse": {"grid": [cmlp.cfg.nx, cmlp.cfg.ny, cmlp.cfg.nz], "dx_m": cmlp.cfg.dx, "dt_s": cmlp.cfg.dt,
                   "filter": R_FILTER},
        "training": {"samples": int(n), "heldout_samples": int(Xv.shape[0]), "steps": a.train_steps,
                     "batch": a.batch, "lr": a.lr, "history": history},
        "a_posteriori": res,
        "profile_reference_t_s": [e * a.eval_every * fine.dt for e in range(a.evals + 1)],
    }
    np.savez(os.path.join(a.out, "closure_les40m.npz"), params=params, norm=nrm)
    with open(os.path.join(a.out, "closure_les40m.json"), "w") as fh:
        json.dump(report, fh, indent=1)
    _log(f"done in {time.time() - t_start:.0f} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
