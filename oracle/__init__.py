"""Python access to the FP64 CPU oracle (oracle/liberf_oracle.so).

TEST INFRASTRUCTURE ONLY.  Imported by tests, ``__graft_entry__.smoke`` and the
``cpu_baseline`` leg of ``bench.py``; the product path never imports it.  It
shares no code with the HIP library.

State dictionaries hold numpy float64 arrays:
    rho, rt : (nz, ny, nx)       density and rho*theta at cell centres
    ru, rv  : (nz, ny, nx)       x-/y-face momenta (face i between cells i-1, i)
    rw      : (nz+1, ny, nx)     z-face momentum (face k below cell k)
    rq      : (nq, nz, ny, nx)   rho*q of the passive scalars
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liberf_oracle.so")
_lib = None
_lock = threading.Lock()

FIELDS = ("rho", "rt", "ru", "rv", "rw", "rq")


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.POINTER(C.c_double)),
                ("terrain", C.POINTER(C.c_double)), ("terrain_beta", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_substeps", C.c_int32), ("beta_s", C.c_double),
                ("beta_d", C.c_double), ("adv_order_h", C.c_int32), ("adv_order_v", C.c_int32),
                ("scalar_scheme", C.c_int32), ("n_scalars", C.c_int32), ("sgs", C.c_int32),
                ("Cs", C.c_double), ("Pr_t", C.c_double), ("nu_m", C.c_double),
                ("alpha_m", C.c_double), ("f_cor", C.c_double), ("Ug", C.c_double),
                ("Vg", C.c_double), ("surf_heat_flux", C.c_double), ("grav", C.c_double),
                ("mlp_params", C.POINTER(C.c_double)), ("mlp_norm", C.POINTER(C.c_double)),
                ("mlp_bf16", C.c_int32), ("moist", C.c_int32), ("anelastic", C.c_int32),
                ("p_anel", C.POINTER(C.c_double)), ("most_z0", C.c_double)]


class _Base(C.Structure):
    _fields_ = [("rho0", C.POINTER(C.c_double)), ("theta0", C.POINTER(C.c_double)),
                ("p0", C.POINTER(C.c_double)), ("pi0", C.POINTER(C.c_double)),
                ("qv0", C.POINTER(C.c_double))]


class _State(C.Structure):
    _fields_ = [(f, C.POINTER(C.c_double)) for f in FIELDS]


_DP = C.POINTER(C.c_double)


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                from . import build as _b
                _b.build()
            L = C.CDLL(_SO)
            L.orc_const.restype = C.c_double
            L.orc_const.argtypes = [C.c_int]
            L.orc_eos_p.restype = C.c_double
            L.orc_eos_p.argtypes = [C.c_double]
            L.orc_eos_pprime.restype = C.c_double
            L.orc_eos_pprime.argtypes = [C.c_double, C.c_double, C.c_double]
            L.orc_eos_p_moist.restype = C.c_double
            L.orc_eos_p_moist.argtypes = [C.c_double, C.c_double]
            L.orc_eos_pprime_moist.restype = C.c_double
            L.orc_eos_pprime_moist.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
            L.orc_base_state_moist.argtypes = [C.c_int32, _DP, _DP, _DP, C.c_double, C.c_double, _DP, _DP, _DP]
            L.orc_interp.restype = C.c_double
            L.orc_interp.argtypes = [C.c_int32, _DP, C.c_double]
            L.orc_weno5.restype = C.c_double
            L.orc_weno5.argtypes = [_DP, C.c_double, C.c_double]
            L.orc_thomas.argtypes = [C.c_int32, _DP, _DP, _DP, _DP, _DP]
            L.orc_base_state.argtypes = [C.c_int32, _DP, _DP, C.c_double, C.c_double, _DP, _DP, _DP]
            L.orc_terrain_heights.argtypes = [C.POINTER(_Grid), _DP, _DP]
            L.orc_base_state_columns.argtypes = [C.POINTER(_Grid), _DP, _DP, C.c_double, _DP, _DP, _DP]
            L.orc_slow_rhs.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                       C.POINTER(_State), C.POINTER(_State)]
            L.orc_acoustic_substeps.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                                C.POINTER(_State), C.POINTER(_State), C.POINTER(_State),
                                                C.c_int32, C.c_double, C.POINTER(_State), _DP, _DP, _DP]
            L.orc_scalar_advance.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_State),
                                             C.POINTER(_State), _DP, _DP, _DP, C.c_double, _DP, _DP]
            L.orc_most_ustar.restype = C.c_double
            L.orc_most_ustar.argtypes = [C.c_double] * 6
            L.orc_rk3_step.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                       C.POINTER(_State)]
            L.orc_diagnostics.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                          C.POINTER(_State), _DP]
            L.orc_kessler.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base), C.POINTER(_State),
                                      C.c_double, _DP]
            L.orc_esat.restype = C.c_double
            L.orc_esat.argtypes = [C.c_double]
            L.orc_qvsat.restype = C.c_double
            L.orc_qvsat.argtypes = [C.c_double, C.c_double]
            L.orc_sat_adjust.restype = C.c_double
            L.orc_sat_adjust.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
            L.orc_bf16.restype = C.c_double
            L.orc_bf16.argtypes = [C.c_double]
            L.orc_mlp_forward.argtypes = [_DP, _DP, C.c_int64, _DP, C.c_int]
            L.orc_mlp_loss_grad.argtypes = [_DP, _DP, _DP, C.c_int64, C.c_int, _DP, _DP]
            L.orc_mlp_grad_abs.argtypes = [_DP, _DP, _DP, C.c_int64, C.c_int, _DP]
            L.orc_mlp_unit_margins.argtypes = [_DP, _DP, C.c_int64, _DP, C.POINTER(C.c_int32),
                                               C.POINTER(C.c_int32), _DP]
            L.orc_adam.argtypes = [_DP, _DP, _DP, _DP, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                   C.c_double, C.c_double]
            L.orc_sgs_features.argtypes = [C.POINTER(_Grid), C.POINTER(_State), _DP]
            L.orc_box_filter.argtypes = [C.POINTER(_Grid), C.POINTER(_State), C.c_int32, C.c_double, C.c_double,
                                         C.POINTER(_State), _DP]
            L.orc_divergence.argtypes = [C.POINTER(_Grid), _DP, _DP, _DP, _DP]
            L.orc_poisson.argtypes = [C.POINTER(_Grid), _DP, _DP]
            L.orc_project.argtypes = [C.POINTER(_Grid), _DP, _DP, _DP, C.c_double, _DP]
            L.orc_ssprk2_step.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                          C.POINTER(_State), _DP]
            L.orc_slow_rhs_mlp.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Base),
                                           C.POINTER(_State), _DP, _DP, C.c_int, C.POINTER(_State),
                                           C.POINTER(C.c_int64)]
            _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def const(name: str) -> float:
    return lib().orc_const({"R_d": 0, "c_p": 1, "c_v": 2, "gamma": 3, "P00": 4, "R_v": 5}[name])


class Oracle:
    """Oracle bound to one grid and one parameter set (a workloads.Config)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.nx, self.ny, self.nz = cfg.nx, cfg.ny, cfg.nz
        self.dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
        self._grid = _Grid(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, _p(self.dz), None, 0.0)
        self.terrain = None
        self._params = _Params(cfg.dt, cfg.n_substeps, cfg.beta_s, cfg.beta_d, cfg.adv_order_h,
                               cfg.adv_order_v, cfg.scalar_scheme, cfg.n_scalars, cfg.sgs, cfg.Cs,
                               cfg.Pr_t, cfg.nu_m, cfg.alpha_m, cfg.f_cor, cfg.Ug, cfg.Vg,
                               cfg.surf_heat_flux, cfg.grav, None, None, 0, int(cfg.moist),
                               int(getattr(cfg, "anelastic", 0)), None, float(getattr(cfg, "most_z0", 0.0)))
        self.base = None
        # anelastic mode: the lagged perturbation pressure (Sec. 3.2)
        self.p_anel = np.zeros((cfg.nz, cfg.ny, cfg.nx))
        self._params.p_anel = _p(self.p_anel)
        self._mlp = None

    def set_mlp(self, params, norm, bf16: bool = False):
        """Closure weights for sgs == 2 (kept alive by this object)."""
        pa = np.ascontiguousarray(params, dtype=np.float64)
        no = np.ascontiguousarray(norm, dtype=np.float64)
        if pa.size != mlp_nparams() or no.size != 38:
            raise ValueError("MLP parameters must have mlp_nparams() values and norm 38")
        self._mlp = (pa, no)
        self._params.mlp_params = _p(pa)
        self._params.mlp_norm = _p(no)
        self._params.mlp_bf16 = int(bool(bf16))

    # -- terrain-following coordinates (App. A, App. B) -------------------------
    def set_terrain(self, h_nodes, beta: float = 1.0):
        """Terrain heights h[ny][nx] at the nodes (node (i, j) the low-x, low-y
        corner of cell (i, j)); beta 1 basic terrain following, 3 Sullivan.
        Set before the base state, which then holds one value per cell."""
        h = np.ascontiguousarray(h_nodes, dtype=np.float64)
        if h.shape != (self.ny, self.nx):
            raise ValueError("terrain heights must be (ny, nx)")
        self.terrain = h
        self._grid.terrain = _p(h)
        self._grid.terrain_beta = float(beta)
        self.base = None

    def terrain_heights(self):
        """(Hc, zc): physical cell heights and centre heights, (nz, ny, nx)."""
        Hc, zc = np.zeros((self.nz, self.ny, self.nx)), np.zeros((self.nz, self.ny, self.nx))
        self._check(lib().orc_terrain_heights(C.byref(self._grid), _p(Hc), _p(zc)), "orc_terrain_heights")
        return Hc, zc

    def init_base_state_columns(self, theta0, p_surf):
        """Hydrostatic base state of every column from theta0 (nz, ny, nx) at
        the cell centres and the ground pressure p_surf (ny, nx)."""
        shp = (self.nz, self.ny, self.nx)
        th = np.ascontiguousarray(np.broadcast_to(theta0, shp), dtype=np.float64)
        ps = np.ascontiguousarray(np.broadcast_to(p_surf, shp[1:]), dtype=np.float64)
        rho0, p0, pi0 = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        self._check(lib().orc_base_state_columns(C.byref(self._grid), _p(th), _p(ps), self.cfg.grav,
                                                 _p(rho0), _p(p0), _p(pi0)), "orc_base_state_columns")
        self.base = {"rho0": rho0, "theta0": th, "p0": p0, "pi0": pi0, "qv0": None}
        self._base = _Base(_p(rho0), _p(th), _p(p0), _p(pi0), None)
        return self.base

    # -- base state -------------------------------------------------------
    def init_base_state(self, theta0: np.ndarray, p_surface: float, qv0=None):
        """Hydrostatic base state; qv0[nz] (None: dry) is the base-state water
        vapour mixing ratio of the moist EOS."""
        nz = self.nz
        th = np.ascontiguousarray(theta0, dtype=np.float64)
        qv = None if qv0 is None else np.ascontiguousarray(qv0, dtype=np.float64)
        rho0, p0, pi0 = np.zeros(nz), np.zeros(nz), np.zeros(nz)
        rc = lib().orc_base_state_moist(nz, _p(self.dz), _p(th), None if qv is None else _p(qv), p_surface,
                                        self.cfg.grav, _p(rho0), _p(p0), _p(pi0))
        if rc != 0:
            raise RuntimeError(f"orc_base_state failed ({rc})")
        self.base = {"rho0": rho0, "theta0": th, "p0": p0, "pi0": pi0,
                     "qv0": np.zeros(nz) if qv is None else qv}
        self._base = _Base(_p(rho0), _p(th), _p(p0), _p(pi0), None if qv is None else _p(qv))
        return self.base

    # -- helpers ----------------------------------------------------------
    def zeros_state(self):
        nx, ny, nz, nq = self.nx, self.ny, self.nz, self.cfg.n_scalars
        return {"rho": np.zeros((nz, ny, nx)), "rt": np.zeros((nz, ny, nx)),
                "ru": np.zeros((nz, ny, nx)), "rv": np.zeros((nz, ny, nx)),
                "rw": np.zeros((nz + 1, ny, nx)), "rq": np.zeros((max(nq, 0), nz, ny, nx))}

    def _st(self, S):
        arrs = {}
        for f in FIELDS:
            a = S[f]
            if not (a.dtype == np.float64 and a.flags.c_contiguous):
                raise TypeError(f"field {f} must be C-contiguous float64")
            arrs[f] = _p(a) if a.size else C.cast(C.c_void_p(0), _DP)
        return _State(**arrs)

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with status {rc}")

    # -- the calls ---------------------------------------------------------
    def slow_rhs(self, S):
        R = self.zeros_state()
        self._check(lib().orc_slow_rhs(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                       C.byref(self._st(S)), C.byref(self._st(R))), "orc_slow_rhs")
        return R

    def acoustic_substeps(self, Sn, St, Rt, n_sub: int, dtau: float):
        out = self.zeros_state()
        nx, ny, nz = self.nx, self.ny, self.nz
        Fu, Fv, Fw = np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.zeros((nz + 1, ny, nx))
        self._check(lib().orc_acoustic_substeps(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                                C.byref(self._st(Sn)), C.byref(self._st(St)),
                                                C.byref(self._st(Rt)), n_sub, dtau, C.byref(self._st(out)),
                                                _p(Fu), _p(Fv), _p(Fw)), "orc_acoustic_substeps")
        return out, (Fu, Fv, Fw)

    def scalar_advance(self, Sn, St, F, dts: float, src=None):
        """src: the Deardorff closure's source of rho e at S^t (slow_rhs's
        R["rq"]), required with that closure."""
        rq = np.zeros_like(Sn["rq"])
        Fu, Fv, Fw = (np.ascontiguousarray(f, dtype=np.float64) for f in F)
        sp = None if src is None else np.ascontiguousarray(src, dtype=np.float64)
        self._check(lib().orc_scalar_advance(C.byref(self._grid), C.byref(self._params), C.byref(self._st(Sn)),
                                             C.byref(self._st(St)), _p(Fu), _p(Fv), _p(Fw), dts,
                                             None if sp is None else _p(sp),
                                             _p(rq) if rq.size else C.cast(C.c_void_p(0), _DP)),
                    "orc_scalar_advance")
        return rq

    def rk3_step(self, S):
        """Advance S (modified in place) by one RK3 step; with the workload's
        microphysics switched on, the Kessler step over dt follows (the rain
        reaching the ground accumulates in self.precip)."""
        self._check(lib().orc_rk3_step(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                       C.byref(self._st(S))), "orc_rk3_step")
        if getattr(self.cfg, "microphysics", 0):
            self.kessler(S, self.cfg.dt)
        return S

    # -- anelastic mode (Sec. 2.2, Sec. 3.2) --------------------------------
    def divergence(self, ru, rv, rw):
        """Finite-volume divergence of face momenta at the cell centres."""
        D = np.zeros((self.nz, self.ny, self.nx))
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (ru, rv, rw)]
        self._check(lib().orc_divergence(C.byref(self._grid), _p(a[0]), _p(a[1]), _p(a[2]), _p(D)),
                    "orc_divergence")
        return D

    def poisson(self, D):
        """phi with D(G(phi)) = D (gauge: the horizontal mean of phi in the
        lowest cell is zero)."""
        Dc = np.ascontiguousarray(D, dtype=np.float64)
        phi = np.zeros_like(Dc)
        self._check(lib().orc_poisson(C.byref(self._grid), _p(Dc), _p(phi)), "orc_poisson")
        return phi

    def project(self, S, dt: float, pp=None):
        """Project the face momenta of S in place; pp (in place, may be None)
        gains psi = phi / dt."""
        self._check(lib().orc_project(C.byref(self._grid), _p(S["ru"]), _p(S["rv"]), _p(S["rw"]), float(dt),
                                      None if pp is None else _p(pp)), "orc_project")
        return S

    def ssprk2_step(self, S):
        """One anelastic SSP-RK2 step in place; self.p_anel is the lagged
        perturbation pressure, updated in place."""
        self._check(lib().orc_ssprk2_step(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                          C.byref(self._st(S)), _p(self.p_anel)), "orc_ssprk2_step")
        return S

    def kessler(self, S, dt: float):
        """Kessler warm-rain microphysics over dt, in place (Sec. 2.4); the rain
        reaching the ground [kg/m^2] accumulates in self.precip [ny][nx]."""
        if getattr(self, "precip", None) is None:
            self.precip = np.zeros((self.ny, self.nx))
        self._check(lib().orc_kessler(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                      C.byref(self._st(S)), float(dt), _p(self.precip)), "orc_kessler")
        return S

    def diagnostics(self, S):
        out = np.zeros(5 + max(self.cfg.n_scalars, 0))
        self._check(lib().orc_diagnostics(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                          C.byref(self._st(S)), _p(out)), "orc_diagnostics")
        d = {"mass": out[0], "theta_mass": out[1], "energy": out[2], "max_w": out[3],
             "nonfinite": int(out[4])}
        d["scalar_mass"] = out[5:].copy()
        return d


    # -- learned closure ---------------------------------------------------
    def sgs_features(self, S):
        n = self.nx * self.ny * self.nz
        feat = np.zeros((n, 10))
        self._check(lib().orc_sgs_features(C.byref(self._grid), C.byref(self._st(S)), _p(feat)),
                    "orc_sgs_features")
        return feat

    def box_filter(self, S, r: int, Cs: float = 0.0, Pr_t: float = 1.0 / 3.0):
        """Coarse state (rho, rt, ru, rv, rw; rq empty) and targets[nc][9];
        Cs > 0 adds the block mean of the fine Smagorinsky stresses."""
        nx, ny, nz = self.nx // r, self.ny // r, self.nz // r
        Cst = {"rho": np.zeros((nz, ny, nx)), "rt": np.zeros((nz, ny, nx)), "ru": np.zeros((nz, ny, nx)),
               "rv": np.zeros((nz, ny, nx)), "rw": np.zeros((nz + 1, ny, nx)), "rq": np.zeros((0, nz, ny, nx))}
        tg = np.zeros((nx * ny * nz, 9))
        Sx = dict(S)
        Sx["rq"] = np.zeros((0,) + S["rho"].shape)
        self._check(lib().orc_box_filter(C.byref(self._grid), C.byref(self._st(Sx)), r, Cs, Pr_t,
                                         C.byref(self._st(Cst)), _p(tg)), "orc_box_filter")
        return Cst, tg

    def slow_rhs_mlp(self, S, params, norm, bf16: bool = False):
        """Slow RHS with the learned closure; returns (R, number of fallback cells)."""
        R = self.zeros_state()
        pa = np.ascontiguousarray(params, dtype=np.float64)
        no = np.ascontiguousarray(norm, dtype=np.float64)
        nfb = C.c_int64(0)
        self._check(lib().orc_slow_rhs_mlp(C.byref(self._grid), C.byref(self._params), C.byref(self._base),
                                           C.byref(self._st(S)), _p(pa), _p(no), int(bool(bf16)),
                                           C.byref(self._st(R)), C.byref(nfb)), "orc_slow_rhs_mlp")
        return R, int(nfb.value)


# -- learned closure: network helpers ----------------------------------------
def mlp_nparams() -> int:
    return int(lib().orc_mlp_nparams())


def bf16(x: float) -> float:
    return lib().orc_bf16(float(x))


def mlp_forward(params, x, bf16: bool = False):
    pa = np.ascontiguousarray(params, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 10)
    y = np.zeros((xa.shape[0], 9))
    lib().orc_mlp_forward(_p(pa), _p(xa), xa.shape[0], _p(y), int(bool(bf16)))
    return y


def mlp_loss_grad(params, x, t, bf16: bool = False):
    pa = np.ascontiguousarray(params, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 10)
    ta = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, 9)
    assert xa.shape[0] == ta.shape[0]
    loss = C.c_double(0.0)
    g = np.zeros(pa.size)
    lib().orc_mlp_loss_grad(_p(pa), _p(xa), _p(ta), xa.shape[0], int(bool(bf16)), C.byref(loss), _p(g))
    return loss.value, g


def mlp_grad_abs(params, x, t, bf16: bool = False):
    """Per parameter, the sum of the magnitudes of the terms of its gradient."""
    pa = np.ascontiguousarray(params, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 10)
    ta = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, 9)
    assert xa.shape[0] == ta.shape[0]
    g = np.zeros(pa.size)
    lib().orc_mlp_grad_abs(_p(pa), _p(xa), _p(ta), xa.shape[0], int(bool(bf16)), _p(g))
    return g


def mlp_unit_margins(params, x):
    """Per sample and hidden unit (n, 192; layers 1..3 of 64 units): the
    relative distance of the unit's value to a bfloat16 rounding boundary (or
    to zero) in the BF16-mode forward pass."""
    pa = np.ascontiguousarray(params, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 10)
    m = np.zeros((xa.shape[0], 192))
    lib().orc_mlp_unit_margins(_p(pa), _p(xa), xa.shape[0], _p(m), None, None, None)
    return m


def mlp_forward_margin(params, x):
    """Per sample, the smallest relative distance of a hidden value to a
    bfloat16 rounding boundary (or to zero) in the BF16-mode forward pass."""
    return mlp_unit_margins(params, x).min(axis=1)


def mlp_forward_flipped(params, x, units):
    """BF16-mode outputs (n, 9) with, in sample s, hidden unit units[s] (0..191,
    layer-major; -1: none) rounded to the bfloat16 neighbour on the other side
    of its value instead of the nearest."""
    pa = np.ascontiguousarray(params, dtype=np.float64)
    xa = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 10)
    u = np.asarray(units, dtype=np.int64).reshape(-1)
    assert u.size == xa.shape[0]
    layer = np.ascontiguousarray(np.where(u >= 0, u // 64, -1), dtype=np.int32)
    unit = np.ascontiguousarray(np.where(u >= 0, u % 64, 0), dtype=np.int32)
    y = np.zeros((xa.shape[0], 9))
    P32 = C.POINTER(C.c_int32)
    lib().orc_mlp_unit_margins(_p(pa), _p(xa), xa.shape[0], None, layer.ctypes.data_as(P32),
                               unit.ctypes.data_as(P32), _p(y))
    return y


def adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on float64 arrays, in place."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(_p(params), _p(grad), _p(m), _p(v), params.size, step, lr, beta1, beta2, eps)


# -- pointwise helpers used by the pin tests ---------------------------------
def most_ustar(U: float, z1: float, z0: float, Qs: float, th1: float, grav: float = 9.81) -> float:
    """Friction velocity of the Monin-Obukhov surface layer."""
    return lib().orc_most_ustar(U, z1, z0, Qs, th1, grav)


def interp(order: int, q6, sgn: float) -> float:
    q = np.ascontiguousarray(q6, dtype=np.float64)
    return lib().orc_interp(order, _p(q), sgn)


def weno5(q6, sgn: float, eps: float = 1e-6) -> float:
    q = np.ascontiguousarray(q6, dtype=np.float64)
    return lib().orc_weno5(_p(q), sgn, eps)


def thomas(a, b, c, r):
    n = len(b)
    a, b, c, r = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, r))
    x = np.zeros(n)
    lib().orc_thomas(n, _p(a), _p(b), _p(c), _p(r), _p(x))
    return x


def eos_p(Theta: float) -> float:
    return lib().orc_eos_p(Theta)


def eos_pprime(Theta: float, Theta0: float, p0: float) -> float:
    return lib().orc_eos_pprime(Theta, Theta0, p0)


def esat(T: float) -> float:
    return lib().orc_esat(T)


def qvsat(T: float, p: float) -> float:
    return lib().orc_qvsat(T, p)


def sat_adjust(T: float, p: float, qv: float, qc: float) -> float:
    return lib().orc_sat_adjust(T, p, qv, qc)


def eos_p_moist(Theta: float, qv: float) -> float:
    return lib().orc_eos_p_moist(Theta, qv)


def eos_pprime_moist(Theta: float, qv: float, Theta0: float, qv0: float, p0: float) -> float:
    return lib().orc_eos_pprime_moist(Theta, qv, Theta0, qv0, p0)


def base_state(dz, theta0, p_surface: float, grav: float = 9.81, qv0=None):
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    th = np.ascontiguousarray(theta0, dtype=np.float64)
    qv = None if qv0 is None else np.ascontiguousarray(qv0, dtype=np.float64)
    nz = len(dz)
    rho0, p0, pi0 = np.zeros(nz), np.zeros(nz), np.zeros(nz)
    rc = lib().orc_base_state_moist(nz, _p(dz), _p(th), None if qv is None else _p(qv), p_surface, grav,
                                    _p(rho0), _p(p0), _p(pi0))
    if rc != 0:
        raise RuntimeError("orc_base_state failed")
    return rho0, p0, pi0
