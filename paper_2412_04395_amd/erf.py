"""Thin Python binding of liberf.so (include/erf.h).

Argument marshalling only: every step of the RK3 path runs in the HIP kernels
of liberf.so.  torch supplies device memory and the stream.  There is no CPU
fallback: if the library is missing, or no GPU is present, the calls raise.

State dictionaries hold torch tensors on the GPU (float64 in FP64 mode):
    rho, rt : (nz, ny, nx)     rho and rho*theta at cell centres
    ru, rv  : (nz, ny, nx)     x-/y-face momenta (face i between cells i-1, i)
    rw      : (nz+1, ny, nx)   z-face momentum (face k below cell k)
    rq      : (nq, nz, ny, nx) rho*q of the advected scalars
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liberf.so")
FIELDS = ("rho", "rt", "ru", "rv", "rw", "rq")

ERF_OK, ERF_E_ARG, ERF_E_SHAPE, ERF_E_HIP, ERF_E_NONFINITE, ERF_E_UNSUPPORTED, ERF_E_NOMEM, ERF_E_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
ERF_FP64, ERF_FP32_MIXED = 0, 1

ERF_SGS_NONE, ERF_SGS_SMAGORINSKY, ERF_SGS_MLP = 0, 1, 2
MLP_NPARAMS, MLP_NNORM = 9609, 38
MLP_NOALLOC_MAX_BATCH = 8192  # ERF_MLP_NOALLOC_MAX_BATCH of include/erf_mlp.h

# every symbol include/erf.h, include/erf_mlp.h and include/erf_ensemble.h declare
EXPORTS = ("erf_base_state_host", "erf_create", "erf_destroy", "erf_last_error", "erf_workspace_bytes",
           "erf_init_base_state", "erf_slow_rhs", "erf_acoustic_substeps", "erf_scalar_advance",
           "erf_rk3_step", "erf_kessler", "erf_precipitation", "erf_project", "erf_ssprk2_step",
           "erf_anelastic_pressure", "erf_diagnostics", "erf_timing_begin", "erf_timing_end", "erf_layout", "erf_autotune",
           "erf_mlp_set_weights", "erf_mlp_get_weights", "erf_mlp_forward", "erf_mlp_features",
           "erf_box_filter", "erf_mlp_fit_norm", "erf_mlp_standardize", "erf_mlp_loss_grad",
           "erf_mlp_train_step", "erf_mlp_loss_grad_noalloc", "erf_mlp_fallback_count",
           "erf_ensemble_create", "erf_ensemble_destroy", "erf_ensemble_last_error", "erf_ensemble_member",
           "erf_ensemble_set_branches", "erf_ensemble_branches", "erf_ensemble_set_batched", "erf_ensemble_batched",
           "erf_ensemble_rk3_step", "erf_ensemble_autotune", "erf_set_terrain", "erf_terrain_heights",
           "erf_init_base_state_columns")
_NOT_STATUS = ("erf_destroy", "erf_last_error", "erf_workspace_bytes", "erf_ensemble_destroy",
               "erf_ensemble_last_error", "erf_ensemble_member", "erf_ensemble_branches", "erf_ensemble_batched")


class ErfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (erf_status {status})")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double),
                ("dy", C.c_double), ("dz", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_substeps", C.c_int32), ("beta_s", C.c_double),
                ("beta_d", C.c_double), ("adv_order_h", C.c_int32), ("adv_order_v", C.c_int32),
                ("scalar_scheme", C.c_int32), ("n_scalars", C.c_int32), ("sgs", C.c_int32),
                ("Cs", C.c_double), ("Pr_t", C.c_double), ("nu_m", C.c_double), ("alpha_m", C.c_double),
                ("f_cor", C.c_double), ("Ug", C.c_double), ("Vg", C.c_double),
                ("surf_heat_flux", C.c_double), ("grav", C.c_double), ("precision", C.c_int32),
                ("moist", C.c_int32), ("microphysics", C.c_int32), ("anelastic", C.c_int32),
                ("most_z0", C.c_double)]


class State(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("rhotheta", C.c_void_p), ("rhou", C.c_void_p),
                ("rhov", C.c_void_p), ("rhow", C.c_void_p), ("rhoq", C.c_void_p)]


class FieldLayout(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("components", C.c_int32),
                ("stride_y", C.c_int64), ("stride_z", C.c_int64), ("stride_c", C.c_int64), ("count", C.c_int64),
                ("bytes", C.c_int64), ("elem_bytes", C.c_int32), ("perturbation", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("levels_per_wave", C.c_int32), ("tile_rows", C.c_int32), ("ms_per_step", C.c_double),
                ("from_cache", C.c_int32)]


# erf_field ids, in the order of the state dictionaries' keys
FIELD_IDS = {"rho": 0, "rt": 1, "ru": 2, "rv": 3, "rw": 4, "rq": 5}


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("theta_mass", C.c_double), ("energy", C.c_double),
                ("max_w", C.c_double), ("nonfinite", C.c_int64), ("scalar_mass", C.c_double * 8)]


_lib = None
_lock = threading.Lock()
_DP = C.POINTER(C.c_double)


def load(path: str = LIB_PATH):
    """Load liberf.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
            # torch first: the library must bind to the HIP runtime torch
            # allocates with, not to a second copy of it
            import torch  # noqa: F401
            L = C.CDLL(path)
            L.erf_base_state_host.argtypes = [C.c_int32, _DP, _DP, _DP, C.c_double, C.c_double, _DP, _DP, _DP]
            L.erf_create.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)]
            L.erf_destroy.argtypes = [C.c_void_p]
            L.erf_destroy.restype = None
            L.erf_last_error.argtypes = [C.c_void_p]
            L.erf_last_error.restype = C.c_char_p
            L.erf_workspace_bytes.argtypes = [C.c_void_p]
            L.erf_workspace_bytes.restype = C.c_int64
            L.erf_init_base_state.argtypes = [C.c_void_p, _DP, _DP, C.c_double, _DP, _DP, _DP]
            L.erf_slow_rhs.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(State)]
            L.erf_set_terrain.argtypes = [C.c_void_p, _DP, C.c_double]
            L.erf_terrain_heights.argtypes = [C.c_void_p, _DP, _DP]
            L.erf_init_base_state_columns.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP]
            L.erf_acoustic_substeps.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(State), C.POINTER(State),
                                                C.c_int32, C.c_double, C.POINTER(State), C.POINTER(State)]
            L.erf_scalar_advance.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(State), C.POINTER(State),
                                             C.c_double, C.c_void_p]
            L.erf_rk3_step.argtypes = [C.c_void_p, C.POINTER(State)]
            L.erf_kessler.argtypes = [C.c_void_p, C.POINTER(State), C.c_double, C.c_void_p]
            L.erf_precipitation.argtypes = [C.c_void_p, _DP, C.c_int32]
            L.erf_project.argtypes = [C.c_void_p, C.POINTER(State), C.c_double]
            L.erf_ssprk2_step.argtypes = [C.c_void_p, C.POINTER(State)]
            L.erf_anelastic_pressure.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
            L.erf_diagnostics.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Diag)]
            L.erf_timing_begin.argtypes = [C.c_void_p, C.c_char_p, C.c_int32]
            L.erf_timing_end.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
            L.erf_layout.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int32, C.POINTER(FieldLayout)]
            L.erf_autotune.argtypes = [C.c_void_p, C.POINTER(State), C.c_int32, C.c_char_p, C.POINTER(Tuning)]
            _FP = C.POINTER(C.c_float)
            L.erf_mlp_set_weights.argtypes = [C.c_void_p, _FP, _DP]
            L.erf_mlp_get_weights.argtypes = [C.c_void_p, _FP, _DP]
            L.erf_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
            L.erf_mlp_features.argtypes = [C.c_void_p, C.POINTER(State), C.c_void_p]
            L.erf_box_filter.argtypes = [C.c_void_p, C.POINTER(State), C.c_int32, C.c_double, C.c_double,
                                         C.POINTER(State), C.c_void_p]
            L.erf_mlp_fit_norm.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
            L.erf_mlp_standardize.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                              C.c_void_p]
            L.erf_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, _DP]
            L.erf_mlp_loss_grad_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                                    C.c_void_p]
            L.erf_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, _DP]
            L.erf_mlp_fallback_count.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
            L.erf_ensemble_create.argtypes = [C.c_int32, C.POINTER(Grid), C.POINTER(Params), C.c_void_p,
                                              C.POINTER(C.c_void_p)]
            L.erf_ensemble_destroy.argtypes = [C.c_void_p]
            L.erf_ensemble_destroy.restype = None
            L.erf_ensemble_last_error.argtypes = [C.c_void_p]
            L.erf_ensemble_last_error.restype = C.c_char_p
            L.erf_ensemble_member.argtypes = [C.c_void_p, C.c_int32]
            L.erf_ensemble_member.restype = C.c_void_p
            L.erf_ensemble_set_branches.argtypes = [C.c_void_p, C.c_int32]
            L.erf_ensemble_branches.argtypes = [C.c_void_p]
            L.erf_ensemble_branches.restype = C.c_int32
            L.erf_ensemble_set_batched.argtypes = [C.c_void_p, C.c_int32]
            L.erf_ensemble_batched.argtypes = [C.c_void_p]
            L.erf_ensemble_batched.restype = C.c_int32
            L.erf_ensemble_rk3_step.argtypes = [C.c_void_p, C.POINTER(State)]
            L.erf_ensemble_autotune.argtypes = [C.c_void_p, C.POINTER(State), C.c_int32, C.POINTER(C.c_int32),
                                                C.POINTER(C.c_double)]
            for name in EXPORTS:
                fn = getattr(L, name)
                if name not in _NOT_STATUS:
                    fn.restype = C.c_int32
            _lib = L
    return _lib


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _opt_ptr(a, n: int):
    """Pointer to a float64 copy of a length-n array, or NULL for None."""
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected {n} values, got shape {a.shape}")
    return a, _np_ptr(a)


def base_state_host(dz, theta0, p_surface: float, grav: float = 9.81, qv0=None):
    """Hydrostatic base state computed by the library's host code (no GPU);
    qv0: base-state water vapour mixing ratio [nz] or None (dry)."""
    L = load()
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    th = np.ascontiguousarray(theta0, dtype=np.float64)
    nz = len(dz)
    qv, qp = _opt_ptr(qv0, nz)
    rho0, p0, pi0 = np.zeros(nz), np.zeros(nz), np.zeros(nz)
    st = L.erf_base_state_host(nz, _np_ptr(dz), _np_ptr(th), qp, p_surface, grav, _np_ptr(rho0), _np_ptr(p0),
                               _np_ptr(pi0))
    if st != ERF_OK:
        raise ErfError(st, "erf_base_state_host")
    return rho0, p0, pi0


def params_from_config(cfg) -> Params:
    prec = {"fp64": ERF_FP64, "fp32": ERF_FP32_MIXED}[cfg.prec]
    return Params(cfg.dt, cfg.n_substeps, cfg.beta_s, cfg.beta_d, cfg.adv_order_h, cfg.adv_order_v,
                  cfg.scalar_scheme, cfg.n_scalars, cfg.sgs, cfg.Cs, cfg.Pr_t, cfg.nu_m, cfg.alpha_m,
                  cfg.f_cor, cfg.Ug, cfg.Vg, cfg.surf_heat_flux, cfg.grav, prec, int(getattr(cfg, "moist", 0)),
                  int(getattr(cfg, "microphysics", 0)), int(getattr(cfg, "anelastic", 0)),
                  float(getattr(cfg, "most_z0", 0.0)))


def layout(cfg, field: str) -> dict:
    """Layout of one state field ("rho", "rt", "ru", "rv", "rw" or "rq") as the
    library stores it (erf_layout; host only, no GPU needed)."""
    L = load()
    dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
    grid = Grid(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, _np_ptr(dz))
    out = FieldLayout()
    st = L.erf_layout(C.byref(grid), C.byref(params_from_config(cfg)), FIELD_IDS[field], C.byref(out))
    if st != ERF_OK:
        raise ErfError(st, f"erf_layout({field})")
    return {name: getattr(out, name) for name, _ in FieldLayout._fields_}


class Solver:
    """One liberf context: a grid, a parameter set and a HIP stream."""

    def __init__(self, cfg, stream=None, _handle=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liberf needs a GPU; none is visible")
        self.torch = torch
        self.cfg = cfg
        self.L = load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.dtype = torch.float64 if cfg.prec == "fp64" else torch.float32
        self._dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
        self._grid = Grid(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, _np_ptr(self._dz))
        self._params = params_from_config(cfg)
        self._owned = _handle is None
        if _handle is not None:      # a member context owned by an Ensemble
            self.h = C.c_void_p(_handle)
        else:
            h = C.c_void_p()
            st = self.L.erf_create(C.byref(self._grid), C.byref(self._params),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
            if st != ERF_OK:
                raise ErfError(st, "erf_create")
            self.h = h
        self.base = None

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value and self._owned:
            self.L.erf_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != ERF_OK:
            msg = self.L.erf_last_error(self.h)
            raise ErfError(st, f"{what}: {msg.decode() if msg else ''}")

    @property
    def workspace_bytes(self) -> int:
        return int(self.L.erf_workspace_bytes(self.h))

    # -- base state ----------------------------------------------------------
    def init_base_state(self, theta0, p_surface=None, qv0=None):
        """erf_init_base_state; qv0 [nz]: base-state water vapour of a moist
        context (None: dry)."""
        nz = self.cfg.nz
        th = np.ascontiguousarray(theta0, dtype=np.float64)
        qv, qp = _opt_ptr(qv0, nz)
        rho0, p0, pi0 = np.zeros(nz), np.zeros(nz), np.zeros(nz)
        ps = self.cfg.p_surface if p_surface is None else p_surface
        self._check(self.L.erf_init_base_state(self.h, _np_ptr(th), qp, ps, _np_ptr(rho0), _np_ptr(p0),
                                               _np_ptr(pi0)), "erf_init_base_state")
        self.base = {"rho0": rho0, "theta0": th, "p0": p0, "pi0": pi0, "qv0": np.zeros(nz) if qv is None else qv}
        return self.base

    # -- terrain-following coordinates ------------------------------------------
    def set_terrain(self, h_nodes, beta: float = 1.0):
        """erf_set_terrain: terrain heights h[ny][nx] at the nodes (node (i, j)
        the low-x, low-y corner of cell (i, j)); beta 1 basic, 3 Sullivan."""
        cfg = self.cfg
        h = np.ascontiguousarray(h_nodes, dtype=np.float64)
        if h.shape != (cfg.ny, cfg.nx):
            raise ValueError("terrain heights must be (ny, nx)")
        self._check(self.L.erf_set_terrain(self.h, _np_ptr(h), float(beta)), "erf_set_terrain")
        self.base = None

    def terrain_heights(self):
        """(Hc, zc): physical cell heights and centre heights, (nz, ny, nx)."""
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        Hc, zc = np.zeros(shp), np.zeros(shp)
        self._check(self.L.erf_terrain_heights(self.h, _np_ptr(Hc), _np_ptr(zc)), "erf_terrain_heights")
        return Hc, zc

    def init_base_state_columns(self, theta0, p_surf):
        """erf_init_base_state_columns: theta0 (nz, ny, nx) at the cell centres,
        p_surf (ny, nx) at each column's ground."""
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        th = np.ascontiguousarray(np.broadcast_to(theta0, shp), dtype=np.float64)
        ps = np.ascontiguousarray(np.broadcast_to(p_surf, shp[1:]), dtype=np.float64)
        rho0, p0, pi0 = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        self._check(self.L.erf_init_base_state_columns(self.h, _np_ptr(th), _np_ptr(ps), _np_ptr(rho0), _np_ptr(p0),
                                                       _np_ptr(pi0)), "erf_init_base_state_columns")
        self.base = {"rho0": rho0, "theta0": th, "p0": p0, "pi0": pi0, "qv0": None}
        return self.base

    # -- states ----------------------------------------------------------------
    def shapes(self):
        """Tensor shapes of the state fields, from the library's erf_layout."""
        out = {}
        for f in FIELDS:
            lay = layout(self.cfg, f)
            shape = (lay["nz"], lay["ny"], lay["nx"])
            out[f] = (lay["components"],) + shape if f == "rq" else shape
        return out

    def empty_state(self):
        t = self.torch
        return {f: t.zeros(s, dtype=self.dtype, device=self.device) for f, s in self.shapes().items()}

    def to_device(self, S_np):
        t = self.torch
        return {f: t.from_numpy(np.ascontiguousarray(S_np[f])).to(self.device, self.dtype) for f in FIELDS}

    @staticmethod
    def to_numpy(S):
        return {f: S[f].detach().cpu().double().numpy() for f in FIELDS}

    # The FP32 storage keeps rho and rho*theta as perturbations about the base
    # state (include/erf.h); these two convert a full FP64 host state to and
    # from the context's storage.
    def _base_cols(self):
        if self.base is None:
            raise RuntimeError("init_base_state must come first")
        rho0 = self.base["rho0"][:, None, None]
        return rho0, (self.base["rho0"] * self.base["theta0"])[:, None, None]

    def from_full(self, S_np):
        S = dict(S_np)
        if self.cfg.prec == "fp32":
            rho0, T0 = self._base_cols()
            S["rho"] = S_np["rho"] - rho0
            S["rt"] = S_np["rt"] - T0
        return self.to_device(S)

    def to_full(self, S):
        out = self.to_numpy(S)
        if self.cfg.prec == "fp32":
            rho0, T0 = self._base_cols()
            out["rho"] = out["rho"] + rho0
            out["rt"] = out["rt"] + T0
        return out

    def _st(self, S, fields=FIELDS):
        vals = {}
        for f, name in zip(FIELDS, ("rho", "rhotheta", "rhou", "rhov", "rhow", "rhoq")):
            t = S.get(f) if S is not None else None
            if t is None or f not in fields or t.numel() == 0:
                vals[name] = None
                continue
            if not (t.is_cuda and t.is_contiguous() and t.dtype == self.dtype):
                raise TypeError(f"field {f} must be a contiguous {self.dtype} CUDA tensor")
            if tuple(t.shape) != self.shapes()[f]:
                raise ValueError(f"field {f} has shape {tuple(t.shape)}, expected {self.shapes()[f]}")
            vals[name] = t.data_ptr()
        return State(**vals)

    # -- the calls -------------------------------------------------------------
    def slow_rhs(self, S, R=None):
        R = self.empty_state() if R is None else R
        self._check(self.L.erf_slow_rhs(self.h, C.byref(self._st(S)), C.byref(self._st(R))), "erf_slow_rhs")
        return R

    def acoustic_substeps(self, Sn, St, Rt, n_sub: int, dtau: float, out=None, flux=None, sums: bool = True):
        """erf_acoustic_substeps; with sums=False no stage-averaged momenta are
        kept (flux_avg = NULL) and the returned flux is None."""
        out = self.empty_state() if out is None else out
        if sums:
            flux = self.empty_state() if flux is None else flux
            fp = C.byref(self._st(flux))
        else:
            flux, fp = None, None
        self._check(self.L.erf_acoustic_substeps(self.h, C.byref(self._st(Sn)), C.byref(self._st(St)),
                                                 C.byref(self._st(Rt)), int(n_sub), float(dtau),
                                                 C.byref(self._st(out)), fp),
                    "erf_acoustic_substeps")
        return out, flux

    def scalar_advance(self, Sn, St, flux, dts: float, out=None):
        t = self.torch
        out = t.zeros_like(Sn["rq"]) if out is None else out
        self._check(self.L.erf_scalar_advance(self.h, C.byref(self._st(Sn)), C.byref(self._st(St)),
                                              C.byref(self._st(flux)), float(dts), C.c_void_p(out.data_ptr())),
                    "erf_scalar_advance")
        return out

    def rk3_step(self, S):
        self._check(self.L.erf_rk3_step(self.h, C.byref(self._st(S))), "erf_rk3_step")
        return S

    # -- anelastic contexts (Sec. 2.2, Sec. 3.2) ----------------------------
    def ssprk2_step(self, S):
        """erf_ssprk2_step: one anelastic SSP-RK2 step with projections, in place."""
        self._check(self.L.erf_ssprk2_step(self.h, C.byref(self._st(S))), "erf_ssprk2_step")
        return S

    def project(self, S, dt: float):
        """erf_project: project the face momenta of S in place; the context's
        perturbation pressure gains psi."""
        self._check(self.L.erf_project(self.h, C.byref(self._st(S)), float(dt)), "erf_project")
        return S

    def anelastic_pressure(self, set_to=None):
        """The context's perturbation pressure as a float64 tensor [nz][ny][nx]
        (a copy); with set_to (a tensor of that shape) it is replaced first."""
        t = self.torch
        shp = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        if set_to is not None:
            self._check(self.L.erf_anelastic_pressure(self.h, self._dev(set_to, t.float64, shp, "p"), 1),
                        "erf_anelastic_pressure")
        out = t.empty(shp, dtype=t.float64, device=self.device)
        self._check(self.L.erf_anelastic_pressure(self.h, C.c_void_p(out.data_ptr()), 0), "erf_anelastic_pressure")
        return out

    def kessler(self, S, dt: float, precip=None):
        """erf_kessler: Kessler microphysics over dt on S in place; precip (a
        float64 tensor [ny][nx] on the device) accumulates the rain reaching
        the ground, else the context's own accumulator does."""
        self._check(self.L.erf_kessler(self.h, C.byref(self._st(S)), float(dt),
                                       None if precip is None else
                                       self._dev(precip, self.torch.float64, (self.cfg.ny, self.cfg.nx), "precip")),
                    "erf_kessler")
        return S

    def precipitation(self, reset: bool = False) -> np.ndarray:
        """The context's accumulated precipitation [kg/m^2], [ny][nx]."""
        out = np.zeros((self.cfg.ny, self.cfg.nx))
        self._check(self.L.erf_precipitation(self.h, _np_ptr(out), int(bool(reset))), "erf_precipitation")
        return out

    def autotune(self, S, trials: int = 3, cache_path: str | None = None) -> dict:
        """erf_autotune: time the acoustic substep's launch shapes on S (which
        advances) or read the choice from cache_path; returns the choice."""
        out = Tuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.L.erf_autotune(self.h, C.byref(self._st(S)), int(trials), path, C.byref(out)),
                    "erf_autotune")
        return {name: getattr(out, name) for name, _ in Tuning._fields_}

    def timing_begin(self, kernel: str, max_launches: int = 4096):
        self._check(self.L.erf_timing_begin(self.h, kernel.encode(), int(max_launches)), "erf_timing_begin")

    def timing_end(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(self.L.erf_timing_end(self.h, C.byref(ms), C.byref(n)), "erf_timing_end")
        return ms.value, n.value

    # -- learned closure (include/erf_mlp.h) -----------------------------------
    def _dev(self, t, dtype, shape=None, what="tensor"):
        torch = self.torch
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype):
            raise TypeError(f"{what} must be a contiguous {dtype} CUDA tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    def mlp_set_weights(self, params, norm=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_NPARAMS:
            raise ValueError(f"params must hold {MLP_NPARAMS} values")
        n = None if norm is None else np.ascontiguousarray(norm, dtype=np.float64)
        if n is not None and n.size != MLP_NNORM:
            raise ValueError(f"norm must hold {MLP_NNORM} values")
        self._check(self.L.erf_mlp_set_weights(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                               None if n is None else _np_ptr(n)), "erf_mlp_set_weights")

    def mlp_get_weights(self):
        p = np.zeros(MLP_NPARAMS, dtype=np.float32)
        n = np.zeros(MLP_NNORM)
        self._check(self.L.erf_mlp_get_weights(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), _np_ptr(n)),
                    "erf_mlp_get_weights")
        return p, n

    def mlp_forward(self, x):
        n = x.shape[0]
        y = self.torch.empty((n, 9), dtype=self.torch.float32, device=self.device)
        self._check(self.L.erf_mlp_forward(self.h, self._dev(x, self.torch.float32, (n, 10), "x"), n,
                                           C.c_void_p(y.data_ptr())), "erf_mlp_forward")
        return y

    def mlp_features(self, S):
        c = self.cfg
        f = self.torch.empty((c.nx * c.ny * c.nz, 10), dtype=self.torch.float64, device=self.device)
        self._check(self.L.erf_mlp_features(self.h, C.byref(self._st(S)), C.c_void_p(f.data_ptr())),
                    "erf_mlp_features")
        return f

    def box_filter(self, S, r: int, Cs: float = 0.0, Pr_t: float = 1.0 / 3.0):
        """Coarse state (float64 full values, dict of tensors) and targets (nc, 9)."""
        torch, c = self.torch, self.cfg
        nx, ny, nz = c.nx // r, c.ny // r, c.nz // r
        z = lambda *s: torch.zeros(s, dtype=torch.float64, device=self.device)
        Cst = {"rho": z(nz, ny, nx), "rt": z(nz, ny, nx), "ru": z(nz, ny, nx), "rv": z(nz, ny, nx),
               "rw": z(nz + 1, ny, nx), "rq": z(0, nz, ny, nx)}
        tg = z(nx * ny * nz, 9)
        cs = State(Cst["rho"].data_ptr(), Cst["rt"].data_ptr(), Cst["ru"].data_ptr(), Cst["rv"].data_ptr(),
                   Cst["rw"].data_ptr(), None)
        self._check(self.L.erf_box_filter(self.h, C.byref(self._st(S)), int(r), float(Cs), float(Pr_t),
                                          C.byref(cs), C.c_void_p(tg.data_ptr())), "erf_box_filter")
        return Cst, tg

    def mlp_fit_norm(self, feat, targets):
        n = feat.shape[0]
        self._check(self.L.erf_mlp_fit_norm(self.h, self._dev(feat, self.torch.float64, (n, 10), "feat"),
                                            self._dev(targets, self.torch.float64, (n, 9), "targets"), n),
                    "erf_mlp_fit_norm")

    def mlp_standardize(self, feat, targets=None):
        torch = self.torch
        n = feat.shape[0]
        x = torch.empty((n, 10), dtype=torch.float32, device=self.device)
        t = None if targets is None else torch.empty((n, 9), dtype=torch.float32, device=self.device)
        self._check(self.L.erf_mlp_standardize(self.h, self._dev(feat, torch.float64, (n, 10), "feat"),
                                               None if targets is None else
                                               self._dev(targets, torch.float64, (n, 9), "targets"), n,
                                               C.c_void_p(x.data_ptr()),
                                               None if t is None else C.c_void_p(t.data_ptr())),
                    "erf_mlp_standardize")
        return x, t

    def mlp_loss_grad(self, x, t):
        torch = self.torch
        n = x.shape[0]
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=self.device)
        loss = C.c_double()
        self._check(self.L.erf_mlp_loss_grad(self.h, self._dev(x, torch.float32, (n, 10), "x"),
                                             self._dev(t, torch.float32, (n, 9), "t"), n,
                                             C.c_void_p(g.data_ptr()), C.byref(loss)), "erf_mlp_loss_grad")
        return loss.value, g

    def mlp_loss_grad_noalloc(self, x, t, grad=None, loss=None):
        """erf_mlp_loss_grad_noalloc: gradient into grad (float32[9609]) and the
        loss into loss (float64[1]) on the device, with nothing allocated by
        the library and nothing waited for."""
        torch = self.torch
        n = x.shape[0]
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=self.device) if grad is None else grad
        self._check(self.L.erf_mlp_loss_grad_noalloc(self.h, self._dev(x, torch.float32, (n, 10), "x"),
                                                     self._dev(t, torch.float32, (n, 9), "t"), n,
                                                     self._dev(g, torch.float32, (MLP_NPARAMS,), "grad"),
                                                     None if loss is None else
                                                     self._dev(loss, torch.float64, (1,), "loss")),
                    "erf_mlp_loss_grad_noalloc")
        return g

    def mlp_train_step(self, x, t, lr: float, want_loss: bool = True):
        torch = self.torch
        n = x.shape[0]
        loss = C.c_double()
        self._check(self.L.erf_mlp_train_step(self.h, self._dev(x, torch.float32, (n, 10), "x"),
                                              self._dev(t, torch.float32, (n, 9), "t"), n, float(lr),
                                              C.byref(loss) if want_loss else None), "erf_mlp_train_step")
        return loss.value if want_loss else None

    def mlp_fallback_count(self) -> int:
        v = C.c_int64()
        self._check(self.L.erf_mlp_fallback_count(self.h, C.byref(v)), "erf_mlp_fallback_count")
        return v.value

    def diagnostics(self, S, allow_nonfinite: bool = False):
        d = Diag()
        st = self.L.erf_diagnostics(self.h, C.byref(self._st(S)), C.byref(d))
        if st != ERF_OK and not (allow_nonfinite and st == ERF_E_NONFINITE):
            self._check(st, "erf_diagnostics")
        return {"mass": d.mass, "theta_mass": d.theta_mass, "energy": d.energy, "max_w": d.max_w,
                "nonfinite": int(d.nonfinite), "scalar_mass": np.array(d.scalar_mass[:self.cfg.n_scalars])}


class Ensemble:
    """Independent members stepped together (include/erf_ensemble.h): one HIP
    graph launch per ensemble step."""

    def __init__(self, cfgs, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liberf needs a GPU; none is visible")
        self.torch = torch
        self.L = load()
        self.cfgs = list(cfgs)
        n = len(self.cfgs)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._dz = [np.ascontiguousarray(c.dz, dtype=np.float64) for c in self.cfgs]
        grids = (Grid * n)(*[Grid(c.nx, c.ny, c.nz, c.dx, c.dy, _np_ptr(d)) for c, d in zip(self.cfgs, self._dz)])
        params = (Params * n)(*[params_from_config(c) for c in self.cfgs])
        h = C.c_void_p()
        st = self.L.erf_ensemble_create(n, grids, params, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != ERF_OK:
            raise ErfError(st, "erf_ensemble_create")
        self.h = h
        self.members = [Solver(c, stream=self.stream, _handle=self.L.erf_ensemble_member(h, m))
                        for m, c in enumerate(self.cfgs)]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            for s in self.members:
                s.h = None
            self.L.erf_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != ERF_OK:
            msg = self.L.erf_ensemble_last_error(self.h)
            raise ErfError(st, f"{what}: {msg.decode() if msg else ''}")

    def _states(self, states):
        if len(states) != len(self.members):
            raise ValueError("one state per member")
        return (State * len(states))(*[m._st(S) for m, S in zip(self.members, states)])

    @property
    def branches(self) -> int:
        return int(self.L.erf_ensemble_branches(self.h))

    def set_branches(self, n: int):
        self._check(self.L.erf_ensemble_set_branches(self.h, int(n)), "erf_ensemble_set_branches")

    @property
    def batched(self) -> bool:
        return bool(self.L.erf_ensemble_batched(self.h))

    def set_batched(self, on: bool):
        self._check(self.L.erf_ensemble_set_batched(self.h, int(bool(on))), "erf_ensemble_set_batched")

    def rk3_step(self, states):
        self._states_keep = self._states(states)
        self._check(self.L.erf_ensemble_rk3_step(self.h, self._states_keep), "erf_ensemble_rk3_step")

    def autotune(self, states, trials: int = 3):
        nb, ms = C.c_int32(), C.c_double()
        self._check(self.L.erf_ensemble_autotune(self.h, self._states(states), int(trials), C.byref(nb),
                                                 C.byref(ms)), "erf_ensemble_autotune")
        return nb.value, ms.value
