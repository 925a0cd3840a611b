"""Thin ctypes binding of liblbmletkf.so (declared in include/lbmletkf.h).

Argument marshalling only: every step of the forecast-analysis cycle runs in
the library's HIP kernels.  Device buffers are torch CUDA tensors (float64,
contiguous) and launches go to torch's current stream.  If the library is
not built, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch  # imported before the library so that one HIP runtime is shared

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmletkf.so")

LBMLETKF_OK = 0
LBMLETKF_ENONFINITE, LBMLETKF_EDIVERGED, LBMLETKF_EEIG = -4, -5, -6
DIAG_LEN = 8
NSTAGES = 7
STAGES = ("stream_collide", "observe", "obs_stats", "analysis", "diagnostics", "adjoint",
          "misfit")
ROUTE_AUTO, ROUTE_ENSEMBLE, ROUTE_OBSERVATION = 0, 1, 2
STORAGE_F64, STORAGE_F32_DEV = 0, 1

_c_int32 = ctypes.c_int32
_c_double = ctypes.c_double
_vp = ctypes.c_void_p


class LbmParams(ctypes.Structure):
    _fields_ = [("nx", _c_int32), ("ny", _c_int32), ("members", _c_int32),
                ("tau0", _c_double), ("cs", _c_double), ("mu", _c_double),
                ("storage", _c_int32)]


class ObsParams(ctypes.Structure):
    _fields_ = [("n_points", _c_int32), ("points", ctypes.POINTER(_c_int32)),
                ("nvar", _c_int32), ("sigma", _c_double * 3), ("d_cut", _c_double),
                ("beta", _c_double), ("route", _c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("forecast_blocks", _c_int32), ("tile_rows", _c_int32),
                ("bucket_granularity", _c_int32), ("use_graph", _c_int32),
                ("steps_per_launch", _c_int32), ("analysis_queue", _c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LbmLetkfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbmletkf status {status}: {msg}")
        self.status = status


# every symbol include/lbmletkf.h declares, with (restype, argtypes)
SIGNATURES = {
    "lbmletkf_workspace_bytes": (_c_int32, [ctypes.POINTER(LbmParams), ctypes.POINTER(ObsParams),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "lbmletkf_create": (_c_int32, [ctypes.POINTER(LbmParams), ctypes.POINTER(ObsParams), _vp, _vp,
                                   ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lbmletkf_destroy": (_c_int32, [_vp]),
    "lbmletkf_init_equilibrium": (_c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "lbmletkf_import": (_c_int32, [_vp, _vp, _vp, _vp]),
    "lbmletkf_export": (_c_int32, [_vp, _vp, _vp, _vp]),
    "lbm_ensemble_step": (_c_int32, [_vp, _vp, _c_int32, _vp]),
    "observe": (_c_int32, [_vp, _vp, _vp, _vp]),
    "letkf_analyze": (_c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "lbmletkf_diagnostics": (_c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "run_cycle": (_c_int32, [_vp, _vp, _c_int32, _vp, _vp, _vp, _vp]),
    "lbmletkf_moments": (_c_int32, [_vp, _vp, _vp, _vp]),
    "lbmletkf_diagnostics_noalloc": (_c_int32, [ctypes.POINTER(LbmParams), _vp, _vp, _vp, _vp]),
    "lbmletkf_set_checks": (_c_int32, [_vp, _c_int32, _c_double, _c_int32]),
    "lbmletkf_set_matrix_core_transform": (_c_int32, [_vp, _c_int32]),
    "lbmletkf_check": (_c_int32, [_vp, _vp, _vp]),
    "lbmletkf_energy_spectrum": (_c_int32, [_vp, _vp, _vp, _c_int32, _vp]),
    "lbmletkf_synth_obs": (_c_int32, [_vp, _vp, _vp, _vp, _c_int32, _vp]),
    "lbmletkf_plan": (_c_int32, [ctypes.POINTER(LbmParams), ctypes.POINTER(ObsParams),
                                 ctypes.POINTER(_c_int32), ctypes.POINTER(_c_int32),
                                 ctypes.POINTER(_c_int32)]),
    "lbmletkf_info": (_c_int32, [_vp, ctypes.POINTER(_c_int32), ctypes.POINTER(_c_int32),
                                 ctypes.POINTER(_c_int32)]),
    "lbmletkf_local_histogram": (_c_int32, [_vp, ctypes.POINTER(_c_int32), _c_int32]),
    "lbmletkf_adjoint_workspace_bytes": (_c_int32, [ctypes.POINTER(LbmParams), _c_int32,
                                                    _c_int32, _c_int32,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "lbmletkf_misfit_forward": (_c_int32, [_vp, _vp, _c_double, _c_int32, _c_int32, _vp, _vp,
                                           _vp, ctypes.c_size_t, _vp]),
    "lbmletkf_misfit_backward": (_c_int32, [_vp, _vp, _c_double, _c_int32, _c_int32, _vp, _vp,
                                            ctypes.c_size_t, _vp, _vp, _vp]),
    "lbmletkf_batch_workspace_bytes": (_c_int32, [ctypes.POINTER(_vp), _c_int32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "lbmletkf_batch_create": (_c_int32, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _c_int32,
                                         _c_int32, ctypes.POINTER(BatchConfig), _vp,
                                         ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lbmletkf_batch_run_cycle": (_c_int32, [_vp, ctypes.POINTER(_vp), _vp]),
    "lbmletkf_batch_get_config": (_c_int32, [_vp, ctypes.POINTER(BatchConfig)]),
    "lbmletkf_batch_set_config": (_c_int32, [_vp, ctypes.POINTER(BatchConfig), _vp]),
    "lbmletkf_batch_tune": (_c_int32, [_vp, _c_int32, ctypes.POINTER(BatchConfig),
                                       ctypes.POINTER(_c_double), ctypes.POINTER(_c_double),
                                       _vp]),
    "lbmletkf_batch_destroy": (_c_int32, [_vp]),
    "lbmletkf_set_profiling": (_c_int32, [_vp, _c_int32]),
    "lbmletkf_profile_collect": (_c_int32, [_vp, ctypes.POINTER(_c_double),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "lbmletkf_status_string": (ctypes.c_char_p, [_c_int32]),
    "lbmletkf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2308_03972_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != LBMLETKF_OK:
        msg = load().lbmletkf_last_error().decode(errors="replace")
        raise LbmLetkfError(status, msg)


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: Optional[torch.Tensor], numel: Optional[int] = None, name: str = "tensor",
         dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# C entry points under their own names
# ---------------------------------------------------------------------------
def lbm_ensemble_step(ctx: "Context", f: torch.Tensor, nsteps: int, stream=None) -> None:
    _check(load().lbm_ensemble_step(ctx.handle, ctx._state(f), int(nsteps), _stream(stream)))


def observe(ctx: "Context", f: torch.Tensor, yf: torch.Tensor, stream=None) -> None:
    _check(load().observe(ctx.handle, ctx._state(f), _dev(yf, ctx.members * ctx.n_obs, "yf"),
                          _stream(stream)))


def letkf_analyze(ctx: "Context", f: torch.Tensor, yf: torch.Tensor, yo: torch.Tensor,
                  stream=None) -> None:
    _check(load().letkf_analyze(ctx.handle, ctx._state(f),
                                _dev(yf, ctx.members * ctx.n_obs, "yf"),
                                _dev(yo, ctx.n_obs, "yo"), _stream(stream)))


def run_cycle(ctx: "Context", f: torch.Tensor, nsteps: int, yo: torch.Tensor,
              truth_uv: Optional[torch.Tensor] = None, diag: Optional[torch.Tensor] = None,
              stream=None) -> None:
    _check(load().run_cycle(ctx.handle, ctx._state(f), int(nsteps),
                            _dev(yo, ctx.n_obs, "yo"), _dev(truth_uv, 2 * ctx.plane, "truth_uv"),
                            _dev(diag, 2 * DIAG_LEN, "diag"), _stream(stream)))


def lbmletkf_misfit_forward(ctx: "Context", f0: torch.Tensor, cs: float, steps_per_obs: int,
                            yo: torch.Tensor, J: torch.Tensor, work: "AdjointWorkspace",
                            stream=None) -> None:
    n_times = work.n_times
    _check(load().lbmletkf_misfit_forward(
        ctx.handle, ctx._state(f0), float(cs), int(steps_per_obs), int(n_times),
        _dev(yo, n_times * ctx.n_obs, "yo"), _dev(J, 1, "J"), work.ptr, work.nbytes,
        _stream(stream)))


def lbmletkf_misfit_backward(ctx: "Context", f0: torch.Tensor, cs: float, steps_per_obs: int,
                             yo: torch.Tensor, work: "AdjointWorkspace", grad_f0: torch.Tensor,
                             grad_cs: Optional[torch.Tensor] = None, stream=None) -> None:
    n_times = work.n_times
    _check(load().lbmletkf_misfit_backward(
        ctx.handle, ctx._state(f0), float(cs), int(steps_per_obs), int(n_times),
        _dev(yo, n_times * ctx.n_obs, "yo"), work.ptr, work.nbytes,
        _dev(grad_f0, ctx.state_numel, "grad_f0"), _dev(grad_cs, 1, "grad_cs"), _stream(stream)))


class AdjointWorkspace:
    """Device workspace of the misfit sweeps (checkpoints, recomputed states,
    adjoint states) for one (steps_per_obs, n_times)."""

    def __init__(self, ctx: "Context", steps_per_obs: int, n_times: int):
        n = ctypes.c_size_t(0)
        _check(load().lbmletkf_adjoint_workspace_bytes(ctypes.byref(ctx._lbm),
                                                       int(ctx.n_points), int(steps_per_obs),
                                                       int(n_times), ctypes.byref(n)))
        self.steps_per_obs, self.n_times = int(steps_per_obs), int(n_times)
        self.nbytes = int(n.value)
        self.buffer = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=ctx.device)
        self.ptr = (self.buffer.data_ptr() + 255) // 256 * 256


class ForecastMisfit(torch.autograd.Function):
    """J(f0, C_s) of lbmletkf_misfit_forward as an autograd node; its backward
    is the library's reverse sweep (lbmletkf_misfit_backward)."""

    @staticmethod
    def forward(actx, f0, cs, ctx, steps_per_obs, yo):
        cs_val = float(cs)
        f = ctx.import_canonical(f0.detach().contiguous())
        yo = yo.detach().contiguous()
        work = AdjointWorkspace(ctx, steps_per_obs, yo.shape[0])
        J = torch.empty(1, dtype=torch.float64, device=ctx.device)
        lbmletkf_misfit_forward(ctx, f, cs_val, steps_per_obs, yo, J, work)
        ctx._last_forward = (f.data_ptr(), cs_val, int(steps_per_obs), work.ptr)
        actx.saved = (ctx, f, cs_val, int(steps_per_obs), yo, work)
        actx.cs_like = cs if torch.is_tensor(cs) else None
        return J[0]

    @staticmethod
    def backward(actx, gJ):
        ctx, f, cs_val, steps, yo, work = actx.saved
        if ctx._last_forward != (f.data_ptr(), cs_val, steps, work.ptr):
            # another forward sweep ran on this context since: rebuild the checkpoints
            J = torch.empty(1, dtype=torch.float64, device=ctx.device)
            lbmletkf_misfit_forward(ctx, f, cs_val, steps, yo, J, work)
            ctx._last_forward = (f.data_ptr(), cs_val, steps, work.ptr)
        g = ctx.new_canonical()
        gcs = torch.empty(1, dtype=torch.float64, device=ctx.device)
        lbmletkf_misfit_backward(ctx, f, cs_val, steps, yo, work, g, gcs)
        gf = g * gJ
        gc = None
        if actx.cs_like is not None:
            gc = (gcs[0] * gJ).to(actx.cs_like.device, actx.cs_like.dtype).reshape(
                actx.cs_like.shape)
        return gf, gc, None, None, None


def forecast_misfit(ctx: "Context", f0: torch.Tensor, cs, steps_per_obs: int,
                    yo: torch.Tensor) -> torch.Tensor:
    """Differentiable J = sum_c sum_m sum_q (H_q(f_m(c s)) - y^o_{c,q})^2.

    f0: canonical FP64 [M][9][ny][nx] CUDA tensor; cs: float or 0-dim tensor
    (the Smagorinsky constant, differentiable when a tensor); yo:
    [n_times][n_obs]; s = steps_per_obs.  Gradients flow to f0 and cs.
    """
    return ForecastMisfit.apply(f0, cs, ctx, int(steps_per_obs), yo)


def plan(nx: int, ny: int, members: int, points, nvar: int, sigma: Sequence[float],
         d_cut: float, beta: float, tau0: float = 0.6, cs: float = 0.1, mu: float = 0.0,
         route: int = ROUTE_AUTO, storage: int = STORAGE_F64) -> Tuple[int, int, int]:
    """Host-only: (max local points, eigenproblem size, route) -- no GPU needed."""
    lbm, obs, _keep = _params(nx, ny, members, tau0, cs, mu, points, nvar, sigma, d_cut, beta,
                              route, storage)
    a, b, c = _c_int32(), _c_int32(), _c_int32()
    _check(load().lbmletkf_plan(ctypes.byref(lbm), ctypes.byref(obs), ctypes.byref(a),
                                ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def workspace_bytes(nx: int, ny: int, members: int, points, nvar: int, sigma: Sequence[float],
                    d_cut: float, beta: float, tau0: float = 0.6, cs: float = 0.1,
                    mu: float = 0.0, route: int = ROUTE_AUTO, storage: int = STORAGE_F64) -> int:
    """Host-only: bytes of device workspace a context needs."""
    lbm, obs, _keep = _params(nx, ny, members, tau0, cs, mu, points, nvar, sigma, d_cut, beta,
                              route, storage)
    n = ctypes.c_size_t(0)
    _check(load().lbmletkf_workspace_bytes(ctypes.byref(lbm), ctypes.byref(obs), ctypes.byref(n)))
    return int(n.value)


def _params(nx, ny, members, tau0, cs, mu, points, nvar, sigma, d_cut, beta, route,
            storage=STORAGE_F64):
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 2))
    lbm = LbmParams(int(nx), int(ny), int(members), float(tau0), float(cs), float(mu),
                    int(storage))
    sig = list(sigma) + [1.0] * (3 - len(sigma))
    dc = float(d_cut) if math.isfinite(d_cut) else 0.0
    obs = ObsParams(len(pts), pts.ctypes.data_as(ctypes.POINTER(_c_int32)), int(nvar),
                    (_c_double * 3)(*sig), dc, float(beta), int(route))
    return lbm, obs, pts


def diagnostics_noalloc(nx: int, ny: int, members: int, f: torch.Tensor,
                        truth_uv: Optional[torch.Tensor] = None,
                        out: Optional[torch.Tensor] = None, storage: int = STORAGE_F64,
                        stream=None) -> torch.Tensor:
    """lbmletkf_diagnostics_noalloc: the ensemble diagnostics of f (storage
    layout) without a context or workspace (static device scratch)."""
    lbm = LbmParams(int(nx), int(ny), int(members), 0.6, 0.0, 0.0, int(storage))
    dtype = torch.float32 if storage == STORAGE_F32_DEV else torch.float64
    plane = int(nx) * int(ny)
    if out is None:
        out = torch.empty(DIAG_LEN, dtype=torch.float64, device=f.device)
    _check(load().lbmletkf_diagnostics_noalloc(
        ctypes.byref(lbm), _dev(f, members * 9 * plane, "f", dtype),
        _dev(truth_uv, 2 * plane, "truth_uv"), _dev(out, DIAG_LEN, "diag"), _stream(stream)))
    return out


def synth_obs(y: torch.Tensor, eps: torch.Tensor, sigma: torch.Tensor, stream=None) -> torch.Tensor:
    n = y.numel()
    yo = torch.empty_like(y)
    _check(load().lbmletkf_synth_obs(_dev(y, n, "y"), _dev(eps, n, "eps"), _dev(sigma, n, "sigma"),
                                     _dev(yo, n, "yo"), n, _stream(stream)))
    return yo


class Context:
    """One ensemble (M members on an nx x ny grid) with its observing network.

    Owns the device workspace (a torch uint8 tensor) and the library context.
    """

    def __init__(self, nx: int, ny: int, members: int, tau0: float, cs: float,
                 points, nvar: int, sigma: Sequence[float], d_cut: float, beta: float,
                 mu: float = 0.0, force: Optional[torch.Tensor] = None,
                 route: int = ROUTE_AUTO, device: str = "cuda", storage: int = STORAGE_F64):
        lib = load()
        self.storage = int(storage)
        self.state_dtype = torch.float32 if self.storage == STORAGE_F32_DEV else torch.float64
        self.nx, self.ny, self.members, self.nvar = int(nx), int(ny), int(members), int(nvar)
        self.tau0, self.cs, self.mu = float(tau0), float(cs), float(mu)
        self._last_forward = None
        self.plane = self.nx * self.ny
        self.state_numel = self.members * 9 * self.plane
        self.points = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 2))
        self.n_points = len(self.points)
        self.n_obs = self.n_points * self.nvar
        self.device = torch.device(device)
        self._lbm, self._obs, self.points = _params(self.nx, self.ny, self.members, tau0, cs, mu,
                                                    self.points, self.nvar, sigma, d_cut, beta,
                                                    route, self.storage)
        nbytes = ctypes.c_size_t(0)
        _check(lib.lbmletkf_workspace_bytes(ctypes.byref(self._lbm), ctypes.byref(self._obs),
                                            ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._force = None
        if force is not None:
            self._force = force
        h = _vp()
        _check(lib.lbmletkf_create(ctypes.byref(self._lbm), ctypes.byref(self._obs),
                                   _dev(force, 2 * self.plane, "force"), aligned,
                                   ctypes.c_size_t(nbytes.value), _stream(None), ctypes.byref(h)))
        self.handle = h
        lmax, n, r = _c_int32(), _c_int32(), _c_int32()
        _check(lib.lbmletkf_info(self.handle, ctypes.byref(lmax), ctypes.byref(n), ctypes.byref(r)))
        self.max_local_points, self.eig_size, self.route = lmax.value, n.value, r.value

    # -- construction from a configuration object (inputs.CycleConfig) --------
    @classmethod
    def from_config(cls, cfg, members: Optional[int] = None, force: Optional[torch.Tensor] = None,
                    route: int = ROUTE_AUTO, points=None,
                    storage: int = STORAGE_F64) -> "Context":
        from . import inputs
        pts = inputs.observation_points(cfg) if points is None else points
        return cls(cfg.n, cfg.n, cfg.members if members is None else members, cfg.tau0, cfg.cs,
                   pts, cfg.nvar, cfg.sigmas, cfg.d_cut, cfg.beta, mu=cfg.mu, force=force,
                   route=route, storage=storage)

    def _state(self, f: torch.Tensor):
        return _dev(f, self.state_numel, "f", self.state_dtype)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.lbmletkf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ---------------------------------------------------------------
    def new_state(self) -> torch.Tensor:
        """A state buffer in the storage layout [y][x][a][member]."""
        return torch.empty((self.ny, self.nx, 9, self.members), dtype=self.state_dtype,
                           device=self.device)

    def new_canonical(self) -> torch.Tensor:
        return torch.empty((self.members, 9, self.ny, self.nx), dtype=torch.float64,
                           device=self.device)

    def init_equilibrium(self, uv: torch.Tensor, rho: Optional[torch.Tensor] = None,
                         stream=None) -> torch.Tensor:
        f = self.new_state()
        _check(load().lbmletkf_init_equilibrium(
            self.handle, _dev(rho, self.members * self.plane, "rho"),
            _dev(uv, self.members * 2 * self.plane, "uv"), self._state(f), _stream(stream)))
        return f

    def import_canonical(self, canon: torch.Tensor, stream=None) -> torch.Tensor:
        f = self.new_state()
        _check(load().lbmletkf_import(self.handle, _dev(canon, self.state_numel, "canonical"),
                                      self._state(f), _stream(stream)))
        return f

    def export_canonical(self, f: torch.Tensor, stream=None) -> torch.Tensor:
        out = self.new_canonical()
        _check(load().lbmletkf_export(self.handle, self._state(f), _dev(out), _stream(stream)))
        return out

    # -- the hot path ------------------------------------------------------------
    def step(self, f: torch.Tensor, nsteps: int, stream=None) -> None:
        lbm_ensemble_step(self, f, nsteps, stream)

    def observe(self, f: torch.Tensor, yf: Optional[torch.Tensor] = None, stream=None):
        if yf is None:
            yf = torch.empty((self.members, self.n_obs), dtype=torch.float64, device=self.device)
        observe(self, f, yf, stream)
        return yf

    def analyze(self, f: torch.Tensor, yf: torch.Tensor, yo: torch.Tensor, stream=None) -> None:
        letkf_analyze(self, f, yf, yo, stream)

    def run_cycle(self, f: torch.Tensor, nsteps: int, yo: torch.Tensor,
                  truth_uv: Optional[torch.Tensor] = None, diag: Optional[torch.Tensor] = None,
                  stream=None) -> None:
        run_cycle(self, f, nsteps, yo, truth_uv, diag, stream)

    # -- diagnostics ---------------------------------------------------------------
    def diagnostics(self, f: torch.Tensor, truth_uv: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(DIAG_LEN, dtype=torch.float64, device=self.device)
        _check(load().lbmletkf_diagnostics(self.handle, self._state(f),
                                           _dev(truth_uv, 2 * self.plane, "truth_uv"),
                                           _dev(out, DIAG_LEN, "diag"), _stream(stream)))
        return out

    def moments(self, f: torch.Tensor, stream=None) -> torch.Tensor:
        out = torch.empty((self.members, 3, self.ny, self.nx), dtype=torch.float64,
                          device=self.device)
        _check(load().lbmletkf_moments(self.handle, self._state(f), _dev(out), _stream(stream)))
        return out

    def energy_spectrum(self, f: torch.Tensor, kmax: Optional[int] = None,
                        stream=None) -> torch.Tensor:
        """Member-mean shell energy spectrum E[0..kmax] (default kmax = n // 2)."""
        kmax = self.nx // 2 if kmax is None else int(kmax)
        out = torch.empty(kmax + 1, dtype=torch.float64, device=self.device)
        _check(load().lbmletkf_energy_spectrum(self.handle, self._state(f), _dev(out), kmax,
                                               _stream(stream)))
        return out

    # -- health checks -------------------------------------------------------------
    def set_checks(self, max_sweeps: int = 30, diverge_limit: float = 0.0,
                   check_every_cycle: bool = False) -> None:
        _check(load().lbmletkf_set_checks(self.handle, int(max_sweeps), float(diverge_limit),
                                          int(bool(check_every_cycle))))

    def set_matrix_core_transform(self, enable: bool) -> None:
        """FP32 storage: B = dX Z^T and the transform on BF16 matrix cores."""
        _check(load().lbmletkf_set_matrix_core_transform(self.handle, int(bool(enable))))

    def check(self, diag: Optional[torch.Tensor] = None, stream=None) -> None:
        """Raises LbmLetkfError (status ENONFINITE, EEIG or EDIVERGED) if unhealthy."""
        _check(load().lbmletkf_check(self.handle, _dev(diag, 2 * DIAG_LEN, "diag"),
                                     _stream(stream)))

    def local_histogram(self) -> np.ndarray:
        """Nodes per number of local observation points (index = count)."""
        n = self.n_points + 1
        buf = (_c_int32 * n)()
        _check(load().lbmletkf_local_histogram(self.handle, buf, n))
        return np.array(buf[:], dtype=np.int64)

    # -- differentiation form ------------------------------------------------------
    def adjoint_workspace(self, steps_per_obs: int, n_times: int) -> AdjointWorkspace:
        return AdjointWorkspace(self, steps_per_obs, n_times)

    def misfit_forward(self, f0: torch.Tensor, cs: float, steps_per_obs: int, yo: torch.Tensor,
                       work: AdjointWorkspace, stream=None) -> torch.Tensor:
        """J (a 1-element device tensor) and the checkpoints in ``work``."""
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        lbmletkf_misfit_forward(self, f0, cs, steps_per_obs, yo, J, work, stream)
        self._last_forward = (f0.data_ptr(), float(cs), int(steps_per_obs), work.ptr)
        return J

    def misfit_backward(self, f0: torch.Tensor, cs: float, steps_per_obs: int,
                        yo: torch.Tensor, work: AdjointWorkspace,
                        stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
        """(dJ/df0 canonical [M][9][ny][nx], dJ/dC_s 1-element) on the device."""
        g = self.new_canonical()
        gcs = torch.empty(1, dtype=torch.float64, device=self.device)
        lbmletkf_misfit_backward(self, f0, cs, steps_per_obs, yo, work, g, gcs, stream)
        return g, gcs

    def set_profiling(self, enable) -> None:
        """False/0: off; True/1: an event pair per launch; 2: one pair per forecast
        call (all its steps) and one per analysis."""
        level = 2 if (not isinstance(enable, bool) and enable == 2) else (1 if enable else 0)
        _check(load().lbmletkf_set_profiling(self.handle, level))

    def profile_collect(self) -> Tuple[np.ndarray, np.ndarray]:
        ms = (_c_double * NSTAGES)()
        cnt = (ctypes.c_int64 * NSTAGES)()
        _check(load().lbmletkf_profile_collect(self.handle, ms, cnt))
        return np.array(ms[:]), np.array(cnt[:])


class Batch:
    """Many contexts advanced together (lbmletkf_batch_*): one persistent
    forecast launch per step for all problems, analyses grouped by eigenproblem
    size across problems, the cycle captured as a hipGraph."""

    def __init__(self, contexts: Sequence[Context], states: Sequence[torch.Tensor], nsteps: int,
                 config: Optional[dict] = None, stream=None):
        lib = load()
        if len(contexts) != len(states) or not contexts:
            raise ValueError("need one state per context")
        self.contexts = list(contexts)
        self.states = list(states)
        self.nsteps = int(nsteps)
        n = len(contexts)
        self._ctxs = (_vp * n)(*[c.handle.value for c in contexts])
        self._fs = (_vp * n)(*[c._state(f) for c, f in zip(contexts, states)])
        nbytes = ctypes.c_size_t(0)
        _check(lib.lbmletkf_batch_workspace_bytes(self._ctxs, n, ctypes.byref(nbytes)))
        dev = contexts[0].device
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        cfg = None
        if config is not None:
            cfg = BatchConfig(**{"steps_per_launch": 1, **{k: int(v) for k, v in config.items()}})
        h = _vp()
        _check(lib.lbmletkf_batch_create(self._ctxs, self._fs, n, self.nsteps,
                                         ctypes.byref(cfg) if cfg is not None else None, aligned,
                                         ctypes.c_size_t(nbytes.value), _stream(stream),
                                         ctypes.byref(h)))
        self.handle = h

    def run_cycle(self, yo: Sequence[torch.Tensor], stream=None) -> None:
        n = len(self.contexts)
        if len(yo) != n:
            raise ValueError("need one observation vector per problem")
        ptrs = (_vp * n)(*[_dev(y, c.n_obs, "yo") for c, y in zip(self.contexts, yo)])
        self._yo_keep = list(yo)
        _check(load().lbmletkf_batch_run_cycle(self.handle, ptrs, _stream(stream)))

    @property
    def config(self) -> dict:
        cfg = BatchConfig()
        _check(load().lbmletkf_batch_get_config(self.handle, ctypes.byref(cfg)))
        return cfg.as_dict()

    def set_config(self, config: dict, stream=None) -> None:
        cfg = BatchConfig(**{"steps_per_launch": 1, **{k: int(v) for k, v in config.items()}})
        _check(load().lbmletkf_batch_set_config(self.handle, ctypes.byref(cfg), _stream(stream)))

    def tune(self, reps: int = 3, stream=None) -> Tuple[dict, float, float]:
        cfg = BatchConfig()
        fms, ams = _c_double(), _c_double()
        _check(load().lbmletkf_batch_tune(self.handle, int(reps), ctypes.byref(cfg),
                                          ctypes.byref(fms), ctypes.byref(ams), _stream(stream)))
        return cfg.as_dict(), fms.value, ams.value

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.lbmletkf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
