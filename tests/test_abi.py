"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and its host-side validation, planning and workspace sizing behave
as documented.  No call here touches a GPU."""
import math
import os
import re

import numpy as np
import pytest

from paper_2308_03972_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmletkf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lbmletkf_status|const char\s*\*)\s*(\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2308_03972_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lbmletkf.h but not exported"
        assert n in binding.SIGNATURES, f"{n} has no ctypes signature in the binding"
    assert set(binding.SIGNATURES) == set(names)


def test_status_strings(lib):
    assert lib.lbmletkf_status_string(0) == b"ok"
    assert lib.lbmletkf_status_string(-1) == b"invalid argument"
    assert lib.lbmletkf_status_string(-7) == b"workspace missing or too small"
    assert lib.lbmletkf_status_string(123) == b"unknown status"


def _plan(**kw):
    cfg = inputs.CONFIGS[kw.pop("cfg", "paper")]
    args = dict(nx=cfg.n, ny=cfg.n, members=cfg.members, points=inputs.observation_points(cfg),
                nvar=cfg.nvar, sigma=cfg.sigmas, d_cut=cfg.d_cut, beta=cfg.beta,
                tau0=cfg.tau0, cs=cfg.cs)
    args.update(kw)
    return binding.plan(**args)


def test_plan_matches_brute_force_local_counts(lib):
    """The planner's support count uses |xi - eta| < 2 d_cut (minimum image)."""
    for name in ("tiny", "paper"):
        cfg = inputs.CONFIGS[name]
        lmax, n, route = _plan(cfg=name)
        pts = inputs.observation_points(cfg)
        xs, ys = np.meshgrid(np.arange(cfg.n), np.arange(cfg.n))
        dx = np.abs(xs.ravel()[:, None] - pts[None, :, 0])
        dy = np.abs(ys.ravel()[:, None] - pts[None, :, 1])
        dx = np.minimum(dx, cfg.n - dx)
        dy = np.minimum(dy, cfg.n - dy)
        counts = ((dx * dx + dy * dy) < 4 * cfg.d_cut ** 2).sum(axis=1)
        assert lmax == counts.max()
        nz = cfg.nvar * lmax
        if name == "paper":
            # 8x8 points every 32 cells, d_cut = 16 sqrt(3): at most 12 points
            assert lmax == 12 and route == binding.ROUTE_OBSERVATION and n == 24 == nz
        else:
            # M = 8 members < 2 * lmax local observations: ensemble route
            assert route == binding.ROUTE_ENSEMBLE and n == 8


def test_plan_routes_and_limits(lib):
    assert _plan(route=binding.ROUTE_ENSEMBLE)[1:] == (64, binding.ROUTE_ENSEMBLE)
    # no localization: every node sees all 64 points = 128 observations
    lmax, n, r = _plan(d_cut=math.inf)
    assert lmax == 64 and r == binding.ROUTE_ENSEMBLE and n == 64
    with pytest.raises(binding.LbmLetkfError) as e:
        _plan(d_cut=math.inf, route=binding.ROUTE_OBSERVATION)
    assert e.value.status == -8


@pytest.mark.parametrize("kw,status", [
    (dict(tau0=0.5), -1), (dict(tau0=float("nan")), -1), (dict(members=0), -2),
    (dict(members=65), -2), (dict(cs=-0.1), -1), (dict(nvar=4), -1),
    (dict(sigma=(0.0, 0.1)), -1), (dict(beta=0.0), -1), (dict(nx=2), -2),
    (dict(points=np.array([[256, 0]])), -1), (dict(points=np.array([[0, -1]])), -1),
    (dict(route=7), -1), (dict(mu=-1.0), -1),
])
def test_validation_rejects_bad_arguments(lib, kw, status):
    with pytest.raises(binding.LbmLetkfError) as e:
        _plan(**kw)
    assert e.value.status == status
    assert lib.lbmletkf_last_error()


def test_workspace_accounts_for_state_and_tables(lib):
    cfg = inputs.CONFIGS["paper"]
    nbytes = binding.workspace_bytes(cfg.n, cfg.n, cfg.members, inputs.observation_points(cfg),
                                     cfg.nvar, cfg.sigmas, cfg.d_cut, cfg.beta)
    state = cfg.n * cfg.n * 9 * cfg.members * 8
    table = cfg.n * cfg.n * 12 * (4 + 8)
    # per-node G (n x n) and h (n) between the two analysis kernels, n the
    # eigenproblem size of the node's local-observation count
    lmax, _, _ = binding.plan(cfg.n, cfg.n, cfg.members, inputs.observation_points(cfg),
                              cfg.nvar, cfg.sigmas, cfg.d_cut, cfg.beta)
    gmin = cfg.n * cfg.n * (16 * 16 + 16) * 8
    gmax = cfg.n * cfg.n * (24 * 24 + 24) * 8
    # run_cycle's diagnostics: five fields per node for the forecast and the analysis
    diag = 2 * cfg.n * cfg.n * 5 * 8
    assert state + table + gmin + diag < nbytes < state + table + gmax + diag + 4 * 2**20
    assert nbytes % 256 == 0


def _adjoint_bytes(lib, n, members, storage, n_points, steps, times):
    import ctypes
    lbm = binding.LbmParams(n, n, members, 0.52, 0.1, 0.0, storage)
    out = ctypes.c_size_t(0)
    st = lib.lbmletkf_adjoint_workspace_bytes(ctypes.byref(lbm), n_points, steps, times,
                                              ctypes.byref(out))
    return st, int(out.value)


def test_adjoint_workspace_holds_checkpoints_segment_and_adjoints(lib):
    """Differentiation workload (128^2, 16 members, 64 points, 10 times 20 steps
    apart): 10 checkpoints + two sets of 19 recomputed states in the storage type,
    two FP64 adjoint states, per-(member, point) misfit terms and per-block
    partials."""
    def align(v):
        return (v + 255) // 256 * 256
    for storage, elem in ((binding.STORAGE_F32_DEV, 4), (binding.STORAGE_F64, 8)):
        st, nbytes = _adjoint_bytes(lib, 128, 16, storage, 64, 20, 10)
        assert st == 0
        plane = 128 * 128
        state = align(plane * 9 * 16 * elem)
        expect = (state * 10 + 2 * state * 19 + 2 * align(plane * 9 * 16 * 8)
                  + align(16 * 64 * 8) + align(16 * (plane // 256) * 8))
        assert nbytes == expect
    st, _ = _adjoint_bytes(lib, 128, 16, 0, 64, 0, 10)
    assert st == -1
    st, _ = _adjoint_bytes(lib, 128, 16, 0, 64, 20, 0)
    assert st == -1
    st, _ = _adjoint_bytes(lib, 2, 16, 0, 64, 20, 1)
    assert st == -2


def test_misfit_entries_validate_before_any_gpu_call(lib):
    import ctypes
    st = lib.lbmletkf_misfit_forward(None, None, 0.1, 20, 10, None, None, None, 0, None)
    assert st == -1
    st = lib.lbmletkf_misfit_backward(None, None, 0.1, 20, 10, None, None, 0, None, None, None)
    assert st == -1
    assert b"NULL" in lib.lbmletkf_last_error()
