"""GPU tests of the failure detection on the C ABI (lbmletkf_set_checks,
lbmletkf_check, run_cycle with per-cycle checks): every status is forced
from the host with data, never by faulting a kernel -- a NaN planted in the
ensemble or in the observations (arithmetic only; every loop of the
eigensolver is bounded by its sweep cap), a sweep cap of one, and a
divergence limit that a growing spread crosses.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2308_03972_amd import binding, inputs
from gpu_helpers import config_state, context, cuda, host, need_gpu, say

pytestmark = pytest.mark.gpu

TINY = inputs.CONFIGS["tiny"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _setup(cfg, route=binding.ROUTE_AUTO):
    ft, fe = config_state(cfg, spin_steps=2)
    ctx = context(cfg, route=route)
    tctx = context(cfg, members=1)
    f = ctx.import_canonical(cuda(fe))
    truth = tctx.import_canonical(cuda(ft))
    return ctx, tctx, f, truth


def _obs(cfg, tctx, truth, cycle):
    tctx.step(truth, cfg.steps_per_cycle)
    y = tctx.observe(truth)[0].contiguous()
    yo = binding.synth_obs(y, cuda(inputs.observation_noise(cfg, cycle)),
                           cuda(inputs.sigma_vector(cfg)))
    return yo, tctx.moments(truth)[0, 1:].contiguous()


def _status(fn):
    try:
        fn()
    except binding.LbmLetkfError as e:
        return e.status, str(e)
    return 0, ""


@pytest.mark.parametrize("route", [binding.ROUTE_ENSEMBLE, binding.ROUTE_OBSERVATION])
def test_healthy_cycles_report_ok(route):
    say(f"checks: healthy tiny cycles route={route}")
    ctx, tctx, f, truth = _setup(TINY, route)
    ctx.set_checks(max_sweeps=30, diverge_limit=1.0, check_every_cycle=True)
    diag = torch.zeros(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
    for c in range(1, 4):
        yo, tuv = _obs(TINY, tctx, truth, c)
        ctx.run_cycle(f, TINY.steps_per_cycle, yo, tuv, diag)   # raises if unhealthy
    ctx.check(diag)


@pytest.mark.parametrize("route", [binding.ROUTE_ENSEMBLE, binding.ROUTE_OBSERVATION])
def test_nan_in_ensemble_gives_nonfinite_and_counts_eigensolves(route):
    say(f"checks: NaN member route={route}")
    ctx, tctx, f, truth = _setup(TINY, route)
    ctx.set_checks(check_every_cycle=True)
    # one population of member 3 at one node becomes NaN
    f[5, 7, 2, 3] = float("nan")
    yo, tuv = _obs(TINY, tctx, truth, 1)
    diag = torch.zeros(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
    st, msg = _status(lambda: ctx.run_cycle(f, TINY.steps_per_cycle, yo, tuv, diag))
    assert st == binding.LBMLETKF_ENONFINITE, msg
    # the NaN reached the observed node's perturbations, so eigensolves hit the cap
    assert "at the sweep cap" in msg and not msg.rstrip().endswith(" 0 node eigensolves at the sweep cap")
    d = host(diag)
    assert d[2] > 0 and d[binding.DIAG_LEN + 2] > 0


def test_nan_in_observations_gives_nonfinite_without_eigen_failure():
    say("checks: NaN observation")
    ctx, tctx, f, truth = _setup(TINY, binding.ROUTE_OBSERVATION)
    yo, tuv = _obs(TINY, tctx, truth, 1)
    yo[3] = float("nan")
    diag = torch.zeros(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
    # checks off by default: run_cycle returns OK and does not wait
    ctx.run_cycle(f, TINY.steps_per_cycle, yo, tuv, diag)
    st, msg = _status(lambda: ctx.check(diag))
    assert st == binding.LBMLETKF_ENONFINITE, msg
    d = host(diag)
    assert d[2] == 0 and d[binding.DIAG_LEN + 2] > 0     # forecast fine, analysis not
    assert "0 node eigensolves at the sweep cap" in msg   # y^o does not enter S


@pytest.mark.parametrize("route", [binding.ROUTE_ENSEMBLE, binding.ROUTE_OBSERVATION])
def test_sweep_cap_of_one_gives_eeig_and_counter_clears(route):
    say(f"checks: sweep cap 1 route={route}")
    ctx, tctx, f, truth = _setup(TINY, route)
    ctx.set_checks(max_sweeps=1)
    yo, tuv = _obs(TINY, tctx, truth, 1)
    ctx.run_cycle(f, TINY.steps_per_cycle, yo)
    st, msg = _status(lambda: ctx.check())
    assert st == binding.LBMLETKF_EEIG, msg
    assert "within 1 Jacobi sweeps" in msg
    # the check cleared the counter; with the default cap the next cycle is healthy
    ctx.set_checks(max_sweeps=30)
    yo, tuv = _obs(TINY, tctx, truth, 2)
    ctx.run_cycle(f, TINY.steps_per_cycle, yo)
    ctx.check()


def test_divergence_limit():
    """A limit below the analysis spread gives EDIVERGED; so does a run whose
    spread grows: four members, one observation point, inflation 1.5 per
    cycle, against a limit of four observation errors."""
    say("checks: divergence limit")
    ctx, tctx, f, truth = _setup(TINY)
    ctx.set_checks(diverge_limit=1e-9, check_every_cycle=True)
    yo, tuv = _obs(TINY, tctx, truth, 1)
    diag = torch.zeros(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
    st, msg = _status(lambda: ctx.run_cycle(f, TINY.steps_per_cycle, yo, tuv, diag))
    assert st == binding.LBMLETKF_EDIVERGED, msg
    cfg = TINY.replace(members=4, obs_side=1, beta=1.5)
    ctx, tctx, f, truth = _setup(cfg)
    limit = 4 * cfg.sigma
    ctx.set_checks(diverge_limit=limit, check_every_cycle=True)
    spreads = []
    status = 0
    for c in range(1, 41):
        yo, tuv = _obs(cfg, tctx, truth, c)
        status, msg = _status(lambda: ctx.run_cycle(f, cfg.steps_per_cycle, yo, tuv, diag))
        spreads.append(float(host(diag)[binding.DIAG_LEN + 1]))
        if status:
            break
    assert status == binding.LBMLETKF_EDIVERGED, (status, spreads)
    assert spreads[-1] > limit and spreads[0] < limit


def test_set_checks_validation():
    say("checks: argument validation")
    ctx = context(TINY)
    for bad in ((0, 0.0, 0), (101, 0.0, 0), (30, float("nan"), 0), (30, 0.0, 2)):
        st, _ = _status(lambda: binding._check(binding.load().lbmletkf_set_checks(
            ctx.handle, bad[0], bad[1], bad[2])))
        assert st == -1, bad


@pytest.mark.parametrize("cfg_name", ["paper", "precision"])
def test_nan_stays_inside_the_localization_of_its_observation(cfg_name):
    """A NaN in one member at an observed node reaches, through that
    observation's perturbation, only the nodes whose local observation set
    holds it (squared distance < (2 d_cut)^2, periodic, Sec. 3.2.2) and the
    node itself; every other node -- also those sharing a wavefront, a
    segment pass or a batch of LDS reads with an affected node in the eigen
    and apply kernels -- stays finite and keeps the clean run's analysis to
    rounding: a wavefront sweeps until all of its nodes converge, so a node
    beside a NaN node takes the sweep cap's further (vanishing) rotations."""
    cfg = inputs.CONFIGS[cfg_name]
    say(f"checks: NaN localization {cfg_name}")
    _, fe = config_state(cfg)
    ctx = context(cfg)
    pts = inputs.observation_points(cfg)
    x0, y0 = (int(v) for v in pts[len(pts) // 2])
    fe_nan = fe.copy()
    fe_nan[3, 0, y0, x0] = float("nan")        # rest population: stays at (x0, y0)
    outs, yo = [], None
    for canon in (fe, fe_nan):
        f = ctx.import_canonical(cuda(canon))
        yf = ctx.observe(f)
        if yo is None:                          # the same observations for both runs
            yo = (yf.mean(dim=0) + 1e-3).contiguous()
        ctx.analyze(f, yf, yo)
        outs.append(host(ctx.export_canonical(f)))
    clean, dirty = outs
    assert np.isfinite(clean).all()
    changed = ~(dirty == clean).all(axis=(0, 1))   # [y][x]
    dev = np.nan_to_num(np.abs(dirty - clean), nan=np.inf).max(axis=(0, 1))
    n = cfg.n
    ys, xs = np.mgrid[0:n, 0:n]
    dx = np.minimum(np.abs(xs - x0), n - np.abs(xs - x0))
    dy = np.minimum(np.abs(ys - y0), n - np.abs(ys - y0))
    inside = (dx * dx + dy * dy) < 4.0 * cfg.d_cut ** 2
    say(f"  changed nodes {int(changed.sum())}, inside the support {int(inside.sum())}")
    say(f"  outside: changed {int((changed & ~inside).sum())}, max |diff| {dev[~inside].max():.2e}")
    assert changed[y0, x0] and not np.isfinite(dirty[:, :, y0, x0]).all()
    assert np.isfinite(dirty[:, :, ~inside]).all()
    assert dev[~inside].max() <= 1e-14
