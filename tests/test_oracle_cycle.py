"""Pins of the oracle's cycle-level functions: the ensemble spread, the
member-mean spectrum and the forecast-analysis workflow of Sec. 3 (ii)-(v)
in ``run_cycles``.

Each pin is fixed independently of the function it checks: pure-Python loops
over nodes and members, closed forms (two members, the no-information limit of
the analysis), and the order of the workflow written out step by step.  Every
test also shows that a plausible slip -- a 1/M divisor, observing the truth
before it is advanced, taking the forecast RMSE after the analysis -- fails it.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2308_03972_amd import inputs


def _velocities_brute_force(f):
    """u, v of every member and node by explicit sums over the nine populations."""
    cx, cy, _ = oracle.lattice()
    M, _, ny, nx = f.shape
    u = np.zeros((M, ny, nx))
    v = np.zeros((M, ny, nx))
    for m in range(M):
        for y in range(ny):
            for x in range(nx):
                rho = sum(f[m, a, y, x] for a in range(9))
                u[m, y, x] = sum(cx[a] * f[m, a, y, x] for a in range(9)) / rho
                v[m, y, x] = sum(cy[a] * f[m, a, y, x] for a in range(9)) / rho
    return u, v


def _spread_brute_force(f, divisor):
    u, v = _velocities_brute_force(f)
    M, ny, nx = u.shape
    acc = 0.0
    for y in range(ny):
        for x in range(nx):
            ub = sum(u[m, y, x] for m in range(M)) / M
            vb = sum(v[m, y, x] for m in range(M)) / M
            acc += sum((u[m, y, x] - ub) ** 2 + (v[m, y, x] - vb) ** 2 for m in range(M)) / divisor
    return math.sqrt(acc / (nx * ny))


# ---------------------------------------------------------------------------
# spread: sqrt(N^-1 sum_xi (M-1)^-1 sum_m |u_m - u_bar|^2)
# ---------------------------------------------------------------------------
def test_spread_brute_force_and_two_member_closed_form():
    rng = np.random.default_rng(31)
    M, ny, nx = 3, 3, 4
    f = oracle.equilibrium(1.0 + 0.01 * rng.standard_normal((M, ny, nx)),
                           0.02 * rng.standard_normal((M, ny, nx)),
                           0.02 * rng.standard_normal((M, ny, nx)))
    f = f * (1.0 + 0.01 * rng.standard_normal(f.shape))   # off equilibrium
    ref = _spread_brute_force(f, M - 1)
    assert oracle.spread(f) == pytest.approx(ref, rel=1e-13)
    # the slip 1/M instead of 1/(M-1) is sqrt(2/3) away and fails the pin
    assert abs(_spread_brute_force(f, M) / ref - 1) > 0.1
    # two members: (M-1)^-1 sum_m |u_m - u_bar|^2 = |u_1 - u_2|^2 / 2
    u = 0.02 * rng.standard_normal((2, ny, nx))
    v = 0.02 * rng.standard_normal((2, ny, nx))
    f2 = oracle.equilibrium(np.ones((2, ny, nx)), u, v)
    uu, vv = _velocities_brute_force(f2)
    closed = math.sqrt(np.mean(((uu[0] - uu[1]) ** 2 + (vv[0] - vv[1]) ** 2) / 2))
    assert oracle.spread(f2) == pytest.approx(closed, rel=1e-13)


# ---------------------------------------------------------------------------
# member-mean spectrum (Sec. 4.3.2)
# ---------------------------------------------------------------------------
def test_member_mean_spectrum_single_modes_and_parseval():
    n = 16
    x = np.arange(n)
    # member 0: u = cos(2 pi 3 x / n) (shell 3, energy 1/4); member 1: v = cos(2 pi 5 y / n)
    u0 = np.cos(2 * np.pi * 3 * x / n)[None, :].repeat(n, 0)
    v1 = np.cos(2 * np.pi * 5 * x / n)[:, None].repeat(n, 1)
    zero = np.zeros((n, n))
    f = oracle.equilibrium(np.ones((2, n, n)), np.stack([0.01 * u0, zero]),
                           np.stack([zero, 0.01 * v1]))
    E = oracle.member_mean_spectrum(f)
    # each mode carries (0.01)^2 / 4 in its own member; the mean halves it
    assert E[3] == pytest.approx(0.25e-4 / 2, rel=1e-9)
    assert E[5] == pytest.approx(0.25e-4 / 2, rel=1e-9)
    assert E.sum() == pytest.approx(0.25e-4, rel=1e-9)
    # Parseval: summed over shells, half the mean squared speed, averaged over members
    rng = np.random.default_rng(32)
    g = oracle.equilibrium(np.ones((3, n, n)), 0.02 * rng.standard_normal((3, n, n)),
                           0.02 * rng.standard_normal((3, n, n)))
    uu, vv = _velocities_brute_force(g)
    assert oracle.member_mean_spectrum(g).sum() == pytest.approx(
        0.5 * np.mean(uu * uu + vv * vv), rel=1e-12)


# ---------------------------------------------------------------------------
# run_cycles: the workflow of Sec. 3, written out step by step
# ---------------------------------------------------------------------------
SMALL = inputs.CONFIGS["tiny"].replace(name="small16", n=16, members=4, obs_side=4, loc_r=3.0,
                                       steps_per_cycle=3, cycles=2)


def _small_start():
    truth_uv, mem_uv = inputs.initial_velocities(SMALL)
    ft = oracle.equilibrium(np.ones((1, SMALL.n, SMALL.n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((SMALL.members, SMALL.n, SMALL.n)), mem_uv[:, 0],
                            mem_uv[:, 1])
    return ft, fe


def test_run_cycles_follows_the_workflow_order():
    cfg = SMALL
    ft0, fe0 = _small_start()
    force = inputs.body_force(cfg)
    pts = inputs.observation_points(cfg)
    noise = inputs.all_observation_noise(cfg, 2)
    sig = inputs.sigma_vector(cfg)
    s = cfg.steps_per_cycle
    out = oracle.run_cycles(fe0, ft0, cfg, force, pts, noise, 2, keep_states=True)

    # truth at the analysis times: advanced c * s steps (one call each), then observed
    t1 = oracle.lbm_steps(ft0, s, cfg.tau0, cfg.cs, force)
    t2 = oracle.lbm_steps(ft0, 2 * s, cfg.tau0, cfg.cs, force)
    np.testing.assert_array_equal(out["yo"][0], oracle.observe(t1, pts)[0] + sig * noise[0])
    np.testing.assert_allclose(out["yo"][1], oracle.observe(t2, pts)[0] + sig * noise[1],
                               rtol=0, atol=1e-15)
    # the slip "observe, then advance the truth" gives other observations
    stale = oracle.observe(ft0, pts)[0] + sig * noise[0]
    assert np.max(np.abs(stale - out["yo"][0])) > 10 * cfg.sigma * 1e-3

    # cycle 1: forecast, its RMSE and spread, analysis, its RMSE and spread
    f1 = oracle.lbm_steps(fe0, s, cfg.tau0, cfg.cs, force)
    yo1 = oracle.observe(t1, pts)[0] + sig * noise[0]
    a1 = oracle.letkf_analysis(f1, oracle.observe(f1, pts), yo1, pts, cfg.sigmas, cfg.d_cut,
                               cfg.beta)
    assert out["rmse_f"][0] == oracle.rmse(f1, t1)
    assert out["spread_f"][0] == oracle.spread(f1)
    np.testing.assert_array_equal(out["states"][0], a1)
    assert out["rmse_a"][0] == oracle.rmse(a1, t1)
    assert out["spread_a"][0] == oracle.spread(a1)
    # cycle 2 starts from the analysis of cycle 1
    f2 = oracle.lbm_steps(a1, s, cfg.tau0, cfg.cs, force)
    yo2 = out["yo"][1]
    a2 = oracle.letkf_analysis(f2, oracle.observe(f2, pts), yo2, pts, cfg.sigmas, cfg.d_cut,
                               cfg.beta)
    assert out["rmse_f"][1] == pytest.approx(oracle.rmse(f2, t2), rel=1e-14)
    assert out["rmse_a"][1] == pytest.approx(oracle.rmse(a2, t2), rel=1e-14)
    np.testing.assert_allclose(out["f_ens"], a2, rtol=0, atol=1e-15)
    # the slips "RMSE_f after the analysis" and "RMSE_a before it" are detectable:
    # the analysis moves the mean by much more than the comparison's rounding
    assert abs(oracle.rmse(a1, t1) / out["rmse_f"][0] - 1) > 1e-6
    assert abs(oracle.rmse(f1, t1) / out["rmse_a"][0] - 1) > 1e-6


def test_run_cycles_uninformative_observations_inflate_only():
    """With observation errors so large that the observations carry no weight,
    the LETKF keeps the mean populations and multiplies their perturbations
    by sqrt(beta) (w_bar -> 0, dW -> sqrt(beta) I), so RMSE_a = RMSE_f and
    spread_a = sqrt(beta) spread_f each cycle, up to the second-order change
    that u = j / rho (nonlinear in the populations) brings (~1e-6 relative
    here).  Fails if spread_a were taken before the analysis, or spread_f
    after it."""
    cfg = SMALL.replace(sigma_uv=1e7, beta=1.21)
    ft0, fe0 = _small_start()
    out = oracle.run_cycles(fe0, ft0, cfg, inputs.body_force(cfg), inputs.observation_points(cfg),
                            inputs.all_observation_noise(cfg, 2), 2)
    np.testing.assert_allclose(out["rmse_a"], out["rmse_f"], rtol=1e-4)
    np.testing.assert_allclose(out["spread_a"], math.sqrt(1.21) * out["spread_f"], rtol=1e-4)
    assert np.all(np.abs(out["spread_a"] / out["spread_f"] - 1) > 0.09)


def test_tiny_run_rmse_settles_below_the_observation_noise():
    """The paper's qualitative check (Sec. 4.3.2): with the LETKF the analysis
    error settles below the observation noise sqrt(2) sigma (the rms error of
    an observed velocity vector); tiny configuration, all 20 cycles, time
    average over the second half.  The run must also stay finite with a
    spread of the same order as the error (no collapse, no divergence)."""
    cfg = inputs.CONFIGS["tiny"]
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    ft = oracle.equilibrium(np.ones((1, cfg.n, cfg.n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((cfg.members, cfg.n, cfg.n)), mem_uv[:, 0], mem_uv[:, 1])
    out = oracle.run_cycles(fe, ft, cfg, inputs.body_force(cfg), inputs.observation_points(cfg),
                            inputs.all_observation_noise(cfg, cfg.cycles), cfg.cycles,
                            report_every=10)
    ra = out["rmse_a"]
    assert np.all(np.isfinite(ra)) and np.all(np.isfinite(out["spread_a"]))
    assert ra[cfg.cycles // 2:].mean() < math.sqrt(2.0) * cfg.sigma
    ratio = out["spread_a"][cfg.cycles // 2:] / ra[cfg.cycles // 2:]
    assert np.all((ratio > 0.2) & (ratio < 5.0))
    # spectra at the report cycles: the analysis keeps the energy-containing
    # range of the truth's spectrum (shells 1..8 within a factor of two)
    assert list(out["report_cycle"]) == [10, 20]
    for Ea, Et in zip(out["spectrum_a"], out["spectrum_t"]):
        k = np.arange(1, 9)
        assert np.all(np.abs(np.log(Ea[k] / Et[k])) < math.log(2.0))
