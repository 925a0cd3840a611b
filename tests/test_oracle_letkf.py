"""Pins of the oracle's LETKF (Sec. 3.2.1) and R-localization (Sec. 3.2.2)
against results fixed independently of its own code path: the exact Kalman
update on linear-Gaussian cases, the Sherman-Morrison closed form for one
observation, the empty-neighbourhood limit, a brute-force global ETKF in
observation space, and the smoothness the printed Gaspari-Cohn polynomial
must have."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_03972_amd import inputs


# ---------------------------------------------------------------------------
# Gaspari-Cohn (Sec. 3.2.2)
# ---------------------------------------------------------------------------
def _gc_branch_derivs(d, branch):
    """Value and first two derivatives of one branch, by central differences."""
    h = 1e-4

    def g(x):
        if branch == 1:
            return -0.25 * x**5 + 0.5 * x**4 + 0.625 * x**3 - 5 / 3 * x**2 + 1
        return x**5 / 12 - 0.5 * x**4 + 0.625 * x**3 + 5 / 3 * x**2 - 5 * x + 4 - 2 / (3 * x)

    return g(d), (g(d + h) - g(d - h)) / (2 * h), (g(d + h) - 2 * g(d) + g(d - h)) / h**2


def test_gaspari_cohn_anchor_values():
    """G(0) = 1, G = 0 for d >= 2 (the paper's reason to cut there), 0 <= G <= 1."""
    d = np.linspace(0, 3, 3001)
    g = oracle.gaspari_cohn(d)
    assert g[0] == 1.0
    assert np.all(g[d >= 2.0] == 0.0)
    assert np.all((g >= 0) & (g <= 1))
    assert np.all(np.diff(g[d <= 2.0]) <= 1e-15)   # monotone non-increasing


def test_gaspari_cohn_is_c2_at_the_knots():
    """The two printed pieces must join with matching value, slope and
    curvature at d = 1, and vanish to second order at d = 2 (Gaspari-Cohn's
    function is twice differentiable).  A typo in any coefficient breaks this."""
    v1, s1, c1 = _gc_branch_derivs(1.0, 1)
    v2, s2, c2 = _gc_branch_derivs(1.0, 2)
    assert v1 == pytest.approx(v2, abs=1e-12)
    assert s1 == pytest.approx(s2, abs=1e-7)
    assert c1 == pytest.approx(c2, abs=1e-5)
    v, s, c = _gc_branch_derivs(2.0, 2)
    assert abs(v) < 1e-12 and abs(s) < 1e-7 and abs(c) < 1e-5
    # the oracle evaluates the same pieces on each side of d = 1
    assert oracle.gaspari_cohn(np.array([1.0]))[0] == pytest.approx(v1, abs=1e-15)
    assert oracle.gaspari_cohn(np.array([1.5]))[0] == pytest.approx(
        _gc_branch_derivs(1.5, 2)[0], abs=1e-15)
    # slope zero at the origin (no linear term)
    assert _gc_branch_derivs(0.0, 1)[1] == pytest.approx(0.0, abs=1e-7)


def test_gaspari_cohn_is_nearly_gaussian():
    """The paper describes G as a close approximation of exp(-1.5 d^2)."""
    d = np.linspace(0, 2, 2001)
    dev = np.max(np.abs(oracle.gaspari_cohn(d) - np.exp(-1.5 * d * d)))
    assert dev < 0.025


def test_periodic_distance_brute_force():
    n = 7
    for x0 in range(n):
        for y0 in range(n):
            best = min(math.hypot(x0 - 3 + a * n, y0 - 5 + b * n)
                       for a in (-1, 0, 1) for b in (-1, 0, 1))
            assert oracle.periodic_distance(n, x0, y0, 3, 5) == pytest.approx(best, abs=1e-15)


# ---------------------------------------------------------------------------
# LETKF core (Sec. 3.2.1 with the inflation of Sec. 3.2.2)
# ---------------------------------------------------------------------------
def _linear_case(rng, n_state=6, M=7, n_obs=4):
    H = rng.standard_normal((n_obs, n_state))
    X = rng.standard_normal((n_state, M)) + 3.0
    sig = 0.3 + rng.random(n_obs)
    yo = H @ X.mean(axis=1) + sig * rng.standard_normal(n_obs)
    return H, X, sig, yo


@pytest.mark.parametrize("beta", [1.0, 1.05, 1.7])
def test_letkf_equals_kalman_update_linear_gaussian(beta):
    """For linear H the analysis mean and covariance equal the Kalman update
    with the inflated prior P^f = beta dX dX^T / (M-1)."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        H, X, sig, yo = _linear_case(rng)
        M = X.shape[1]
        Xa = oracle.letkf_core(X[None], H @ X, yo, (1 / sig**2)[None], beta)[0]
        xbar = X.mean(axis=1)
        dX = X - xbar[:, None]
        Pf = beta * dX @ dX.T / (M - 1)
        R = np.diag(sig**2)
        K = Pf @ H.T @ np.linalg.inv(H @ Pf @ H.T + R)
        xa_mean = xbar + K @ (yo - H @ xbar)
        Pa = (np.eye(len(xbar)) - K @ H) @ Pf
        np.testing.assert_allclose(Xa.mean(axis=1), xa_mean, rtol=1e-12, atol=1e-12)
        dXa = Xa - Xa.mean(axis=1)[:, None]
        np.testing.assert_allclose(dXa @ dXa.T / (M - 1), Pa, rtol=1e-10, atol=1e-12)


def test_single_observation_closed_form():
    """One observation: A = aI + s s^T (a = (M-1)/beta), so by Sherman-Morrison
    w_bar = s (sqrt(g) d / sigma) / (a + |s|^2) and
    dW = sqrt(beta) [I + (sqrt(a / (a + |s|^2)) - 1) s s^T / |s|^2]."""
    rng = np.random.default_rng(12)
    M, beta, sigma, g = 9, 1.2, 0.4, 0.37
    X = rng.standard_normal((9, M))
    yf = rng.standard_normal((1, M))
    yo = np.array([0.8])
    Xa = oracle.letkf_core(X[None], yf, yo, np.array([[g / sigma**2]]), beta)[0]
    a = (M - 1) / beta
    dy = yf[0] - yf[0].mean()
    s = math.sqrt(g) * dy / sigma
    d = yo[0] - yf[0].mean()
    wbar = s * math.sqrt(g) * d / (sigma * (a + s @ s))
    dW = math.sqrt(beta) * (np.eye(M) + (math.sqrt(a / (a + s @ s)) - 1) * np.outer(s, s) / (s @ s))
    xbar = X.mean(axis=1)
    ref = xbar[:, None] + (X - xbar[:, None]) @ (wbar[:, None] + dW)
    np.testing.assert_allclose(Xa, ref, rtol=1e-12, atol=1e-13)


def test_no_local_observation_inflates_only():
    """rinv = 0 (all observations beyond 2 d_cut): x^a = x_bar + sqrt(beta) dX."""
    rng = np.random.default_rng(13)
    X = rng.standard_normal((9, 5))
    Xa = oracle.letkf_core(X[None], rng.standard_normal((3, 5)), np.zeros(3),
                           np.zeros((1, 3)), 1.05)[0]
    xbar = X.mean(axis=1)[:, None]
    np.testing.assert_allclose(Xa, xbar + math.sqrt(1.05) * (X - xbar), rtol=1e-13, atol=1e-14)


def test_member_permutation_equivariance_and_mean():
    rng = np.random.default_rng(14)
    H, X, sig, yo = _linear_case(rng, M=8)
    rinv = (1 / sig**2)[None]
    Xa = oracle.letkf_core(X[None], H @ X, yo, rinv, 1.1)[0]
    perm = rng.permutation(8)
    Xp = oracle.letkf_core(X[None][:, :, perm], (H @ X)[:, perm], yo, rinv, 1.1)[0]
    np.testing.assert_allclose(Xp, Xa[:, perm], rtol=1e-12, atol=1e-12)
    # mean(x^a) = x_bar + dX w_bar, and the analysis perturbations sum to zero
    dXa = Xa - Xa.mean(axis=1)[:, None]
    np.testing.assert_allclose(dXa.sum(axis=1), 0, atol=1e-12)


# ---------------------------------------------------------------------------
# grid-level analysis
# ---------------------------------------------------------------------------
def _small_grid_problem(n=6, M=5, seed=15):
    rng = np.random.default_rng(seed)
    u = 0.03 * rng.standard_normal((M, n, n))
    v = 0.03 * rng.standard_normal((M, n, n))
    f = oracle.equilibrium(1 + 0.01 * rng.standard_normal((M, n, n)), u, v)
    f = f * (1 + 0.01 * rng.standard_normal(f.shape))
    pts = np.array([[0, 0], [3, 0], [0, 3], [3, 3]], dtype=np.int32)
    yf = oracle.observe(f, pts)
    yo = yf.mean(axis=0) + 0.01 * rng.standard_normal(yf.shape[1])
    return f, pts, yf, yo


def test_infinite_radius_is_global_etkf_in_observation_space():
    """d_cut = inf: every node sees every observation with weight 1, so the
    analysis is the global ETKF.  Its mean is checked against the Kalman-gain
    form solved in observation space, K = dX dY^T (dY dY^T + (M-1)/beta R)^-1,
    and its covariance against P^a = P^f - K P_yx."""
    f, pts, yf, yo = _small_grid_problem()
    M, _, n, _ = f.shape
    sig, beta = 0.01, 1.1
    fa = oracle.letkf_analysis(f, yf, yo, pts, (sig, sig), math.inf, beta)
    X = f.reshape(M, -1).T                        # global state, one column per member
    Xa = fa.reshape(M, -1).T
    dX = X - X.mean(axis=1)[:, None]
    Y = yf.T
    dY = Y - Y.mean(axis=1)[:, None]
    R = sig**2 * np.eye(len(yo))
    K = dX @ dY.T @ np.linalg.inv(dY @ dY.T + (M - 1) / beta * R)
    mean_ref = X.mean(axis=1) + K @ (yo - Y.mean(axis=1))
    np.testing.assert_allclose(Xa.mean(axis=1), mean_ref, rtol=1e-11, atol=1e-13)
    Pf = beta * dX @ dX.T / (M - 1)
    Pyx = beta * dY @ dX.T / (M - 1)
    dXa = Xa - Xa.mean(axis=1)[:, None]
    np.testing.assert_allclose(dXa @ dXa.T / (M - 1), Pf - K @ Pyx, rtol=1e-9, atol=1e-14)


def test_localized_analysis_matches_per_node_brute_force():
    """Each node uses only observations with G > 0, weighted by G / sigma^2.
    Checked against a loop that builds each node's local problem explicitly,
    keeping only the observations inside 2 d_cut, and solves it with the
    Kalman-gain form."""
    f, pts, yf, yo = _small_grid_problem(n=8, M=6, seed=16)
    pts = np.array([[1, 1], [5, 2], [2, 6]], dtype=np.int32)
    yf = oracle.observe(f, pts)
    yo = yf.mean(axis=0) + 0.01 * np.arange(len(yf[0]))
    M, _, n, _ = f.shape
    sig, beta, d_cut = 0.02, 1.05, 1.6
    fa = oracle.letkf_analysis(f, yf, yo, pts, (sig, sig), d_cut, beta)
    for node in range(n * n):
        x, y = node % n, node // n
        keep, wts = [], []
        for k, (px, py) in enumerate(pts):
            dist = oracle.periodic_distance(n, x, y, px, py)
            if dist < 2 * d_cut:
                g = float(oracle.gaspari_cohn(np.array([dist / d_cut]))[0])
                keep += [2 * k, 2 * k + 1]
                wts += [g, g]
        X = f[:, :, y, x].T
        xbar = X.mean(axis=1)
        dX = X - xbar[:, None]
        if not keep:
            ref = xbar[:, None] + math.sqrt(beta) * dX
        else:
            Y = yf[:, keep].T
            dY = Y - Y.mean(axis=1)[:, None]
            Rl = np.diag(sig**2 / np.asarray(wts))
            K = dX @ dY.T @ np.linalg.inv(dY @ dY.T + (M - 1) / beta * Rl)
            mean_ref = xbar + K @ (yo[keep] - Y.mean(axis=1))
            Xa = fa[:, :, y, x].T
            np.testing.assert_allclose(Xa.mean(axis=1), mean_ref, rtol=1e-11, atol=1e-13)
            continue
        np.testing.assert_allclose(fa[:, :, y, x].T, ref, rtol=1e-12, atol=1e-14)


def test_subset_of_nodes_matches_full_grid():
    f, pts, yf, yo = _small_grid_problem()
    full = oracle.letkf_analysis(f, yf, yo, pts, (0.01, 0.01), 2.0, 1.05)
    nodes = np.array([0, 7, 13, 35])
    sub = oracle.letkf_analysis(f, yf, yo, pts, (0.01, 0.01), 2.0, 1.05, nodes=nodes)
    M = f.shape[0]
    np.testing.assert_array_equal(sub, full.reshape(M, 9, -1)[:, :, nodes])


def test_observe_recovers_velocity_of_equilibrium():
    """H(f^eq(rho, u)) = u (and rho for nvar = 3)."""
    rng = np.random.default_rng(17)
    rho = 1 + 0.01 * rng.random((2, 4, 4))
    u = 0.05 * rng.standard_normal((2, 4, 4))
    v = 0.05 * rng.standard_normal((2, 4, 4))
    f = oracle.equilibrium(rho, u, v)
    pts = np.array([[1, 2], [3, 0]], dtype=np.int32)
    y = oracle.observe(f, pts)
    np.testing.assert_allclose(y[:, 0], u[:, 2, 1], rtol=1e-14)
    np.testing.assert_allclose(y[:, 1], v[:, 2, 1], rtol=1e-14)
    np.testing.assert_allclose(y[:, 2], u[:, 0, 3], rtol=1e-14)
    y3 = oracle.observe(f, pts, nvar=3)
    np.testing.assert_allclose(y3[:, 0], rho[:, 2, 1], rtol=1e-14)
    np.testing.assert_allclose(y3[:, 4], u[:, 0, 3], rtol=1e-14)


# ---------------------------------------------------------------------------
# diagnostics and inputs
# ---------------------------------------------------------------------------
def test_spectrum_parseval_and_single_mode():
    rng = np.random.default_rng(18)
    n = 16
    u, v = rng.standard_normal((2, n, n))
    E = oracle.energy_spectrum(u, v)
    assert E.sum() == pytest.approx(0.5 * np.mean(u * u + v * v), rel=1e-12)
    # a single Fourier mode at k = (3, 0) puts all energy in shell 3
    x = np.arange(n)
    uu = np.cos(2 * np.pi * 3 * x / n)[None, :].repeat(n, 0)
    E = oracle.energy_spectrum(uu, np.zeros_like(uu))
    assert E[3] == pytest.approx(0.25, rel=1e-12)
    assert E.sum() == pytest.approx(0.25, rel=1e-12)


def test_rmse_brute_force():
    rng = np.random.default_rng(19)
    f = oracle.equilibrium(np.ones((3, 4, 4)), 0.01 * rng.standard_normal((3, 4, 4)),
                           0.01 * rng.standard_normal((3, 4, 4)))
    t = oracle.equilibrium(np.ones((1, 4, 4)), 0.01 * rng.standard_normal((1, 4, 4)),
                           0.01 * rng.standard_normal((1, 4, 4)))
    mo, mt = oracle.moments(f), oracle.moments(t)
    acc = 0.0
    for j in range(16):
        y, x = divmod(j, 4)
        ub = sum(mo[1, m, y, x] for m in range(3)) / 3
        vb = sum(mo[2, m, y, x] for m in range(3)) / 3
        acc += (ub - mt[1, 0, y, x]) ** 2 + (vb - mt[2, 0, y, x]) ** 2
    assert oracle.rmse(f, t) == pytest.approx(math.sqrt(acc / 16), rel=1e-13)


def test_initial_field_spectrum_divergence_and_rms():
    cfg = inputs.CONFIGS["tiny"]
    truth, members = inputs.initial_velocities(cfg)
    n = cfg.n
    assert math.sqrt(np.mean(truth[0] ** 2 + truth[1] ** 2)) == pytest.approx(cfg.urms, rel=1e-12)
    pert = members - truth[None]
    for p in pert:
        assert math.sqrt(np.mean(p[0] ** 2 + p[1] ** 2)) == pytest.approx(
            cfg.member_amp * cfg.urms, rel=1e-12)
    # spectral divergence is zero
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    div = 1j * k1[None, :] * np.fft.fft2(truth[0]) + 1j * k1[:, None] * np.fft.fft2(truth[1])
    assert np.max(np.abs(div)) < 1e-12 * np.max(np.abs(np.fft.fft2(truth[0])))
    # shell spectrum proportional to k^4 exp(-(k/4)^2) / per-mode counts
    uh, vh = np.fft.fft2(truth[0]), np.fft.fft2(truth[1])
    kmag = np.hypot(k1[None, :], k1[:, None])
    shell = np.rint(kmag).astype(int)
    e = np.abs(uh) ** 2 + np.abs(vh) ** 2
    keep = (kmag > 0) & (np.abs(k1[None, :]) != n // 2) & (np.abs(k1[:, None]) != n // 2)
    Es = np.bincount(shell[keep], weights=e[keep])
    ks = np.arange(1, len(Es))
    target = ks.astype(float) ** 4 * np.exp(-(ks / 4.0) ** 2)
    ratio = Es[1:] / target
    np.testing.assert_allclose(ratio, ratio[0], rtol=1e-10)


def test_observation_layout_and_noise_are_reproducible():
    cfg = inputs.CONFIGS["paper"]
    pts = inputs.observation_points(cfg)
    assert pts.shape == (64, 2) and pts.max() == 224 and pts[1].tolist() == [32, 0]
    a = inputs.all_observation_noise(cfg, 3)
    b = inputs.all_observation_noise(cfg, 3)
    np.testing.assert_array_equal(a, b)
    assert a.shape == (3, 128)
    assert not np.allclose(a[0], a[1])


def test_shell_forcing_is_divergence_free_and_in_its_shell():
    """Sec. 4.1: F = dx grad(F_e) x i_z is solenoidal and has Fourier support
    only on ||k| - k_f| <= dk."""
    cfg = inputs.CONFIGS["paper_physics"].replace(n=64)
    F = inputs.body_force(cfg)
    n = cfg.n
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    Fx, Fy = np.fft.fft2(F[0]), np.fft.fft2(F[1])
    div = k1[None, :] * Fx + k1[:, None] * Fy
    assert np.max(np.abs(div)) < 1e-12 * np.max(np.abs(Fx))
    kmag = np.hypot(k1[None, :], k1[:, None])
    outside = np.abs(kmag - cfg.force_k) > cfg.shell_width
    power = np.abs(Fx) ** 2 + np.abs(Fy) ** 2
    assert power[outside].sum() < 1e-24 * power.sum()
    assert math.sqrt(np.mean(F[0] ** 2 + F[1] ** 2)) == pytest.approx(cfg.amplitude / math.sqrt(2),
                                                                      rel=1e-12)
    # deterministic from the seed
    np.testing.assert_array_equal(F, inputs.body_force(cfg))


def test_paper_physics_relaxation_time_from_table_1():
    """tau0 = 1/2 + 3 nu dt / dx^2 with nu = 1e-4, dt = 0.001232, dx = 2 pi / 256."""
    cfg = inputs.CONFIGS["paper_physics"]
    nu_lat = (cfg.tau0 - 0.5) / 3
    assert nu_lat == pytest.approx(1e-4 * 0.001232 / (2 * math.pi / 256) ** 2, rel=1e-12)
    assert cfg.d_cut == pytest.approx(256 / 8, rel=1e-12)
    assert cfg.nvar == 3 and cfg.cs == 0.2
