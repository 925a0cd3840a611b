"""Pins of the oracle's lattice-Boltzmann step (Sec. 2) against facts the
paper and the mathematics fix: lattice moment identities, conservation laws,
symmetries, the Smagorinsky relation solved by a different method, and the
Taylor-Green vortex decay against its closed form."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_03972_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _random_state(rng, m, n, amp=0.03):
    u = amp * rng.standard_normal((m, n, n))
    v = amp * rng.standard_normal((m, n, n))
    rho = 1.0 + 0.01 * rng.standard_normal((m, n, n))
    f = oracle.equilibrium(rho, u, v)
    # add a non-equilibrium part so that the Smagorinsky term is active
    return f * (1.0 + 0.02 * rng.standard_normal(f.shape))


def test_lattice_moments_are_exact():
    """Sec. 2 velocity set and weights: sum w = 1, sum w c = 0, sum w c c = I/3."""
    cx, cy, w = oracle.lattice()
    assert w.sum() == pytest.approx(1.0, abs=1e-16)
    assert abs((w * cx).sum()) < 1e-16 and abs((w * cy).sum()) < 1e-16
    assert (w * cx * cx).sum() == pytest.approx(1 / 3, abs=1e-16)
    assert (w * cy * cy).sum() == pytest.approx(1 / 3, abs=1e-16)
    assert abs((w * cx * cy).sum()) < 1e-16
    # the set of Sec. 2: rest, 4 axis (speed 1), 4 diagonal (speed sqrt 2)
    speeds = sorted(cx * cx + cy * cy)
    assert speeds == [0, 1, 1, 1, 1, 2, 2, 2, 2]
    assert set(zip(cx.tolist(), cy.tolist())) == {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1),
                                                  (1, 1), (-1, -1), (1, -1), (-1, 1)}


def test_equilibrium_moments():
    """f^eq has density rho, momentum rho u and momentum flux rho/3 I + rho u u."""
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.random((1, 4, 5))
    u = 0.1 * rng.standard_normal((1, 4, 5))
    v = 0.1 * rng.standard_normal((1, 4, 5))
    f = oracle.equilibrium(rho, u, v)[0]
    cx, cy, _ = oracle.lattice()
    sx = np.einsum("ayx,a->yx", f, cx * 1.0)
    sy = np.einsum("ayx,a->yx", f, cy * 1.0)
    np.testing.assert_allclose(f.sum(0), rho[0], rtol=1e-15)
    np.testing.assert_allclose(sx, rho[0] * u[0], atol=1e-16)
    np.testing.assert_allclose(sy, rho[0] * v[0], atol=1e-16)
    pxx = np.einsum("ayx,a->yx", f, cx * cx * 1.0)
    pxy = np.einsum("ayx,a->yx", f, cx * cy * 1.0)
    np.testing.assert_allclose(pxx, rho[0] / 3 + rho[0] * u[0] ** 2, atol=1e-15)
    np.testing.assert_allclose(pxy, rho[0] * u[0] * v[0], atol=1e-16)
    # moments() inverts it
    mo = oracle.moments(f[None])
    np.testing.assert_allclose(mo[1, 0], u[0], atol=1e-15)
    np.testing.assert_allclose(mo[2, 0], v[0], atol=1e-15)


def test_mass_and_momentum_conserved_without_force():
    """Collision conserves mass and momentum; streaming permutes populations.
    Over 1000 steps the drift stays at the round-off level (<= 1e-15 per step)."""
    rng = np.random.default_rng(2)
    f = _random_state(rng, 2, 12)
    cx, cy, _ = oracle.lattice()
    g = oracle.lbm_steps(f, 1000, 0.52, 0.1)
    mass0, mass1 = f.sum(), g.sum()
    px0 = np.einsum("maij,a->", f, cx * 1.0)
    px1 = np.einsum("maij,a->", g, cx * 1.0)
    py0 = np.einsum("maij,a->", f, cy * 1.0)
    py1 = np.einsum("maij,a->", g, cy * 1.0)
    assert abs(mass1 - mass0) / mass0 < 1e-12
    scale = np.einsum("maij->", np.abs(f))
    assert abs(px1 - px0) / scale < 1e-12
    assert abs(py1 - py0) / scale < 1e-12


def test_force_adds_rho_F_per_step():
    """sum_a F_a = 0 and sum_a F_a c_a = rho F: momentum grows by sum rho F each step."""
    rng = np.random.default_rng(3)
    n = 10
    f = _random_state(rng, 1, n)
    force = 1e-4 * rng.standard_normal((2, n, n))
    cx, cy, _ = oracle.lattice()
    rho = oracle.moments(f)[0, 0]
    g = oracle.lbm_steps(f, 1, 0.6, 0.1, force)
    dpx = np.einsum("maij,a->", g - f, cx * 1.0)
    dpy = np.einsum("maij,a->", g - f, cy * 1.0)
    assert dpx == pytest.approx((rho * force[0]).sum(), rel=1e-11, abs=1e-17)
    assert dpy == pytest.approx((rho * force[1]).sum(), rel=1e-11, abs=1e-17)
    assert abs(g.sum() - f.sum()) / f.sum() < 1e-15


def test_friction_decelerates_uniform_flow_exactly():
    """With F = -mu u on a uniform flow, u(t+1) = u(t) (1 - mu) exactly (no gradients)."""
    n, mu = 6, 0.01
    u0 = 0.02
    f = oracle.equilibrium(np.ones((1, n, n)), np.full((1, n, n), u0), np.zeros((1, n, n)))
    g = oracle.lbm_steps(f, 1, 0.7, 0.1, None, mu)
    mo = oracle.moments(g)
    np.testing.assert_allclose(mo[1], u0 * (1 - mu), rtol=1e-13)


def test_uniform_flow_is_stationary():
    """A uniform equilibrium has Pi^neq = 0, so tau = tau0 and nothing changes."""
    n = 8
    f = oracle.equilibrium(np.full((1, n, n), 1.02), np.full((1, n, n), 0.04),
                           np.full((1, n, n), -0.03))
    g = oracle.lbm_steps(f, 50, 0.52, 0.2)
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-15)


def test_translation_and_rotation_equivariance():
    rng = np.random.default_rng(4)
    n = 8
    f = _random_state(rng, 1, n)
    g = oracle.lbm_steps(f, 5, 0.55, 0.15)
    # translation by one cell in x and two in y
    ft = np.roll(f, (2, 1), axis=(2, 3))
    gt = oracle.lbm_steps(ft, 5, 0.55, 0.15)
    np.testing.assert_allclose(gt, np.roll(g, (2, 1), axis=(2, 3)), atol=1e-15)
    # rotation by 90 degrees: (x, y) -> (-y, x) maps velocity a to rot[a]
    cx, cy, _ = oracle.lattice()
    rot = [int(np.where((cx == -cy[a]) & (cy == cx[a]))[0][0]) for a in range(9)]

    def rotate(h):
        # new[y'][x'] with x' = -y, y' = x  (indices mod n)
        out = np.empty_like(h)
        for a in range(9):
            plane = h[:, a]
            # new(x', y') = old(x = y', y = -x')
            yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
            out[:, rot[a]] = plane[:, (-xx) % n, yy]
        return out

    gr = oracle.lbm_steps(rotate(f), 5, 0.55, 0.15)
    np.testing.assert_allclose(gr, rotate(g), atol=1e-15)


def test_smagorinsky_tau_solves_its_defining_relation():
    """tau from the closed form satisfies nu + nu_SGS = (tau - 1/2)/3 with
    nu_SGS = C_s^2 |S| and S_ij = -Pi_ij / (2 rho c_s^2 tau), found here by a
    fixed-point iteration instead of the quadratic's root."""
    rng = np.random.default_rng(5)
    cx, cy, w = oracle.lattice()
    for trial in range(20):
        rho = 1 + 0.05 * rng.standard_normal()
        u, v = 0.05 * rng.standard_normal(2)
        feq = rho * w * (1 + 3 * (cx * u + cy * v) + 4.5 * (cx * u + cy * v) ** 2
                         - 1.5 * (u * u + v * v))
        f9 = feq + 1e-3 * rng.standard_normal(9) * w
        # make the perturbation conserve mass and momentum so Pi is the only change
        f9 = f9 - w * (f9 - feq).sum()
        tau0, cs = 0.5 + 0.3 * rng.random() + 0.01, 0.3 * rng.random()
        tau = oracle.relaxation_time(f9, tau0, cs)
        r = f9.sum()
        ux, uy = (f9 * cx).sum() / r, (f9 * cy).sum() / r
        fe = r * w * (1 + 3 * (cx * ux + cy * uy) + 4.5 * (cx * ux + cy * uy) ** 2
                      - 1.5 * (ux * ux + uy * uy))
        pi = np.array([[((f9 - fe) * cx * cx).sum(), ((f9 - fe) * cx * cy).sum()],
                       [((f9 - fe) * cx * cy).sum(), ((f9 - fe) * cy * cy).sum()]])
        nu0 = (tau0 - 0.5) / 3
        t = tau0
        for _ in range(200):
            S = -pi / (2 * r * t / 3)
            absS = math.sqrt(2 * (S * S).sum())
            t = 0.5 + 3 * (nu0 + cs * cs * absS)
        assert tau == pytest.approx(t, rel=1e-13)
        assert tau >= tau0


def test_cs_zero_is_plain_bgk():
    """C_s = 0 gives tau = tau0 at every node."""
    rng = np.random.default_rng(6)
    f = _random_state(rng, 1, 4)
    for i in range(16):
        f9 = f[0, :, i // 4, i % 4]
        assert oracle.relaxation_time(f9, 0.61, 0.0) == 0.61


def test_brute_force_single_step_tiny_grid():
    """One step on a 3x4 grid against a pure-Python collide-then-stream loop
    that takes tau by fixed-point iteration of the Smagorinsky relation."""
    rng = np.random.default_rng(7)
    nx, ny = 4, 3
    f = np.abs(_random_state(rng, 1, 4)[:, :, :ny, :nx])
    force = 1e-3 * rng.standard_normal((2, ny, nx))
    tau0, cs, mu = 0.57, 0.18, 0.003
    cx, cy, w = oracle.lattice()
    ref = np.zeros_like(f)
    for y in range(ny):
        for x in range(nx):
            f9 = f[0, :, y, x]
            r = f9.sum()
            ux, uy = (f9 * cx).sum() / r, (f9 * cy).sum() / r
            cu = cx * ux + cy * uy
            fe = r * w * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
            pxx, pyy, pxy = (((f9 - fe) * cx * cx).sum(), ((f9 - fe) * cy * cy).sum(),
                             ((f9 - fe) * cx * cy).sum())
            t = tau0
            for _ in range(300):
                absS = 3 / (2 * r * t) * math.sqrt(2 * (pxx * pxx + pyy * pyy + 2 * pxy * pxy))
                t = tau0 + 3 * cs * cs * absS
            Fx, Fy = force[0, y, x] - mu * ux, force[1, y, x] - mu * uy
            for a in range(9):
                fs = f9[a] - (f9[a] - fe[a]) / t + 3 * w[a] * r * (Fx * cx[a] + Fy * cy[a])
                ref[0, a, (y + cy[a]) % ny, (x + cx[a]) % nx] = fs
    got = oracle.lbm_steps(f, 1, tau0, cs, force, mu)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-16)


def _taylor_green_rate_error(n, tau0=0.8, u0=0.01, frac=0.5):
    k = 2 * np.pi / n
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    u = -u0 * np.cos(k * X) * np.sin(k * Y)
    v = u0 * np.sin(k * X) * np.cos(k * Y)
    p = -(u0 ** 2 / 4) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    f = oracle.equilibrium(1 + 3 * p, u, v)
    nu = (tau0 - 0.5) / 3
    steps = int(round(frac / (2 * nu * k * k)))
    basis = np.sin(k * X) * np.cos(k * Y)

    def amp(h):
        return (oracle.moments(h)[2, 0] * basis).sum() / (basis * basis).sum()

    t1 = steps // 2
    f1 = oracle.lbm_steps(f, t1, tau0, 0.0)
    f2 = oracle.lbm_steps(f1, steps - t1, tau0, 0.0)
    rate = math.log(amp(f1) / amp(f2)) / (steps - t1)
    return rate / (2 * nu * k * k) - 1.0


def test_taylor_green_decay_second_order():
    """Amplitude decays as exp(-2 nu k^2 t), nu = (tau0 - 1/2)/3 (viscosity-tau
    relation of Sec. 2); the error in the rate falls ~4x per grid doubling."""
    errs = [abs(_taylor_green_rate_error(n)) for n in (16, 32, 64)]
    assert errs[1] < 2e-3 and errs[2] < 5e-4
    order1 = math.log2(errs[0] / errs[1])
    order2 = math.log2(errs[1] / errs[2])
    assert 1.7 < order1 < 2.5 and 1.7 < order2 < 2.5


def test_kolmogorov_forcing_drives_its_laminar_profile():
    """At low Reynolds number the sinusoidal force's steady flow is
    u = A/(nu k^2) sin(k y); the configured amplitude gives rms urms."""
    cfg = inputs.CycleConfig(name="t", n=16, members=1, tau0=1.0, cs=0.0, obs_side=2,
                             loc_r=2.0, steps_per_cycle=1, cycles=1, force_k=1)
    force = inputs.body_force(cfg)
    f = oracle.equilibrium(np.ones((1, 16, 16)), np.zeros((1, 16, 16)), np.zeros((1, 16, 16)))
    f = oracle.lbm_steps(f, 3000, cfg.tau0, 0.0, force)
    u = oracle.moments(f)[1, 0]
    rms = math.sqrt(np.mean(u * u))
    assert rms == pytest.approx(cfg.urms, rel=3e-2)


def test_lattice_matches_printed_table():
    """Weights and speed classes against the fixture transcribed from Sec. 2."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "d2q9_sec2.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    cx, cy, w = oracle.lattice()
    assert len(rows) == 9
    for a, c2, wt in rows:
        a = int(a)
        assert cx[a] ** 2 + cy[a] ** 2 == int(c2)
        assert w[a] == float(Fraction(wt))
    # opposite pairs adjacent: c_{2j-1} = -c_{2j}
    for j in (1, 3, 5, 7):
        assert (cx[j], cy[j]) == (-cx[j + 1], -cy[j + 1])
