"""Pins of the oracle's misfit gradient (differentiation form).

The oracle takes every partial derivative by complex step and assembles the
reverse sweep by hand; these tests tie it to things outside itself: the C
oracle's forward step, central finite differences of the C oracle's misfit
(every entry on a tiny lattice), the complex-step derivative of the whole
misfit along random directions, the conservation laws that fix column sums of
the collision Jacobian, the finite propagation speed of the lattice, and the
affine dependence of the gradient on the observations.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint


def _state(rng, m, ny, nx, spin=3, tau0=0.56, cs=0.15):
    """A non-equilibrium state: a random-velocity equilibrium advanced a few steps."""
    rho = 1.0 + 0.02 * rng.standard_normal((m, ny, nx))
    u = 0.05 * rng.standard_normal((m, ny, nx))
    v = 0.05 * rng.standard_normal((m, ny, nx))
    f = oracle.equilibrium(rho, u, v)
    f = f + 1e-3 * rng.standard_normal(f.shape) * oracle.lattice()[2][None, :, None, None]
    return oracle.lbm_steps(f, spin, tau0, cs)


def _problem(rng, m, ny, nx, npts, nvar, n_times, s, tau0=0.56, cs=0.15, mu=2e-3):
    f0 = _state(rng, m, ny, nx)
    force = 1e-4 * rng.standard_normal((2, ny, nx))
    flat = rng.choice(nx * ny, size=npts, replace=False)
    pts = np.stack([flat % nx, flat // nx], axis=1)
    # observations near the forecast so the residuals are of a realistic size
    f = f0
    yo = []
    for _ in range(n_times):
        f = oracle.lbm_steps(f, s, tau0, cs, force, mu)
        y = oracle.observe(f, pts, nvar).mean(axis=0)
        yo.append(y + 0.01 * rng.standard_normal(y.shape))
    return dict(f0=f0, steps_per_obs=s, yo=np.array(yo), points=pts, nvar=nvar, tau0=tau0,
                cs=cs, force=force, mu=mu)


def _J(p, f0=None, cs=None):
    return adjoint.misfit(p["f0"] if f0 is None else f0, p["steps_per_obs"], p["yo"],
                          p["points"], p["nvar"], p["tau0"], p["cs"] if cs is None else cs,
                          p["force"], p["mu"])


def _grad(p):
    return adjoint.misfit_gradient(p["f0"], p["steps_per_obs"], p["yo"], p["points"],
                                   p["nvar"], p["tau0"], p["cs"], p["force"], p["mu"])


def test_numpy_collision_matches_c_oracle():
    rng = np.random.default_rng(11)
    f = _state(rng, 2, 10, 12)
    force = 1e-4 * rng.standard_normal((2, 10, 12))
    ref = oracle.lbm_steps(f, 4, 0.53, 0.17, force, 1e-3)
    g = f
    for _ in range(4):
        g = adjoint.step(g, 0.53, 0.17, force, 1e-3)
    assert np.max(np.abs(g - ref)) < 1e-15
    np.testing.assert_allclose(adjoint.observe_any(g, [[1, 2], [5, 7]], 3),
                               oracle.observe(g, [[1, 2], [5, 7]], 3), rtol=1e-14)


def test_collision_jacobian_column_sums_follow_conservation():
    """sum_a C_a = rho, so sum_a dC_a/df_b = 1; sum_a c_a C_a = j + rho F - mu j,
    so sum_a c_ax dC_a/df_b = c_bx (1 - mu) + F_x (any tau, any C_s)."""
    rng = np.random.default_rng(12)
    f = _state(rng, 2, 6, 7)
    force = 1e-3 * rng.standard_normal((2, 6, 7))
    mu = 0.03
    jac = adjoint.collision_jacobian(f, 0.51, 0.2, force, mu)
    cx, cy, _ = oracle.lattice()
    np.testing.assert_allclose(jac.sum(axis=1), 1.0, atol=1e-13)
    mx = np.einsum("a,mabyx->mbyx", cx.astype(float), jac)
    my = np.einsum("a,mabyx->mbyx", cy.astype(float), jac)
    ex = cx[None, :, None, None] * (1 - mu) + force[0][None, None]
    ey = cy[None, :, None, None] * (1 - mu) + force[1][None, None]
    np.testing.assert_allclose(mx, np.broadcast_to(ex, mx.shape), atol=1e-13)
    np.testing.assert_allclose(my, np.broadcast_to(ey, my.shape), atol=1e-13)
    # the relaxation does depend on C_s away from equilibrium
    assert np.max(np.abs(adjoint.collision_dcs(f, 0.51, 0.2, force, mu))) > 1e-8


@pytest.mark.parametrize("nvar", [2, 3])
def test_gradient_matches_central_differences_every_entry(nvar):
    """Tiny lattice (4 x 3, 2 members, 2 observation times of 2 steps): all 216
    entries of dJ/df0 and dJ/dC_s against central differences, h = 1e-6."""
    rng = np.random.default_rng(13 + nvar)
    p = _problem(rng, 2, 3, 4, npts=2, nvar=nvar, n_times=2, s=2)
    J, g, gcs = _grad(p)
    assert abs(J - _J(p)) <= 1e-14 * J
    h = 1e-6
    fd = np.empty_like(g)
    f0 = p["f0"]
    for idx in np.ndindex(f0.shape):
        fp = f0.copy()
        fm = f0.copy()
        fp[idx] += h
        fm[idx] -= h
        fd[idx] = (_J(p, f0=fp) - _J(p, f0=fm)) / (2 * h)
    scale = np.max(np.abs(g))
    assert scale > 1e-4
    assert np.max(np.abs(fd - g)) < 1e-7 * scale
    fdcs = (_J(p, cs=p["cs"] + h) - _J(p, cs=p["cs"] - h)) / (2 * h)
    assert abs(fdcs - gcs) < 1e-6 * abs(gcs)


@pytest.mark.parametrize("nvar", [2, 3])
def test_gradient_matches_complex_step_of_whole_misfit(nvar):
    """<dJ/df0, d> = Im J(f0 + i h d)/h along random directions d, and the same
    for C_s, with the complex forecast run end to end (16 x 12, 3 members)."""
    rng = np.random.default_rng(21 + nvar)
    p = _problem(rng, 3, 12, 16, npts=6, nvar=nvar, n_times=3, s=4)
    _, g, gcs = _grad(p)
    h = 1e-30
    for _ in range(2):
        d = rng.standard_normal(g.shape)
        Jc = adjoint.misfit_any(p["f0"] + 1j * h * d, p["steps_per_obs"], p["yo"], p["points"],
                                nvar, p["tau0"], p["cs"], p["force"], p["mu"])
        ref = Jc.imag / h
        assert abs(np.sum(g * d) - ref) < 1e-11 * np.sum(np.abs(g * d))
    Jc = adjoint.misfit_any(p["f0"].astype(np.complex128), p["steps_per_obs"], p["yo"],
                            p["points"], nvar, p["tau0"], p["cs"] + 1j * h, p["force"], p["mu"])
    assert abs(gcs - Jc.imag / h) < 1e-11 * abs(gcs)


def test_gradient_confined_to_the_light_cone():
    """After N steps one observation node sees f0 only within Chebyshev distance N."""
    rng = np.random.default_rng(31)
    p = _problem(rng, 1, 20, 20, npts=1, nvar=2, n_times=1, s=4)
    p["points"] = np.array([[9, 11]])
    _, g, _ = _grad(p)
    yy, xx = np.mgrid[0:20, 0:20]
    cheb = np.maximum(np.abs(xx - 9), np.abs(yy - 11))
    mag = np.abs(g[0]).max(axis=0)
    assert np.all(mag[cheb > 4] == 0.0)
    assert np.all(mag[cheb < 4] > 0.0)
    assert mag[cheb == 4].max() > 0.0


def test_gradient_is_affine_in_the_observations_and_zero_at_a_perfect_fit():
    rng = np.random.default_rng(41)
    p = _problem(rng, 2, 8, 8, npts=3, nvar=3, n_times=2, s=3)
    q = dict(p)
    q["yo"] = p["yo"] + 0.02 * rng.standard_normal(p["yo"].shape)
    r = dict(p)
    r["yo"] = 0.5 * (p["yo"] + q["yo"])
    _, g1, c1 = _grad(p)
    _, g2, c2 = _grad(q)
    _, gm, cm = _grad(r)
    np.testing.assert_allclose(g1 + g2, 2 * gm, atol=1e-12 * np.abs(g1).max())
    assert abs(c1 + c2 - 2 * cm) < 1e-10 * abs(c1)
    # observations equal to the member's own forecast: J = 0, gradient 0
    z = dict(p)
    z["f0"] = p["f0"][:1]
    f = z["f0"]
    yo = []
    for _ in range(2):
        f = oracle.lbm_steps(f, 3, p["tau0"], p["cs"], p["force"], p["mu"])
        yo.append(oracle.observe(f, p["points"], 3)[0])
    z["yo"] = np.array(yo)
    J, g, c = _grad(z)
    # zero up to the rounding of the two observation-operator evaluations
    assert J < 1e-30 and np.max(np.abs(g)) < 1e-14 and abs(c) < 1e-14
    assert np.max(np.abs(g1)) > 1e-3
