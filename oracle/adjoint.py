"""FP64 oracle of the differentiation form -- TEST INFRASTRUCTURE ONLY.

The gradient of the observation misfit of an ensemble LBM forecast,

    J(f0, C_s) = sum_{c=1..C} sum_m sum_q (H_q(f_m(c s)) - y^o_{c,q})^2,

with respect to the initial populations f0 = f(t=0) (every member) and the
Smagorinsky constant C_s.  f(t) is the pre-collision state after t steps of
the LBE of Sec. 2 (BGK relaxation with the Smagorinsky relaxation time, force
term with the external field and friction), H the observation operator of
Sec. 3 ((u, v) or (rho, u, v) at the observation nodes), s the number of steps
between observation times.  Like the rest of the oracle it is only for the
tests, the smoke check and the benchmark's CPU leg, and shares no code with
the GPU library.

Method (reverse mode written out, nothing hand-differentiated):
one step is f^{n+1}_a(x + c_a) = C_a(f^n(x)), C the per-node collision, so
the adjoint lam^n = dJ/df^n obeys

    lam^n_b(x) = sum_a lam^{n+1}_a(x + c_a) dC_a/df_b(f^n(x)) + dJ_n/df^n_b(x),

J_n the misfit term at step n (zero unless n is an observation time), and
dJ/dC_s = sum_n sum_x sum_a lam^{n+1}_a(x + c_a) dC_a/dC_s(f^n(x)).
Every partial derivative (the 9 x 9 collision Jacobian at each node, dC/dC_s
and dJ_n/df) is taken by the complex-step derivative of Squire and Trapp
(SIAM Review 40, 1998): d g(x)/dx = Im g(x + i h)/h with h = 1e-30, exact to
rounding for an analytic g.  The collision is written below with analytic
operations only (no abs, no branches on the state), so it can be evaluated at
complex arguments.  At |Pi| = 0 the complex step returns 0 for the
derivative of |Pi|: the subgradient 0.

The forward trajectory comes from the C oracle step (``oracle.lbm_steps``);
``collide`` below is the same Sec. 2 collision in NumPy, pinned to it.
"""
from __future__ import annotations

import numpy as np

from . import lbm_steps as _c_steps
from . import lattice as _lattice

_H = 1e-30


def _lat():
    cx, cy, w = _lattice()
    return cx, cy, w


def collide(f, tau0, cs, force=None, mu: float = 0.0):
    """Post-collision populations C(f) of every node (Sec. 2), any float or complex dtype.

    f [M][9][ny][nx] pre-collision; force [2][ny][nx] or None.
    """
    cx, cy, w = _lat()
    cxf = cx.astype(np.float64)[None, :, None, None]
    cyf = cy.astype(np.float64)[None, :, None, None]
    wf = w[None, :, None, None]
    rho = f.sum(axis=1, keepdims=True)
    u = (cxf * f).sum(axis=1, keepdims=True) / rho
    v = (cyf * f).sum(axis=1, keepdims=True) / rho
    cu = cxf * u + cyf * v
    feq = rho * wf * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u * u + v * v))
    fneq = f - feq
    pxx = (cxf * cxf * fneq).sum(axis=1, keepdims=True)
    pyy = (cyf * cyf * fneq).sum(axis=1, keepdims=True)
    pxy = (cxf * cyf * fneq).sum(axis=1, keepdims=True)
    pnorm = np.sqrt(pxx * pxx + pyy * pyy + 2.0 * pxy * pxy)
    tau = 0.5 * (tau0 + np.sqrt(tau0 * tau0 + 18.0 * np.sqrt(2.0) * cs * cs * pnorm / rho))
    gx = -mu * u
    gy = -mu * v
    if force is not None:
        gx = gx + np.asarray(force)[0][None, None]
        gy = gy + np.asarray(force)[1][None, None]
    Fa = 3.0 * wf * rho * (cxf * gx + cyf * gy)
    return f - fneq / tau + Fa


def stream(f):
    """Push streaming: out_a(x + c_a) = f_a(x), doubly periodic."""
    cx, cy, _ = _lat()
    out = np.empty_like(f)
    for a in range(9):
        out[:, a] = np.roll(f[:, a], shift=(cy[a], cx[a]), axis=(-2, -1))
    return out


def step(f, tau0, cs, force=None, mu: float = 0.0):
    return stream(collide(f, tau0, cs, force, mu))


def observe_any(f, points, nvar: int):
    """H(f) of every member, [M][n_points * nvar], any dtype (Sec. 3)."""
    cx, cy, _ = _lat()
    pts = np.asarray(points)
    fo = f[:, :, pts[:, 1], pts[:, 0]]                       # [M][9][K]
    rho = fo.sum(axis=1)
    u = (cx.astype(np.float64)[None, :, None] * fo).sum(axis=1) / rho
    v = (cy.astype(np.float64)[None, :, None] * fo).sum(axis=1) / rho
    cols = [u, v] if nvar == 2 else [rho, u, v]
    return np.stack(cols, axis=-1).reshape(f.shape[0], -1)


def _residual_terms(f, points, nvar, yo_c):
    """[M][K]: sum over the variables of point k of (H - y^o)^2."""
    r = observe_any(f, points, nvar) - np.asarray(yo_c)[None, :]
    return (r * r).reshape(f.shape[0], len(points), nvar).sum(axis=-1)


def misfit(f0, steps_per_obs: int, yo, points, nvar: int, tau0, cs, force=None,
           mu: float = 0.0) -> float:
    """J with the C oracle forecast; yo [C][n_points * nvar]."""
    f = np.array(f0, dtype=np.float64)
    J = 0.0
    for yo_c in np.asarray(yo):
        f = _c_steps(f, steps_per_obs, tau0, cs, force, mu)
        J += float(_residual_terms(f, points, nvar, yo_c).sum())
    return J


def misfit_any(f0, steps_per_obs: int, yo, points, nvar: int, tau0, cs, force=None,
               mu: float = 0.0):
    """J with the NumPy forecast, for complex arguments (complex-step checks)."""
    f = np.array(f0)
    J = 0.0
    for yo_c in np.asarray(yo):
        for _ in range(steps_per_obs):
            f = step(f, tau0, cs, force, mu)
        J = J + _residual_terms(f, points, nvar, yo_c).sum()
    return J


def _misfit_state_gradient(f, points, nvar, yo_c):
    """dJ_n/df of one observation time, [M][9][ny][nx] (nonzero at observation nodes)."""
    pts = np.asarray(points)
    g = np.zeros(f.shape)
    for b in range(9):
        fc = f.astype(np.complex128)
        # one complex step on f_b of every observation node; each term R[m, k]
        # depends on the populations of node k only
        fc[:, b, pts[:, 1], pts[:, 0]] = f[:, b, pts[:, 1], pts[:, 0]] + 1j * _H
        dR = _residual_terms(fc, points, nvar, yo_c).imag / _H        # [M][K]
        gb = np.zeros(f.shape[:1] + f.shape[2:])
        for k in range(len(pts)):
            gb[:, pts[k, 1], pts[k, 0]] += dR[:, k]
        g[:, b] = gb
    return g


def collision_jacobian(f, tau0, cs, force=None, mu: float = 0.0):
    """dC_a/df_b at every node: [M][9 (a)][9 (b)][ny][nx]."""
    jac = np.empty(f.shape[:2] + (9,) + f.shape[2:])
    for b in range(9):
        fc = f.astype(np.complex128)
        fc[:, b] += 1j * _H
        jac[:, :, b] = collide(fc, tau0, cs, force, mu).imag / _H
    return jac


def collision_dcs(f, tau0, cs, force=None, mu: float = 0.0):
    """dC_a/dC_s at every node: [M][9][ny][nx]."""
    return collide(f.astype(np.complex128), tau0, cs + 1j * _H, force, mu).imag / _H


def misfit_gradient(f0, steps_per_obs: int, yo, points, nvar: int, tau0, cs, force=None,
                    mu: float = 0.0):
    """(J, dJ/df0 [M][9][ny][nx], dJ/dC_s) by the reverse sweep described above."""
    f0 = np.array(f0, dtype=np.float64)
    yo = np.asarray(yo, dtype=np.float64)
    n_times = yo.shape[0]
    nsteps = n_times * steps_per_obs
    cx, cy, _ = _lat()
    # forward trajectory f^0 .. f^N
    traj = [f0]
    for _ in range(nsteps):
        traj.append(_c_steps(traj[-1], 1, tau0, cs, force, mu))
    J = 0.0
    for c in range(1, n_times + 1):
        J += float(_residual_terms(traj[c * steps_per_obs], points, nvar, yo[c - 1]).sum())
    # reverse sweep
    lam = _misfit_state_gradient(traj[nsteps], points, nvar, yo[n_times - 1])
    dcs = 0.0
    for n in range(nsteps - 1, -1, -1):
        fn = traj[n]
        # lam^{n+1}_a(x + c_a), gathered to node x
        shifted = np.empty_like(lam)
        for a in range(9):
            shifted[:, a] = np.roll(lam[:, a], shift=(-cy[a], -cx[a]), axis=(-2, -1))
        jac = collision_jacobian(fn, tau0, cs, force, mu)
        dcs += float((shifted * collision_dcs(fn, tau0, cs, force, mu)).sum())
        lam = np.einsum("mabyx,mayx->mbyx", jac, shifted)
        if n > 0 and n % steps_per_obs == 0:
            lam = lam + _misfit_state_gradient(fn, points, nvar, yo[n // steps_per_obs - 1])
    return J, lam, dcs
