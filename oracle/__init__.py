"""FP64 CPU oracle of the LBM-LETKF forecast-analysis cycle.

TEST INFRASTRUCTURE.  This package is the plain, slow, obviously correct
reference the GPU library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does.  It shares no code with the GPU library: the lattice-Boltzmann
step is plain C (``lbm_oracle.c``), the rest is NumPy written from the paper
(Hasegawa et al., "Continuous data assimilation of large eddy simulation by
lattice Boltzmann method and local ensemble transform Kalman filter").

Contents and the passage each follows:

* ``lbm_steps`` / ``equilibrium`` / ``moments`` / ``relaxation_time`` --
  Sec. 2 (D2Q9 set, LBE with BGK and force, moments, equilibrium,
  viscosity-tau relation, Smagorinsky model, force term); see lbm_oracle.c.
* ``observe`` -- the observation operator y = H x with y = (u, v) (or
  (rho, u, v)) at the observation nodes (Sec. 3, state and observation
  vectors).
* ``gaspari_cohn`` / ``localization_weights`` -- R-localization with the
  Gaspari-Cohn weight, R_loc^-1 = G o R^-1 for diagonal R (Sec. 3.2.2).
* ``letkf_core`` / ``letkf_analysis`` -- the LETKF of Sec. 3.2.1 with the
  localized, inflated forms of Sec. 3.2.2: ensemble means and
  perturbations, P~a = [(M-1)/beta I + dY^T R_loc^-1 dY]^-1 by a symmetric
  eigendecomposition, w_bar = P~a dY^T R_loc^-1 (y^o - y_bar),
  dW = [(M-1) P~a]^(1/2) (symmetric square root),
  x_m^a = x_bar + dX (w_bar + dW[:, m]).
* ``rmse`` -- RMSE of the ensemble-mean velocity (Sec. 4.3.1).
* ``energy_spectrum`` -- shell-summed energy spectrum (Sec. 4.1);
  ``member_mean_spectrum`` -- the ensemble's spectrum as the mean of the
  members' spectra (Sec. 4.3.2).
* ``run_cycles`` -- the workflow of Sec. 3: forecast s steps, observe the
  truth, analyse, repeat.
* ``oracle.adjoint`` (submodule) -- the gradient of the observation misfit
  of a forecast with respect to the initial populations and C_s, by a
  reverse sweep over complex-step partial derivatives of the Sec. 2 step.

Readings of points the paper leaves open (the same readings the GPU path
documents): the analysis sign is +K (the printed generic update has a sign
slip; the LETKF formulas add the increment); y_bar is the mean of H(x_m); the
square root is the symmetric principal root; the distance is the
minimum-image periodic distance in cells; shells of the spectrum are
half-open [k - 1/2, k + 1/2).

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force on tiny inputs and the exact
Kalman update; none is pinned to the paper's printed RMSE values, which
come from a different configuration (parity with the paper's own numbers is
unpinned).
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIBPATH)
        lib.oracle_lattice.argtypes = [_ip, _ip, _dp]
        lib.oracle_equilibrium.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]
        lib.oracle_moments.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int]
        lib.oracle_relaxation_time.argtypes = [_dp, ctypes.c_double, ctypes.c_double]
        lib.oracle_relaxation_time.restype = ctypes.c_double
        lib.oracle_lbm_steps.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, _dp,
                                         ctypes.c_double, ctypes.c_int]
        lib.oracle_lbm_steps.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# lattice Boltzmann (Sec. 2)
# ---------------------------------------------------------------------------
def lattice():
    """(cx, cy, w) of the D2Q9 set in the oracle's velocity order."""
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    _load().oracle_lattice(cx, cy, w)
    return np.array(cx[:]), np.array(cy[:]), np.array(w[:])


def equilibrium(rho, ux, uy) -> np.ndarray:
    """f^eq of every node; inputs [M][ny][nx] (or [ny][nx]), output [M][9][ny][nx]."""
    rho, ux, uy = (_c64(a) for a in np.broadcast_arrays(rho, ux, uy))
    if rho.ndim == 2:
        rho, ux, uy = rho[None], ux[None], uy[None]
    rho, ux, uy = _c64(rho), _c64(ux), _c64(uy)
    m, ny, nx = rho.shape
    f = np.empty((m, 9, ny, nx))
    _load().oracle_equilibrium(_ptr(rho), _ptr(ux), _ptr(uy), _ptr(f), nx, ny, m)
    return f


def moments(f) -> np.ndarray:
    """(rho, u, v) of every node, shape [3][M][ny][nx]."""
    f = _c64(f)
    m, _, ny, nx = f.shape
    out = np.empty((3, m, ny, nx))
    _load().oracle_moments(_ptr(f), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), nx, ny, m)
    return out


def relaxation_time(f9, tau0: float, cs: float) -> float:
    f9 = _c64(f9)
    return _load().oracle_relaxation_time(_ptr(f9), tau0, cs)


def lbm_steps(f, nsteps: int, tau0: float, cs: float, force=None, mu: float = 0.0) -> np.ndarray:
    """Advance a copy of f ([M][9][ny][nx], pre-collision) by nsteps steps."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    m, nine, ny, nx = f.shape
    assert nine == 9
    fp = None
    if force is not None:
        force = _c64(force)
        assert force.shape == (2, ny, nx)
        fp = _ptr(force)
    rc = _load().oracle_lbm_steps(_ptr(f), nx, ny, m, tau0, cs, fp, mu, int(nsteps))
    if rc != 0:
        raise MemoryError("oracle_lbm_steps could not allocate its buffer")
    return f


# ---------------------------------------------------------------------------
# observation operator (Sec. 3, eqs. for x and y)
# ---------------------------------------------------------------------------
def observe(f, points, nvar: int = 2) -> np.ndarray:
    """y_m = H(x_m): [M][nvar * n_points], q = nvar*k + var, var = (u, v) or (rho, u, v)."""
    f = np.asarray(f, dtype=np.float64)
    cx, cy, _ = lattice()
    pts = np.asarray(points)
    fo = f[:, :, pts[:, 1], pts[:, 0]]                 # [M][9][K]
    rho = fo.sum(axis=1)
    u = np.einsum("mak,a->mk", fo, cx.astype(np.float64)) / rho
    v = np.einsum("mak,a->mk", fo, cy.astype(np.float64)) / rho
    cols = [u, v] if nvar == 2 else [rho, u, v]
    return np.stack(cols, axis=-1).reshape(f.shape[0], -1)


# ---------------------------------------------------------------------------
# localization (Sec. 3.2.2)
# ---------------------------------------------------------------------------
def gaspari_cohn(d) -> np.ndarray:
    """The printed piecewise Gaspari-Cohn weight G(d), d >= 0."""
    d = np.asarray(d, dtype=np.float64)
    g = np.zeros_like(d)
    a = d <= 1.0
    b = (d > 1.0) & (d < 2.0)
    x = d[a]
    g[a] = -0.25 * x**5 + 0.5 * x**4 + 0.625 * x**3 - (5.0 / 3.0) * x**2 + 1.0
    x = d[b]
    g[b] = (x**5 / 12.0 - 0.5 * x**4 + 0.625 * x**3 + (5.0 / 3.0) * x**2 - 5.0 * x + 4.0
            - (2.0 / 3.0) / x)
    return g


def periodic_distance(n: int, x0, y0, x1, y1) -> np.ndarray:
    """Minimum-image Euclidean distance on the n x n periodic lattice."""
    dx = np.abs(np.asarray(x0) - np.asarray(x1)) % n
    dy = np.abs(np.asarray(y0) - np.asarray(y1)) % n
    dx = np.minimum(dx, n - dx)
    dy = np.minimum(dy, n - dy)
    return np.hypot(dx, dy)


def localization_weights(n: int, points, d_cut: float, nodes=None) -> np.ndarray:
    """G[node][k] = GC(|xi - eta_k| / d_cut); node index = y*n + x; d_cut=inf: all 1."""
    pts = np.asarray(points)
    nodes = np.arange(n * n) if nodes is None else np.asarray(nodes)
    nx_, ny_ = nodes % n, nodes // n
    if not math.isfinite(d_cut):
        return np.ones((len(nodes), len(pts)))
    dist = periodic_distance(n, nx_[:, None], ny_[:, None], pts[None, :, 0], pts[None, :, 1])
    return gaspari_cohn(dist / d_cut)


# ---------------------------------------------------------------------------
# LETKF (Sec. 3.2.1 and Sec. 3.2.2)
# ---------------------------------------------------------------------------
def letkf_core(X, Yf, yo, rinv, beta: float) -> np.ndarray:
    """Analysis ensemble of a batch of local problems.

    X    [B][n_state][M]  forecast states x_m^f (one column per member)
    Yf   [n_obs][M] or [B][n_obs][M]  forecast observations y_m^f = H x_m^f
    yo   [n_obs]          observations y^o
    rinv [B][n_obs]       diagonal of R_loc^-1 = G o R^-1
    Returns X^a [B][n_state][M].
    """
    X = np.asarray(X, dtype=np.float64)
    Yf = np.asarray(Yf, dtype=np.float64)
    rinv = np.asarray(rinv, dtype=np.float64)
    M = X.shape[-1]
    ybar = Yf.mean(axis=-1)                                   # y_bar^f
    dY = Yf - ybar[..., None]                                 # dY^f
    d = np.asarray(yo, dtype=np.float64) - ybar               # y^o - y_bar^f
    xbar = X.mean(axis=-1)                                    # x_bar^f
    dX = X - xbar[..., None]                                  # dX^f
    dYt = np.swapaxes(dY, -1, -2)                             # dY^T
    # (M-1)/beta I + dY^T R_loc^-1 dY   (its inverse is P~a)
    A = dYt @ (rinv[..., :, None] * dY) + ((M - 1) / beta) * np.eye(M)
    lam, Q = np.linalg.eigh(A)
    Qt = np.swapaxes(Q, -1, -2)
    Pa = Q @ (Qt / lam[..., :, None])                         # Q Lambda^-1 Q^T
    wbar = (Pa @ (dYt @ (rinv * d)[..., None]))[..., 0]      # P~a dY^T R_loc^-1 d
    dW = Q @ (np.sqrt((M - 1) / lam)[..., :, None] * Qt)      # [(M-1) P~a]^(1/2)
    T = wbar[..., :, None] + dW                               # column m: w_bar + dW[:, m]
    return xbar[..., None] + dX @ T


def letkf_analysis(f, yf, yo, points, sigmas: Sequence[float], d_cut: float, beta: float,
                   nodes=None, chunk: int = 1024) -> np.ndarray:
    """LETKF analysis of every node (or of ``nodes``), each node its own local problem.

    f [M][9][ny][nx] forecast populations (pre-collision), yf [M][n_obs],
    yo [n_obs], sigmas: observation-error std per variable.
    Returns the analysis f^a [M][9][ny][nx] (nodes=None) or [M][9][len(nodes)].
    """
    f = np.asarray(f, dtype=np.float64)
    M, _, ny, nx = f.shape
    assert nx == ny
    nvar = len(sigmas)
    rinv_var = 1.0 / np.asarray(sigmas, dtype=np.float64) ** 2
    Yf = np.asarray(yf, dtype=np.float64).T                   # [n_obs][M]
    all_nodes = np.arange(nx * ny) if nodes is None else np.asarray(nodes)
    flat = f.reshape(M, 9, nx * ny)
    out = np.empty((M, 9, len(all_nodes)))
    for s in range(0, len(all_nodes), chunk):
        nd = all_nodes[s:s + chunk]
        G = localization_weights(nx, points, d_cut, nodes=nd)            # [B][K]
        rinv = (G[:, :, None] * rinv_var[None, None, :]).reshape(len(nd), -1)
        X = np.transpose(flat[:, :, nd], (2, 1, 0))                      # [B][9][M]
        Xa = letkf_core(X, Yf, yo, rinv, beta)
        out[:, :, s:s + chunk] = np.transpose(Xa, (2, 1, 0))
    if nodes is None:
        return out.reshape(M, 9, ny, nx)
    return out


# ---------------------------------------------------------------------------
# diagnostics (Sec. 4.1, Sec. 4.3.1)
# ---------------------------------------------------------------------------
def ensemble_mean_velocity(f) -> np.ndarray:
    """u^DA = M^-1 sum_m u_m, shape [2][ny][nx]."""
    mo = moments(f)
    return np.stack([mo[1].mean(axis=0), mo[2].mean(axis=0)])


def rmse(f_ens, f_truth) -> float:
    """sqrt(N^-1 sum_xi |u^DA - u^t|^2), u^DA the ensemble-mean velocity."""
    ue = ensemble_mean_velocity(f_ens)
    mt = moments(f_truth)
    du = ue[0] - mt[1, 0]
    dv = ue[1] - mt[2, 0]
    return float(np.sqrt(np.mean(du * du + dv * dv)))


def spread(f_ens) -> float:
    """sqrt(N^-1 sum_xi (M-1)^-1 sum_m |u_m - u_bar|^2)."""
    mo = moments(f_ens)
    M = mo.shape[1]
    du = mo[1] - mo[1].mean(axis=0)
    dv = mo[2] - mo[2].mean(axis=0)
    return float(np.sqrt(np.mean((du * du + dv * dv).sum(axis=0) / (M - 1))))


def energy_spectrum(u, v) -> np.ndarray:
    """E(k) = sum over the shell k - 1/2 <= |k'| < k + 1/2 of |u_hat(k')|^2 / 2.

    u_hat = N^-2 sum u exp(-i k.xi); returns E for k = 0 .. ceil(n/sqrt2).
    """
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[0]
    uh = np.fft.fft2(u) / (n * n)
    vh = np.fft.fft2(np.asarray(v, dtype=np.float64)) / (n * n)
    e = 0.5 * (np.abs(uh) ** 2 + np.abs(vh) ** 2)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kmag = np.hypot(k1[None, :], k1[:, None])
    shell = np.floor(kmag + 0.5).astype(np.int64)
    return np.bincount(shell.ravel(), weights=e.ravel())


def member_mean_spectrum(f) -> np.ndarray:
    """Ensemble spectrum M^-1 sum_m E_m(k), E_m the spectrum of member m's
    velocity (the mean of the members' spectra, Sec. 4.3.2); f [M][9][n][n]."""
    mo = moments(f)
    specs = [energy_spectrum(mo[1, m], mo[2, m]) for m in range(mo.shape[1])]
    return np.mean(np.stack(specs), axis=0)


# ---------------------------------------------------------------------------
# forecast-analysis cycle (Sec. 3 workflow, Sec. 4.3 OSSE)
# ---------------------------------------------------------------------------
def run_cycles(f_ens, f_truth, params, force, points, noise, cycles: Optional[int] = None,
               keep_states: bool = False, analyze=None,
               report_every: int = 0) -> Dict[str, object]:
    """Run ``cycles`` forecast-analysis cycles (Sec. 3 workflow (ii)-(v)).

    params: any object with n, tau0, cs, mu, steps_per_cycle, nvar, sigmas,
    d_cut, beta.  noise: [cycles][n_obs] standard normals; observation
    q of cycle c is y^o = H(truth) + sigma_q * noise[c-1][q], taken from the
    truth after it has been advanced to the analysis time c * s.  RMSE_f and
    spread_f are those of the forecast (before the analysis), RMSE_a and
    spread_a those of the analysis.  ``analyze``: the analysis function
    (default ``letkf_analysis``; any callable with its signature and result,
    e.g. the same function mapped over node subsets).  With report_every = k
    > 0 the member-mean spectrum of the analysis ensemble and the truth's
    spectrum are recorded at every k-th cycle.
    """
    cycles = len(noise) if cycles is None else cycles
    analyze = letkf_analysis if analyze is None else analyze
    sig = np.tile(np.asarray(params.sigmas, dtype=np.float64), len(points))
    f_ens = np.array(f_ens, dtype=np.float64)
    f_truth = np.array(f_truth, dtype=np.float64)
    hist = {"rmse_f": [], "rmse_a": [], "spread_f": [], "spread_a": [], "yo": [],
            "report_cycle": [], "spectrum_a": [], "spectrum_t": []}
    states = []
    for c in range(1, cycles + 1):
        # (ii) forecast: truth and members advance s steps
        f_truth = lbm_steps(f_truth, params.steps_per_cycle, params.tau0, params.cs, force,
                            params.mu)
        f_ens = lbm_steps(f_ens, params.steps_per_cycle, params.tau0, params.cs, force,
                          params.mu)
        # (iii) observe the truth at the analysis time
        yo = observe(f_truth, points, params.nvar)[0] + sig * np.asarray(noise[c - 1])
        yf = observe(f_ens, points, params.nvar)
        hist["rmse_f"].append(rmse(f_ens, f_truth))
        hist["spread_f"].append(spread(f_ens))
        # (iv) analysis
        f_ens = analyze(f_ens, yf, yo, points, params.sigmas, params.d_cut, params.beta)
        hist["rmse_a"].append(rmse(f_ens, f_truth))
        hist["spread_a"].append(spread(f_ens))
        hist["yo"].append(yo)
        if report_every > 0 and c % report_every == 0:
            mt = moments(f_truth)
            hist["report_cycle"].append(c)
            hist["spectrum_a"].append(member_mean_spectrum(f_ens))
            hist["spectrum_t"].append(energy_spectrum(mt[1, 0], mt[2, 0]))
        if keep_states:
            states.append(f_ens.copy())
    out = {k: np.asarray(v) for k, v in hist.items()}
    out["f_ens"] = f_ens
    out["f_truth"] = f_truth
    if keep_states:
        out["states"] = states
    return out
