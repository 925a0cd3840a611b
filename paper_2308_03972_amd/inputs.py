"""Seeded synthetic inputs for the LBM-LETKF forecast-analysis cycle.

This module is the only code shared by the GPU path and the FP64 oracle, and
it holds none of the method's arithmetic: no lattice-Boltzmann update, no
moment, no observation operator, no Kalman algebra.  It only

* defines the run configurations (grid, ensemble, observing network,
  localization, inflation, cycle length),
* draws the random initial velocity fields, the member perturbations and the
  observation noise from fixed seeds,
* lays out the body-force field and the observation points.

The paper runs an observing-system simulation experiment on synthetic forced
2D turbulence (Sec. 4.1, Sec. 4.3); no dataset is involved.  Its truth and
ensemble start from mutually uncorrelated random states (Sec. 4.3); here the
initial fields follow the readings listed below.

Readings of points the paper leaves open (all are explicit config fields):

* lattice units, dx = dt = c = 1 (the paper's c = dx/dt, Sec. 2);
* initial velocity: random-phase streamfunction with shell spectrum
  E(k) ~ k^4 exp(-(k/4)^2), zero mean, Nyquist lines removed, rescaled to
  rms |u| = urms = 0.05 c_s (c_s = 1/sqrt(3));
* members = truth + an independent field of the same spectrum at
  ``member_amp`` * urms;
* steady body force F = (A sin(2 pi k y / n), 0) at k = 4, with A chosen so
  that the laminar Kolmogorov flow it drives has rms velocity urms; or, for the
  paper's own physics, the shell forcing of Sec. 4.1, F = dx grad(F_e) x i_z,
  F_e = sum over the integer wavevectors with ||k| - k_f| <= dk of
  r1.k cos(k.xi) + r2.k sin(k.xi) with Gaussian random vectors r1, r2 per
  wavevector, drawn once (steady), and F_e0 fixed by the reading that the force
  has the same rms as the sinusoidal force;
* observation points on a uniform lattice (a*p, b*p), p = n / obs_side,
  point index k = b*obs_side + a, observation index q = nvar*k + var,
  var = (u, v) for nvar = 2 and (rho, u, v) for nvar = 3 (eq. for y, Sec. 3);
* observation error sigma = 0.1 urms for u and v (the paper's 10 % of the
  reference velocity, Sec. 4.3), 0.01 for rho;
* the localization length r is the length of the Gaussian that the
  Gaspari-Cohn function approximates, so d_cut = sqrt(3) r (Sec. 3.2.2);
* all randomness comes from numpy PCG64 streams spawned from one seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED = 230803972
CS2 = 1.0 / 3.0  # lattice speed of sound squared, lattice units


@dataclasses.dataclass(frozen=True)
class CycleConfig:
    """One forecast-analysis experiment (Sec. 3 workflow, Sec. 4.3 OSSE)."""

    name: str
    n: int                      # grid is n x n, doubly periodic
    members: int                # ensemble size M
    tau0: float                 # molecular relaxation time (lattice units)
    cs: float                   # Smagorinsky constant C_s (filter width = dx)
    obs_side: int               # observation points per side
    loc_r: float                # Gaussian localization length in cells; <= 0: none
    steps_per_cycle: int        # s, LBM steps between analyses
    cycles: int
    beta: float = 1.05          # multiplicative inflation
    force_k: int = 4
    force_amp: Optional[float] = None   # None: the Kolmogorov-rms reading
    mu: float = 0.0             # linear friction coefficient (Sec. 4.1)
    urms: float = 0.05 * math.sqrt(CS2)
    member_amp: float = 0.2
    nvar: int = 2               # 2: (u, v); 3: (rho, u, v)
    forcing: str = "kolmogorov"  # "kolmogorov" (sinusoidal) or "shell" (Sec. 4.1)
    shell_width: float = 2.0    # dk of the shell forcing
    sigma_uv: Optional[float] = None    # None: 0.1 * urms
    sigma_rho: float = 0.01
    seed: int = SEED

    # ---- derived quantities (configuration readings, not method steps) ----
    @property
    def nu0(self) -> float:
        return (self.tau0 - 0.5) * CS2

    @property
    def amplitude(self) -> float:
        if self.force_amp is not None:
            return self.force_amp
        kphys = 2.0 * math.pi * self.force_k / self.n
        return math.sqrt(2.0) * self.urms * self.nu0 * kphys * kphys

    @property
    def sigma(self) -> float:
        return 0.1 * self.urms if self.sigma_uv is None else self.sigma_uv

    @property
    def sigmas(self) -> Tuple[float, ...]:
        """Observation-error standard deviation per observed variable."""
        if self.nvar == 2:
            return (self.sigma, self.sigma)
        return (self.sigma_rho, self.sigma, self.sigma)

    @property
    def obs_spacing(self) -> int:
        return self.n // self.obs_side

    @property
    def n_points(self) -> int:
        return self.obs_side * self.obs_side

    @property
    def n_obs(self) -> int:
        return self.nvar * self.n_points

    @property
    def d_cut(self) -> float:
        """Gaspari-Cohn cutoff; infinite when localization is off."""
        return math.sqrt(3.0) * self.loc_r if self.loc_r > 0 else math.inf

    def replace(self, **kw) -> "CycleConfig":
        return dataclasses.replace(self, **kw)


CONFIGS: Dict[str, CycleConfig] = {
    # 32^2, 8 members, 4x4 observations, r = 4, s = 10, 20 cycles, FP64.
    "tiny": CycleConfig(name="tiny", n=32, members=8, tau0=0.52, cs=0.1,
                        obs_side=4, loc_r=4.0, steps_per_cycle=10, cycles=20),
    # 256^2, 64 members, 8x8 observations, r = 16, s = 20, 200 cycles, FP64.
    "paper": CycleConfig(name="paper", n=256, members=64, tau0=0.52, cs=0.1,
                         obs_side=8, loc_r=16.0, steps_per_cycle=20, cycles=200),
    # 512^2, 64 members, 16x16 observations, 100 cycles (precision form).
    "precision": CycleConfig(name="precision", n=512, members=64, tau0=0.52,
                             cs=0.1, obs_side=16, loc_r=16.0,
                             steps_per_cycle=20, cycles=100),
    # The paper's own physics (Sec. 4.1, Table 1, Sec. 4.3) on 256^2: nu = 1e-4,
    # dt = 0.001232, dx = 2 pi / 256 give tau0 = 1/2 + 3 nu dt / dx^2; C_s = 0.2;
    # friction mu dt per step; shell forcing k_f = 4, dk = 2; (rho, u, v)
    # observed every p = 32 cells; d_cut = p (so r = p / sqrt 3); s = 200.
    "paper_physics": CycleConfig(
        name="paper_physics", n=256, members=64,
        tau0=0.5 + 3.0 * 1e-4 * 0.001232 / (2.0 * math.pi / 256) ** 2, cs=0.2,
        obs_side=8, loc_r=32.0 / math.sqrt(3.0), steps_per_cycle=200, cycles=20,
        mu=5e-4 * 0.001232, nvar=3, forcing="shell"),
    # Differentiation form: 128^2, 16 members, 8x8 observations of (u, v),
    # FP32 populations; the misfit covers 10 observation times 20 steps apart
    # (200 steps, a checkpoint at every observation time).
    "differentiation": CycleConfig(name="differentiation", n=128, members=16, tau0=0.52,
                                   cs=0.1, obs_side=8, loc_r=16.0, steps_per_cycle=20,
                                   cycles=10),
}


def batch_configs() -> List[CycleConfig]:
    """The twelve problems of the batching form: grids {128, 192, 256, 384}^2 x
    members {16, 32, 64}, problem i = 3 g + m (g grid index, m member index),
    observation grid side [4, 8, 16, 32][(g + m) mod 4] and localization length
    r = [0.15, 0.5, 0.73][(g + 2 m) mod 3] x the observation spacing, which gives
    0-4, 16-24 and 32-44 local observations per node.  Every problem draws its
    own fields (seed offset i); other parameters as the paper-scale configuration."""
    base = CONFIGS["paper"]
    out = []
    for g, n in enumerate((128, 192, 256, 384)):
        for m, members in enumerate((16, 32, 64)):
            side = (4, 8, 16, 32)[(g + m) % 4]
            ratio = (0.15, 0.5, 0.73)[(g + 2 * m) % 3]
            out.append(base.replace(name=f"batch{3 * g + m}", n=n, members=members,
                                    obs_side=side, loc_r=ratio * n / side,
                                    seed=base.seed + 1 + 3 * g + m))
    return out


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------
def streams(cfg: CycleConfig, cycles: Optional[int] = None) -> Dict[str, object]:
    """Independent PCG64 generators: truth IC, one per member, one per cycle.

    Child streams depend only on their index, so asking for more cycles than
    the configuration holds leaves the first ones unchanged."""
    n_noise = max(cfg.cycles, cycles or 0) + 1
    root = np.random.SeedSequence(cfg.seed)
    truth_ss, member_ss, noise_ss, force_ss = root.spawn(4)
    return {
        "force": np.random.Generator(np.random.PCG64(force_ss)),
        "truth": np.random.Generator(np.random.PCG64(truth_ss)),
        "members": [np.random.Generator(np.random.PCG64(s))
                    for s in member_ss.spawn(cfg.members)],
        "noise": [np.random.Generator(np.random.PCG64(s))
                  for s in noise_ss.spawn(n_noise)],
    }


def spectral_velocity(n: int, rng: np.random.Generator, rms: float,
                      kpeak: float = 4.0) -> np.ndarray:
    """Divergence-free random-phase velocity field, shape [2][n][n] = (u, v).

    Streamfunction modes psi(k) = exp(i phi_k) sqrt(E(k_s)/n_s) / |k| with
    integer shell k_s = round|k|, n_s the number of retained modes in the
    shell, E(k) = k^4 exp(-(k/kpeak)^2); phi odd in k (Hermitian field), the
    k = 0 mode and the Nyquist lines removed.  u = d psi/dy, v = -d psi/dx,
    then the field is scaled to rms sqrt(<u^2 + v^2>) = ``rms``.
    Array index order is [y][x].
    """
    k1 = np.fft.fftfreq(n, d=1.0 / n)            # integer wavenumbers
    kx = np.broadcast_to(k1[None, :], (n, n))
    ky = np.broadcast_to(k1[:, None], (n, n))
    kmag = np.hypot(kx, ky)
    shell = np.rint(kmag).astype(np.int64)
    keep = (kmag > 0) & (np.abs(kx) != n // 2) & (np.abs(ky) != n // 2)
    counts = np.bincount(shell[keep], minlength=shell.max() + 1)
    spec = shell.astype(np.float64) ** 4 * np.exp(-(shell / kpeak) ** 2)
    amp = np.zeros((n, n))
    amp[keep] = np.sqrt(spec[keep] / counts[shell[keep]]) / kmag[keep]
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(n, n))
    neg = (-np.arange(n)) % n
    phase = phi - phi[np.ix_(neg, neg)]          # odd in k => real field
    psi = amp * np.exp(1j * phase)
    scale = 2.0 * np.pi / n
    u = np.fft.ifft2(1j * ky * scale * psi).real
    v = np.fft.ifft2(-1j * kx * scale * psi).real
    norm = math.sqrt(float(np.mean(u * u + v * v)))
    return np.stack([u, v]) * (rms / norm)


def initial_velocities(cfg: CycleConfig) -> Tuple[np.ndarray, np.ndarray]:
    """Truth velocity [2][n][n] and member velocities [M][2][n][n]."""
    st = streams(cfg)
    truth = spectral_velocity(cfg.n, st["truth"], cfg.urms)
    members = np.stack([
        truth + spectral_velocity(cfg.n, g, cfg.member_amp * cfg.urms)
        for g in st["members"]])
    return truth, members


def body_force(cfg: CycleConfig) -> np.ndarray:
    """Steady acceleration field [2][n][n] = (Fx, Fy), index [.][y][x]."""
    if cfg.forcing == "shell":
        return shell_force(cfg)
    y = np.arange(cfg.n, dtype=np.float64)
    fx_row = cfg.amplitude * np.sin(2.0 * np.pi * cfg.force_k * y / cfg.n)
    force = np.zeros((2, cfg.n, cfg.n))
    force[0] = fx_row[:, None]
    return force


def shell_force(cfg: CycleConfig) -> np.ndarray:
    """Divergence-free random shell forcing (Sec. 4.1), [2][n][n].

    F_e(xi) = sum_k r1_k.k cos(k.xi) + r2_k.k sin(k.xi) over integer wavevectors
    with ||k| - k_f| <= dk on the 2 pi periodic box (xi = 2 pi (x, y) / n),
    r1_k, r2_k independent standard-normal 2-vectors; F = (dF_e/dy, -dF_e/dx),
    scaled to rms sqrt(<Fx^2 + Fy^2>) = A / sqrt 2 (the sinusoidal force's rms).
    """
    rng = streams(cfg)["force"]
    n = cfg.n
    xi = 2.0 * np.pi * np.arange(n) / n
    X, Y = np.meshgrid(xi, xi)                      # [y][x]
    kmax = int(np.ceil(cfg.force_k + cfg.shell_width))
    fx = np.zeros((n, n))
    fy = np.zeros((n, n))
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            km = math.hypot(kx, ky)
            if km == 0 or abs(km - cfg.force_k) > cfg.shell_width:
                continue
            r1 = rng.standard_normal(2)
            r2 = rng.standard_normal(2)
            a = r1[0] * kx + r1[1] * ky
            b = r2[0] * kx + r2[1] * ky
            ph = kx * X + ky * Y
            # d/dxi of a cos(ph) + b sin(ph) = (-a sin(ph) + b cos(ph)) * k
            dphase = -a * np.sin(ph) + b * np.cos(ph)
            fx += ky * dphase          # dF_e/dy
            fy -= kx * dphase          # -dF_e/dx
    rms = math.sqrt(float(np.mean(fx * fx + fy * fy)))
    scale = (cfg.amplitude / math.sqrt(2.0)) / rms
    return np.stack([fx, fy]) * scale


def observation_points(cfg: CycleConfig) -> np.ndarray:
    """Observation node coordinates, int32 [n_points][2] = (x, y)."""
    p = cfg.obs_spacing
    pts = [(a * p, b * p) for b in range(cfg.obs_side) for a in range(cfg.obs_side)]
    return np.asarray(pts, dtype=np.int32)


def observation_noise(cfg: CycleConfig, cycle: int) -> np.ndarray:
    """Standard-normal draws for the observations of ``cycle`` (1-based)."""
    return streams_noise(cfg, cycle)[cycle].standard_normal(cfg.n_obs)


def streams_noise(cfg: CycleConfig, cycles: Optional[int] = None) -> List[np.random.Generator]:
    return streams(cfg, cycles)["noise"]


def all_observation_noise(cfg: CycleConfig, cycles: Optional[int] = None) -> np.ndarray:
    """Noise for cycles 1..cycles, shape [cycles][n_obs]."""
    cycles = cfg.cycles if cycles is None else cycles
    gens = streams_noise(cfg, cycles)
    return np.stack([gens[c].standard_normal(cfg.n_obs) for c in range(1, cycles + 1)])


def sigma_vector(cfg: CycleConfig) -> np.ndarray:
    """Observation-error standard deviation per observation index q."""
    return np.tile(np.asarray(cfg.sigmas, dtype=np.float64), cfg.n_points)
