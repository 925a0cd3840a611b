"""Helpers shared by the GPU parity tests (test-side only)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2308_03972_amd import binding, inputs


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def cuda(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def random_state(rng, m, ny, nx, amp=0.03, neq=0.02):
    """Canonical populations near equilibrium plus a non-equilibrium part."""
    u = amp * rng.standard_normal((m, ny, nx))
    v = amp * rng.standard_normal((m, ny, nx))
    rho = 1.0 + 0.01 * rng.standard_normal((m, ny, nx))
    f = oracle.equilibrium(rho, u, v)
    return f * (1.0 + neq * rng.standard_normal(f.shape))


def config_state(cfg, spin_steps=0):
    """Canonical truth [1][9][n][n] and ensemble [M][9][n][n] of a config,
    built by the oracle from the seeded velocity fields."""
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    ft = oracle.equilibrium(np.ones((1, cfg.n, cfg.n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((cfg.members, cfg.n, cfg.n)), mem_uv[:, 0], mem_uv[:, 1])
    if spin_steps:
        force = inputs.body_force(cfg)
        ft = oracle.lbm_steps(ft, spin_steps, cfg.tau0, cfg.cs, force, cfg.mu)
        fe = oracle.lbm_steps(fe, spin_steps, cfg.tau0, cfg.cs, force, cfg.mu)
    return ft, fe


def context(cfg, members=None, route=binding.ROUTE_AUTO, points=None, force=True, **over):
    cfg = cfg.replace(**over) if over else cfg
    fz = cuda(inputs.body_force(cfg)) if force else None
    return binding.Context.from_config(cfg, members=members, force=fz, route=route,
                                       points=points)
