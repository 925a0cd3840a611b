"""GPU parity for the paper's own physics (Sec. 4.1, Table 1, Sec. 4.3):
tau0 = 0.500614 (nu = 1e-4 at dt = 0.001232), C_s = 0.2, random shell forcing,
linear friction, (rho, u, v) observed, d_cut = p, s = 200."""
import numpy as np
import pytest
import torch

import oracle
from paper_2308_03972_amd import binding, inputs
from gpu_helpers import cuda, host, need_gpu, rel_max, say

pytestmark = pytest.mark.gpu

PP = inputs.CONFIGS["paper_physics"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _states(cfg):
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    ft = oracle.equilibrium(np.ones((1, cfg.n, cfg.n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((cfg.members, cfg.n, cfg.n)), mem_uv[:, 0], mem_uv[:, 1])
    return ft, fe


def test_paper_physics_forecast_200_steps_full_scale():
    say("paper physics: 200 steps 256x256 M=64")
    ft, fe = _states(PP)
    force = inputs.body_force(PP)
    ctx = binding.Context.from_config(PP, force=cuda(force))
    f = ctx.import_canonical(cuda(fe))
    ctx.step(f, PP.steps_per_cycle)
    got = host(ctx.export_canonical(f))
    ref = oracle.lbm_steps(fe, PP.steps_per_cycle, PP.tau0, PP.cs, force, PP.mu)
    assert rel_max(got, ref) < 1e-12


def test_paper_physics_osse_reduced():
    """64^2, 16 members, 4x4 (rho, u, v) points, d_cut = p = 16, s = 50, 4 cycles."""
    cfg = PP.replace(n=64, members=16, obs_side=4, loc_r=16 / np.sqrt(3.0),
                     steps_per_cycle=50, cycles=4)
    say("paper physics: reduced OSSE")
    ft, fe = _states(cfg)
    force = inputs.body_force(cfg)
    tctx = binding.Context.from_config(cfg, members=1, force=cuda(force))
    ectx = binding.Context.from_config(cfg, force=cuda(force))
    gt = tctx.import_canonical(cuda(ft))
    ge = ectx.import_canonical(cuda(fe))
    noise = inputs.all_observation_noise(cfg, cfg.cycles)
    sig = cuda(inputs.sigma_vector(cfg))
    diags = []
    for c in range(cfg.cycles):
        tctx.step(gt, cfg.steps_per_cycle)
        yo = binding.synth_obs(tctx.observe(gt)[0].contiguous(), cuda(noise[c]), sig)
        tm = tctx.moments(gt)[0, 1:].contiguous()
        d = torch.empty(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
        ectx.run_cycle(ge, cfg.steps_per_cycle, yo, tm, d)
        diags.append(host(d))
    diags = np.array(diags)
    ref = oracle.run_cycles(fe, ft, cfg, force, inputs.observation_points(cfg), noise,
                            cfg.cycles)
    assert np.max(np.abs(diags[:, 0] / ref["rmse_f"] - 1)) < 1e-6
    assert np.max(np.abs(diags[:, 8] / ref["rmse_a"] - 1)) < 1e-6
    assert rel_max(host(ectx.export_canonical(ge)), ref["f_ens"]) < 1e-9
