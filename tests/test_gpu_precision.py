"""GPU parity of the precision form: populations stored as FP32 deviations
g = f - w (LBMLETKF_F32_DEV); the forecast relaxes g in FP32 arithmetic
(rho = 1 + sum g); the analysis forms its Gram matrices on FP32 matrix cores
(optionally also B = dX Z^T and the transform on BF16 ones) and keeps its
eigensolve and square root in FP64.

Tolerances: storing a deviation (|g| <~ 0.02 here) in FP32 rounds it by
|g| 2^-24 <= 1.2e-9.  The FP32 relaxation adds a few FP32 roundings of
quantities no larger than the state's largest deviation max|g| (the moments,
the equilibrium deviation, the non-equilibrium part), multiplied by at most
omega = 1/tau < 2: one step from an identical (already rounded) state agrees
with the FP64 oracle to 32 * 2^-24 * max|g| (a generous count of roundings; a
wrong term would miss by ~1e-4 and more).  A single analysis from an identical
state agrees to ~1e-9 absolute plus, with the matrix-core transform
(lbmletkf_set_matrix_core_transform: the observation route's ensemble-space
contractions on BF16 matrix cores with a hi/lo split of each FP32 operand,
~2^-16 per product), 2^-12 of the increment's size; the eigensolve and the
weights stay FP64.  Over a run the velocity
RMSE must stay within 1e-3 of the observation-error standard deviation sigma
(|dRMSE| < 1e-3 sigma = 2.9e-6) of the FP64 result.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2308_03972_amd import binding, inputs
from gpu_helpers import config_state, cuda, host, need_gpu, random_state, rel_max, say

pytestmark = pytest.mark.gpu

TINY = inputs.CONFIGS["tiny"]
F32 = binding.STORAGE_F32_DEV


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _ctx(cfg, storage=F32, members=None, route=binding.ROUTE_AUTO):
    return binding.Context.from_config(cfg, members=members, force=cuda(inputs.body_force(cfg)),
                                       route=route, storage=storage)


def test_f32_storage_roundtrip_and_layout():
    say("f32 import/export")
    rng = np.random.default_rng(200)
    canon = random_state(rng, 3, 20, 24)
    ctx = binding.Context(24, 20, 3, 0.6, 0.1, [[1, 2]], 2, (0.1, 0.1), 4.0, 1.05, storage=F32)
    f = ctx.import_canonical(cuda(canon))
    assert f.dtype == torch.float32
    back = host(ctx.export_canonical(f))
    _, _, w = oracle.lattice()
    dev = canon - w[None, :, None, None]
    assert np.max(np.abs(back - canon)) <= np.max(np.abs(dev)) * 2.0**-24 * 1.01
    # stored values are the deviations (in the shifted storage slots, [y][x][a][m])
    cx, cy, _ = oracle.lattice()
    st = host(f).astype(np.float64)
    for a in range(9):
        exp = np.roll(dev[:, a], shift=(-cy[a], -cx[a]), axis=(1, 2))
        np.testing.assert_allclose(np.moveaxis(st[:, :, a, :], -1, 0), exp, rtol=2**-23,
                                   atol=1e-12)


@pytest.mark.parametrize("members", [1, 4, 5, 64])
def test_f32_stream_collide_step_matches_oracle(members):
    """Even ensembles take two members per thread (8-byte accesses), odd ones one."""
    say(f"f32 stream_collide one step, {members} members")
    rng = np.random.default_rng(201)
    canon = random_state(rng, members, 23, 37)
    force = 1e-4 * rng.standard_normal((2, 23, 37))
    ctx = binding.Context(37, 23, members, 0.55, 0.15, [[0, 0]], 2, (0.1, 0.1), 2.0, 1.05,
                          force=cuda(force), storage=F32)
    f = ctx.import_canonical(cuda(canon))
    start = host(ctx.export_canonical(f))          # the FP32-rounded input
    ctx.step(f, 1)
    got = host(ctx.export_canonical(f))
    ref = oracle.lbm_steps(start, 1, 0.55, 0.15, force)
    w = oracle.lattice()[2][None, :, None, None]
    gmax = np.max(np.abs(start - w))
    err = np.max(np.abs(got - ref))
    say(f"  max error {err:.2e} = {err / (2.0**-24 * gmax):.2f} x 2^-24 max|g|")
    assert err < 32 * 2.0**-24 * gmax


@pytest.mark.parametrize("route,mfma", [(binding.ROUTE_ENSEMBLE, False),
                                        (binding.ROUTE_OBSERVATION, False),
                                        (binding.ROUTE_OBSERVATION, True)])
def test_f32_analysis_matches_oracle(route, mfma):
    say(f"f32 analysis route={route} matrix-core transform={mfma}")
    ft, fe = config_state(TINY, spin_steps=10)
    ctx = _ctx(TINY, route=route)
    ctx.set_matrix_core_transform(mfma)
    f = ctx.import_canonical(cuda(fe))
    start = host(ctx.export_canonical(f))
    pts = inputs.observation_points(TINY)
    sig = inputs.sigma_vector(TINY)
    yo = oracle.observe(ft, pts)[0] + sig * np.random.default_rng(3).standard_normal(len(sig))
    yf = ctx.observe(f)
    ctx.analyze(f, yf, cuda(yo))
    got = host(ctx.export_canonical(f))
    ref = oracle.letkf_analysis(start, oracle.observe(start, pts), yo, pts, TINY.sigmas,
                                TINY.d_cut, TINY.beta)
    inc = ref - start
    # matrix-core transform: B = dX Z^T and the transform on BF16 matrix cores (each
    # FP32 operand split hi + lo, ~2^-16 per product, FP32 accumulation), so the
    # increment is good to ~2^-14 of its size; otherwise they stay FP64 and only the
    # Gram matrices (K, Z^T Z) come from FP32 matrix cores
    rel_inc = 2.0**-12 if mfma else 1e-6
    err = np.max(np.abs(got - ref))
    err_inc = np.max(np.abs((got - start) - inc)) / np.max(np.abs(inc))
    say(f"  max error {err:.2e}; increment error {err_inc:.2e} of max|increment| "
        f"{np.max(np.abs(inc)):.2e}")
    assert err < 2e-9 + rel_inc * np.max(np.abs(inc))
    assert err_inc * np.max(np.abs(inc)) < rel_inc * np.max(np.abs(inc)) + 2e-9


def _osse(cfg, cycles, storage):
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    tctx = _ctx(cfg, storage=binding.STORAGE_F64, members=1)
    ectx = _ctx(cfg, storage=storage)
    ft = tctx.init_equilibrium(cuda(truth_uv[None]))
    fe = ectx.init_equilibrium(cuda(mem_uv))
    noise = inputs.all_observation_noise(cfg, cycles)
    sig = cuda(inputs.sigma_vector(cfg))
    diags = []
    for c in range(cycles):
        tctx.step(ft, cfg.steps_per_cycle)
        yo = binding.synth_obs(tctx.observe(ft)[0].contiguous(), cuda(noise[c]), sig)
        tm = tctx.moments(ft)[0, 1:].contiguous()
        d = torch.empty(2 * binding.DIAG_LEN, dtype=torch.float64, device="cuda")
        ectx.run_cycle(fe, cfg.steps_per_cycle, yo, tm, d)
        diags.append(host(d))
    mo = host(ectx.moments(fe))
    return np.array(diags), mo


def test_f32_tiny_run_rmse_within_tolerance_of_fp64_oracle():
    say("f32 tiny run vs oracle")
    cycles = TINY.cycles
    diags, _ = _osse(TINY, cycles, F32)
    truth_uv, mem_uv = inputs.initial_velocities(TINY)
    ft = oracle.equilibrium(np.ones((1, 32, 32)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((TINY.members, 32, 32)), mem_uv[:, 0], mem_uv[:, 1])
    ref = oracle.run_cycles(fe, ft, TINY, inputs.body_force(TINY),
                            inputs.observation_points(TINY),
                            inputs.all_observation_noise(TINY, cycles), cycles)
    tol = 1e-3 * TINY.sigma
    assert np.max(np.abs(diags[:, 0] - ref["rmse_f"])) < tol
    assert np.max(np.abs(diags[:, 8] - ref["rmse_a"])) < tol


def test_f32_precision_config_matches_fp64_form():
    """512^2, 64 members, 16x16 observations: the FP32-deviation form against the
    FP64 GPU form (itself parity-tested against the oracle) over 10 cycles;
    RMSE within 1e-3 sigma and the ensemble-mean energy spectrum within 1e-3
    relative for k <= 32 (the error up to k = n/3 is printed)."""
    say("f32 precision config 10 cycles")
    cfg = inputs.CONFIGS["precision"]
    d64, m64 = _osse(cfg, 10, binding.STORAGE_F64)
    d32, m32 = _osse(cfg, 10, F32)
    tol = 1e-3 * cfg.sigma
    assert np.max(np.abs(d64[:, 8] - d32[:, 8])) < tol
    assert np.max(np.abs(d64[:, 0] - d32[:, 0])) < tol
    e64 = oracle.energy_spectrum(m64[:, 1].mean(0), m64[:, 2].mean(0))
    e32 = oracle.energy_spectrum(m32[:, 1].mean(0), m32[:, 2].mean(0))
    rel = np.abs(e32 - e64) / e64
    k = np.arange(1, cfg.n // 3)
    worst = int(k[np.argmax(rel[k])])
    say(f"spectrum rel. error: max over k<=32 {rel[1:33].max():.2e}, over k<n/3 "
        f"{rel[k].max():.2e} at k={worst} (E={e64[worst]:.2e}, E(4)={e64[4]:.2e})")
    # energy-containing scales must agree closely; the dissipation range (E
    # many decades below E(4)) is reported, not bounded
    assert rel[1:33].max() < 1e-3
