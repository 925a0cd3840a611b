"""GPU tests of the batching form (lbmletkf_batch_*): many problems per cycle in
one persistent forecast launch per step and size-grouped analysis launches
under a captured hipGraph.

The batched kernels run the same per-node arithmetic as the single-problem
path (itself parity-tested against the oracle), so with the default bucket
granularity (eigenproblem size as the single path chooses it) the batch must
reproduce each problem's own run_cycle bit for bit; coarser granularities pad
the eigenproblems, which changes only the rounding (1e-12 of the state's
scale).  One small batch is also compared with the oracle directly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2308_03972_amd import binding, inputs
from gpu_helpers import cuda, host, need_gpu, say

pytestmark = pytest.mark.gpu

F64, F32 = binding.STORAGE_F64, binding.STORAGE_F32_DEV


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _problem(cfg, storage, force=True):
    """Context, truth context, initial member fields and the force of a config."""
    fz = cuda(inputs.body_force(cfg)) if force else None
    ctx = binding.Context.from_config(cfg, force=fz, storage=storage)
    tctx = binding.Context.from_config(cfg, members=1, force=fz, storage=F64)
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    return ctx, tctx, cuda(truth_uv[None]), cuda(mem_uv)


def _observations(cfg, tctx, truth_uv, cycles):
    ft = tctx.init_equilibrium(truth_uv)
    noise = cuda(inputs.all_observation_noise(cfg, cycles))
    sig = cuda(inputs.sigma_vector(cfg))
    out = []
    for c in range(cycles):
        tctx.step(ft, cfg.steps_per_cycle)
        out.append(binding.synth_obs(tctx.observe(ft)[0].contiguous(), noise[c].contiguous(), sig))
    return out


def _setup(cfgs, storage, cycles):
    probs = []
    for cfg in cfgs:
        ctx, tctx, tuv, muv = _problem(cfg, storage)
        yo = _observations(cfg, tctx, tuv, cycles)
        probs.append((cfg, ctx, muv, yo))
    return probs


def _single_runs(probs, cycles):
    out = []
    for cfg, ctx, muv, yo in probs:
        f = ctx.init_equilibrium(muv)
        for c in range(cycles):
            ctx.run_cycle(f, cfg.steps_per_cycle, yo[c])
        out.append(host(f).copy())
    return out


def _batch_runs(probs, cycles, config=None, tune=False):
    states = [ctx.init_equilibrium(muv) for _, ctx, muv, _ in probs]
    b = binding.Batch([p[1] for p in probs], states, probs[0][0].steps_per_cycle, config=config)
    if tune:
        before = [host(f).copy() for f in states]
        cfg, fms, ams = b.tune(reps=1)
        say(f"tuned {cfg}: forecast {fms:.3f} ms/step, analysis {ams:.3f} ms")
        for f, f0 in zip(states, before):
            assert np.array_equal(host(f), f0)          # tuning leaves the states alone
    for c in range(cycles):
        b.run_cycle([p[3][c] for p in probs])
    res = [host(f).copy() for f in states]
    b.close()
    return res


def _mixed_configs():
    """Four small problems: both analysis routes, empty and full neighbourhoods,
    ragged grids, members 8..64."""
    base = inputs.CONFIGS["tiny"]
    return [
        base,                                                             # 32^2, M=8: ensemble route
        base.replace(name="b1", n=48, members=16, obs_side=4, loc_r=3.0, seed=11),   # l = 0..4
        base.replace(name="b2", n=40, members=32, obs_side=8, loc_r=4.0, seed=12),   # obs route
        base.replace(name="b3", n=24, members=64, obs_side=6, loc_r=3.0, seed=13),   # obs route
    ]


@pytest.mark.parametrize("storage,mfma", [(F64, False), (F32, False), (F32, True)])
def test_batch_reproduces_each_problems_run_cycle(storage, mfma):
    say(f"batch vs single storage={storage} matrix-core transform={mfma}")
    probs = _setup(_mixed_configs(), storage, cycles=3)
    for p in probs:
        p[1].set_matrix_core_transform(mfma)
    single = _single_runs(probs, 3)
    batched = _batch_runs(probs, 3)
    diffs = [float(np.max(np.abs(s.astype(np.float64) - b))) for s, b in zip(single, batched)]
    say(f"  max |batched - single| per problem: {diffs}")
    for s, b in zip(single, batched):
        assert np.array_equal(s, b)


@pytest.mark.parametrize("storage", [F64, F32])
def test_batch_two_step_launches_reproduce_run_cycle(storage):
    """Problems with 16 | M: the batch's two-step launch over every problem's
    (tile, member group) blocks, with an odd step count (the last step single),
    against each problem's own run_cycle, bit for bit, graph and eager."""
    say(f"batch two-step launches storage={storage}")
    base = inputs.CONFIGS["tiny"]
    cfgs = [base.replace(name="t1", n=32, members=16, steps_per_cycle=7, seed=21),
            base.replace(name="t2", n=37, members=32, obs_side=4, loc_r=3.0, steps_per_cycle=7,
                         seed=22),
            base.replace(name="t3", n=26, members=64, obs_side=4, loc_r=5.0, steps_per_cycle=7,
                         seed=23)]
    probs = _setup(cfgs, storage, cycles=3)
    single = _single_runs(probs, 3)
    for graph in (1, 0):
        batched = _batch_runs(probs, 3, config=dict(forecast_blocks=0, tile_rows=2,
                                                    bucket_granularity=2, use_graph=graph,
                                                    steps_per_launch=2))
        for s_, b_ in zip(single, batched):
            assert np.array_equal(s_, b_)


@pytest.mark.parametrize("storage", [F64, F32])
def test_batch_analysis_work_queue_reproduces_run_cycle(storage):
    """analysis_queue = 1: persistent eigen and apply launches whose blocks take
    the (problem, node tile) items from a queue; each problem's states equal its
    own run_cycle bit for bit, graph (the counters cleared by a kernel inside
    it) and eager, over three cycles."""
    say(f"batch analysis work queue storage={storage}")
    base = inputs.CONFIGS["tiny"]
    # plus a problem whose every node sees all 50 observations: the split-row
    # eigen kernel (N = 56, two wavefronts per block) through the queue
    cfgs = _mixed_configs() + [base.replace(name="b4", n=20, members=64, obs_side=5, loc_r=0.0,
                                            seed=14)]
    probs = _setup(cfgs, storage, cycles=3)
    single = _single_runs(probs, 3)
    for graph in (1, 0):
        batched = _batch_runs(probs, 3, config=dict(forecast_blocks=0, tile_rows=2,
                                                    bucket_granularity=2, use_graph=graph,
                                                    steps_per_launch=1, analysis_queue=1))
        for s_, b_ in zip(single, batched):
            assert np.array_equal(s_, b_)


def test_batch_graph_replays_match_eager_launches():
    """Three cycles replayed from the captured graph against the same cycles
    issued launch by launch, compared after every cycle."""
    say("batch graph vs eager")
    probs = _setup(_mixed_configs(), F64, cycles=3)
    sa = [ctx.init_equilibrium(muv) for _, ctx, muv, _ in probs]
    sb = [ctx.init_equilibrium(muv) for _, ctx, muv, _ in probs]
    s = probs[0][0].steps_per_cycle
    ga = binding.Batch([p[1] for p in probs], sa, s,
                       config=dict(forecast_blocks=512, tile_rows=2, bucket_granularity=2,
                                   use_graph=1))
    gb = binding.Batch([p[1] for p in probs], sb, s,
                       config=dict(forecast_blocks=512, tile_rows=2, bucket_granularity=2,
                                   use_graph=0))
    for c in range(3):
        ga.run_cycle([p[3][c] for p in probs])
        torch.cuda.synchronize()
        gb.run_cycle([p[3][c] for p in probs])
        for x, y in zip(sa, sb):
            assert torch.equal(x, y)
    ga.close()
    gb.close()


def test_batch_tuning_and_coarse_buckets():
    say("batch tune, granularity 8")
    probs = _setup(_mixed_configs(), F64, cycles=2)
    single = _single_runs(probs, 2)
    tuned = _batch_runs(probs, 2, tune=True)
    coarse = _batch_runs(probs, 2, config=dict(forecast_blocks=256, tile_rows=8,
                                               bucket_granularity=8, use_graph=1))
    for s, t, c in zip(single, tuned, coarse):
        scale = np.max(np.abs(s))
        # the tuner may pick a coarser granularity: rounding-level differences only
        assert np.max(np.abs(t - s)) <= 1e-12 * scale
        assert np.max(np.abs(c - s)) <= 1e-12 * scale


def test_batch_one_block_per_tile():
    """forecast_blocks = 0 launches one block per tile instead of a fixed-stride
    persistent grid; the states must still equal each problem's run_cycle."""
    say("batch one block per tile")
    probs = _setup(_mixed_configs(), F64, cycles=2)
    single = _single_runs(probs, 2)
    for rows in (1, 3):
        batched = _batch_runs(probs, 2, config=dict(forecast_blocks=0, tile_rows=rows,
                                                    bucket_granularity=2, use_graph=1))
        for s_, b_ in zip(single, batched):
            assert np.array_equal(s_, b_)


def test_batch_against_oracle():
    """Two problems (ensemble and observation route) over two cycles against the
    oracle's own forecast-analysis cycles."""
    say("batch vs oracle")
    cfgs = _mixed_configs()[:3:2]
    probs = _setup(cfgs, F64, cycles=2)
    batched = _batch_runs(probs, 2)
    for (cfg, ctx, muv, yo), got in zip(probs, batched):
        truth_uv, mem_uv = inputs.initial_velocities(cfg)
        n = cfg.n
        fe = oracle.equilibrium(np.ones((cfg.members, n, n)), mem_uv[:, 0], mem_uv[:, 1])
        ft = oracle.equilibrium(np.ones((1, n, n)), truth_uv[0][None], truth_uv[1][None])
        ref = oracle.run_cycles(fe, ft, cfg, inputs.body_force(cfg),
                                inputs.observation_points(cfg),
                                inputs.all_observation_noise(cfg, 2), 2)
        canon = host(ctx.export_canonical(torch.from_numpy(got).cuda()))
        assert np.max(np.abs(canon - ref["f_ens"])) <= 1e-11 * np.max(np.abs(ref["f_ens"]))


def test_batching_configuration_twelve_problems():
    """The batching form's twelve problems (grids 128-384, 16-64 members, 0-44
    local observations, FP32 storage): one cycle batched against each problem's
    own run_cycle (the single-problem path is the one pinned to the oracle)."""
    say("batch: twelve-problem configuration")
    cfgs = inputs.batch_configs()
    probs = _setup(cfgs, F32, cycles=1)
    single = _single_runs(probs, 1)
    batched = _batch_runs(probs, 1)
    for cfg, s, b in zip(cfgs, single, batched):
        assert np.array_equal(s, b), cfg.name


def test_batch_argument_errors():
    say("batch argument errors")
    base = inputs.CONFIGS["tiny"]
    c1, _, _, m1 = _problem(base, F64)
    c2, _, _, m2 = _problem(base.replace(name="x", members=3, seed=5), F64)
    f1 = c1.init_equilibrium(m1)
    f2 = c2.init_equilibrium(m2)
    with pytest.raises(binding.LbmLetkfError) as e:      # 3 members do not divide 256
        binding.Batch([c1, c2], [f1, f2], 10)
    assert e.value.status == -8
    c3, _, _, m3 = _problem(base, F32)
    f3 = c3.init_equilibrium(m3)
    with pytest.raises(binding.LbmLetkfError) as e:      # mixed storage
        binding.Batch([c1, c3], [f1, f3], 10)
    assert e.value.status == -8
    c4, _, _, m4 = _problem(base, F64)
    with pytest.raises(binding.LbmLetkfError) as e:      # one state bound twice
        binding.Batch([c1, c4], [f1, f1], 10)
    assert e.value.status == -1
    c5, _, _, m5 = _problem(base, F64)
    c6 = binding.Context.from_config(base, members=1, storage=F64)
    f6 = c6.init_equilibrium(m5[:1].contiguous())
    with pytest.raises(binding.LbmLetkfError) as e:      # one member: no analysis
        binding.Batch([c5, c6], [c5.init_equilibrium(m5), f6], 10)
    assert e.value.status == -1
    # two steps per launch need 16 | members (tiny has 8); the count must be 1 or 2
    with pytest.raises(binding.LbmLetkfError) as e:
        binding.Batch([c1], [f1], 10, config=dict(forecast_blocks=0, tile_rows=2,
                                                  bucket_granularity=2, use_graph=0,
                                                  steps_per_launch=2))
    assert e.value.status == -8
    with pytest.raises(binding.LbmLetkfError) as e:
        binding.Batch([c1], [f1], 10, config=dict(forecast_blocks=0, tile_rows=2,
                                                  bucket_granularity=2, use_graph=0,
                                                  steps_per_launch=3))
    assert e.value.status == -1
