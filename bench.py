"""Benchmark of the LBM-LETKF forecast-analysis cycle on one MI355X.

One "step" is one full data-assimilation cycle of the hot path: s = 20
stream-collide steps of all 64 members on 256^2, the observation operator,
the observation-space statistics, the per-node LETKF analysis and the cycle
diagnostics (forecast and analysis RMSE against the truth).  The truth run
and the noisy observations are generated on the GPU before the timed region
and stay resident in HBM.

Prints one JSON line: DA cycles/s (value), GLUPS*member, the mean analysis
RMSE and spread of the timed cycles, the energy spectrum against the nature
run at the report cycles (an untimed re-run of the same cycles), the run
against the FP64 oracle's stored series (tests/golden, when present), the
roofline of the dominant kernel measured with HIP events on the launch
stream, and the FP64 oracle timed on the host cores (cpu_baseline: two whole
cycles, every node analysed).

    python bench.py [--steps K] [--warmup W] [--config paper] [--route auto|ensemble|observation]
"""
from __future__ import annotations

import argparse
import json
import math
import mmap
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("DA cycles/s and GLUPS·member at 256² / 64 members vs plain GPU form, "
          "at equal RMSE")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector, TFLOP/s
BYTES_PER_NODE_MEMBER = 144.0  # 9 loads + 9 stores of FP64 per node and member


def traffic_record(kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 PMC summary in
    profiles/ (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy), or
    None when the kernel's sources changed after the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel") != kernel:
                continue
            h = hashlib.sha256()
            for src in rec["sources"]:
                h.update(open(os.path.join(ROOT, src), "rb").read())
            if h.hexdigest() == rec["sources_sha256"]:
                return rec
    return None


def two_step_bytes(n: int, members: int, elem: int) -> int:
    """Algorithmic bytes of one two-step launch over an n x n grid: per member,
    every 6 x 6 tile's 8 x 8 node region read once (9 populations) and the
    interior written once; the intermediate step stays on chip."""
    tiles = (-(-n // 6)) ** 2
    return members * (tiles * 64 + n * n) * 9 * elem


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def analysis_flops_per_node(route: int, members: int, n_local: float, n_eig: int) -> float:
    """Algorithmic FP64 work of one node's analysis, textbook operation counts.

    Ensemble route: A = aI + Z^T Z (l M^2), the M x M symmetric
    eigendecomposition with vectors counted at the textbook 9 M^3, the
    weights (2 M^3) and the transform of the 9 populations (2*9*M^2).
    Observation route: S = Z Z^T from the Gram matrix (l^2), the l x l
    eigendecomposition (9 l^3), the weight factors (4 l^2 + ...), B = dX Z^T
    and the transform (2 * 2*9*l*M)."""
    M, l = float(members), float(n_local)
    if route == 2:
        return 2 * l * l + 9 * l ** 3 + 4 * l * l + 2 * 2 * 9 * l * M + 2 * 9 * l * l
    return 2 * l * M * M + 9 * M ** 3 + 2 * M ** 3 + 2 * 9 * M * M


_CPU_JOB = {}


def _cpu_analysis_chunk(nodes):
    """Worker: the oracle analysis of `nodes`, written into the shared output.
    One BLAS thread per worker: the workers already fill the cores, and
    NumPy's BLAS would otherwise start OMP_NUM_THREADS threads in each."""
    import oracle
    from threadpoolctl import threadpool_limits
    j = _CPU_JOB
    with threadpool_limits(limits=1):
        j["out"][:, :, nodes] = oracle.letkf_analysis(j["f"], j["yf"], j["yo"], j["pts"],
                                                      j["sigmas"], j["d_cut"], j["beta"],
                                                      nodes=nodes)
    return len(nodes)


def cpu_baseline(cfg, force, pts, sample_cycles: int, procs: int):
    """The FP64 oracle on the host: `sample_cycles` whole cycles of the
    workload (s LBM steps of the full ensemble in the C oracle on OpenMP
    threads, H, and the oracle analysis of every node, mapped over node
    subsets in `procs` processes), timed per stage.  Runs before the GPU is
    initialised (the analysis workers are forked)."""
    import multiprocessing as mp
    import oracle
    from paper_2308_03972_amd import inputs
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    fe = oracle.equilibrium(np.ones((cfg.members, cfg.n, cfg.n)), mem_uv[:, 0], mem_uv[:, 1])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nodes = np.arange(cfg.n * cfg.n)
    t_lbm = t_an = 0.0
    for c in range(sample_cycles):
        t0 = time.perf_counter()
        fe = oracle.lbm_steps(fe, cfg.steps_per_cycle, cfg.tau0, cfg.cs, force, cfg.mu)
        t_lbm += time.perf_counter() - t0
        yf = oracle.observe(fe, pts, cfg.nvar)
        t0 = time.perf_counter()
        # the workers (forked) write into a shared anonymous mapping
        shared = mmap.mmap(-1, fe.nbytes)
        out = np.frombuffer(shared, dtype=np.float64).reshape(cfg.members, 9, cfg.n * cfg.n)
        _CPU_JOB.update(f=fe, yf=yf, yo=yf.mean(axis=0), pts=pts, sigmas=cfg.sigmas,
                        d_cut=cfg.d_cut, beta=cfg.beta, out=out)
        with mp.get_context("fork").Pool(procs) as pool:
            pool.map(_cpu_analysis_chunk, np.array_split(nodes, 8 * procs))
        fe = out.reshape(fe.shape).copy()
        _CPU_JOB.clear()
        del out
        shared.close()
        t_an += time.perf_counter() - t0
    t_cycle = (t_lbm + t_an) / sample_cycles
    # one LBM step on one thread, and one node's analysis in this process
    t_step1 = None
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        oracle.lbm_steps(fe, 1, cfg.tau0, cfg.cs, force, cfg.mu)
        t_step1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
    except OSError:
        pass
    yf = oracle.observe(fe, pts, cfg.nvar)
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        oracle.letkf_analysis(fe, yf, yf.mean(axis=0), pts, cfg.sigmas, cfg.d_cut, cfg.beta,
                              nodes=nodes[:2048])
    t_node1 = (time.perf_counter() - t0) / 2048
    return {
        "value": 1.0 / t_cycle, "unit": "cycles/s", "cores": max(threads, procs), "kind": "oracle",
        "sample": (f"{sample_cycles} whole oracle cycles of the {cfg.n}^2 x {cfg.members} workload: "
                   f"{cfg.steps_per_cycle} LBM steps (C, OpenMP {threads} threads) + the analysis "
                   f"of all {cfg.n * cfg.n} nodes (NumPy/LAPACK eigh, node subsets in {procs} "
                   "processes)"),
        "cores_per_leg": {"lbm_openmp_threads": threads, "analysis_processes": procs},
        "s_per_lbm_step": t_lbm / (sample_cycles * cfg.steps_per_cycle),
        "s_per_analysis": t_an / sample_cycles,
        "s_per_lbm_step_1_thread": t_step1,
        "s_per_node_analysis_1_process": t_node1,
    }


def observations(cfg, tctx, total: int, report=()):
    """Truth run (M = 1 context) and the observation sets of `total` cycles,
    resident on the GPU: y_o per cycle, the truth velocity per cycle, and the
    truth's energy spectrum at the report cycles (1-based)."""
    import torch
    from paper_2308_03972_amd import binding, inputs
    dev = torch.device("cuda:0")
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    truth_uv, _ = inputs.initial_velocities(cfg)
    noise = cuda(inputs.all_observation_noise(cfg, total))
    sig = cuda(inputs.sigma_vector(cfg))
    ft = tctx.init_equilibrium(cuda(truth_uv[None]))
    yo_all = torch.empty((total, cfg.n_obs), dtype=torch.float64, device=dev)
    tuv_all = torch.empty((total, 2, cfg.n, cfg.n), dtype=torch.float64, device=dev)
    spectra = {}
    for c in range(total):
        tctx.step(ft, cfg.steps_per_cycle)
        ytrue = tctx.observe(ft)[0].contiguous()
        yo_all[c] = binding.synth_obs(ytrue, noise[c].contiguous(), sig)
        tuv_all[c] = tctx.moments(ft)[0, 1:]
        if c + 1 in report:
            spectra[c + 1] = tctx.energy_spectrum(ft, cfg.n // 2).cpu().numpy()
    torch.cuda.synchronize()
    return yo_all, tuv_all, spectra


def spectra_pass(ctx, cfg, yo_all, tuv_all, report):
    """Untimed re-run of the cycles from the initial ensemble (the same
    deterministic states as the timed runs): member-mean energy spectrum of
    the analysis ensemble at the report cycles, and every cycle's diagnostics."""
    import torch
    from paper_2308_03972_amd import binding, inputs
    dev = torch.device("cuda:0")
    _, mem_uv = inputs.initial_velocities(cfg)
    fe = ctx.init_equilibrium(torch.from_numpy(np.ascontiguousarray(mem_uv)).to(dev))
    total = yo_all.shape[0]
    diag = torch.zeros((total, 2 * binding.DIAG_LEN), dtype=torch.float64, device=dev)
    spectra = {}
    for c in range(total):
        ctx.run_cycle(fe, cfg.steps_per_cycle, yo_all[c], tuv_all[c], diag[c])
        if c + 1 in report:
            spectra[c + 1] = ctx.energy_spectrum(fe, cfg.n // 2).cpu().numpy()
    ctx.check(diag[-1])   # raises on a non-finite, unconverged or diverged run
    return spectra, diag.cpu().numpy()


def spectrum_error(got, ref, n, kmax=None):
    """max over 1 <= k <= kmax (default n/3) of |E_got(k) - E_ref(k)| / E_ref(k)."""
    k = np.arange(1, (n // 3 if kmax is None else kmax) + 1)
    return float(np.max(np.abs(got[k] - ref[k]) / ref[k]))


def golden(name):
    """The FP64 oracle's stored series (tests/golden, written by the oracle's
    own script), or None."""
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    return dict(np.load(path, allow_pickle=False))


def versus_oracle(g, d, spectra, n, cycles):
    """Per-cycle RMSE and spread of a run (diagnostics d, cycles 1..len(d)) and its
    analysis spectra at report cycles against the oracle's stored series."""
    m = min(len(d), len(g["rmse_a"]), cycles)
    out = {"cycles_compared": int(m)}
    for k, col in (("rmse_f", 0), ("rmse_a", 8), ("spread_f", 1), ("spread_a", 9)):
        ref = g[k][:m]
        out[f"max_rel_diff_{k}"] = float(np.max(np.abs(d[:m, col] / ref - 1)))
        out[f"max_abs_diff_{k}"] = float(np.max(np.abs(d[:m, col] - ref)))
    errs = [spectrum_error(spectra[int(c)], g["spectrum_a"][i][: n // 2 + 1], n)
            for i, c in enumerate(g["report_cycle"]) if int(c) in spectra]
    if errs:
        out["spectrum_error_vs_oracle_max_k_le_n3"] = max(errs)
        # FP32 storage: the tail k > 32 falls below the state's rounding floor
        out["spectrum_error_vs_oracle_max_k_le_32"] = max(
            spectrum_error(spectra[int(c)], g["spectrum_a"][i][: n // 2 + 1], n, 32)
            for i, c in enumerate(g["report_cycle"]) if int(c) in spectra)
        out["spectrum_report_cycles"] = [int(c) for c in g["report_cycle"] if int(c) in spectra]
    return out


def run_form(ctx, cfg, yo_all, tuv_all, warmup: int, steps: int, repeats: int = 1,
             breakdown_cycles: int = 5):
    """Warmup + timed cycles of one form, `repeats` times from the same initial
    ensemble.  Returns per repeat (elapsed s, diagnostics of the timed cycles,
    stage ms and launch counts of the timed region) and the stage ms per cycle of
    a per-launch pass after the last repeat."""
    import torch
    from paper_2308_03972_amd import binding, inputs
    dev = torch.device("cuda:0")
    _, mem_uv = inputs.initial_velocities(cfg)
    mem = torch.from_numpy(np.ascontiguousarray(mem_uv, dtype=np.float64)).to(dev)
    s, total = cfg.steps_per_cycle, warmup + steps
    runs = []
    for _ in range(repeats):
        diag = torch.zeros((total, 2 * binding.DIAG_LEN), dtype=torch.float64, device=dev)
        fe = ctx.init_equilibrium(mem)
        for c in range(warmup):
            ctx.run_cycle(fe, s, yo_all[c], tuv_all[c], diag[c])
        torch.cuda.synchronize()
        # timed region: HIP events on the launch stream around each cycle's
        # forecast steps and around each analysis (level 2: one pair each)
        ctx.set_profiling(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(warmup, total):
            ctx.run_cycle(fe, s, yo_all[c], tuv_all[c], diag[c])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ms, n = ctx.profile_collect()
        ctx.set_profiling(False)
        runs.append((el, diag[warmup:].cpu().numpy(), ms, n))
    # stage breakdown: a few more cycles with an event pair around every launch
    scratch = torch.zeros(2 * binding.DIAG_LEN, dtype=torch.float64, device=dev)
    ctx.set_profiling(True)
    for c in range(total - breakdown_cycles, total):
        ctx.run_cycle(fe, s, yo_all[c], tuv_all[c], scratch)
    ms1, _ = ctx.profile_collect()
    ctx.set_profiling(False)
    breakdown = {binding.STAGES[k]: round(ms1[k] / breakdown_cycles, 4)
                 for k in range(binding.NSTAGES)}
    return runs, breakdown


def median_run(runs):
    """The repeat with the median elapsed time."""
    return sorted(runs, key=lambda r: r[0])[len(runs) // 2]


def f32_forecast_roofline(cfg, t_step: float) -> dict:
    """The FP32 two-step forecast kernel (stream_collide2_dev) against the HBM
    roofline at its own bytes; `t_step` is the library's per-step time (two
    steps per launch when 16 divides the member count)."""
    two = cfg.members % 16 == 0
    t = t_step * (2 if two else 1)
    b = two_step_bytes(cfg.n, cfg.members, 4) if two else 72 * cfg.n * cfg.n * cfg.members
    kname = "stream_collide2_dev_kernel" if two else "stream_collide_kernel"
    rec = traffic_record(kname) if two and cfg.name == "paper" else None
    gbs = b / t / 1e9
    return {"kernel": kname.replace("_kernel", ""), "bound": "hbm", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": rec["bytes_per_launch"] if rec else None, "algorithmic_bytes": int(b),
            "steps_per_launch": 2 if two else 1, "avg_launch_us": round(t * 1e6, 2)}


def precision_config_form(cycles: int):
    """The precision form at its own configuration (512^2, 64 members, 16x16
    (u, v) observations, s = 20) beside the plain FP64 form on the same
    observations, each run `cycles` cycles from the initial ensemble (5 warmup
    cycles, the rest timed): cycles/s of both, the RMSE difference between
    them, and both runs against the FP64 oracle's stored series (per-cycle
    RMSE and the analysis spectrum at the report cycles), when present."""
    from paper_2308_03972_amd import binding, inputs
    import torch
    cfg = inputs.CONFIGS["precision"]
    warmup, steps = 5, cycles - 5
    dev = torch.device("cuda:0")
    force = torch.from_numpy(np.ascontiguousarray(inputs.body_force(cfg))).to(dev)
    tctx = binding.Context.from_config(cfg, members=1, force=force)
    g = golden("cycle_512x512x64_100cycles.npz")
    report = [int(c) for c in g["report_cycle"] if int(c) <= cycles] if g is not None else []
    yo_all, tuv_all, tspec = observations(cfg, tctx, cycles, report)
    out = {"workload": (f"{cfg.n}x{cfg.n}, {cfg.members} members, {cfg.obs_side}x{cfg.obs_side} "
                        f"(u,v) observations, s={cfg.steps_per_cycle}, r={cfg.loc_r:g}, "
                        f"{cycles} cycles ({warmup} warmup)")}
    res = {}
    for name, storage, mfma in (("plain", binding.STORAGE_F64, False),
                                ("f32_dev", binding.STORAGE_F32_DEV, False),
                                ("f32_dev_mfma_transform", binding.STORAGE_F32_DEV, True)):
        ctx = binding.Context.from_config(cfg, force=force, storage=storage)
        ctx.set_matrix_core_transform(mfma)
        runs, _ = run_form(ctx, cfg, yo_all, tuv_all, warmup, steps, 1, breakdown_cycles=1)
        el, d, ms, n = runs[0]
        res[name] = (el, d)
        out[f"{name}_cycles_per_s"] = round(steps / el, 3)
        out[f"{name}_stream_collide_us_per_step"] = round(1e3 * ms[0] / max(n[0], 1), 2)
        out[f"{name}_analysis_ms"] = round(ms[3] / max(n[3], 1), 4)
        if storage == binding.STORAGE_F32_DEV and not mfma:
            out[f"{name}_roofline_forecast"] = f32_forecast_roofline(cfg, 1e-3 * ms[0]
                                                                     / max(n[0], 1))
        if g is not None:
            spec, dall = spectra_pass(ctx, cfg, yo_all, tuv_all, report)
            out[f"{name}_vs_fp64_oracle"] = versus_oracle(g, dall, spec, cfg.n, cycles)
        ctx.close()
    out["speedup_vs_plain"] = round(res["plain"][0] / res["f32_dev"][0], 4)
    out["mfma_transform_speedup_vs_f32_dev"] = round(res["f32_dev"][0]
                                                     / res["f32_dev_mfma_transform"][0], 4)
    out["max_abs_rmse_a_diff_vs_plain"] = float(np.max(np.abs(
        res["f32_dev"][1][:, binding.DIAG_LEN] - res["plain"][1][:, binding.DIAG_LEN])))
    out["tolerance_1e-3_sigma"] = 1e-3 * cfg.sigma
    tctx.close()
    return out


def differentiation_form(reps: int, storage: int):
    """Misfit gradient of the differentiation workload (128^2, 16 members, 8x8
    (u, v) observations, 10 observation times 20 steps apart, a checkpoint at
    each): forward sweep + reverse sweep, inputs resident on the GPU."""
    import torch
    from paper_2308_03972_amd import binding, inputs
    cfg = inputs.CONFIGS["differentiation"]
    dev = torch.device("cuda:0")
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    s, times = cfg.steps_per_cycle, cfg.cycles
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    force = cuda(inputs.body_force(cfg))
    tctx = binding.Context.from_config(cfg, members=1, force=force)
    ctx = binding.Context.from_config(cfg, force=force, storage=storage)
    # members and truth spun up one observation interval from their fields
    f0 = ctx.init_equilibrium(cuda(mem_uv))
    ctx.step(f0, s)
    ft = tctx.init_equilibrium(cuda(truth_uv[None]))
    tctx.step(ft, s)
    noise = cuda(inputs.all_observation_noise(cfg, times))
    sig = cuda(inputs.sigma_vector(cfg))
    yo = torch.empty((times, cfg.n_obs), dtype=torch.float64, device=dev)
    for c in range(times):
        tctx.step(ft, s)
        yo[c] = binding.synth_obs(tctx.observe(ft)[0].contiguous(), noise[c].contiguous(), sig)
    work = ctx.adjoint_workspace(s, times)

    def one():
        J = ctx.misfit_forward(f0, cfg.cs, s, yo, work)
        g, gcs = ctx.misfit_backward(f0, cfg.cs, s, yo, work)
        return J, g, gcs

    for _ in range(3):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        J, g, gcs = one()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # per-kernel durations: HIP events around every launch, a second pass
    ctx.set_profiling(True)
    for _ in range(reps):
        one()
    ms, n = ctx.profile_collect()
    ctx.set_profiling(False)
    plane = cfg.n * cfg.n
    elem = 4 if storage == binding.STORAGE_F32_DEV else 8
    # adjoint step: 9 state loads (storage type), 9 FP64 adjoint loads and 9 stores
    adj_bytes = (9 * elem + 2 * 9 * 8) * plane * cfg.members
    t_adj = ms[5] / max(n[5], 1) * 1e-3
    t_col = ms[0] / max(n[0], 1) * 1e-3
    gbs = adj_bytes / t_adj / 1e9
    rec = traffic_record("adjoint_step_kernel") if storage == binding.STORAGE_F32_DEV else None
    return {
        "workload": (f"{cfg.n}x{cfg.n}, {cfg.members} members, {cfg.obs_side}x{cfg.obs_side} "
                     f"(u,v) observations, {times} observation times {s} steps apart "
                     f"({times * s} steps, a checkpoint every {s})"),
        "storage": "FP32 f - w" if elem == 4 else "FP64",
        "gradients_per_s": round(reps / el, 3),
        "ms_per_gradient": round(1e3 * el / reps, 4),
        # the library counts forecast steps, two per two-step launch
        "forecast_steps_per_gradient": int(n[0] // reps),
        "launches_per_gradient": {"adjoint": int(n[5] // reps), "misfit": int(n[6] // reps)},
        "J": float(J.item()), "dJ_dCs": float(gcs.item()),
        "grad_f0_norm": float(torch.linalg.vector_norm(g).item()),
        "stream_collide_us_per_step": round(t_col * 1e6, 2),
        "roofline_adjoint": {"kernel": "adjoint_step", "bound": "hbm", "achieved": round(gbs, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "traffic": rec["bytes_per_launch"] if rec else None,
                             "algorithmic_bytes": int(adj_bytes),
                             "avg_launch_us": round(t_adj * 1e6, 2)},
    }


def batching_form(cycles: int, warmup: int):
    """The twelve-problem batch (grids 128-384, 16-64 members, 0-44 local
    observations, FP32 storage, s = 20): autotuned, cycle replayed from its
    hipGraph, against the same problems run one after another through
    run_cycle (no graph)."""
    import torch
    from paper_2308_03972_amd import binding, inputs
    dev = torch.device("cuda:0")
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    cfgs = inputs.batch_configs()
    total = warmup + cycles
    ctxs, mem, yos = [], [], []
    for cfg in cfgs:
        force = cuda(inputs.body_force(cfg))
        ctx = binding.Context.from_config(cfg, force=force, storage=binding.STORAGE_F32_DEV)
        tctx = binding.Context.from_config(cfg, members=1, force=force)
        truth_uv, mem_uv = inputs.initial_velocities(cfg)
        ft = tctx.init_equilibrium(cuda(truth_uv[None]))
        noise = cuda(inputs.all_observation_noise(cfg, total))
        sig = cuda(inputs.sigma_vector(cfg))
        yo = []
        for c in range(total):
            tctx.step(ft, cfg.steps_per_cycle)
            yo.append(binding.synth_obs(tctx.observe(ft)[0].contiguous(), noise[c].contiguous(),
                                        sig))
        ctxs.append(ctx)
        mem.append(cuda(mem_uv))
        yos.append(yo)
    s = cfgs[0].steps_per_cycle
    node_members = sum(c.n * c.n * c.members for c in cfgs)
    # sequential: every problem through run_cycle, one after another
    states = [c.init_equilibrium(m) for c, m in zip(ctxs, mem)]
    for c in range(warmup):
        for k, ctx in enumerate(ctxs):
            ctx.run_cycle(states[k], s, yos[k][c])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(warmup, total):
        for k, ctx in enumerate(ctxs):
            ctx.run_cycle(states[k], s, yos[k][c])
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    seq_states = [st.clone() for st in states]
    # batched, tuned, graph replay
    states = [c.init_equilibrium(m) for c, m in zip(ctxs, mem)]
    batch = binding.Batch(ctxs, states, s)
    # tune on cycled states: the Jacobi sweep count, hence the analysis cost,
    # grows once the analyses have correlated the members
    for c in range(warmup):
        batch.run_cycle([yos[k][c] for k in range(len(cfgs))])
    cfg_best, fms, ams = batch.tune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(warmup, total):
        batch.run_cycle([yos[k][c] for k in range(len(cfgs))])
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(states, seq_states))
    maxdiff = max(float((a.double() - b.double()).abs().max()) for a, b in zip(states, seq_states))
    batch.close()
    # the tuner's forecast time is per step; with two steps per launch the
    # launch is priced at the two-step kernel's own bytes (region read once,
    # interior written once), else at one step's 72 B per node-member (FP32)
    two = int(cfg_best.get("steps_per_launch", 1)) == 2
    fc_bytes = (sum(two_step_bytes(c.n, c.members, 4) for c in cfgs) if two
                else 72.0 * node_members)
    t_fc = fms * 1e-3 * (2 if two else 1)
    kname = "stream_collide2_batch_kernel" if two else "stream_collide_batch_kernel"
    rec = traffic_record(kname)
    gbs = fc_bytes / t_fc / 1e9
    return {
        "workload": ("12 problems: grids {128,192,256,384}^2 x members {16,32,64}, "
                     "observation grids 4x4..32x32, 0-44 local observations, FP32 f - w, s=20"),
        "node_members_per_step": node_members,
        "cycles_per_s": round(cycles / bt, 3),
        "glups_member": round(node_members * s * cycles / bt / 1e9, 3),
        "sequential_cycles_per_s": round(cycles / seq, 3),
        "speedup_vs_sequential": round(seq / bt, 4),
        "tuned_config": cfg_best,
        "tuned_forecast_ms_per_step": round(fms, 4),
        "tuned_analysis_ms": round(ams, 4),
        "states_equal_to_sequential": same,
        "max_abs_state_diff_vs_sequential": maxdiff,
        "roofline_forecast": {"kernel": kname.replace("_kernel", ""), "bound": "hbm",
                              "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(gbs / HBM_PEAK_GBS, 4),
                              "traffic": rec["bytes_per_launch"] if rec else None,
                              "algorithmic_bytes": int(fc_bytes),
                              "steps_per_launch": 2 if two else 1,
                              "avg_launch_us": round(t_fc * 1e6, 2)},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=190, help="timed DA cycles")
    ap.add_argument("--warmup", type=int, default=10, help="untimed DA cycles before timing")
    ap.add_argument("--config", default="paper")
    ap.add_argument("--route", default="auto", choices=["auto", "ensemble", "observation"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision, batching and differentiation forms")
    ap.add_argument("--batch-cycles", type=int, default=20,
                    help="timed cycles of the batching form")
    ap.add_argument("--grad-reps", type=int, default=20,
                    help="timed misfit gradients of the differentiation form")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs of the plain and precision forms (value: the median)")
    ap.add_argument("--precision-cycles", type=int, default=100,
                    help="timed cycles of each form at the precision configuration (512^2)")
    ap.add_argument("--cpu-cycles", type=int, default=6,
                    help="whole oracle cycles timed for the CPU baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-GPU by design and has no multi-GPU mode.", file=sys.stderr)
        return 2

    from paper_2308_03972_amd import inputs
    cfg = inputs.CONFIGS[args.config]
    cpu = None
    if not args.no_cpu_baseline and not args.calibrate_copy:
        # before the GPU is initialised: the oracle's analysis workers are forked
        log("timing the FP64 oracle on the host (bounded sample)")
        procs = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = cpu_baseline(cfg, inputs.body_force(cfg), inputs.observation_points(cfg),
                           args.cpu_cycles, procs)

    import torch
    from paper_2308_03972_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        # a copy kernel that reads and writes exactly MIB MiB each, 5 launches
        n = args.calibrate_copy * 2**20 // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_mib": args.calibrate_copy, "launches": 5}), flush=True)
        return 0
    route = {"auto": 0, "ensemble": 1, "observation": 2}[args.route]
    total = args.warmup + args.steps
    s = cfg.steps_per_cycle
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    # ---- inputs: seeded fields, force, observing network --------------------
    force_np = inputs.body_force(cfg)
    pts = inputs.observation_points(cfg)
    force = cuda(force_np)
    tctx = binding.Context.from_config(cfg, members=1, force=force)
    ectx = binding.Context.from_config(cfg, force=force, route=route)
    log(f"config {cfg.name}: {cfg.n}^2 x {cfg.members}, route {ectx.route}, eig size "
        f"{ectx.eig_size}, max local points {ectx.max_local_points}")

    # ---- truth run and observations, all resident before timing -------------
    report = [c for c in range(50, total + 1, 50)]
    yo_all, tuv_all, truth_spectra = observations(cfg, tctx, total, report)
    log(f"truth and {total} observation sets ready")

    runs, breakdown = run_form(ectx, cfg, yo_all, tuv_all, args.warmup, args.steps, args.repeats)
    elapsed, d, stage_ms, stage_n = median_run(runs)
    log(f"plain form: timed {args.steps} cycles in " + ", ".join(f"{r[0]:.3f}" for r in runs)
        + f" s (median {elapsed:.3f} s)")
    # ---- spectra at the report cycles (untimed re-run of the same cycles) --------
    spectra, dall = spectra_pass(ectx, cfg, yo_all, tuv_all, report)
    spec = {"report_cycles": report,
            "definition": "member-mean shell spectrum of the analysis ensemble (lbmletkf_energy_"
                          "spectrum) vs the nature run's; error = max over 1 <= k <= n/3 of "
                          "|E_a(k) - E_t(k)| / E_t(k)",
            "error_vs_nature_run": [round(spectrum_error(spectra[c], truth_spectra[c], cfg.n), 5)
                                    for c in report],
            "E_analysis_k1_k4_k16_k64": [[float(spectra[c][k]) for k in (1, 4, 16, 64)
                                          if k < len(spectra[c])] for c in report],
            "E_truth_k1_k4_k16_k64": [[float(truth_spectra[c][k]) for k in (1, 4, 16, 64)
                                       if k < len(truth_spectra[c])] for c in report]}
    g = golden("cycle_256x256x64_200cycles.npz") if cfg.name == "paper" else None
    vs_oracle = versus_oracle(g, dall, spectra, cfg.n, total) if g is not None else None

    forms = {}
    if not args.no_forms:
        f32ctx = binding.Context.from_config(cfg, force=force, route=route,
                                             storage=binding.STORAGE_F32_DEV)
        runs32, _ = run_form(f32ctx, cfg, yo_all, tuv_all, args.warmup, args.steps, args.repeats)
        el32, d32, ms32, n32 = median_run(runs32)
        log(f"precision form: timed {args.steps} cycles in {el32:.3f} s (median)")
        log("precision form at its own configuration (512^2)")
        forms["f32_dev_512"] = precision_config_form(max(args.precision_cycles, 6))
        log(f"precision form at 512^2: {forms['f32_dev_512']['speedup_vs_plain']}x plain")
        log("batching form: twelve problems")
        forms["batching"] = batching_form(args.batch_cycles, 3)
        log(f"batching: {forms['batching']['cycles_per_s']} cycles/s "
            f"({forms['batching']['speedup_vs_sequential']}x sequential)")
        for name, st in (("differentiation", binding.STORAGE_F32_DEV),
                         ("differentiation_f64", binding.STORAGE_F64)):
            forms[name] = differentiation_form(args.grad_reps, st)
            log(f"{name}: {forms[name]['ms_per_gradient']} ms per gradient")
        forms["f32_dev"] = {
            "storage": ("FP32 f - w; FP32 relaxation; Gram matrices on FP32 matrix cores; "
                        "FP64 eigensolve, weights and apply"),
            "cycles_per_s": round(args.steps / el32, 3),
            "speedup_vs_plain": round(elapsed / el32, 4),
            "stream_collide_us_per_step": round(1e3 * ms32[0] / max(n32[0], 1), 2),
            "roofline_forecast": f32_forecast_roofline(cfg, 1e-3 * ms32[0] / max(n32[0], 1)),
            "rmse_a_mean": float(d32[:, binding.DIAG_LEN].mean()),
            "max_abs_rmse_a_diff_vs_plain": float(np.max(np.abs(
                d32[:, binding.DIAG_LEN] - d[:, binding.DIAG_LEN]))),
            "tolerance_1e-3_sigma": 1e-3 * cfg.sigma,
        }

    rmse_f, rmse_a = d[:, 0], d[:, binding.DIAG_LEN]
    nonfinite = float(d[:, 2].sum() + d[:, binding.DIAG_LEN + 2].sum())
    cycles_per_s = args.steps / elapsed
    plane = cfg.n * cfg.n
    glups = plane * cfg.members * s * cycles_per_s / 1e9

    # ---- roofline of the dominant kernel ----------------------------------------
    per_launch = {binding.STAGES[k]: (stage_ms[k] / stage_n[k] if stage_n[k] else 0.0)
                  for k in range(binding.NSTAGES)}
    per_cycle = {binding.STAGES[k]: stage_ms[k] / args.steps for k in range(binding.NSTAGES)}
    t_lbm = per_launch["stream_collide"] * 1e-3  # per step (the timer counts steps)
    t_an = per_launch["analysis"] * 1e-3
    lbm_gbs = BYTES_PER_NODE_MEMBER * plane * cfg.members / t_lbm / 1e9
    # the library runs two steps per launch for FP64 storage when 16 divides M
    # (stream_collide2_kernel); its launch moves two steps' algorithmic bytes
    # and its real HBM traffic (PMC) is below them, since the intermediate
    # state stays on chip
    lbm_steps_per_launch = 2 if cfg.members % 16 == 0 else 1
    # each node priced at its own local observation count (the planner's
    # histogram of local points per node)
    hist = ectx.local_histogram()
    an_flops = float(sum(int(cnt) * analysis_flops_per_node(ectx.route, cfg.members,
                                                            cfg.nvar * k, ectx.eig_size)
                         for k, cnt in enumerate(hist) if cnt))
    n_local = cfg.nvar * float(np.dot(np.arange(len(hist)), hist)) / max(1, int(hist.sum()))
    an_tflops = an_flops / t_an / 1e12
    lbm_kernel = "stream_collide2_kernel" if lbm_steps_per_launch == 2 else "stream_collide_kernel"
    rec = traffic_record(lbm_kernel) if cfg.name == "paper" else None
    an_rec = traffic_record("analysis") if cfg.name == "paper" else None
    t_launch = t_lbm * lbm_steps_per_launch
    single_step_bytes = BYTES_PER_NODE_MEMBER * plane * cfg.members * lbm_steps_per_launch
    if lbm_steps_per_launch == 2:
        # the two-step launch's own algorithmic bytes: per 16-member block, the
        # 8 x 8 node region read once (9 FP64 pulls per node) and the 6 x 6
        # interior written once; the intermediate step stays in LDS
        kernel_bytes = two_step_bytes(cfg.n, cfg.members, 8)
    else:
        kernel_bytes = single_step_bytes
    kernel_gbs = kernel_bytes / t_launch / 1e9
    rl_lbm = {"kernel": lbm_kernel.replace("_kernel", ""), "bound": "hbm",
              "achieved": round(kernel_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(kernel_gbs / HBM_PEAK_GBS, 4),
              "traffic": rec["bytes_per_launch"] if rec else None,
              "algorithmic_bytes": int(kernel_bytes),
              "steps_per_launch": lbm_steps_per_launch,
              "avg_launch_us": round(t_launch * 1e6, 2),
              # the same launch priced at two single steps' bytes (144 B per
              # node-member and step): a rate, not a roofline fraction
              "effective_gbs_single_step_bytes": round(single_step_bytes / t_launch / 1e9, 1)}
    if lbm_steps_per_launch == 2:
        rl_lbm["bytes_note"] = ("algorithmic_bytes: the two-step tile kernel's own reads (8x8 "
                                "region per 6x6 tile) and writes; 288 B per node-member of two "
                                "single steps would exceed the HBM roofline by design")
    if rec:
        rl_lbm["traffic_source"] = ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE summary in profiles/ "
                                    "from the builder's run (sources hash-matched), not this run")
        rl_lbm["hbm_gbs_from_traffic"] = round(rec["bytes_per_launch"] / t_launch / 1e9, 1)
        rl_lbm["frac_from_traffic"] = round(rec["bytes_per_launch"] / t_launch / 1e9
                                            / HBM_PEAK_GBS, 4)
    rl_an = {"kernel": "analysis", "bound": "alu", "achieved": round(an_tflops, 3),
             "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": round(an_tflops / FP64_PEAK_TFLOPS, 4),
             "traffic": an_rec["bytes_per_launch"] if an_rec else None,
             "traffic_note": "HBM bytes of one analysis (all node-group launches)",
             "algorithmic_flops": round(an_flops),
             "mean_local_obs": round(n_local, 3),
             "avg_launch_us": round(per_launch["analysis"] * 1e3, 2)}
    if an_rec:
        rl_an["traffic_source"] = ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE summary in profiles/ "
                                   "from the builder's run (sources hash-matched), not this run")
    dominant = rl_lbm if per_cycle["stream_collide"] >= per_cycle["analysis"] else rl_an
    other = rl_an if dominant is rl_lbm else rl_lbm

    out = {
        "metric": METRIC,
        "value": round(cycles_per_s, 3),
        "unit": "cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"plain FP64 forecast-analysis cycle, {cfg.n}x{cfg.n} D2Q9 "
                         f"BGK-Smagorinsky, {cfg.members} members, {cfg.obs_side}x{cfg.obs_side} "
                         f"(u,v) observations, s={s}, r={cfg.loc_r:g}, beta={cfg.beta}"),
            "grid": cfg.n, "members": cfg.members, "steps_per_cycle": s,
            "obs_points": cfg.n_points, "route": ["", "ensemble", "observation"][ectx.route],
            "eig_size": ectx.eig_size,
        },
        "repeats_cycles_per_s": [round(args.steps / r[0], 3) for r in runs],
        "glups_member": round(glups, 3),
        "glups_member_stream_collide": round(plane * cfg.members / t_lbm / 1e9, 3),
        # the analysis alone: whole-grid analyses per second and local (per-node)
        # LETKF problems solved per second, from its event-timed share of the cycle
        "analyses_per_s": round(1.0 / t_an, 1),
        "node_analyses_per_s": round(plane / t_an, 1),
        "rmse_a_mean": float(rmse_a.mean()),
        "rmse_f_mean": float(rmse_f.mean()),
        "spread_a_mean": float(d[:, binding.DIAG_LEN + 1].mean()),
        "spread_f_mean": float(d[:, 1].mean()),
        "obs_noise_rms": cfg.sigma * math.sqrt(2.0),
        "spectrum": spec,
        "nonfinite": nonfinite,
        "stage_ms_per_cycle": {"stream_collide": round(per_cycle["stream_collide"], 4),
                               "analysis": round(per_cycle["analysis"], 4),
                               "other": round(1e3 * elapsed / args.steps - per_cycle["stream_collide"]
                                              - per_cycle["analysis"], 4)},
        "stage_ms_per_cycle_per_launch_events": breakdown,
        "roofline": dominant,
        "roofline_other": other,
    }
    if vs_oracle is not None:
        out["vs_fp64_oracle"] = vs_oracle
    if forms:
        out["forms"] = forms
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
