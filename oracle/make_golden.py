"""Write the golden series the full-length GPU parity tests compare against.

TEST INFRASTRUCTURE.  Calls only the FP64 oracle (this package) and the seeded
input generators; nothing here comes from the GPU library.  Each run is the
forecast-analysis workflow of Sec. 3 (``oracle.run_cycles``) from the seeded
initial fields, with the analysis of each cycle mapped over node subsets in
worker processes (the per-node problems are independent, so the result is the
same array ``letkf_analysis`` gives for the whole grid).

    python -m oracle.make_golden paper       # 256^2, 64 members, 8x8, 200 cycles
    python -m oracle.make_golden precision   # 512^2, 64 members, 16x16, 100 cycles
    python -m oracle.make_golden batch       # the twelve batching problems, 2 cycles

Output: tests/golden/<name>.npz with, per run, the per-cycle RMSE_f, RMSE_a,
spread_f, spread_a, the member-mean spectrum of the analysis and the truth's
spectrum at the report cycles, and the final analysis ensemble at sampled
nodes (canonical populations [M][9][len(nodes)]).
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2308_03972_amd import inputs  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")

# arguments of the analysis being mapped, visible to the forked workers
_JOB = {}


def _analyse_chunk(nodes):
    j = _JOB
    return oracle.letkf_analysis(j["f"], j["yf"], j["yo"], j["points"], j["sigmas"], j["d_cut"],
                                 j["beta"], nodes=nodes)


def parallel_analysis(procs: int, chunks: int):
    """letkf_analysis of every node, computed over node subsets in `procs` processes."""

    def analyze(f, yf, yo, points, sigmas, d_cut, beta):
        M, _, ny, nx = f.shape
        _JOB.update(f=f, yf=yf, yo=yo, points=points, sigmas=sigmas, d_cut=d_cut, beta=beta)
        parts = np.array_split(np.arange(nx * ny), chunks)
        with mp.get_context("fork").Pool(procs) as pool:
            res = pool.map(_analyse_chunk, parts)
        _JOB.clear()
        return np.concatenate(res, axis=2).reshape(M, 9, ny, nx)

    return analyze


def sample_nodes(n: int, count: int, seed: int) -> np.ndarray:
    """Corners, centre and a seeded random set of nodes (index y * n + x)."""
    fixed = [0, n - 1, (n - 1) * n, n * n - 1, (n // 2) * n + n // 2]
    rng = np.random.default_rng(seed)
    extra = rng.choice(n * n, size=count - len(fixed), replace=False)
    return np.unique(np.concatenate([fixed, extra])).astype(np.int64)


def run(cfg, cycles: int, report_every: int, procs: int, n_sample: int, log):
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    ft = oracle.equilibrium(np.ones((1, cfg.n, cfg.n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((cfg.members, cfg.n, cfg.n)), mem_uv[:, 0], mem_uv[:, 1])
    noise = inputs.all_observation_noise(cfg, cycles)
    t0 = time.time()
    out = oracle.run_cycles(fe, ft, cfg, inputs.body_force(cfg), inputs.observation_points(cfg),
                            noise, cycles, analyze=parallel_analysis(procs, 8 * procs),
                            report_every=report_every)
    log(f"{cfg.name}: {cycles} cycles in {time.time() - t0:.0f} s; RMSE_a last "
        f"{out['rmse_a'][-1]:.4e}")
    nodes = sample_nodes(cfg.n, n_sample, seed=cfg.seed % 1000)
    M = cfg.members
    flat = out["f_ens"].reshape(M, 9, cfg.n * cfg.n)
    res = {k: out[k] for k in ("rmse_f", "rmse_a", "spread_f", "spread_a", "report_cycle",
                               "spectrum_a", "spectrum_t")}
    res["final_nodes"] = nodes
    res["final_f"] = flat[:, :, nodes]
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["paper", "precision", "batch"])
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    log = lambda m: print(f"[golden] {m}", flush=True)
    os.makedirs(GOLDEN, exist_ok=True)
    command = "python -m oracle.make_golden " + args.which
    data = {}
    if args.which == "paper":
        cfg = inputs.CONFIGS["paper"]
        res = run(cfg, cfg.cycles, 50, args.procs, 64, log)
        data.update(res)
        name = "cycle_256x256x64_200cycles.npz"
        desc = ("FP64 oracle, 256^2 D2Q9 BGK-Smagorinsky, 64 members, 8x8 (u,v) observations, "
                "s=20, r=16, beta=1.05, 200 cycles; spectra every 50 cycles")
    elif args.which == "precision":
        cfg = inputs.CONFIGS["precision"]
        res = run(cfg, cfg.cycles, 25, args.procs, 64, log)
        data.update(res)
        name = "cycle_512x512x64_100cycles.npz"
        desc = ("FP64 oracle, 512^2 D2Q9 BGK-Smagorinsky, 64 members, 16x16 (u,v) observations, "
                "s=20, r=16, beta=1.05, 100 cycles; spectra every 25 cycles")
    else:
        cycles = 2
        for i, cfg in enumerate(inputs.batch_configs()):
            res = run(cfg, cycles, cycles, args.procs, 32, log)
            for k, v in res.items():
                data[f"p{i}_{k}"] = v
        name = "batch12_2cycles.npz"
        desc = ("FP64 oracle, the twelve batching problems (grids {128,192,256,384}^2 x members "
                "{16,32,64}), 2 cycles each, spectra at cycle 2")
    data["command"] = np.array(command)
    data["description"] = np.array(desc)
    path = os.path.join(GOLDEN, name)
    np.savez_compressed(path, **data)
    log(f"wrote {path} ({os.path.getsize(path)} bytes)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
