"""GPU parity of the differentiation form: the library's misfit J, its reverse
sweep dJ/df0 and dJ/dC_s (through the C ABI), against the oracle's
complex-step reverse sweep and central differences of the oracle's misfit.

Tolerances:
* FP64 storage, element by element against the oracle's gradient: 1e-11 of
  max |g| (both sides compute the same partials in FP64 in different orders;
  over 15 steps the rounding stays near 1e-14, the margin covers growth).
* FP32-deviation storage: the stored state is rounded every step by
  |f - w| 2^-24 <~ 3e-9; through the residuals H - y^o (~1e-2) that moves the
  gradient by ~1e-6 relative over the short runs and ~1e-5 over 200 steps;
  the bounds are 5e-5 and 1e-4 of the gradient's scale.
* Central differences of the FP64 oracle (h = 1e-6): truncation ~h^2 and
  rounding ~1e-16 J / h, both below 1e-8 relative here.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as oadj
from paper_2308_03972_amd import binding, inputs
from gpu_helpers import cuda, host, need_gpu, say

pytestmark = pytest.mark.gpu

F64, F32 = binding.STORAGE_F64, binding.STORAGE_F32_DEV


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _round_f32_dev(f):
    """The rounding the F32_DEV storage applies: w + fp32(f - w)."""
    w = oracle.lattice()[2][None, :, None, None]
    return w + (f - w).astype(np.float32).astype(np.float64)


def _problem(seed, m, ny, nx, npts, nvar, n_times, s, tau0=0.56, cs=0.15, mu=2e-3,
             spin=3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.standard_normal((m, ny, nx))
    f0 = oracle.equilibrium(rho, 0.05 * rng.standard_normal((m, ny, nx)),
                            0.05 * rng.standard_normal((m, ny, nx)))
    f0 = oracle.lbm_steps(f0, spin, tau0, cs)       # away from equilibrium
    force = 1e-4 * rng.standard_normal((2, ny, nx))
    flat = rng.choice(nx * ny, size=npts, replace=False)
    pts = np.stack([flat % nx, flat // nx], axis=1).astype(np.int32)
    f = f0
    yo = []
    for _ in range(n_times):
        f = oracle.lbm_steps(f, s, tau0, cs, force, mu)
        y = oracle.observe(f, pts, nvar).mean(axis=0)
        yo.append(y + 0.01 * rng.standard_normal(y.shape))
    return dict(f0=f0, s=s, yo=np.array(yo), pts=pts, nvar=nvar, tau0=tau0, cs=cs,
                force=force, mu=mu)


def _ctx(p, storage=F64, points=None):
    m, _, ny, nx = p["f0"].shape
    pts = p["pts"] if points is None else points
    return binding.Context(nx, ny, m, p["tau0"], p["cs"], pts, p["nvar"], (0.1,) * p["nvar"],
                           4.0, 1.05, mu=p["mu"], force=cuda(p["force"]), storage=storage)


def _gpu_gradient(p, storage=F64, repeat=1):
    ctx = _ctx(p, storage)
    f = ctx.import_canonical(cuda(p["f0"]))
    yo = cuda(p["yo"])
    work = ctx.adjoint_workspace(p["s"], len(p["yo"]))
    J = ctx.misfit_forward(f, p["cs"], p["s"], yo, work)
    outs = [ctx.misfit_backward(f, p["cs"], p["s"], yo, work) for _ in range(repeat)]
    return (float(host(J)[0]),) + tuple((host(g), float(host(c)[0])) for g, c in outs)


def _oracle_gradient(p, f0=None):
    return oadj.misfit_gradient(p["f0"] if f0 is None else f0, p["s"], p["yo"], p["pts"],
                                p["nvar"], p["tau0"], p["cs"], p["force"], p["mu"])


@pytest.mark.parametrize("nvar", [2, 3])
def test_misfit_gradient_matches_oracle_fp64(nvar):
    """40 x 24 lattice (960 nodes: 3 full 256-node blocks and a ragged one),
    3 members, 3 observation times 5 steps apart, force and friction."""
    say(f"adjoint fp64 nvar={nvar}")
    p = _problem(100 + nvar, 3, 24, 40, npts=7, nvar=nvar, n_times=3, s=5)
    J, (g, gcs) = _gpu_gradient(p)
    Jr, gr, gcsr = _oracle_gradient(p)
    scale = np.max(np.abs(gr))
    say(f"J {J:.6e} vs {Jr:.6e}; grad rel {np.max(np.abs(g - gr)) / scale:.2e}; "
        f"dJ/dCs {gcs:.6e} vs {gcsr:.6e}")
    assert abs(J - Jr) <= 1e-13 * Jr
    assert np.max(np.abs(g - gr)) <= 1e-11 * scale
    assert abs(gcs - gcsr) <= 1e-11 * abs(gcsr)
    assert np.count_nonzero(gr) > 0.5 * gr.size     # the sensitivity has spread


def test_misfit_gradient_two_step_forward_fp64():
    """16 members in FP64 storage: the forward sweep takes pairs of steps per
    launch, and s = 5 leaves one single step per interval (the reverse sweep
    recomputes single steps); 24 x 20 lattice, 3 observation times."""
    say("adjoint fp64, 16 members, two-step forward")
    p = _problem(801, 16, 20, 24, npts=6, nvar=2, n_times=3, s=5)
    J, (g, gcs) = _gpu_gradient(p)
    Jr, gr, gcsr = _oracle_gradient(p)
    scale = np.max(np.abs(gr))
    say(f"J {J:.6e} vs {Jr:.6e}; grad rel {np.max(np.abs(g - gr)) / scale:.2e}; "
        f"dJ/dCs {gcs:.6e} vs {gcsr:.6e}")
    assert abs(J - Jr) <= 1e-13 * Jr
    assert np.max(np.abs(g - gr)) <= 1e-11 * scale
    assert abs(gcs - gcsr) <= 1e-11 * abs(gcsr)


@pytest.mark.parametrize("case", ["one_step", "cs_zero_single_member", "min_grid"])
def test_misfit_gradient_edge_cases(case):
    say(f"adjoint edge {case}")
    if case == "one_step":          # a checkpoint after every step
        p = _problem(201, 2, 9, 11, npts=3, nvar=2, n_times=1, s=1)
    elif case == "cs_zero_single_member":
        p = _problem(202, 1, 12, 10, npts=4, nvar=3, n_times=2, s=3, cs=0.0)
    else:                           # 3 x 3 periodic lattice, every node observed
        p = _problem(203, 2, 3, 3, npts=9, nvar=3, n_times=2, s=2)
    J, (g, gcs) = _gpu_gradient(p)
    Jr, gr, gcsr = _oracle_gradient(p)
    assert abs(J - Jr) <= 1e-13 * Jr
    assert np.max(np.abs(g - gr)) <= 1e-11 * np.max(np.abs(gr))
    if p["cs"] == 0.0:
        assert gcs == 0.0 and gcsr == 0.0
    else:
        assert abs(gcs - gcsr) <= 1e-11 * abs(gcsr)


def test_misfit_gradient_f32_storage_matches_oracle():
    say("adjoint f32 storage")
    p = _problem(301, 3, 24, 40, npts=7, nvar=3, n_times=3, s=5)
    p["f0"] = _round_f32_dev(p["f0"])              # the state the FP32 form starts from
    J, (g, gcs) = _gpu_gradient(p, F32)
    Jr, gr, gcsr = _oracle_gradient(p)
    rel = np.max(np.abs(g - gr)) / np.max(np.abs(gr))
    say(f"f32: J rel {abs(J - Jr) / Jr:.2e}, grad rel {rel:.2e}, "
        f"dCs rel {abs(gcs - gcsr) / abs(gcsr):.2e}")
    assert abs(J - Jr) <= 1e-6 * Jr
    assert rel <= 5e-5
    assert abs(gcs - gcsr) <= 5e-5 * abs(gcsr)


def test_misfit_backward_is_deterministic_and_repeatable():
    say("adjoint determinism")
    p = _problem(401, 2, 16, 20, npts=5, nvar=2, n_times=2, s=4)
    J, (g1, c1), (g2, c2) = _gpu_gradient(p, repeat=2)
    assert np.array_equal(g1, g2) and c1 == c2


def _config5_problem(cfg):
    """Differentiation workload from the seeded fields, built by the oracle:
    members and truth spun up one observation interval from their
    equilibrium fields, y^o = H(truth) + sigma eps at every observation time."""
    truth_uv, mem_uv = inputs.initial_velocities(cfg)
    force = inputs.body_force(cfg)
    n = cfg.n
    ft = oracle.equilibrium(np.ones((1, n, n)), truth_uv[0][None], truth_uv[1][None])
    fe = oracle.equilibrium(np.ones((cfg.members, n, n)), mem_uv[:, 0], mem_uv[:, 1])
    s = cfg.steps_per_cycle
    ft = oracle.lbm_steps(ft, s, cfg.tau0, cfg.cs, force, cfg.mu)
    fe = oracle.lbm_steps(fe, s, cfg.tau0, cfg.cs, force, cfg.mu)
    pts = inputs.observation_points(cfg)
    noise = inputs.all_observation_noise(cfg, cfg.cycles)
    sig = inputs.sigma_vector(cfg)
    yo = []
    for c in range(cfg.cycles):
        ft = oracle.lbm_steps(ft, s, cfg.tau0, cfg.cs, force, cfg.mu)
        yo.append(oracle.observe(ft, pts, cfg.nvar)[0] + sig * noise[c])
    return dict(f0=fe, s=s, yo=np.array(yo), pts=pts, nvar=cfg.nvar, tau0=cfg.tau0,
                cs=cfg.cs, force=force, mu=cfg.mu)


def test_misfit_gradient_full_size_differentiation_config():
    """128^2, 16 members, 8 x 8 (u, v) observations, 200 steps with a
    checkpoint every 20: J against the oracle's misfit, <dJ/df0, d> along two
    random unit directions and dJ/dC_s against central differences of the
    oracle's misfit (h = 1e-6), for the FP32 form (the configuration's
    storage) and the FP64 form."""
    cfg = inputs.CONFIGS["differentiation"]
    p = _config5_problem(cfg)
    p32 = dict(p, f0=_round_f32_dev(p["f0"]))

    def Jo(q, f0=None, cs=None):
        return oadj.misfit(q["f0"] if f0 is None else f0, q["s"], q["yo"], q["pts"], q["nvar"],
                           q["tau0"], q["cs"] if cs is None else cs, q["force"], q["mu"])

    rng = np.random.default_rng(555)
    dirs = [rng.standard_normal(p["f0"].shape) for _ in range(2)]
    dirs = [d / np.linalg.norm(d) for d in dirs]
    h = 1e-6
    for form, q, tol_j, tol_g in ((F32, p32, 1e-5, 1e-4), (F64, p, 1e-12, 1e-7)):
        say(f"adjoint full size form={form}")
        J, (g, gcs) = _gpu_gradient(q, form)
        Jr = Jo(q)
        say(f"J {J:.8e} oracle {Jr:.8e}")
        assert abs(J - Jr) <= tol_j * Jr
        gn = np.linalg.norm(g)
        for d in dirs:
            fd = (Jo(q, f0=q["f0"] + h * d) - Jo(q, f0=q["f0"] - h * d)) / (2 * h)
            say(f"<g,d> {np.sum(g * d):.8e} fd {fd:.8e} |g| {gn:.3e}")
            assert abs(np.sum(g * d) - fd) <= tol_g * gn
        fdcs = (Jo(q, cs=q["cs"] + h) - Jo(q, cs=q["cs"] - h)) / (2 * h)
        say(f"dJ/dCs {gcs:.8e} fd {fdcs:.8e}")
        assert abs(gcs - fdcs) <= tol_g * abs(fdcs)


def test_forecast_misfit_autograd_function():
    """torch.autograd.gradcheck of binding.forecast_misfit on a 6 x 5 lattice,
    then a second backward after an unrelated forward on the same context."""
    say("adjoint autograd")
    p = _problem(601, 2, 5, 6, npts=3, nvar=3, n_times=2, s=2)
    ctx = _ctx(p)
    f0 = cuda(p["f0"]).requires_grad_(True)
    cs = torch.tensor(p["cs"], dtype=torch.float64, requires_grad=True)
    yo = cuda(p["yo"])

    def fn(f, c):
        return binding.forecast_misfit(ctx, f, c, p["s"], yo)

    assert torch.autograd.gradcheck(fn, (f0, cs), eps=1e-6, atol=1e-8, rtol=1e-5)
    J = fn(f0, cs)
    J.backward(retain_graph=True)
    g1, c1 = f0.grad.clone(), cs.grad.clone()
    _ = fn(f0.detach() * 1.0001, cs.detach() + 0.01)   # a newer forward sweep on the context
    f0.grad = None
    cs.grad = None
    J.backward()
    assert torch.equal(f0.grad, g1) and torch.equal(cs.grad, c1)
    Jr, gr, gcsr = _oracle_gradient(p)
    assert abs(float(J.detach()) - Jr) <= 1e-13 * Jr
    assert np.max(np.abs(host(g1) - gr)) <= 1e-11 * np.max(np.abs(gr))


def test_misfit_argument_errors():
    say("adjoint argument errors")
    p = _problem(701, 2, 8, 8, npts=3, nvar=2, n_times=2, s=2)
    ctx = _ctx(p)
    f = ctx.import_canonical(cuda(p["f0"]))
    yo = cuda(p["yo"])
    work = ctx.adjoint_workspace(2, 2)
    g = ctx.new_canonical()
    gcs = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.LbmLetkfError) as e:   # backward before any forward
        binding.lbmletkf_misfit_backward(ctx, f, p["cs"], 2, yo, work, g, gcs)
    assert e.value.status == -1
    ctx.misfit_forward(f, p["cs"], 2, yo, work)
    with pytest.raises(binding.LbmLetkfError) as e:   # different C_s than the forward
        binding.lbmletkf_misfit_backward(ctx, f, p["cs"] + 0.1, 2, yo, work, g, gcs)
    assert e.value.status == -1
    small = ctx.adjoint_workspace(2, 1)
    small.n_times = 2
    with pytest.raises(binding.LbmLetkfError) as e:   # workspace sized for one time
        ctx.misfit_forward(f, p["cs"], 2, yo, small)
    assert e.value.status == -7
    dup = np.array([[1, 1], [1, 1], [2, 3]], dtype=np.int32)
    cd = _ctx(p, points=dup)
    fd = cd.import_canonical(cuda(p["f0"]))
    wd = cd.adjoint_workspace(2, 2)
    yd = torch.zeros((2, cd.n_obs), dtype=torch.float64, device="cuda")
    J = cd.misfit_forward(fd, p["cs"], 2, yd, wd)   # J itself is fine with duplicates
    assert float(host(J)[0]) > 0.0
    with pytest.raises(binding.LbmLetkfError) as e:
        cd.misfit_backward(fd, p["cs"], 2, yd, wd)
    assert e.value.status == -8
