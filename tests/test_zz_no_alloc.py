"""The allocation-free diagnostics entry point (lbmletkf_diagnostics_noalloc,
static device scratch) against lbmletkf_diagnostics (context workspace) on the
same states through the C ABI: the same kernels in the same order, so the
outputs must be equal bit for bit.  Two calls in a row, the second on a
smaller grid (it must not see the first call's partial sums), and the size
limit of the static scratch (rejected on the host, before any launch)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2308_03972_amd import binding, inputs
from gpu_helpers import config_state, context, cuda, host, need_gpu, random_state, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_noalloc_diagnostics_equal_the_workspace_version_twice_and_smaller():
    cfg = inputs.CONFIGS["paper"]
    say("noalloc diagnostics: 256x256 M=64 FP64, then 37x23 M=3 FP32")
    ft, fe = config_state(cfg, spin_steps=2)
    ctx = context(cfg)
    tctx = context(cfg, members=1)
    f = ctx.import_canonical(cuda(fe))
    t = tctx.import_canonical(cuda(ft))
    tuv = tctx.moments(t)[0, 1:].contiguous()
    ref = host(ctx.diagnostics(f, tuv))
    got = host(binding.diagnostics_noalloc(cfg.n, cfg.n, cfg.members, f, tuv))
    np.testing.assert_array_equal(got, ref)
    assert got[0] > 0 and got[1] > 0

    # second call: a smaller grid and ensemble in FP32 storage, with and without truth
    rng = np.random.default_rng(5)
    nx, ny, m = 37, 23, 3
    small = binding.Context(nx, ny, m, 0.6, 0.1, [[1, 1]], 2, (0.1, 0.1), 4.0, 1.05,
                            storage=binding.STORAGE_F32_DEV)
    g = small.import_canonical(cuda(random_state(rng, m, ny, nx)))
    truth = cuda(0.03 * rng.standard_normal((2, ny, nx)))
    for tr in (truth, None):
        ref2 = host(small.diagnostics(g, tr))
        got2 = host(binding.diagnostics_noalloc(nx, ny, m, g, tr,
                                                storage=binding.STORAGE_F32_DEV))
        np.testing.assert_array_equal(got2, ref2)
    assert not np.array_equal(got2, got)


def test_noalloc_rejects_grids_beyond_the_static_scratch():
    say("noalloc diagnostics: size limit")
    lib = binding.load()
    f = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = torch.zeros(binding.DIAG_LEN, dtype=torch.float64, device="cuda")
    # 2591^2 = 6,713,281 nodes > 6,710,848: rejected before any launch
    lbm = binding.LbmParams(2591, 2591, 2, 0.6, 0.1, 0.0, binding.STORAGE_F64)
    st = lib.lbmletkf_diagnostics_noalloc(ctypes.byref(lbm), f.data_ptr(), None, out.data_ptr(),
                                          None)
    assert st == -2
    assert b"static scratch" in lib.lbmletkf_last_error()
