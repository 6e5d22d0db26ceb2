"""The allocation-free surrogate gradient: dpde_mlp_grad_noalloc keeps its
block partials in the library's static device buffer and must give the same
loss and gradient as dpde_mlp_grad, bit for bit (same kernels, same launch
shape, same summation order), on consecutive calls whose second input is
smaller than the first (the buffer keeps the first call's contents)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _system():
    import paper_1507_06643_amd as dp
    n = 200
    L = W.cubic_side(n)
    q, p, e = W.equilibrium_state(n, [L] * 3, seed=4, eps0=25.0)
    return dp, dp.System(dp.Config(n=n, box=[L] * 3, eos=dp.EOS_EINSTEIN,
                                   theta_mode=dp.THETA_MLP), q, p, e)


def test_noalloc_gradient_equals_allocating_entry_point():
    import torch
    assert torch.cuda.is_available()
    dp, s = _system()
    try:
        rng = np.random.default_rng(31)
        w = rng.normal(0, 0.5, dp._lib.MLP_NPARAM).astype(np.float32)
        s.mlp_set(w, np.array([3.0, 3.0, 0.0, 2.3]))
        # 20000 samples fill all 64 block partials; 700 fill 6 of them
        for n in (20000, 700):
            print(f"no-alloc gradient, n = {n}", flush=True)
            x = rng.uniform(-1, 1, n).astype(np.float32)
            t = rng.uniform(-1, 1, n).astype(np.float32)
            l0, g0 = s.mlp_grad_noalloc(x, t)
            l1, g1 = s.mlp_grad(x, t)
            assert np.isfinite(l0) and np.all(np.isfinite(g0))
            assert l0 == l1
            assert np.array_equal(g0, g1)
            assert np.abs(g0).max() > 0.0
        with pytest.raises(dp.DpdeError):
            s.mlp_grad_noalloc(np.zeros(0, np.float32), np.zeros(0, np.float32))
    finally:
        s.close()
