"""The allocation-free loss and gradient (se_mlp_loss_grad_noalloc) against
the allocating entry point (se_mlp_loss_grad), through the C ABI.

Both run the same kernels with the same launch shape and sum the per-block
partials in the same order, so the bar is bit-for-bit equality.  Two calls
in a row, the second on fewer samples (the array keeps the first call's
partials: a stale entry would show), then one at the array's maximum, and
the size check beyond it.  Each call is also held to the FP64 network oracle
at the bars of the selector tests (loss 1e-5 relative, gradient 1e-4 of the
largest entry).
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2210_01255_amd as se
    from oracle import mlp
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return se, mlp, torch


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _case(mlp, seed, n):
    g = np.random.default_rng(seed)
    theta = g.normal(0.0, 0.3, mlp.N_PARAM).astype(np.float32)
    X = g.normal(size=(n, mlp.N_IN)).astype(np.float32)
    T = g.normal(size=(n, mlp.N_OUT)).astype(np.float32)
    return theta, X, T


def _both(se, torch, theta, X, T):
    dev = "cuda:0"
    td, Xd, Td = (torch.tensor(a, device=dev) for a in (theta, X, T))
    n = X.shape[0]
    out = []
    for fn in (se.se_mlp_loss_grad, se.se_mlp_loss_grad_noalloc):
        grad = torch.full((theta.size,), float("nan"), dtype=torch.float32, device=dev)
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        st = fn(_vp(td), _vp(Xd), _vp(Td), n, _vp(grad), _vp(loss), None)
        assert st == se.SE_OK, se.STATUS.get(st, st)
        torch.cuda.synchronize()
        out.append((grad.cpu().numpy(), float(loss.item())))
    return out


@pytest.mark.parametrize("sizes", [(3000, 777)])
def test_noalloc_matches_allocating_entry_point(env, sizes):
    se, mlp, torch = env
    for k, n in enumerate(sizes + (se.MLP_NOALLOC_MAX_N,)):
        print("loss_grad_noalloc call %d, n=%d" % (k, n), flush=True)
        theta, X, T = _case(mlp, 700 + k, n)
        (g_ref, l_ref), (g, l) = _both(se, torch, theta, X, T)
        assert np.array_equal(g, g_ref), np.max(np.abs(g - g_ref))
        assert l == l_ref, (l, l_ref)
        L, go = mlp.loss_grad(theta.astype(np.float64), X, T)
        assert abs(l - L) <= 1e-5 * L
        assert np.max(np.abs(g.astype(np.float64) - go)) <= 1e-4 * np.max(np.abs(go))


def test_noalloc_rejects_sizes_beyond_its_scratch(env):
    se, mlp, torch = env
    n = se.MLP_NOALLOC_MAX_N + 1
    theta, X, T = _case(mlp, 9, n)
    td, Xd, Td = (torch.tensor(a, device="cuda:0") for a in (theta, X, T))
    grad = torch.empty(theta.size, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    st = se.se_mlp_loss_grad_noalloc(_vp(td), _vp(Xd), _vp(Td), n, _vp(grad), _vp(loss), None)
    assert st == se.SE_ERR_SCRATCH
    st = se.se_mlp_loss_grad_noalloc(_vp(td), _vp(Xd), _vp(Td), 0, _vp(grad), _vp(loss), None)
    assert st == se.SE_ERR_ARG
