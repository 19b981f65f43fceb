"""The learned selector's device kernels (forward, loss and gradient, Adam,
training, prediction) against the FP64 network oracle (oracle/mlp.py).

FP32 bars: outputs and the loss within 1e-5 relative; gradients within
1e-4 of the largest gradient entry (sums of up to n products in FP32);
Adam states within 1e-6 relative; 20 training steps within 1e-4 absolute on
the weights.
"""
import ctypes
import os

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


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda:0")


def _case(mlp, seed, n):
    g = np.random.default_rng(seed)
    theta = g.normal(0.0, 0.3, mlp.N_PARAM).astype(np.float32)
    X = g.normal(size=(n, mlp.N_IN)).astype(np.float32)
    T = g.normal(size=(n, mlp.N_OUT)).astype(np.float32)
    return theta, X, T


@pytest.mark.parametrize("n", [1, 31, 32, 33, 257, 2000])
def test_loss_grad_matches_oracle(env, n):
    se, mlp, torch = env
    theta, X, T = _case(mlp, 10 + n, n)
    grad = torch.empty(mlp.N_PARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    print("loss_grad n=%d" % n, flush=True)
    td, Xd, Td = _dev(torch, theta), _dev(torch, X), _dev(torch, T)  # kept alive across the call
    st = se.se_mlp_loss_grad(_vp(td), _vp(Xd), _vp(Td), n, _vp(grad), _vp(loss), None)
    assert st == se.SE_OK
    L, g = mlp.loss_grad(theta.astype(np.float64), X, T)
    assert abs(loss.item() - L) <= 1e-5 * L
    gg = grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gg - g)) <= 1e-4 * np.max(np.abs(g))


@pytest.mark.parametrize("n", [1, 255, 256, 257, 1000])
def test_forward_matches_oracle(env, n):
    se, mlp, torch = env
    theta, X, _ = _case(mlp, 20 + n, n)
    Y = torch.empty((n, mlp.N_OUT), dtype=torch.float32, device="cuda:0")
    td, Xd = _dev(torch, theta), _dev(torch, X)
    st = se.se_mlp_forward(_vp(td), _vp(Xd), n, _vp(Y), None)
    assert st == se.SE_OK
    ref = mlp.forward(theta.astype(np.float64), X)
    assert np.all(np.abs(Y.cpu().numpy() - ref) <= 1e-5 * (1.0 + np.abs(ref)))


# Adam's hyperparameters as the device receives them (FP32 arguments)
LR, B1, B2, EPS = (float(np.float32(v)) for v in (1e-3, 0.9, 0.999, 1e-8))


def test_adam_matches_oracle(env):
    se, mlp, torch = env
    g = np.random.default_rng(5)
    n = 5124
    th = g.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    tg, mg, vg = _dev(torch, th), _dev(torch, m), _dev(torch, v)
    for t in range(1, 6):
        gr = g.normal(size=n).astype(np.float32)
        gd = _dev(torch, gr)
        st = se.se_mlp_adam(_vp(tg), _vp(mg), _vp(vg), _vp(gd), n, t, LR, B1, B2, EPS, None)
        torch.cuda.synchronize()
        assert st == se.SE_OK
        th, m, v = mlp.adam_step(th, m, v, gr.astype(np.float64), t, LR, B1, B2, EPS)
    torch.cuda.synchronize()
    assert np.allclose(tg.cpu().numpy(), th, rtol=1e-6, atol=1e-6)
    assert np.allclose(mg.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
    assert np.allclose(vg.cpu().numpy(), v, rtol=1e-5, atol=1e-9)


def test_training_steps_match_oracle(env):
    """20 full-batch steps of gradient + Adam on the device against the same
    steps in FP64."""
    se, mlp, torch = env
    theta, X, T = _case(mlp, 33, 300)
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    tg, mg, vg = _dev(torch, theta), _dev(torch, m), _dev(torch, v)
    Xd, Td = _dev(torch, X), _dev(torch, T)
    grad = torch.empty(mlp.N_PARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    for t in range(1, 21):
        assert se.se_mlp_loss_grad(_vp(tg), _vp(Xd), _vp(Td), len(X), _vp(grad), _vp(loss), None) == se.SE_OK
        assert se.se_mlp_adam(_vp(tg), _vp(mg), _vp(vg), _vp(grad), mlp.N_PARAM, t, LR, B1, B2, EPS,
                              None) == se.SE_OK
        _, g = mlp.loss_grad(th, X, T)
        th, m, v = mlp.adam_step(th, m, v, g, t, LR, B1, B2, EPS)
    torch.cuda.synchronize()
    assert np.max(np.abs(tg.cpu().numpy() - th)) <= 1e-4


@pytest.fixture
def restore_selector(env):
    se, _, _ = env
    yield
    path = os.path.join(os.path.dirname(se.__file__), "se_selector_weights.bin")
    if os.path.exists(path):
        assert se.se_selector_load(path.encode()) == se.SE_OK


def test_train_predict_save_load(env, tmp_path, restore_selector):
    """se_selector_train lowers the loss on a smooth synthetic map; the
    trained weights and normalisation, run through the oracle, give what
    se_selector_predict gives; a saved file reloads to the same predictions."""
    se, mlp, torch = env
    from paper_2210_01255_amd import selector as S
    g = np.random.default_rng(8)
    n = 600
    X = np.zeros((n, mlp.N_IN), dtype=np.float32)
    X[:, 0] = g.uniform(3, 6, n)
    X[:, 1] = g.uniform(0, np.log(4), n)
    X[np.arange(n), 2 + g.integers(0, 4, n)] = 1
    X[np.arange(n), 6 + g.integers(0, 3, n)] = 1
    X[:, 9] = g.uniform(-10, -4, n)
    Y = np.stack([2.0 + 0.3 * X[:, 0] - 0.1 * X[:, 9], 3.0 + 0.5 * X[:, 0] + 0.2 * X[:, 1],
                  -1.2 * X[:, 9] + X[:, 2], 1.5 + 0.05 * X[:, 9] ** 2 / 10], axis=1).astype(np.float32)
    hist = S.train(X, Y, epochs=300, batch=64, lr=3e-3, seed=4)
    print("loss first %.4g last %.4g" % (hist[0], hist[-1]), flush=True)
    assert hist[-1] < 0.1 * hist[0]
    theta = np.zeros(mlp.N_PARAM, dtype=np.float32)
    norm = np.zeros(se.MLP_NORM, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    assert se.se_selector_get(theta.ctypes.data_as(fp), norm.ctypes.data_as(fp)) == se.SE_OK
    xm, xs, ym, ys = norm[:10], norm[10:20], norm[20:24], norm[24:28]
    ref = mlp.forward(theta.astype(np.float64), (X - xm) / xs) * ys + ym
    got = S.predict(X)
    assert np.all(np.abs(got - ref) <= 1e-4 * (1.0 + np.abs(ref)))
    assert np.sqrt(np.mean((got - Y) ** 2)) < 0.2 * np.std(Y)
    path = str(tmp_path / "w.bin")
    S.save(path)
    S.load(path)
    assert np.array_equal(S.predict(X), got)


def test_learned_path_completes_a_proposal_like_the_analytic_procedure(env, tmp_path, restore_selector):
    """A network whose output is a constant, the outputs of an analytic
    parameter set (fine pollution rule, safety 3), makes the learned path
    return that set: same xi, and the implied safety factor ~3 gives the same
    window and a grid and cut-off within one rounding step.  A proposal whose
    grid exceeds the FFT limits falls back to the analytic parameters."""
    se, mlp, torch = env
    from paper_2210_01255_amd import selector as S
    import importlib
    abi = importlib.import_module("test_library_abi")
    theta = np.zeros(se.MLP_NPARAM, dtype=np.float32)
    p = str(tmp_path / "c.bin")
    for D, kernel, box, tol in [(3, 0, (1, 1, 1), 1e-8), (0, 0, (1, 2, 1), 1e-6), (2, 2, (1, 1, 1.5), 1e-7),
                                (1, 1, (2.5, 1, 1), 1e-5)]:
        kw = dict(kernel=kernel, periodicity=D, box=box, tol=tol, n_src=20000)
        ref = se.select_params(pollution=se.POLLUTION_FINE, safety=3.0, **kw)
        hmin = min(ref["h"][i] for i in range(3) if (i < D or D == 0))
        y = S.targets_of(ref["xi"], hmin, ref["P"], ref["rc"], np.array(box, dtype=float))
        abi._weights_file(p, theta, np.concatenate([np.zeros(10), np.ones(10), y, np.ones(4)]).astype(np.float32))
        S.load(p)
        got = se.select_params(selector=se.SELECT_LEARNED, **kw)
        print(D, kernel, "ref", ref["M"], ref["P"], ref["rc"], "learned", got["M"], got["P"], got["rc"],
              ref["tau_abs"] / got["tau_abs"], flush=True)
        assert abs(got["xi"] - ref["xi"]) <= 1e-5 * ref["xi"]
        assert abs(got["rc"] - ref["rc"]) <= 0.03 * ref["rc"]
        assert got["P"] == ref["P"]
        assert all(abs(a - b) <= 0.1 * b for a, b in zip(got["M"], ref["M"]))
    kw = dict(kernel=0, periodicity=3, box=(1, 1, 1), tol=1e-8, n_src=20000)
    y = np.array([np.log(2000.0), np.log(4000.0), 12.0, np.log(4.0)], dtype=np.float32)
    abi._weights_file(p, theta, np.concatenate([np.zeros(10), np.ones(10), y, np.ones(4)]).astype(np.float32))
    S.load(p)
    plan = se.Plan(selector=se.SELECT_LEARNED, **kw)
    assert "analytic" in plan.message, plan.message
    assert plan.params == se.select_params(**kw)


def test_shipped_weights_beat_plain_at_equal_error(env, restore_selector):
    """The trained selector (weights shipped beside the library) on N = 1e6
    uniform stokeslet systems, D = 3 and D = 0, tol 1e-4 .. 1e-10: every
    learned run meets its tolerance on every target against the GPU direct
    Ewald reference (checked against the oracle in test_gpu_reference.py),
    and the learned parameters take less total time than the plain analytic
    ones (Table 3 n_rc, the paper's pollution rule, safety 10)."""
    se, mlp, torch = env
    from paper_2210_01255_amd import selector as S
    path = os.path.join(os.path.dirname(se.__file__), "se_selector_weights.bin")
    assert os.path.exists(path), "trained weights missing"
    S.load(path)
    rows = S.evaluate(S.METRIC_PROBLEMS)
    for r in rows:
        assert r["learned_msg"] == "learned parameters", r
        assert r["learned_err"] <= r["tol"], r
        assert r["plain_err"] <= r["tol"], r
    tp = sum(r["plain_ms"] for r in rows)
    tl = sum(r["learned_ms"] for r in rows)
    print("plain %.1f ms learned %.1f ms: x%.2f" % (tp, tl, tp / tl), flush=True)
    assert tl < tp


@pytest.mark.parametrize("D", [3, 0])
def test_learned_parameters_against_oracle_sampled(env, restore_selector, D):
    """Learned parameters at N = 1e6, tol 1e-8, against the oracle on 24
    sampled targets."""
    se, mlp, torch = env
    import oracle
    import workloads as W
    path = os.path.join(os.path.dirname(se.__file__), "se_selector_weights.bin")
    se.se_selector_load(path.encode())
    n = 1_000_000
    s = W.system(5100 + D, n, kernel="stokeslet", zero_mean=(D == 3))
    plan = se.Plan(kernel="stokeslet", periodicity=D, tol=1e-8, n_src=n, source_q=float(np.sum(s["f"] ** 2)),
                   selector=se.SELECT_LEARNED)
    assert plan.message == "learned parameters"
    plan.set_geometry(torch.tensor(s["x"], device="cuda:0"))
    u = plan.execute(torch.tensor(s["f"], device="cuda:0")).cpu().numpy()
    plan.sync()
    idx = np.sort(W.rng(5200 + D).choice(n, 24, replace=False)).astype(np.int64)
    ref = oracle.ewald(D, "stokeslet", s["box"], s["x"], f=s["f"], targets=s["x"][idx], self_src=idx)
    ref = ref.total if D else ref["direct"]
    err = oracle.rms_rel_error(u[idx], ref)
    print("D=%d learned sampled err %.3g" % (D, err), flush=True)
    assert err <= 1e-8
