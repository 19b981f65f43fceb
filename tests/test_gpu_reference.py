"""The GPU direct Ewald reference (se_ewald_reference) against the FP64
oracle on small systems, then used as the reference on every target of
large ones: the fast method at N = 1e5 (stokeslet, harmonic) and at the
benchmark's configuration (N = 1e6 triply periodic stokeslet, tol 1e-8, the
learned+batched form's parameters).

Bars: reference vs oracle 1e-12 rms-relative (both truncate near e^{-36} or
below; what remains is summation order); fast method vs reference: the
requested tolerance, on all targets.
"""
import time

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _ref, _q_of, env  # noqa: F401  (shared fixture)

pytestmark = pytest.mark.gpu

KERNELS = ["stokeslet", "rotlet", "stresslet", "harmonic"]


def _dev(torch, a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def _gpu_ref(se, torch, kernel, D, s, targets=None):
    a = s["q"] if kernel == "stresslet" else s["f"]
    u = se.ewald_reference(kernel, D, tuple(s["box"]), _dev(torch, s["x"]), _dev(torch, a),
                           normals=_dev(torch, s.get("nu")), targets=_dev(torch, targets))
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("D,box", [(3, (1.0, 1.0, 1.0)), (3, (1.3, 0.8, 1.9)), (0, (1.0, 1.0, 1.0)),
                                   (2, (1.0, 1.0, 1.0)), (2, (1.2, 0.9, 1.1)), (1, (1.0, 1.0, 1.0)),
                                   (1, (1.3, 0.9, 1.1))])
def test_reference_matches_oracle(env, kernel, D, box):
    se, oracle, torch = env
    n = 800 if D in (0, 3) else 400
    s = W.system(8100 + D, n, box=box, kernel=kernel, zero_mean=(kernel == "stokeslet"), periodicity=D)
    print("case reference %s D=%d box=%s" % (kernel, D, box), flush=True)
    u = _gpu_ref(se, torch, kernel, D, s)
    err = oracle.rms_rel_error(u, _ref(env, kernel, s, D=D))
    t = W.uniform_points(W.rng(8200 + D), 300, box)
    ut = _gpu_ref(se, torch, kernel, D, s, targets=t)
    errt = oracle.rms_rel_error(ut, _ref(env, kernel, s, D=D, targets=t))
    print("  at sources %.3g, off-source targets %.3g" % (err, errt), flush=True)
    assert err <= 1e-12 and errt <= 1e-12


def test_reference_rejects_bad_arguments(env):
    se, _, torch = env
    s = W.system(8300, 50)
    x, f = _dev(torch, s["x"]), _dev(torch, s["f"])
    with pytest.raises(se.SEError):
        se.ewald_reference("stokeslet", 4, (1, 1, 1), x, f)       # no such periodicity
    with pytest.raises(se.SEError):
        se.ewald_reference("stokeslet", 3, (1, 1, 1), x, f, xi=3.0)  # real-space tail beyond L/2
    with pytest.raises(se.SEError):
        se.ewald_reference("stresslet", 3, (1, 1, 1), x, f)       # normals missing


@pytest.mark.parametrize("kernel,tol", [("stokeslet", 1e-8), ("harmonic", 1e-10), ("stresslet", 1e-6)])
def test_fast_method_on_all_targets_n1e5(env, kernel, tol):
    se, oracle, torch = env
    n = 100_000
    s = W.system(8400, n, kernel=kernel, zero_mean=(kernel == "stokeslet"))
    plan = se.Plan(kernel=kernel, periodicity=3, tol=tol, n_src=n, source_q=_q_of(kernel, s), safety=10.0,
                   precision=se.PREC_FP64)
    plan.set_geometry(_dev(torch, s["x"]), _dev(torch, s.get("nu")))
    u = plan.execute(_dev(torch, s["q"] if kernel == "stresslet" else s["f"]))
    plan.sync()
    ref = _gpu_ref(se, torch, kernel, 3, s)
    err = oracle.rms_rel_error(u.cpu().numpy(), ref)
    print("case %s N=1e5 tol=%g: all-target rms-rel err %.3g" % (kernel, tol, err), flush=True)
    assert err <= tol


@pytest.mark.parametrize("D,kernel,tol,prec", [(2, "stokeslet", 1e-8, "fp64"), (2, "stresslet", 1e-6, "fp32"),
                                               (1, "rotlet", 1e-8, "fp64"), (1, "stresslet", 1e-6, "fp64")])
def test_fast_method_on_all_targets_reduced(env, D, kernel, tol, prec):
    """Doubly and singly periodic systems of N = 2e4 (the doubly periodic
    workload's size) on every target."""
    se, oracle, torch = env
    n = 20_000
    s = W.system(8500 + D, n, kernel=kernel, periodicity=D)
    plan = se.Plan(kernel=kernel, periodicity=D, tol=tol, n_src=n, source_q=_q_of(kernel, s), safety=10.0,
                   precision=se.PREC_FP64 if prec == "fp64" else se.PREC_FP32)
    plan.set_geometry(_dev(torch, s["x"]), _dev(torch, s.get("nu")))
    u = plan.execute(_dev(torch, s["q"] if kernel == "stresslet" else s["f"]))
    plan.sync()
    t0 = time.perf_counter()
    ref = _gpu_ref(se, torch, kernel, D, s)
    t1 = time.perf_counter()
    err = oracle.rms_rel_error(u.cpu().numpy(), ref)
    print("case %s D=%d N=2e4 tol=%g %s: all-target rms-rel err %.3g (reference %.2f s)" %
          (kernel, D, tol, prec, err, t1 - t0), flush=True)
    assert err <= tol


def test_benchmark_configuration_on_all_targets(env):
    """The learned+batched form of the benchmark (N = 1e6, tol 1e-8, two of
    its strength sets through one batch) against the reference on every
    target."""
    se, oracle, torch = env
    n = 1_000_000
    s = W.system(5000, n, kernel="stokeslet", zero_mean=True, n_rhs=2)
    Q = float(np.sum(s["f"] ** 2)) / 2
    b = se.Batch([dict(kernel="stokeslet", periodicity=3, tol=1e-8, n_src=n, source_q=Q, n_rhs=2,
                       selector=se.SELECT_LEARNED, precision=se.PREC_FP64)])
    x, f = _dev(torch, s["x"]), _dev(torch, s["f"])
    out = torch.empty_like(f)
    b.set_geometry([x])
    b.execute([f], [out])
    torch.cuda.synchronize()
    print("params", b.plans[0].params["xi"], b.plans[0].params["M"], b.plans[0].params["P"], flush=True)
    for r in range(2):
        sr = {"x": s["x"], "f": s["f"][r], "box": s["box"]}
        t0 = time.perf_counter()
        ref = _gpu_ref(se, torch, "stokeslet", 3, sr)
        t1 = time.perf_counter()
        err = oracle.rms_rel_error(out[r].cpu().numpy(), ref)
        print("rhs %d: all-target rms-rel err %.3g (reference %.2f s)" % (r, err, t1 - t0), flush=True)
        assert err <= 1e-8
    b.close()
