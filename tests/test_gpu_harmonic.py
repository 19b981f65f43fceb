"""Harmonic kernel 1/|r| (three independent charge sets per source) through
the whole path against the FP64 oracle: every periodicity, neutral and
charged sets (the charged ones check the gauges: the neutralising background
for D = 3, -2 pi |z| for D = 2, -2 log(rho) for D = 1), FP64 and FP32, off-
source targets, a pair of right-hand sides (the six-component gridding and
the paired real-space sum), and the real-space part alone at the same split.

Bar: the requested rms-relative tolerance (safety factor 10, as in the other
parity tests); the real-space part within 1e-12 of the oracle's.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _ref, _run, env  # noqa: F401  (shared fixture)

pytestmark = pytest.mark.gpu

CASES = [
    # D, neutral, tol, precision, box
    (3, True, 1e-6, "fp64", (1.0, 1.0, 1.0)),
    (3, False, 1e-10, "fp64", (1.0, 1.0, 1.0)),
    (3, False, 1e-8, "fp64", (1.3, 0.8, 1.9)),
    (3, True, 1e-5, "fp32", (1.0, 1.0, 1.0)),
    (2, True, 1e-8, "fp64", (1.0, 1.0, 1.0)),
    (2, False, 1e-6, "fp64", (1.2, 0.9, 1.0)),
    (1, True, 1e-8, "fp64", (1.0, 1.0, 1.0)),
    (1, False, 1e-6, "fp64", (2.0, 1.0, 1.0)),
    (0, False, 1e-8, "fp64", (1.0, 1.0, 1.0)),
    (0, False, 1e-5, "fp32", (1.0, 0.6, 1.4)),
]


@pytest.mark.parametrize("D,neutral,tol,prec,box", CASES)
def test_harmonic_against_oracle(env, D, neutral, tol, prec, box):
    se, oracle, _ = env
    s = W.system(7100 + 10 * D + int(neutral), 1500, box=box, kernel="harmonic", zero_mean=neutral,
                 periodicity=D)
    p = se.PREC_FP64 if prec == "fp64" else se.PREC_FP32
    plan, u = _run(env, "harmonic", s, D=D, tol=tol, precision=p)
    print("  P=%d M=%s xi=%.3f" % (plan.params["P"], plan.params["M"], plan.params["xi"]), flush=True)
    err = oracle.rms_rel_error(u, _ref(env, "harmonic", s, D=D))
    print("  rel err %.3g" % err, flush=True)
    assert err <= tol


@pytest.mark.parametrize("D", [3, 1])
def test_harmonic_off_source_targets(env, D):
    se, oracle, _ = env
    box = (1.0, 1.0, 1.0)
    s = W.system(7200 + D, 1200, box=box, kernel="harmonic", periodicity=D)
    t = W.uniform_points(W.rng(7300 + D), 700, box)
    _, u = _run(env, "harmonic", s, D=D, tol=1e-8, targets=t)
    err = oracle.rms_rel_error(u, _ref(env, "harmonic", s, D=D, targets=t))
    print("  rel err %.3g" % err, flush=True)
    assert err <= 1e-8


def test_harmonic_pair_of_rhs(env):
    se, oracle, _ = env
    s = W.system(7400, 1500, kernel="harmonic", n_rhs=2)
    _, u = _run(env, "harmonic", s, D=3, tol=1e-8, n_rhs=2)
    for r in range(2):
        sr = dict(s)
        sr["f"] = s["f"][r]
        err = oracle.rms_rel_error(u[r], _ref(env, "harmonic", sr, D=3))
        print("  rhs %d rel err %.3g" % (r, err), flush=True)
        assert err <= 1e-8


def test_harmonic_real_space_part_at_same_split(env):
    se, oracle, _ = env
    s = W.system(7500, 3000, box=(1.0, 1.3, 0.9), kernel="harmonic")
    plan, ur, _ = _run(env, "harmonic", s, tol=1e-9, split=True)
    par = plan.params
    ref = np.zeros_like(ur)
    L = oracle.lib()
    a = np.ascontiguousarray(s["f"])
    n = len(a)
    L.oracle_real_part(3, oracle.KERNELS["harmonic"], oracle._d(np.asarray(s["box"], float)), par["xi"], par["rc"],
                       n, oracle._d(s["x"]), oracle._d(a), None, n, oracle._d(s["x"]),
                       oracle._l(np.arange(n, dtype=np.int64)), oracle._d(ref))
    err = oracle.rms_rel_error(ur, ref)
    print("  real-space rel err %.3g" % err, flush=True)
    assert err <= 1e-12
