"""Truncated-Gaussian window (Sec. 5.3, eq. TG-window) through the whole
path: gridding and gathering with exp(-alpha (r/a)^2) evaluated exactly, the
scaling step with the untruncated Gaussian's transform, against the FP64
oracle at the requested rms-relative tolerance (safety factor 10 as in the
PKB parity tests), for every periodicity and kernel; and PKB against TG on
the same grid, both far below their window errors, which must agree.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _q_of, env  # noqa: F401  (shared fixture)

pytestmark = pytest.mark.gpu

SAFETY = 10.0

CASES = [
    (3, "stokeslet", (1.0, 1.0, 1.0), 1e-6, "fp64"),
    (3, "stresslet", (1.0, 1.0, 1.0), 1e-8, "fp64"),
    (3, "rotlet", (1.0, 1.0, 1.0), 1e-10, "fp64"),
    (3, "stokeslet", (1.0, 1.0, 1.0), 1e-4, "fp32"),
    (2, "rotlet", (1.0, 1.0, 1.0), 1e-6, "fp64"),
    (2, "stresslet", (1.0, 1.0, 1.0), 1e-8, "fp64"),
    (1, "stokeslet", (2.0, 1.0, 1.0), 1e-6, "fp64"),
    (0, "stokeslet", (1.0, 1.0, 1.0), 1e-8, "fp64"),
    (0, "rotlet", (1.0, 1.0, 1.0), 1e-6, "fp32"),
]


def _run(se, torch, s, kernel, D, box, tol, prec, window, manual=None):
    dev = torch.device("cuda:0")
    n = len(s["x"])
    kw = dict(kernel=kernel, periodicity=D, box=box, tol=tol, n_src=n, source_q=_q_of(kernel, s),
              safety=SAFETY, precision=se.PREC_FP64 if prec == "fp64" else se.PREC_FP32, window=window)
    if manual is not None:
        kw["selector"] = se.SELECT_MANUAL
    plan = se.Plan(manual, **kw)
    nu = torch.tensor(s["nu"], device=dev) if kernel == "stresslet" else None
    plan.set_geometry(torch.tensor(s["x"], device=dev), nu)
    u = plan.execute(torch.tensor(s["q"] if kernel == "stresslet" else s["f"], device=dev))
    plan.sync()
    return plan, u.cpu().numpy()


@pytest.mark.parametrize("D,kernel,box,tol,prec", CASES)
def test_tg_window_against_oracle(env, D, kernel, box, tol, prec):
    se, oracle, torch = env
    n = 1500
    s = W.system(5100 + 7 * D, n, box=box, kernel=kernel, periodicity=D, zero_mean=(D == 3))
    plan, u = _run(se, torch, s, kernel, D, box, tol, prec, "tg")
    par = plan.params
    print("case D=%d %s tol=%g %s: P=%d alpha=%.2f M=%s" % (D, kernel, tol, prec, par["P"], par["alpha"],
                                                             par["M"]), flush=True)
    assert par["window"] == se.WINDOW_TG
    xo = 6.0 / float(np.max(np.asarray(box)[:D])) if D in (1, 2) else None
    r = oracle.ewald(D, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"), xi=xo)
    ref = r.total if D else r["direct"]
    err = oracle.rms_rel_error(u, ref)
    print("  rel err %.3g" % err, flush=True)
    assert err <= tol


def test_tg_and_pkb_agree_on_one_grid(env):
    """Same xi, rc and grid; PKB at P = 20 and TG at P = 30 both sit far below
    1e-10 window error, so the two evaluations agree to that level."""
    se, oracle, torch = env
    n = 1500
    s = W.system(5150, n, kernel="stokeslet", zero_mean=True)
    base = se.select_params(kernel="stokeslet", periodicity=3, tol=1e-10, n_src=n, source_q=_q_of("stokeslet", s),
                            safety=SAFETY)
    outs = []
    for window, P in (("pkb", 20), ("tg", 30)):
        m = se.se_params()
        m.struct_size = se.ctypes.sizeof(se.se_params)
        m.xi, m.rc, m.P = base["xi"], base["rc"], P
        for i in range(3):
            m.M[i] = base["M"][i]
        plan, u = _run(se, torch, s, "stokeslet", 3, (1.0, 1.0, 1.0), 1e-10, "fp64", window, manual=m)
        assert plan.params["P"] == P and plan.params["window"] == se.WINDOWS[window]
        outs.append(u)
    d = oracle.rms_rel_error(outs[1], outs[0])
    print("PKB P=20 vs TG P=30: rms-rel difference %.3g" % d, flush=True)
    assert d <= 1e-10
