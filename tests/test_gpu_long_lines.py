"""Transforms with lines longer than the common in-place budget (1536
elements per call): every route to such a line, against the FP64 oracle.

* D = 2: the K_* class along the free axis;
* D = 1: both free axes of the K_* class;
* D = 3: a long z axis (fused z pass), a long y axis and a long x axis
  (half-length over 1536);
* D = 0: the precompute grid of the truncated kernel along z;
each with its longest line between 1537 and 2048 points (checked).

Small N with a given xi makes the grids large while the oracle stays fast.
Bar: the requested rms-relative tolerance.  With xi forced far above its
usual value the estimates sit at the edge of their band (D = 2 at safety 10
measured 1.07 tol), so these cases use safety 30; a transform that dropped
part of a line gives errors of order one.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _q_of, env  # noqa: F401  (shared fixture)

pytestmark = pytest.mark.gpu

SAFETY = 30.0

CASES = [
    (2, "stokeslet", (1.0, 1.0, 1.0), 1e-10, 100.0),
    (1, "rotlet", (1.0, 1.0, 1.0), 1e-8, 130.0),
    (3, "stokeslet", (0.4, 0.4, 45.0), 1e-6, 14.0),
    (3, "rotlet", (0.4, 45.0, 0.4), 1e-6, 15.0),
    (3, "stokeslet", (110.0, 0.8, 0.8), 1e-6, 12.0),
    (0, "stokeslet", (0.2, 0.2, 3.5), 1e-8, 0.0),
]


@pytest.mark.parametrize("D,kernel,box,tol,xi", CASES)
def test_long_transform_lines(env, D, kernel, box, tol, xi):
    se, oracle, torch = env
    n = 2000
    s = W.system(3100 + D, n, box=box, kernel=kernel, periodicity=D)
    plan = se.Plan(kernel=kernel, periodicity=D, box=box, tol=tol, n_src=n, source_q=_q_of(kernel, s), xi=xi,
                   safety=SAFETY, precision=se.PREC_FP64)
    par = plan.params
    lens = [par["n_fft"][0] // 2] + list(par["n_fft"][1:])
    if D in (1, 2):
        lens += list(par["n0_fft"][D:]) + list(par["nstar_fft"][D:])
    if D == 0:
        lens += list(par["n0_fft"])
    print("case D=%d %s box=%s xi=%g: longest line %d" % (D, kernel, box, xi, max(lens)), flush=True)
    assert 1536 < max(lens) <= 2048
    dev = torch.device("cuda:0")
    nu = torch.tensor(s["nu"], device=dev) if kernel == "stresslet" else None
    plan.set_geometry(torch.tensor(s["x"], device=dev), nu)
    u = plan.execute(torch.tensor(s["q"] if kernel == "stresslet" else s["f"], device=dev))
    plan.sync()
    xo = 6.0 / float(np.max(np.asarray(box)[:D])) if D in (1, 2) else None
    r = oracle.ewald(D, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"), xi=xo)
    ref = r.total if D else r["direct"]
    err = oracle.rms_rel_error(u.cpu().numpy(), ref)
    print("  rel err %.3g" % err, flush=True)
    assert err <= tol
