"""Opt-in wrapping of periodic coordinates (se_plan_set_wrap): points moved
by whole periods along the periodic axes give the same result as the
originals when wrapping is on (the sorted copies hold the primary-cell
representatives, which the stresslet's k = 0 term needs), and raise
SE_ERR_OUT_OF_BOX when it is off.  Bar: 1e-12 relative (only the rounding
of x + k L - k L differs)."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _q_of, env  # noqa: F401  (shared fixture)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("D,kernel", [(3, "stokeslet"), (3, "stresslet"), (2, "rotlet"), (1, "stokeslet")])
def test_wrapped_positions_match_the_primary_cell(env, D, kernel):
    se, oracle, torch = env
    dev = torch.device("cuda:0")
    n = 3000
    box = (1.2, 0.9, 1.1)
    s = W.system(9300 + D, n, box=box, kernel=kernel, periodicity=D)
    shift = W.rng(9400 + D).integers(-2, 3, size=(n, 3)).astype(np.float64)
    shift[:, D:] = 0.0
    xs = s["x"] + shift * np.asarray(box)[None, :]
    kw = dict(kernel=kernel, periodicity=D, box=box, tol=1e-8, n_src=n, source_q=_q_of(kernel, s), safety=10.0,
              precision=se.PREC_FP64)
    nu = torch.tensor(s["nu"], device=dev) if kernel == "stresslet" else None
    a = torch.tensor(s["q"] if kernel == "stresslet" else s["f"], device=dev)
    p0 = se.Plan(**kw)
    p0.set_geometry(torch.tensor(s["x"], device=dev), nu)
    u0 = p0.execute(a)
    p0.sync()
    p1 = se.Plan(**kw)
    p1.set_wrap(True)
    p1.set_geometry(torch.tensor(xs, device=dev), nu)
    u1 = p1.execute(a)
    p1.sync()
    err = oracle.rms_rel_error(u1.cpu().numpy(), u0.cpu().numpy())
    print("D=%d %s wrapped vs primary cell %.3g" % (D, kernel, err), flush=True)
    assert err <= 1e-12
    p2 = se.Plan(**kw)
    p2.set_geometry(torch.tensor(xs, device=dev), nu)  # binning flags the points outside the box
    with pytest.raises(se.SEError) as ei:
        p2.sync()
    assert ei.value.status == se.SE_ERR_OUT_OF_BOX
