"""Launch-shape knobs of a plan (se_plan_set_shape): the real-space blocking,
the FFT column bundles and the gridding/gathering work item (candidates per
item, in batches of 64; a tile with more candidates is split into further
items that add their sums atomically) leave the result unchanged up to the
order of the additions; values out of range are refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2210_01255_amd as se
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return se, torch


@pytest.mark.parametrize("D,kernel,n_rhs", [(3, "stokeslet", 2), (1, "rotlet", 1), (0, "stresslet", 1)])
def test_launch_shapes_leave_the_result_unchanged(env, D, kernel, n_rhs):
    se, torch = env
    n, tol = 20000, 1e-8
    box = (1.0, 1.0, 1.0) if D != 1 else (2.0, 1.0, 1.0)
    s = W.system(8400 + D, n, box=box, kernel=kernel, periodicity=D, zero_mean=(D == 3),
                 n_rhs=n_rhs if n_rhs > 1 else None)
    key = "q" if kernel == "stresslet" else "f"
    dev = "cuda:0"
    x = torch.tensor(s["x"], device=dev)
    nu = torch.tensor(s["nu"], device=dev) if kernel == "stresslet" else None
    f = torch.tensor(s[key], device=dev)
    q = float(np.sum(s[key] ** 2)) / n_rhs
    plan = se.Plan(kernel=kernel, periodicity=D, box=box, tol=tol, n_src=n, source_q=q,
                   precision=se.PREC_FP64, n_rhs=n_rhs)
    plan.set_geometry(x, nu)
    assert plan.get_shape() == (0, 0, 0)
    u0 = plan.execute(f)
    plan.sync()
    u0 = u0.cpu().numpy()
    print("D=%d %s M=%s P=%d" % (D, kernel, plan.params["M"], plan.params["P"]), flush=True)
    for shape in [(0, 0, 1), (1, 2, 3), (4, 16, 64), (2, 4, se.TILE_ITEMS_MAX)]:
        plan.set_shape(*shape)
        assert plan.get_shape() == shape
        u = plan.execute(f)
        plan.sync()
        err = float(np.linalg.norm(u.cpu().numpy() - u0) / np.linalg.norm(u0))
        print("  shape", shape, "rel diff", err, flush=True)
        assert err < 1e-12, (shape, err)
    for bad in [(0, 0, -1), (0, 0, se.TILE_ITEMS_MAX + 1), (5, 0, 0), (0, 3, 0)]:
        with pytest.raises(se.SEError):
            plan.set_shape(*bad)
    assert plan.get_shape() == (2, 4, se.TILE_ITEMS_MAX)
