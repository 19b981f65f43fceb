"""The parameter-selection procedure of Sec. 4.6 against the oracle, in the
setting of the paper's validation (Sec. 4.6, first and second tests): N = 1000
sources that are also the targets, strengths scaled to Q = 1, a given xi, and
absolute tolerances tau; all other parameters come from the procedure as the
paper states it (no safety factor, the paper's error-pollution adjustment).
The measured quantity is the rms error of the Fourier-space part, eq.
(abs-rms-error), against the oracle's Fourier-space part at the same xi (its
total minus its real-space part; for D = 0 the direct sum minus the real-space
part).  The paper reports the error within one order of magnitude of tau
until it flattens out at the rounding floor, sometimes below tau/10 for
D = 3.  At L = 1, Q = 1, xi = 10 the oracle's Fourier-space part has rms 1.8
(stokeslet) and 24 (stresslet), the magnitudes the paper reports for this case.
Checked here: no case above 10 tau (or the floor), and the geometric mean
of err/tau within [1e-2, 10] over each sweep.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KERNELS = ("stokeslet", "rotlet", "stresslet")
TOLS = (1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12)
FLOOR = 1e-13  # absolute rms floor of the FP64 evaluation at Q = 1


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2210_01255_amd as se
    import oracle
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)
    return se, oracle, torch


def _system(seed, n, kernel, box, Q):
    g = np.random.default_rng(seed)
    x = g.random((n, 3)) * np.asarray(box)[None, :]
    s = g.standard_normal((n, 3))
    s *= np.sqrt(Q / np.sum(s ** 2))
    nu = None
    if kernel == "stresslet":
        nu = g.standard_normal((n, 3))
        nu /= np.linalg.norm(nu, axis=1)[:, None]
    return x, s, nu


def _oracle_fourier(oracle, D, kernel, box, x, s, nu, xi):
    """Oracle Fourier-space part at splitting parameter xi."""
    kw = dict(q=s, nu=nu) if kernel == "stresslet" else dict(f=s)
    if D > 0:
        r = oracle.ewald(D, kernel, list(box), x, xi=xi, **kw)
        return r.total - r["real"]
    r = oracle.ewald(0, kernel, list(box), x, **kw)
    # real-space part at xi with the single image p = 0
    L = oracle.lib()
    a, b = oracle._sources(kernel, kw.get("f"), kw.get("q"), kw.get("nu"))
    n = x.shape[0]
    ur = np.zeros((n, 3))
    dp = ctypes.POINTER(ctypes.c_double)
    xs = np.ascontiguousarray(x, dtype=np.float64)
    self_src = np.arange(n, dtype=np.int64)
    L.oracle_real_part(0, oracle.KERNELS[kernel], np.ascontiguousarray(box, dtype=np.float64).ctypes.data_as(dp),
                       float(xi), 6.0 / xi, n, xs.ctypes.data_as(dp), a.ctypes.data_as(dp),
                       b.ctypes.data_as(dp) if b is not None else None, n, xs.ctypes.data_as(dp),
                       self_src.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), ur.ctypes.data_as(dp))
    return r["direct"] - ur


def _fourier_errors(env, D, kernel, box, Q, xi, tols, seed):
    se, oracle, torch = env
    n = 1000
    x, s, nu = _system(seed, n, kernel, box, Q)
    ref = _oracle_fourier(oracle, D, kernel, np.asarray(box, dtype=np.float64), x, s, nu, xi)
    dev = "cuda:0"
    xd, sd = torch.tensor(x, device=dev), torch.tensor(s, device=dev)
    nd = torch.tensor(nu, device=dev) if nu is not None else None
    out = []
    for tol in tols:
        plan = se.Plan(kernel=kernel, periodicity=D, box=tuple(box), tol=tol, tol_kind=se.TOL_ABS, n_src=n,
                       source_q=Q, xi=xi, precision=se.PREC_FP64)
        plan.set_geometry(xd, nd)
        ur, uf = plan.execute_split(sd)
        plan.sync()
        err = oracle.rms_abs_error(uf.cpu().numpy(), ref)
        p = plan.params
        print("%s D=%d L=%g Q=%g xi=%g tol=%.0e: E_rms^F %.3e (ratio %.3g) M=%s P=%d" %
              (kernel, D, box[0], Q, xi, tol, err, err / tol, list(p["M"]), p["P"]), flush=True)
        out.append((tol, err))
        del plan
    return out


def _judge(results, label):
    """The paper's claim for its sweeps: the error within one order of
    magnitude of tau until it reaches the rounding floor.  Grid sizes here
    are rounded up to multiples of 4 (the paper's sweeps use 2), which puts
    some errors further below tau.  Asserted: every case at most 10 tau (or
    at the floor), and the geometric mean of err/tau over the cases above
    the floor between 1e-2 and 10 (the procedure does not over-resolve)."""
    over = [(tol, err) for tol, err, floor in results if err > 10 * tol and err > floor]
    live = [err / tol for tol, err, floor in results if err > floor]
    gmean = float(np.exp(np.mean(np.log(live)))) if live else 1.0
    inside = sum(1 for tol, err, floor in results if tol / 10 <= err <= 10 * tol or err <= floor)
    print("%s: %d of %d within [tau/10, 10 tau] (or at the floor); geometric mean err/tau %.3g; above 10 tau: %s" %
          (label, inside, len(results), gmean, ["%.0e: %.2e" % o for o in over]), flush=True)
    assert not over, label
    assert 1e-2 <= gmean <= 10.0, label


@pytest.mark.parametrize("kernel", KERNELS + ("harmonic",))
def test_procedure_meets_absolute_tolerances(env, kernel):
    """First validation test: L = 1, Q = 1, xi = 10, tau = 1e-2 .. 1e-12, D = 3, 2, 1, 0.
    The harmonic kernel (three charge sets; estimates derived in the paper's
    way, not printed in it) is held to the same bar."""
    res = []
    for D in (3, 2, 1, 0):
        res += [(tol, err, FLOOR) for tol, err in
                _fourier_errors(env, D, kernel, (1.0, 1.0, 1.0), 1.0, 10.0, TOLS, 7100 + D)]
    _judge(res, kernel)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("D", [3, 2])
def test_procedure_over_box_size_and_strength(env, kernel, D):
    """Second validation test, reduced to its extremes: (L, Q) = (0.1, 100)
    and (10, 0.01), xi L = 10 and 30, tau = 1e-4 and 1e-8 (absolute)."""
    res = []
    for L, Q in ((0.1, 100.0), (10.0, 0.01)):
        for xil in (10.0, 30.0):
            res += [(tol, err, FLOOR * max(1.0, np.sqrt(Q))) for tol, err in
                    _fourier_errors(env, D, kernel, (L, L, L), Q, xil / L, (1e-4, 1e-8), 7200 + D + int(10 * L))]
    _judge(res, "%s D=%d" % (kernel, D))
