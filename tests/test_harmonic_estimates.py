"""The harmonic kernel's truncation estimates (derived for uncorrelated
charges, the same way Sec. 4 derives the Stokes ones) against truncation
errors measured with the FP64 oracle: the real-space part cut at the
selected r_c against a cut far beyond it, and the k-space lattice sum cut
at |k| = pi/h against a cut far beyond it.  Bar: the measured rms error
within a factor 4 of the estimate (an rms estimate, not a bound)."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def libs():
    import oracle
    import paper_2210_01255_amd as se
    oracle.build(force=False)
    return se, oracle


def _system(n):
    s = W.system(9600, n, kernel="harmonic", zero_mean=True)
    return s["x"], np.ascontiguousarray(s["f"]), float(np.sum(s["f"] ** 2))


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_real_space_estimate(libs, tol):
    se, oracle = libs
    n, xi = 1500, 9.0
    x, f, Q = _system(n)
    p = se.select_params(kernel="harmonic", periodicity=3, tol=tol, tol_kind=se.TOL_ABS, n_src=n, source_q=Q,
                         xi=xi)
    rc, est = p["rc"], p["est_real"]
    L = oracle.lib()
    box = np.ones(3)
    idx = np.arange(n, dtype=np.int64)

    def real(r):
        u = np.zeros((n, 3))
        L.oracle_real_part(3, oracle.KERNELS["harmonic"], oracle._d(box), xi, r, n, oracle._d(x), oracle._d(f),
                           None, n, oracle._d(x), oracle._l(idx), oracle._d(u))
        return u

    err = math.sqrt(np.mean(np.sum((real(0.49) - real(rc)) ** 2, axis=1)))
    print("tol %g: rc %.4f, estimate %.3g, measured %.3g" % (tol, rc, est, err))
    assert est / 4 <= err <= 4 * est


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_fourier_estimate(libs, tol):
    se, oracle = libs
    n, xi = 600, 9.0
    x, f, Q = _system(n)
    p = se.select_params(kernel="harmonic", periodicity=3, tol=tol, tol_kind=se.TOL_ABS, n_src=n, source_q=Q,
                         xi=xi)
    kc = math.pi / min(p["h"])
    est = p["est_fourier"]
    L = oracle.lib()
    box = np.ones(3)

    def fourier(kmax):
        u = np.zeros((n, 3))
        L.oracle_fourier_part_3p(oracle.KERNELS["harmonic"], oracle._d(box), xi, kmax, n, oracle._d(x),
                                 oracle._d(f), None, n, oracle._d(x), oracle._d(u))
        return u

    err = math.sqrt(np.mean(np.sum((fourier(14.0 * xi) - fourier(kc)) ** 2, axis=1)))
    print("tol %g: pi/h %.1f, estimate %.3g, measured %.3g" % (tol, kc, est, err))
    assert est / 4 <= err <= 4 * est
