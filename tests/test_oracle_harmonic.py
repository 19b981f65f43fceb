"""Pins of the oracle's harmonic kernel 1/|r| (Sec. 2, split as in Sec. 2.1
with the classical screening, eq. ewald-screening), carried per component
as three independent charge sets.

* D = 3: the rock-salt Madelung constant (textbook value, golden file);
  independence of xi, also for charge sets that are not neutral (the
  neutralising-background term);
* D = 2, 1: independence of xi, and Richardson-extrapolated image sums of
  neutral charge sets (nothing there uses the Ewald split);
* the self term as the r -> 0 limit of the real-space minus the free kernel;
* D = 0 against a plain double loop.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from test_oracle_pins import _richardson

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rocksalt(L):
    plus = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    minus = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    x = np.array(plus + minus, dtype=np.float64) * L + 0.013 * L  # shifted off the cell faces
    q = np.array([1.0] * 4 + [-1.0] * 4)
    return x, q


def test_madelung_constant_rocksalt(oracle_lib):
    with open(os.path.join(GOLDEN, "madelung_rocksalt.txt")) as fh:
        M = [float(l.split()[1]) for l in fh if l.startswith("M ")][0]
    for L in (1.0, 2.6):
        x, q = _rocksalt(L)
        f = np.stack([q, -2.0 * q, np.zeros_like(q)], axis=1)
        a = L / 2.0
        for xi in (3.0 / L, 7.0 / L):
            u = oracle_lib.ewald(3, "harmonic", [L, L, L], x, f=f, xi=xi).total
            assert np.allclose(u[:, 0], -M / a * q, rtol=1e-11, atol=0)
            assert np.allclose(u[:, 1], 2.0 * M / a * q, rtol=1e-11, atol=0)
            assert np.all(np.abs(u[:, 2]) < 1e-13)


def test_self_term_is_limit_of_real_minus_free(oracle_lib):
    xi = 6.0
    f = np.array([0.7, -1.1, 0.4])
    r = np.array([0.5, 1.0, -0.3]) * 1e-7
    d = oracle_lib.real_kernel("harmonic", xi, r, f) - oracle_lib.free_kernel("harmonic", r, f)
    assert np.allclose(d, -2 * xi / math.sqrt(math.pi) * f, rtol=1e-6)


@pytest.mark.parametrize("D", [3, 2, 1])
@pytest.mark.parametrize("neutral", [True, False])
def test_xi_invariance(oracle_lib, D, neutral):
    box = (1.2, 0.9, 1.1)
    s = W.system(61 + D, 60, box=box, kernel="harmonic", zero_mean=neutral, periodicity=D)
    a = oracle_lib.ewald(D, "harmonic", box, s["x"], f=s["f"], xi=3.5)
    b = oracle_lib.ewald(D, "harmonic", box, s["x"], f=s["f"], xi=6.0)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-11
    assert oracle_lib.rms_rel_error(a["real"], b["real"]) > 1e-3
    t = W.uniform_points(W.rng(960 + D), 30, box)  # seeds apart from the sources
    a = oracle_lib.ewald(D, "harmonic", box, s["x"], f=s["f"], targets=t, xi=3.5)
    b = oracle_lib.ewald(D, "harmonic", box, s["x"], f=s["f"], targets=t, xi=6.0)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-11


@pytest.mark.parametrize("D", [1, 2])
def test_matches_image_sums_for_neutral_sets(oracle_lib, D):
    """Symmetric block sums |p_i| <= K of 1/|r| for neutral charge sets: the
    images at +p and -p cancel the dipole order, the rest is a power series
    in 1/K removed by Richardson extrapolation."""
    box = (1.0, 1.0, 1.0)
    s = W.system(64, 20, box=box, kernel="harmonic", zero_mean=True, periodicity=D)
    ref = oracle_lib.ewald(D, "harmonic", box, s["x"], f=s["f"], xi=5.0).total
    if D == 1:
        Ks, p0, tol = [250, 500, 1000, 2000], 2, 1e-11
    else:
        Ks, p0, tol = [8, 16, 32, 64, 128, 256], 1, 1e-9
    vals = [oracle_lib.image_block_sum(D, "harmonic", box, s["x"], f=s["f"], K=K) for K in Ks]
    assert oracle_lib.rms_rel_error(_richardson(vals, Ks, p0), ref) < tol


def test_free_space_is_the_double_loop(oracle_lib):
    s = W.system(65, 50, kernel="harmonic")
    x, f = s["x"], s["f"]
    u = oracle_lib.ewald(0, "harmonic", [1, 1, 1], x, f=f)["direct"]
    ref = np.zeros_like(f)
    for m in range(len(x)):
        for n in range(len(x)):
            if m != n:
                ref[m] += f[n] / np.linalg.norm(x[m] - x[n])
    assert np.allclose(u, ref, rtol=1e-13, atol=0)
