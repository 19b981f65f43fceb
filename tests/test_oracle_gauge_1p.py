"""Pin of the singly periodic zero-mode constants that scale with the net
source strength (sum_n f_n != 0): the stokeslet at the gauge l_B = 1,
l_H = e^{-1} and the harmonic kernel at l_H = 1 (Sec. 2.3,
eqs. 1p-stokeslet-Q0 and 1p-stokeslet-extra-contribution).

The image sum over a line of period L diverges logarithmically when the net
strength is non-zero.  By Poisson summation, the symmetric sum over |j| <= K
minus (1/L) times the integral of the kernel over the cells of those images,
s in [s0 - X, s0 + X] with X = (K + 1/2) L, tends to the modes k_1 != 0 of the
singly periodic sum; the tail error is a power series in 1/K from K^-2 on,
removed by Richardson extrapolation.  The mode k_1 = 0 is added in closed
form, derived here from the Green's functions rather than read from the
paper's appendix: with B = |r| (laplacian^2 B = -8 pi delta) and H = 1/|r|,
the line averages satisfy laplacian_perp^2 B0 = -(8 pi/L) delta and
laplacian_perp H0 = -(4 pi/L) delta in the plane across the line, so
  B0 = -(1/L) rho^2 ln(rho/l_B),  H0 = -(2/L) ln(rho/l_H),
and the stokeslet S = 2 delta H - grad grad B gives, at l_B = 1 and
l_H = e^{-1} (the pair for which laplacian B0 = 2 H0 holds),
  S0_xx = -(4/L)(ln rho + 1),  S0_x. = 0,
  S0_jl = (1/L)[delta_jl (-2 ln rho - 3) + 2 rho_j rho_l / rho^2]  (j, l in y, z).
Targets are off the source lines (rho > 0 for every pair).  Nothing here uses
the Ewald split or the oracle's zero-mode formulas.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_pins import _richardson


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def _stokeslet_line(r, f, L, K):
    """sum_{|j| <= K} S(r + j L e_x) f - (1/L) int_{-X}^{X} S(r + s e_x) ds f,
    for pair offsets r [m, n, 3] and strengths f [n, 3]; summed over n."""
    j = np.arange(-K, K + 1, dtype=np.float64)
    s = r[..., 0][..., None] + j * L                     # [m, n, J]
    ry, rz = r[..., 1][..., None], r[..., 2][..., None]
    rr2 = s * s + ry * ry + rz * rz
    ir = 1.0 / np.sqrt(rr2)
    ir3 = ir * ir * ir
    comp = (s, np.broadcast_to(ry, s.shape), np.broadcast_to(rz, s.shape))
    u = np.zeros(r.shape[:2] + (3,))
    for a in range(3):
        for b in range(3):
            Sab = (ir if a == b else 0.0) + comp[a] * comp[b] * ir3
            u[..., a] += Sab.sum(axis=-1) * f[None, :, b]
    # exact integral over s in [s0 - X, s0 + X]
    X = (K + 0.5) * L
    rho2 = r[..., 1] ** 2 + r[..., 2] ** 2
    rho = np.sqrt(rho2)

    def prim(sv):
        rv = np.sqrt(sv * sv + rho2)
        ash = np.arcsinh(sv / rho)
        I = np.zeros(r.shape[:2] + (3, 3))
        I[..., 0, 0] = 2.0 * ash - sv / rv                    # 1/r + s^2/r^3
        for a, ra in ((1, r[..., 1]), (2, r[..., 2])):
            I[..., 0, a] = I[..., a, 0] = -ra / rv            # s r_a / r^3
            for b, rb in ((1, r[..., 1]), (2, r[..., 2])):
                I[..., a, b] = (ash if a == b else 0.0) + ra * rb * sv / (rho2 * rv)
        return I

    Iint = prim(r[..., 0] + X) - prim(r[..., 0] - X)
    return u.sum(axis=1) - np.einsum("mnab,nb->ma", Iint, f) / L


def _stokeslet_k0(r, f, L):
    rho2 = r[..., 1] ** 2 + r[..., 2] ** 2
    lr = 0.5 * np.log(rho2)
    S0 = np.zeros(r.shape[:2] + (3, 3))
    S0[..., 0, 0] = -(4.0 / L) * (lr + 1.0)
    for a in (1, 2):
        for b in (1, 2):
            S0[..., a, b] = ((-2.0 * lr - 3.0) if a == b else 0.0) / L + 2.0 * r[..., a] * r[..., b] / (rho2 * L)
    return np.einsum("mnab,nb->ma", S0, f)


def _harmonic_line(r, q, L, K):
    j = np.arange(-K, K + 1, dtype=np.float64)
    s = r[..., 0][..., None] + j * L
    ir = 1.0 / np.sqrt(s * s + (r[..., 1] ** 2 + r[..., 2] ** 2)[..., None])
    u = np.einsum("mn,nc->mc", ir.sum(axis=-1), q)
    rho = np.sqrt(r[..., 1] ** 2 + r[..., 2] ** 2)
    X = (K + 0.5) * L
    I = np.arcsinh((r[..., 0] + X) / rho) - np.arcsinh((r[..., 0] - X) / rho)
    return u - np.einsum("mn,nc->mc", I, q) / L


def _harmonic_k0(r, q, L):
    rho = np.sqrt(r[..., 1] ** 2 + r[..., 2] ** 2)
    return np.einsum("mn,nc->mc", -(2.0 / L) * np.log(rho), q)   # l_H = 1


@pytest.mark.parametrize("kernel", ["stokeslet", "harmonic"])
def test_net_strength_constant_of_the_singly_periodic_sum(oracle_lib, kernel):
    box = (1.3, 0.9, 1.1)
    L = box[0]
    g = W.rng(4711)
    x = W.uniform_points(g, 7, box)
    t = W.uniform_points(g, 5, box)
    f = g.standard_normal((7, 3)) + np.array([0.8, -0.6, 0.5])   # net strength far from zero
    assert np.all(np.abs(f.sum(axis=0)) > 1.0)
    r = t[:, None, :] - x[None, :, :]
    Ks = [200, 400, 800, 1600]
    if kernel == "stokeslet":
        vals = [_stokeslet_line(r, f, L, K) for K in Ks]
        brute = _richardson(vals, Ks, 2) + _stokeslet_k0(r, f, L)
    else:
        vals = [_harmonic_line(r, f, L, K) for K in Ks]
        brute = _richardson(vals, Ks, 2) + _harmonic_k0(r, f, L)
    ref = oracle_lib.ewald(1, kernel, box, x, f=f, targets=t, xi=5.0).total
    err = oracle_lib.rms_rel_error(ref, brute)
    print("%s: oracle vs image sum with the closed-form k1 = 0 mode: %.3g" % (kernel, err))
    assert err < 1e-10
    # the constant matters: shifting the gauge by a small amount is detected
    shift = (0.01 / L) * np.outer(np.ones(len(t)), f.sum(axis=0))
    assert oracle_lib.rms_rel_error(ref + shift, brute) > 1e-4
