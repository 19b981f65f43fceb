"""Pins of the FP64 oracle against facts it does not itself compute.

Each test checks the oracle against something independent of its own code:
symbolic differentiation of the scalar Green's functions, a textbook lattice
constant, invariance under the splitting parameter, the zero-mean-flow
convention and the stresslet integral identity.  Paper: Bagge & Tornberg,
"Fast Ewald summation for Stokes flow with arbitrary periodicity".
"""
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Kernel formulas from the scalar Green's functions by symbolic calculus.
# Sec. 2, eqs. (diffop-rel-1)-(diffop-rel-3): S = (d_jl Lap - d_j d_l) B,
# Omega = -eps_jlm d_m H, T = [(d_jl d_m + d_mj d_l + d_lm d_j) Lap
# - 2 d_j d_l d_m] B, with B = |r|, H = 1/|r|; Sec. 2.1 gives the real-space
# parts by the same operators acting on B^R and H^R.
# --------------------------------------------------------------------------
def _sym_kernels(real_space):
    import sympy as sp

    x, y, z, xi = sp.symbols("x y z xi", real=True, positive=True)
    X = (x, y, z)
    r = sp.sqrt(x * x + y * y + z * z)
    if real_space:
        B = r * sp.erfc(xi * r) - sp.exp(-xi ** 2 * r ** 2) / (sp.sqrt(sp.pi) * xi)
        H = sp.erfc(xi * r) / r
    else:
        B = r
        H = 1 / r

    def lap(e):
        return sum(sp.diff(e, v, 2) for v in X)

    lapB = lap(B)
    S = [[(lapB if j == l else 0) - sp.diff(B, X[j], X[l]) for l in range(3)] for j in range(3)]
    Om = [[-sum(sp.LeviCivita(j, l, m) * sp.diff(H, X[m]) for m in range(3)) for l in range(3)]
          for j in range(3)]
    T = [[[((sp.diff(lapB, X[m]) if j == l else 0) + (sp.diff(lapB, X[l]) if m == j else 0)
            + (sp.diff(lapB, X[j]) if l == m else 0) - 2 * sp.diff(B, X[j], X[l], X[m]))
           for m in range(3)] for l in range(3)] for j in range(3)]
    f = lambda e: sp.lambdify((x, y, z, xi), e, "mpmath")  # noqa: E731
    return ([[f(S[j][l]) for l in range(3)] for j in range(3)],
            [[f(Om[j][l]) for l in range(3)] for j in range(3)],
            [[[f(T[j][l][m]) for m in range(3)] for l in range(3)] for j in range(3)])


@pytest.fixture(scope="module")
def sym_free():
    return _sym_kernels(False)


@pytest.fixture(scope="module")
def sym_real():
    return _sym_kernels(True)


def _contract(kernel, fn, r, xi, f, nu):
    import mpmath as mp

    mp.mp.dps = 30
    S, Om, T = fn
    u = np.zeros(3)
    for j in range(3):
        acc = mp.mpf(0)
        for l in range(3):
            if kernel == "stokeslet":
                acc += S[j][l](*r, xi) * f[l]
            elif kernel == "rotlet":
                acc += Om[j][l](*r, xi) * f[l]
            else:
                for m in range(3):
                    acc += T[j][l][m](*r, xi) * f[l] * nu[m]
        u[j] = float(acc)
    return u


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
def test_free_kernels_match_operator_definition(oracle_lib, sym_free, kernel):
    g = W.rng(11)
    for _ in range(4):
        r = g.uniform(-1, 1, 3) * g.uniform(0.1, 2.0)
        f = g.standard_normal(3)
        nu = W.unit_normals(g, 1)[0]
        want = _contract(kernel, sym_free, r, 1.0, f, nu)
        got = oracle_lib.free_kernel(kernel, r, f, nu)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
def test_real_space_kernels_match_operator_definition(oracle_lib, sym_real, kernel):
    g = W.rng(12)
    for xi in (3.0, 10.0):
        for _ in range(3):
            r = g.uniform(-1, 1, 3) * g.uniform(0.05, 0.4)
            f = g.standard_normal(3)
            nu = W.unit_normals(g, 1)[0]
            want = _contract(kernel, sym_real, r, xi, f, nu)
            got = oracle_lib.real_kernel(kernel, xi, r, f, nu)
            scale = max(np.abs(want).max(), 1e-300)
            assert np.allclose(got, want, rtol=1e-11, atol=1e-11 * scale)


def test_self_term_is_limit_of_real_minus_free(oracle_lib):
    """Eq. (self-term): lim_{r->0} (G^R - G) . f = -4 xi/sqrt(pi) f for S, 0 for Omega."""
    xi = 7.0
    f = np.array([0.3, -1.2, 0.8])
    r = np.array([1.0, -2.0, 0.5]) * 1e-6
    d = oracle_lib.real_kernel("stokeslet", xi, r, f) - oracle_lib.free_kernel("stokeslet", r, f)
    assert np.allclose(d, -4 * xi / math.sqrt(math.pi) * f, rtol=1e-6)
    d = oracle_lib.real_kernel("rotlet", xi, r, f) - oracle_lib.free_kernel("rotlet", r, f)
    assert np.abs(d).max() < 1e-4 * 4 * xi / math.sqrt(math.pi)


def test_hasimoto_single_force_cubic_lattice(oracle_lib):
    with open(os.path.join(GOLDEN, "hasimoto_cubic.txt")) as fh:
        C = [float(l.split()[1]) for l in fh if l.startswith("C ")][0]
    for L in (1.0, 2.5):
        x = np.array([[0.31, 0.47, 0.12]]) * L
        f = np.array([[0.6, -0.2, 1.1]])
        for xi in (4.0 / L, 9.0 / L):
            u = oracle_lib.ewald(3, "stokeslet", [L, L, L], x, f=f, xi=xi).total
            assert np.allclose(u, C * f / L, rtol=1e-9, atol=0)


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.3, 0.8, 1.9)])
def test_xi_invariance_3p(oracle_lib, kernel, box):
    """Eq. (3p-ewald-decomp-self) does not depend on xi."""
    s = W.system(21, 150, box=box, kernel=kernel)
    a = oracle_lib.ewald(3, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"), xi=3.5)
    b = oracle_lib.ewald(3, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"), xi=6.5)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-12
    # the split itself changes a lot: the test is not vacuous
    assert oracle_lib.rms_rel_error(a["real"], b["real"]) > 1e-3
    # off-source targets too (no self term)
    t = W.uniform_points(W.rng(22), 40, box)
    a = oracle_lib.ewald(3, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"),
                         targets=t, xi=3.5)
    b = oracle_lib.ewald(3, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"),
                         targets=t, xi=6.5)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-12


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet"])
def test_zero_mean_flow_3p(oracle_lib, kernel):
    """Eq. (zero-mean-flow): with zero mode 0, <u_j> over the face x_j = 0 vanishes (S, Omega)."""
    g = W.rng(31)
    x = 0.35 + 0.3 * g.random((6, 3))
    f = g.standard_normal((6, 3))
    n = 48
    s = (np.arange(n) + 0.0) / n
    A, B = np.meshgrid(s, s, indexing="ij")
    for j in range(3):
        pts = np.zeros((n * n, 3))
        others = [a for a in range(3) if a != j]
        pts[:, others[0]] = A.ravel()
        pts[:, others[1]] = B.ravel()
        u = oracle_lib.ewald(3, kernel, [1, 1, 1], x, f=f, targets=pts, self_src=None, xi=5.0).total
        mean = u[:, j].mean()
        assert abs(mean) < 1e-9 * np.abs(u[:, j]).max()


def _sphere_quadrature(center, rho, n_t=24, n_p=48):
    ct, wt = np.polynomial.legendre.leggauss(n_t)
    ph = 2 * np.pi * np.arange(n_p) / n_p
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    nu = np.stack([ST * np.cos(PH), ST * np.sin(PH), CT], axis=-1).reshape(-1, 3)
    w = (rho ** 2 * (2 * np.pi / n_p) * np.repeat(wt, n_p)).reshape(-1)
    return np.asarray(center)[None, :] + rho * nu, nu, w


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_stresslet_integral_identity(oracle_lib, D):
    """Eq. (stresslet-identity) for constant q0 on a sphere.

    With nu the OUTWARD normal, T_jlm q_l nu_m integrates to 8 pi q0 inside and
    0 outside: at the centre, r = -rho nu gives 6 nu_j (nu.q0)/rho^2 per unit
    area and the sphere average of nu_j nu_l is delta_jl/3; far away the
    integral vanishes since the sphere integral of nu is zero.  The paper's
    case labels correspond to the inward normal (same identity, sign of nu
    flipped)."""
    y, nu, w = _sphere_quadrature([0.5, 0.5, 0.5], 0.22)
    q0 = np.array([0.7, -0.4, 1.3])
    q = w[:, None] * q0[None, :]
    inside = np.array([[0.5, 0.5, 0.5], [0.55, 0.45, 0.52]])
    outside = np.array([[0.5, 0.5, 0.93], [0.08, 0.9, 0.5]])
    t = np.concatenate([inside, outside])
    xi = 4.0 if D in (1, 2) else None
    r = oracle_lib.ewald(D, "stresslet", [1, 1, 1], y, q=q, nu=nu, targets=t, self_src=None, xi=xi)
    u = r.total if D else r["direct"]
    assert np.allclose(u[:2], 8 * np.pi * q0[None, :], rtol=0, atol=1e-8)
    assert np.allclose(u[2:], 0.0, atol=1e-8)


# --------------------------------------------------------------------------
# Doubly and singly periodic sums (Appendices A and B).
# --------------------------------------------------------------------------
def test_exponential_integral_matches_library(oracle_lib):
    """E1 used by the singly periodic zero mode (eq. 1p-stokeslet-Q0) vs scipy."""
    from scipy.special import exp1

    for x in [1e-12, 1e-6, 1e-3, 0.1, 0.5, 0.999, 1.0, 1.001, 2.0, 7.5, 30.0, 200.0]:
        assert abs(oracle_lib.e1(x) - exp1(x)) <= 4e-15 * exp1(x)


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("D", [2, 1])
def test_xi_invariance_reduced(oracle_lib, D, kernel):
    """Eqs. (2p-ewald-decomp) / (1p-ewald-decomp) do not depend on xi.

    Net force is non-zero here, so the singly periodic stokeslet also checks
    that the gauge of eq. (1p-stokeslet-Q0) is the same for every xi."""
    box = (1.2, 0.9, 1.1)
    s = W.system(23, 60, box=box, kernel=kernel, periodicity=D)
    kw = dict(f=s.get("f"), q=s.get("q"), nu=s.get("nu"))
    a = oracle_lib.ewald(D, kernel, box, s["x"], xi=3.5, **kw)
    b = oracle_lib.ewald(D, kernel, box, s["x"], xi=6.0, **kw)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-11
    assert oracle_lib.rms_rel_error(a["real"], b["real"]) > 1e-3
    assert oracle_lib.rms_rel_error(a["k0"], b["k0"]) > 1e-3
    t = W.uniform_points(W.rng(24), 30, box)
    a = oracle_lib.ewald(D, kernel, box, s["x"], targets=t, xi=3.5, **kw)
    b = oracle_lib.ewald(D, kernel, box, s["x"], targets=t, xi=6.0, **kw)
    assert oracle_lib.rms_rel_error(a.total, b.total) < 1e-11


def _richardson(vals, Ks, p0):
    """Repeated Richardson extrapolation for an error sum_j c_j K^{-(p0 + j)}, K doubling."""
    T = [np.asarray(v) for v in vals]
    p = p0
    while len(T) > 1:
        r = Ks[1] / Ks[0]
        T = [(r ** p * T[i + 1] - T[i]) / (r ** p - 1) for i in range(len(T) - 1)]
        p += 1
    return T[0]


@pytest.mark.parametrize("kernel", ["stokeslet", "rotlet", "stresslet"])
@pytest.mark.parametrize("D", [1, 2])
def test_reduced_matches_image_sums(oracle_lib, D, kernel):
    """Direct image sums of eq. (periodic-potential) over the block |p_i| <= K.

    The kernels decay as |r|^-2 (rotlet, stresslet; stokeslet with zero net
    force), and the images at +p and -p cancel to leading order, so the sum
    converges and its block truncation error is a power series in 1/K
    (from K^-2 for D = 1 and K^-1 for D = 2), removed by Richardson
    extrapolation.  Nothing here uses the Ewald split."""
    box = (1.0, 1.0, 1.0)
    s = W.system(12, 20, box=box, kernel=kernel, zero_mean=(kernel == "stokeslet"), periodicity=D)
    kw = dict(f=s.get("f"), q=s.get("q"), nu=s.get("nu"))
    ref = oracle_lib.ewald(D, kernel, box, s["x"], xi=5.0, **kw).total
    if D == 1:
        Ks, p0, tol = [250, 500, 1000, 2000], 2, 1e-12
    else:
        Ks, p0, tol = [8, 16, 32, 64, 128, 256], 1, 1e-9
    vals = [oracle_lib.image_block_sum(D, kernel, box, s["x"], K=K, **kw) for K in Ks]
    assert oracle_lib.rms_rel_error(_richardson(vals, Ks, p0), ref) < tol


def test_direct_sum_is_translation_invariant_and_antisymmetric(oracle_lib):
    """D = 0 definition: a shift of all points leaves u unchanged; the rotlet/stresslet
    kernels are odd, the stokeslet even (eq. stokes-kernels)."""
    s = W.system(41, 60, kernel="stokeslet")
    a = oracle_lib.ewald(0, "stokeslet", [1, 1, 1], s["x"], f=s["f"])["direct"]
    b = oracle_lib.ewald(0, "stokeslet", [1, 1, 1], s["x"] * 0.5 + 0.2, f=s["f"])["direct"]
    # scaling positions by 1/2 doubles a 1/r kernel
    assert np.allclose(b, 2 * a, rtol=1e-12)
    r = np.array([0.3, -0.1, 0.2])
    f = np.array([1.0, 2.0, -0.5])
    nu = np.array([0.0, 0.6, 0.8])
    assert np.allclose(oracle_lib.free_kernel("rotlet", -r, f), -oracle_lib.free_kernel("rotlet", r, f))
    assert np.allclose(oracle_lib.free_kernel("stresslet", -r, f, nu),
                       -oracle_lib.free_kernel("stresslet", r, f, nu))
    assert np.allclose(oracle_lib.free_kernel("stokeslet", -r, f), oracle_lib.free_kernel("stokeslet", r, f))


# ------------------------------------------------ learned selector network
def _mlp_case(seed, n):
    from oracle import mlp
    g = np.random.default_rng(seed)
    theta = g.normal(0.0, 0.3, mlp.N_PARAM)
    X = g.normal(size=(n, mlp.N_IN))
    T = g.normal(size=(n, mlp.N_OUT))
    return theta, X, T


def test_mlp_gradient_matches_finite_differences():
    """Backpropagated gradient against central differences of the loss on
    every parameter block (all of b3, b1; strided entries of the weights)."""
    from oracle import mlp
    theta, X, T = _mlp_case(7, 9)
    L, g = mlp.loss_grad(theta, X, T)
    assert abs(L - mlp.loss(theta, X, T)) < 1e-15
    idx = list(range(0, mlp.N_PARAM, 37)) + list(range(mlp.N_PARAM - 4, mlp.N_PARAM)) + [640, 703, 704, 4864]
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-8 * max(1.0, abs(g[i])), i


def test_mlp_forward_known_values():
    """Zero first-layer weights make the output W3 tanh(W2 tanh(b1) + b2) + b3
    for every input; a single active path gives tanh(tanh(w x)) scaled."""
    from oracle import mlp
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["b1"][:] = 0.5
    p["W2"][3, :] = 0.1
    p["W3"][2, 3] = 2.0
    p["b3"][:] = [1.0, -1.0, 0.25, 0.0]
    X = np.random.default_rng(3).normal(size=(5, mlp.N_IN))
    y = mlp.forward(mlp.pack(p), X)
    expect = np.array([1.0, -1.0, 0.25 + 2.0 * np.tanh(64 * 0.1 * np.tanh(0.5)), 0.0])
    assert np.allclose(y, expect[None, :], rtol=0, atol=1e-15)
    q = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    q["W1"][0, 4] = 0.7
    q["W2"][1, 0] = 1.3
    q["W3"][0, 1] = 1.0
    y = mlp.forward(mlp.pack(q), X)
    assert np.allclose(y[:, 0], np.tanh(1.3 * np.tanh(0.7 * X[:, 4])), rtol=0, atol=1e-15)
    assert np.all(y[:, 1:] == 0.0)


def test_adam_first_step_closed_form():
    """At t = 1 from zero moments the bias corrections give m_hat = g and
    v_hat = g^2, so the step is -lr g / (|g| + eps)."""
    from oracle import mlp
    g = np.random.default_rng(4).normal(size=50)
    th0 = np.linspace(-1, 1, 50)
    th1, m, v = mlp.adam_step(th0, np.zeros(50), np.zeros(50), g, 1, 1e-3, 0.9, 0.999, 1e-8)
    assert np.allclose(th1, th0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    th, m, v = th0, np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, g, t, 1e-3, 0.9, 0.999, 0.0)
    assert np.allclose(th, th0 - 5e-3 * np.sign(g), rtol=0, atol=1e-12)
