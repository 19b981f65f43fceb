"""FP64 CPU oracle for the Ewald-summed Stokes potentials (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_2210_01255_amd``) and never imports it.

What it computes (Bagge & Tornberg, Sec. 2):
  * D = 3: classical Ewald sum with explicit real-space and k-space lattice
    sums, eq. (3p-ewald-decomp-self) = real part (real-space-potential-3p)
    + k != 0 part (fourier-space-potential-3p) + non-periodic stresslet term
    (k0-stresslet-3p) + self term (self-term);
  * D = 0: the free-space sum (periodic-potential) with the single image p=0,
    summed directly;
  * D = 2, 1: real part with images in the periodic directions only, the
    nonsingular modes k^P != 0 of (2p-fourier-space) / (1p-fourier-space) by
    the trapezoidal rule in the free wavenumbers (``virtual_cell``), and the
    singular modes k^P = 0 in the closed forms of Appendices A.2 and B.2
    (``reduced_oracle.c``), reported as 'k0'.

The harmonic kernel 1/|r| (Sec. 2) is carried per component: f[n][3] holds
three independent charge sets and u[m][3] their potentials, with the
classical Ewald split of Sec. 2.1 and, for D = 2 and 1, the classical zero
modes in the gauges -2 pi |z| and -2 log(rho).

The oracle chooses its own splitting parameter xi_o and truncations from a
cost balance and a fixed damping margin (erfc(xi rc) and exp(-k^2/4xi^2)
both ~ e^{-36}); nothing is taken from the fast method's parameter selector.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libewald_oracle.so")
_SRCS = ["ewald_oracle.c", "reduced_oracle.c"]

KERNELS = {"stokeslet": 0, "rotlet": 1, "stresslet": 2, "harmonic": 3}


def build(force: bool = True) -> str:
    """Compile the oracle's C sources with gcc (FP64, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    srcs = [os.path.join(_HERE, s) for s in _SRCS if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(_SO):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_SO) >= newest:
            return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.oracle_real_part.argtypes = [i, i, dp, d, d, l, dp, dp, dp, l, dp, lp, dp]
        L.oracle_real_part.restype = l
        L.oracle_fourier_part_3p.argtypes = [i, dp, d, d, l, dp, dp, dp, l, dp, dp]
        L.oracle_fourier_part_3p.restype = l
        L.oracle_fourier_part_3p_box.argtypes = [i, dp, d, dp, l, dp, dp, dp, l, dp, dp]
        L.oracle_fourier_part_3p_box.restype = l
        L.oracle_k0_stresslet_3p.argtypes = [dp, l, dp, dp, dp, l, dp, dp]
        L.oracle_k0_stresslet_3p.restype = None
        L.oracle_self_part.argtypes = [i, d, l, lp, dp, dp]
        L.oracle_self_part.restype = None
        L.oracle_direct_0p.argtypes = [i, l, dp, dp, dp, l, dp, lp, dp]
        L.oracle_direct_0p.restype = l
        L.oracle_image_block_sum.argtypes = [i, i, dp, i, l, dp, dp, dp, l, dp, lp, dp]
        L.oracle_image_block_sum.restype = None
        L.oracle_free_kernel.argtypes = [i, dp, dp, dp, dp]
        L.oracle_free_kernel.restype = None
        L.oracle_real_kernel.argtypes = [i, d, dp, dp, dp, dp]
        L.oracle_real_kernel.restype = None
        L.oracle_reduced_fourier_part.argtypes = [i, i, dp, d, d, l, dp, dp, dp, l, dp, dp]
        L.oracle_reduced_fourier_part.restype = l
        L.oracle_zero_mode.argtypes = [i, i, dp, d, l, dp, dp, dp, l, dp, dp]
        L.oracle_zero_mode.restype = None
        L.oracle_e1.argtypes = [d]
        L.oracle_e1.restype = d
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _l(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _prep(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _sources(kernel, f, q, nu):
    if kernel == "stresslet":
        return _prep(q), _prep(nu)
    return _prep(f), None


def free_kernel(kernel, r, f, nu=None):
    """G(r) . f for one separation vector (eq. stokes-kernels)."""
    out = np.zeros(3)
    r = _prep(r)
    f = _prep(f)
    nu = _prep(nu) if nu is not None else np.zeros(3)
    lib().oracle_free_kernel(KERNELS[kernel], _d(r), _d(f), _d(nu), _d(out))
    return out


def real_kernel(kernel, xi, r, f, nu=None):
    """G^R(r; xi) . f for one separation vector (eqs. *-real)."""
    out = np.zeros(3)
    r = _prep(r)
    f = _prep(f)
    nu = _prep(nu) if nu is not None else np.zeros(3)
    lib().oracle_real_kernel(KERNELS[kernel], float(xi), _d(r), _d(f), _d(nu), _d(out))
    return out


class Parts(dict):
    """Named contributions of one oracle evaluation plus scalar diagnostics."""

    PARTS = ("real", "fourier", "k0", "self", "direct")

    @property
    def total(self):
        return sum(self[k] for k in self.PARTS if k in self)


def choose_xi(n_src, n_tgt, box, margin=6.0):
    """Cost-balanced splitting parameter for the direct Ewald sums.

    Real-space work ~ n_tgt n_src (4/3) pi (margin/xi)^3 / V pairs and k-space
    work ~ (n_src + n_tgt) (2/3) pi (2 margin xi / 2 pi)^3 V terms; equal when
    xi^6 = c n_tgt n_src / ((n_src + n_tgt) V^2) with c = 2 pi^3 w, where
    w = 16 weighs one real-space pair (erfc, exp, image search) against one
    k-space term (measured on this code).
    """
    V = float(np.prod(box))
    c = 2.0 * math.pi ** 3 * 16.0
    return (c * n_tgt * n_src / ((n_src + n_tgt) * V * V)) ** (1.0 / 6.0)


def ewald(D, kernel, box, x, f=None, q=None, nu=None, targets=None, self_src=None,
          xi=None, margin=6.0):
    """Oracle potential u^{DP} (or u^{DP*}) at the targets.

    x: [ns,3] sources in [0,L); targets: [nt,3] (default: the sources, with the
    self interaction omitted).  self_src[m] = index of the source coinciding
    with target m, or -1.  Returns a Parts dict with 'real', 'fourier', 'k0',
    'self' (D>0) or 'direct' (D=0), and .total.
    """
    box = _prep(box)
    x = _prep(x)
    ns = x.shape[0]
    if targets is None:
        targets = x
        if self_src is None:
            self_src = np.arange(ns, dtype=np.int64)
    xt = _prep(targets)
    nt = xt.shape[0]
    if self_src is not None:
        self_src = np.ascontiguousarray(np.asarray(self_src, dtype=np.int64))
    a, b = _sources(kernel, f, q, nu)
    kid = KERNELS[kernel]
    L = lib()
    out = Parts()
    if D == 0:
        u = np.zeros((nt, 3))
        nco = L.oracle_direct_0p(kid, ns, _d(x), _d(a), _d(b) if b is not None else None,
                                 nt, _d(xt), _l(self_src), _d(u))
        out["direct"] = u
        out["coincident"] = int(nco)
        return out
    if xi is None:
        xi = choose_xi(ns, nt, box, margin)
    rc = margin / xi
    kmax = 2.0 * margin * xi
    ur = np.zeros((nt, 3))
    nco = L.oracle_real_part(D, kid, _d(box), float(xi), float(rc), ns, _d(x), _d(a),
                             _d(b) if b is not None else None, nt, _d(xt), _l(self_src), _d(ur))
    out["real"] = ur
    out["coincident"] = int(nco)
    uf = np.zeros((nt, 3))
    if D == 3:
        nk = L.oracle_fourier_part_3p(kid, _d(box), float(xi), float(kmax), ns, _d(x), _d(a),
                                      _d(b) if b is not None else None, nt, _d(xt), _d(uf))
    else:
        Lv = virtual_cell(D, box)
        nk = L.oracle_reduced_fourier_part(D, kid, _d(Lv), float(xi), float(kmax), ns, _d(x), _d(a),
                                           _d(b) if b is not None else None, nt, _d(xt), _d(uf))
        out["virtual_cell"] = tuple(float(v) for v in Lv)
    out["fourier"] = uf
    out["n_k"] = int(nk)
    u0 = np.zeros((nt, 3))
    if D == 3 and kernel == "stresslet":
        L.oracle_k0_stresslet_3p(_d(box), ns, _d(x), _d(a), _d(b), nt, _d(xt), _d(u0))
    elif D == 3 and kernel == "harmonic":
        # uniform neutralising background of each charge set: the k -> 0
        # limit of (4 pi/k^2)(gammaE - 1) Q/V = -pi Q / (V xi^2)
        V = float(box[0]) * float(box[1]) * float(box[2])
        u0[:] = -math.pi / (V * float(xi) ** 2) * np.sum(a, axis=0)[None, :]
    elif D in (1, 2):
        L.oracle_zero_mode(D, kid, _d(box), float(xi), ns, _d(x), _d(a), _d(b) if b is not None else None,
                           nt, _d(xt), _d(u0))
    out["k0"] = u0
    us = np.zeros((nt, 3))
    if self_src is not None:
        L.oracle_self_part(kid, float(xi), nt, _l(self_src), _d(a), _d(us))
    out["self"] = us
    out["xi"] = float(xi)
    return out


def virtual_cell(D, box, decay=7.0):
    """Period P_v of the trapezoidal rule in the free directions (D = 2, 1).

    For a mode with k^P != 0 the integrand over the free wavenumbers is
    analytic in a strip of half-width |k^P| >= 2 pi / max(L_periodic), so the
    trapezoidal rule with step 2 pi / P_v is in error by about
    exp(-2 pi (P_v - extent) / max(L_periodic)); decay = 7 puts that below
    e^{-43}.
    """
    box = np.asarray(box, dtype=np.float64)
    lp = float(np.max(box[:D]))
    ext = float(np.max(box[D:]))
    pv = ext + decay * lp
    Lv = box.copy()
    Lv[D:] = pv
    return np.ascontiguousarray(Lv)


def e1(x):
    """Exponential integral E1 as implemented in the oracle (pinned in tests)."""
    return float(lib().oracle_e1(float(x)))


def image_block_sum(D, kernel, box, x, f=None, q=None, nu=None, targets=None, self_src=None, K=10):
    """Symmetric-block truncation |pbar_i| <= K of eq. (periodic-potential)."""
    box = _prep(box)
    x = _prep(x)
    ns = x.shape[0]
    if targets is None:
        targets = x
        if self_src is None:
            self_src = np.arange(ns, dtype=np.int64)
    xt = _prep(targets)
    nt = xt.shape[0]
    if self_src is not None:
        self_src = np.ascontiguousarray(np.asarray(self_src, dtype=np.int64))
    a, b = _sources(kernel, f, q, nu)
    u = np.zeros((nt, 3))
    lib().oracle_image_block_sum(D, KERNELS[kernel], _d(box), int(K), ns, _d(x), _d(a),
                                 _d(b) if b is not None else None, nt, _d(xt), _l(self_src), _d(u))
    return u


def rms_rel_error(u, ref):
    """E_rms,rel of eq. (rel-rms-error): rms of |u - ref| over rms of |ref|."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    num = np.sqrt(np.mean(np.sum((u - ref) ** 2, axis=1)))
    den = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
    return float(num / den)


def rms_abs_error(u, ref):
    """E_rms of eq. (abs-rms-error)."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    return float(np.sqrt(np.mean(np.sum((u - ref) ** 2, axis=1))))
