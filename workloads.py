"""Seeded synthetic particle systems shaped like the paper's workloads.

This module only draws random numbers; it holds none of the method's
arithmetic and is shared by the tests, the benchmark and the smoke entry
point so that the oracle and the GPU path see byte-identical inputs.

Recipes (paper, "Numerical results" and the error-estimate examples):
  * uniform systems: positions iid uniform in the primary cell;
  * clustered systems: points drawn around cluster centres (Gaussian clouds),
    or the paper's two-corner layout [0,1/3)^3 U [2/3,1)^3;
  * strengths: components iid N(0,1), optionally with the mean removed
    (zero net force);
  * stresslet sources f_lm = q_l nu_m with q ~ N(0,1)^3 and nu uniform on
    the unit sphere.

Draw order inside one call is fixed: positions, then strengths, then normals.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_points(g: np.random.Generator, n: int, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    x = g.random((n, 3)) * box[None, :]
    # keep strictly inside [0, L)
    return np.minimum(x, np.nextafter(box, 0.0)[None, :])


def corner_clustered_points(g: np.random.Generator, n: int, box) -> np.ndarray:
    """Points only in [0,L/3)^3 U [2L/3,L)^3 (the paper's clustered system)."""
    box = np.asarray(box, dtype=np.float64)
    x = g.random((n, 3)) * (box[None, :] / 3.0)
    half = g.random(n) < 0.5
    x[half] += 2.0 * box[None, :] / 3.0
    return np.minimum(x, np.nextafter(box, 0.0)[None, :])


def gaussian_clustered_points(g: np.random.Generator, n: int, box, n_clusters: int,
                              sigma: float, periodicity: int) -> np.ndarray:
    """Gaussian clouds around uniform centres; periodic axes wrap, free axes redraw."""
    box = np.asarray(box, dtype=np.float64)
    centres = g.random((n_clusters, 3)) * box[None, :]
    which = g.integers(0, n_clusters, size=n)
    x = centres[which] + sigma * g.standard_normal((n, 3))
    for ax in range(3):
        if ax < periodicity:
            x[:, ax] = np.mod(x[:, ax], box[ax])
        else:
            bad = (x[:, ax] < 0) | (x[:, ax] >= box[ax])
            while np.any(bad):
                k = int(bad.sum())
                x[bad, ax] = centres[which[bad], ax] + sigma * g.standard_normal(k)
                bad = (x[:, ax] < 0) | (x[:, ax] >= box[ax])
    return np.minimum(np.maximum(x, 0.0), np.nextafter(box, 0.0)[None, :])


def mixed_points(g, n, box, n_clusters=10, sigma=0.02, periodicity=3):
    """Half uniform, half in Gaussian clusters."""
    n_u = n // 2
    a = uniform_points(g, n_u, box)
    b = gaussian_clustered_points(g, n - n_u, box, n_clusters, sigma, periodicity)
    return np.concatenate([a, b], axis=0)


def normal_strengths(g: np.random.Generator, n: int, zero_mean: bool = False,
                     n_rhs: int | None = None) -> np.ndarray:
    shape = (n, 3) if n_rhs is None else (n_rhs, n, 3)
    f = g.standard_normal(shape)
    if zero_mean:
        f = f - f.mean(axis=-2, keepdims=True)
    return f


def unit_normals(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def loguniform_sizes(g: np.random.Generator, count: int, lo: float, hi: float) -> np.ndarray:
    return np.round(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def aspect_box(g: np.random.Generator, lo: float = 1.0, hi: float = 4.0) -> np.ndarray:
    """Unit box with one random axis stretched by a ~ U[lo, hi]."""
    box = np.ones(3)
    box[int(g.integers(0, 3))] = g.uniform(lo, hi)
    return box


def system(seed: int, n: int, box=(1.0, 1.0, 1.0), kernel: str = "stokeslet",
           layout: str = "uniform", zero_mean: bool = False, periodicity: int = 3,
           n_rhs: int | None = None):
    """One seeded system: dict with x, and f (S/Rotlet) or q and nu (stresslet)."""
    g = rng(seed)
    if layout == "uniform":
        x = uniform_points(g, n, box)
    elif layout == "corners":
        x = corner_clustered_points(g, n, box)
    elif layout == "mixed":
        x = mixed_points(g, n, box, periodicity=periodicity)
    else:
        raise ValueError(layout)
    out = {"x": x, "box": np.asarray(box, dtype=np.float64)}
    if kernel == "stresslet":
        out["q"] = normal_strengths(g, n, zero_mean=zero_mean, n_rhs=n_rhs)
        out["nu"] = unit_normals(g, n)
    else:
        out["f"] = normal_strengths(g, n, zero_mean=zero_mean, n_rhs=n_rhs)
    return out
