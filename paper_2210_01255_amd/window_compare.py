"""Window comparison of Sec. 5.3 (PKB against the truncated Gaussian): time of
gridding plus gathering against the rms-relative error of the Fourier-space
part, triply periodic, uniform sources.

Setup as in the paper's comparison: N = 1e5 uniform sources in the unit cube
with Q = 1, xi from its table of decomposition parameters (uniform system,
D = 3), a grid fine enough that the truncation error is negligible (M = 196
stokeslet, 192 stresslet; 210 rotlet, the nearest size with radices 2-7 to the
paper's 208), window support P = 2 .. 14 (PKB) and 2 .. 24 (TG), and as
reference the same grid with the PKB window at P = 20.  Errors and times are
averaged over several seeded point configurations.

Usage: python -m paper_2210_01255_amd.window_compare [--configs 5] [--out FILE]
Prints one JSON line per (kernel, window, P) and a summary table.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

XI = {"stokeslet": 43.0296, "stresslet": 39.4021, "rotlet": 45.4936}
GRID = {"stokeslet": 196, "stresslet": 192, "rotlet": 210}
P_RANGE = {"pkb": list(range(2, 15, 2)), "tg": list(range(2, 25, 2))}
P_REF = 20


def _inputs(kernel, seed, n):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.random((n, 3))
    if kernel == "stresslet":
        q = g.standard_normal((n, 3))
        nu = g.standard_normal((n, 3))
        nu /= np.linalg.norm(nu, axis=1)[:, None]
        q /= np.sqrt(np.sum(q ** 2))  # Q = sum |q|^2 |nu|^2 = 1
        return x, q, nu
    f = g.standard_normal((n, 3))
    f -= f.mean(axis=0)
    f /= np.sqrt(np.sum(f ** 2))      # Q = sum |f|^2 = 1
    return x, f, None


def _fourier_part(se, torch, kernel, window, P, x, a, nu, reps):
    n = len(x)
    xi = XI[kernel]
    m = se.se_params()
    m.struct_size = se.ctypes.sizeof(se.se_params)
    m.xi, m.rc, m.P = xi, 3.5 / xi, P
    for i in range(3):
        m.M[i] = GRID[kernel]
    plan = se.Plan(m, kernel=kernel, periodicity=3, tol=1e-8, n_src=n, source_q=1.0,
                   selector=se.SELECT_MANUAL, precision=se.PREC_FP64, window=window)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev)
    at = torch.tensor(a, device=dev)
    nut = torch.tensor(nu, device=dev) if nu is not None else None
    plan.set_geometry(xt, nut)
    _, uf = plan.execute_split(at)
    plan.sync()
    plan.set_timing(True)
    for _ in range(reps):
        plan.execute_split(at)
    plan.sync()
    ph = plan.phase_times()
    ms = sum(ph[k][0] for k in ("spread", "gather")) / reps
    out = uf.cpu().numpy()
    plan.close()
    return out, ms


def run(configs=5, n=100_000, reps=3, kernels=("stokeslet", "rotlet", "stresslet"), out=None):
    import torch

    import paper_2210_01255_amd as se
    rows = []
    for kernel in kernels:
        acc = {}
        for c in range(configs):
            x, a, nu = _inputs(kernel, 7700 + c, n)
            ref, _ = _fourier_part(se, torch, kernel, "pkb", P_REF, x, a, nu, 1)
            rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
            for window, Ps in P_RANGE.items():
                for P in Ps:
                    u, ms = _fourier_part(se, torch, kernel, window, P, x, a, nu, reps)
                    err = np.sqrt(np.mean(np.sum((u - ref) ** 2, axis=1))) / rms
                    e, t = acc.get((window, P), (0.0, 0.0))
                    acc[(window, P)] = (e + err / configs, t + ms / configs)
            print("%s: configuration %d done" % (kernel, c), flush=True)
        for (window, P), (err, ms) in sorted(acc.items()):
            row = {"kernel": kernel, "window": window, "P": P, "M": GRID[kernel], "xi": XI[kernel], "n": n,
                   "configs": configs, "err_fourier_rms_rel": err, "spread_gather_ms": ms}
            rows.append(row)
            print(json.dumps(row), flush=True)
    # time to reach each error level with either window
    print("\n| kernel | error level | PKB: P, ms | TG: P, ms | TG/PKB time |")
    print("|---|---|---|---|---|")
    for kernel in kernels:
        for lvl in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11):
            best = {}
            for w in ("pkb", "tg"):
                ok = [r for r in rows if r["kernel"] == kernel and r["window"] == w and r["err_fourier_rms_rel"] <= lvl]
                best[w] = min(ok, key=lambda r: r["P"]) if ok else None
            if best["pkb"] and best["tg"]:
                print("| %s | %.0e | %d, %.3f | %d, %.3f | %.2f |" % (
                    kernel, lvl, best["pkb"]["P"], best["pkb"]["spread_gather_ms"], best["tg"]["P"],
                    best["tg"]["spread_gather_ms"], best["tg"]["spread_gather_ms"] / best["pkb"]["spread_gather_ms"]))
    if out:
        with open(out, "w") as fh:
            json.dump(rows, fh, indent=1)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--configs", type=int, default=5)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--kernels", default="stokeslet,rotlet,stresslet")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    run(a.configs, a.n, a.reps, tuple(a.kernels.split(",")), a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
