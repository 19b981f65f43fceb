"""Throughput of one kernel and periodicity with analytic parameters.

One step binds the geometry and evaluates n_rhs strength sets on it, replayed
as one HIP graph (the batched form); the per-phase durations come from the
library's own HIP events on eager launches of the same plan.  Inputs: N
uniform sources = targets in the box, N(0,1) strengths (zero mean for
D = 3), seeded.  Prints one JSON line.

Usage: python -m paper_2210_01255_amd.kernel_bench --kernel harmonic --D 3
       [--n 1000000] [--tol 1e-8] [--nrhs 16] [--steps 5] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def run(kernel="harmonic", D=3, n=1_000_000, tol=1e-8, nrhs=16, steps=5, warmup=2, precision="fp64",
        safety=10.0, seed=6000):
    import torch

    import paper_2210_01255_amd as se
    dev = torch.device("cuda:0")
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.random((n, 3))
    f = g.standard_normal((nrhs, n, 3))
    if D == 3:
        f -= f.mean(axis=1, keepdims=True)
    nu = None
    if kernel == "stresslet":
        nu = g.standard_normal((n, 3))
        nu /= np.linalg.norm(nu, axis=1)[:, None]
    Q = float(np.sum(f ** 2)) / nrhs
    if kernel == "stresslet":
        Q = float(np.sum((f[..., :, None] * nu[None, :, None, :]) ** 2)) / nrhs
    xt = torch.tensor(x, device=dev)
    ft = torch.tensor(f if nrhs > 1 else f[0], device=dev)
    nut = torch.tensor(nu, device=dev) if nu is not None else None
    prob = dict(kernel=kernel, periodicity=D, tol=tol, n_src=n, source_q=Q, n_rhs=nrhs, safety=safety,
                precision=se.PREC_FP64 if precision == "fp64" else se.PREC_FP32)
    batch = se.Batch([prob])
    plan = batch.plans[0]
    out = torch.empty_like(ft)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def step():
        batch.set_geometry([xt], [nut] if nut is not None else None, stream=side)
        batch.execute([ft], [out], stream=side)

    with torch.cuda.stream(side):
        for _ in range(max(1, warmup)):
            step()
    side.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        for _ in range(steps):
            step()
    side.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # per-phase durations (eager launches, library events)
    plan.set_timing(True)
    plan.set_geometry(xt, nut)
    plan.execute(ft, out=out)
    plan.sync()
    ph = plan.phase_times()
    par = plan.params
    res = {"kernel": kernel, "D": D, "n": n, "tol": tol, "n_rhs": nrhs, "precision": precision,
           "ms_per_step": round(ms, 4), "targets_per_s": round(nrhs * n / (ms * 1e-3), 1),
           "params": {"xi": par["xi"], "rc": par["rc"], "M": par["M"], "P": par["P"]},
           "phases_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in ph.items() if v[1]}}
    batch.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kernel", default="harmonic")
    ap.add_argument("--D", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    a = ap.parse_args(argv)
    print(json.dumps(run(a.kernel, a.D, a.n, a.tol, a.nrhs, a.steps, a.warmup, a.precision)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
