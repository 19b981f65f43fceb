"""Benchmark: N = 1e6 triply periodic stokeslet at 1e-8 rms-relative error on one MI355X.

One step = one pass of the whole hot path over the batch: se_set_geometry (cell
list) + the evaluation (gridding, FFT, scaling, IFFT, gathering, real-space
sum, self term).  Two forms run on the same inputs: plain (analytic
parameters, one strength set per step) and learned+batched (learned
parameters, 16 strength sets on the shared geometry, binding and evaluation
replayed as HIP graphs); `value` is the latter's targets/s.  Inputs are resident in
HBM before the timed regions start.
Prints ONE JSON line, with the roofline of the dominant kernel (algorithmic
work per launch over its live duration, against the MI355X peak) and the FP64
oracle timed on a bounded sample of targets as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--nrhs", type=int, default=16,
                    help="strength sets on the shared geometry in the learned+batched form")
    ap.add_argument("--safety", type=float, default=10.0,
                    help="plain form: tau_abs divisor; 10 makes 'error <= tol' hold across the estimate's band")
    ap.add_argument("--nrc", type=float, default=0.0,
                    help="plain form: expected sources within rc (0: the paper's table value)")
    ap.add_argument("--pollution", type=int, default=0,
                    help="plain form: error-pollution rule, 0 (h/1.05, P+4) as the paper applies it for D = 3, "
                         "or 1 (h/1.1, P+2)")
    ap.add_argument("--cpu-sample", type=int, default=2000, help="targets in the oracle sample (0: skip)")
    ap.add_argument("--tune", type=int, default=0, help="run the batch autotuner before timing (1; at the default "
                    "workload it keeps the automatic shapes) or use the automatic launch shapes (0)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the run, one plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


# Algorithmic FP64 work of one real-space pair (r^2, erfc, exp, the stokeslet
# tensor contraction), counted as in the cost model of the real-space sum.
REAL_FLOP_PER_PAIR = 70.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_metric_stokeslet_1e6.json")
KERNEL_SOURCES = {"real_space": "se_real.hip", "spread": "se_spread.hip", "gather": "se_spread.hip",
                  "fft_fwd_xy": "se_fft.hip", "fft_z_scale": "se_fft.hip", "fft_inv_yx": "se_fft.hip"}


def source_digest(phase):
    import hashlib
    path = os.path.join(ROOT, "paper_2210_01255_amd", "csrc", KERNEL_SOURCES[phase])
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(phase):
    """HBM bytes per launch of the phase's kernel in the learned+batched form,
    from the committed FETCH_SIZE / WRITE_SIZE counter runs (scaled by the
    copy-kernel calibration), or None when they were taken on another version
    of the kernel's source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh).get("phases", {}).get(phase)
    except (OSError, ValueError, AttributeError):
        return None
    if not t or t.get("source_sha") != source_digest(phase):
        return None
    return t.get("bytes_per_launch")


def roofline_for(phase, ms_per_launch, par, n_src, n_tgt, ncomp, fp64, box_vol=1.0, slots=1):
    """Algorithmic work of one launch of the phase divided by its duration
    (a launch covers `slots` right-hand sides)."""
    r = _roofline_one(phase, ms_per_launch / slots, par, n_src, n_tgt, ncomp, fp64, box_vol)
    if r is not None:
        r["work_per_launch"] *= slots
    return r


def hbm_bytes(phase, par, n_src, n_tgt, ncomp, fp64, slots=1):
    """Algorithmic HBM bytes of one launch of a phase: every input read once
    and every output written once (a launch covers `slots` right-hand sides,
    `ncomp` components each)."""
    rs = 8 if fp64 else 4
    M = par["M"]
    grid = M[0] * M[1] * M[2] * rs
    nc = ncomp * slots
    if phase == "spread":   # positions, strengths -> grid
        return n_src * (24 + 8 * nc) + nc * grid
    if phase == "gather":   # grid, positions -> FP64 accumulators
        return nc * grid + n_tgt * (24 + 8 * nc)
    if phase == "real_space":  # positions and strengths of sources and targets -> u
        return n_src * (24 + 8 * nc) + n_tgt * (24 + 8 * nc)
    r = _roofline_one(phase, 1.0, par, n_src, n_tgt, ncomp, fp64)
    return r["work_per_launch"] * slots if r is not None and r["unit"] == "GB/s" else None


def _roofline_one(phase, ms_per_launch, par, n_src, n_tgt, ncomp, fp64, box_vol=1.0):
    P = par["P"]
    M = par["M"]
    sec = ms_per_launch * 1e-3
    if phase == "real_space":
        # pairs within rc of a uniform system: N (N - 1) (4 pi/3) rc^3 / V
        pairs = n_tgt * (n_src - 1) * (4.0 * math.pi / 3.0) * par["rc"] ** 3 / box_vol
        flops = REAL_FLOP_PER_PAIR * pairs
        return {"bound": "alu", "achieved": flops / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "work_per_launch": flops}
    if phase == "spread":
        flops = 2.0 * P ** 3 * ncomp * n_src  # P^3 ncomp FMAs per source
        return {"bound": "alu", "achieved": flops / sec / 1e12,
                "peak": PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "work_per_launch": flops}
    if phase == "gather":
        flops = 2.0 * P ** 3 * 3 * n_tgt
        return {"bound": "alu", "achieved": flops / sec / 1e12,
                "peak": PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "work_per_launch": flops}
    rs = 8 if fp64 else 4
    hx = M[0] // 2 + 1
    spec = hx * M[1] * M[2] * 2 * rs  # one complex half-spectrum component
    grid = M[0] * M[1] * M[2] * rs
    if phase == "fft_fwd_xy":
        byt = ncomp * (grid + spec) + ncomp * 2 * spec  # x: read grid, write spec; y: read+write
    elif phase == "fft_z_scale":
        byt = ncomp * spec + 3 * spec
    elif phase == "fft_inv_yx":
        byt = 3 * 2 * spec + 3 * (spec + grid)
    else:
        return None
    return {"bound": "hbm", "achieved": byt / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "work_per_launch": byt}


def cpu_model():
    """The host CPU's model name (lscpu's "Model name" field)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (--gpus %d requested); nothing is launched."
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2210_01255_amd as se

    dev = torch.device("cuda:0")
    n, nrhs = args.n, max(1, args.nrhs)
    s = W.system(args.seed, n, kernel="stokeslet", zero_mean=True, n_rhs=nrhs)
    x = torch.tensor(s["x"], device=dev)
    f = torch.tensor(s["f"], device=dev)         # [nrhs, n, 3]
    f0 = f[0].contiguous()                         # the plain form's strengths: the first set
    Q = float(np.sum(s["f"] ** 2)) / nrhs          # per right-hand side
    common = dict(kernel="stokeslet", periodicity=3, box=(1.0, 1.0, 1.0), tol=args.tol, tol_kind=se.TOL_REL,
                  n_src=n, source_q=Q, precision=se.PREC_FP64)

    # ---- plain: analytic parameters (Sec. 4.6 with the paper's table values), one rhs
    plan = se.Plan(safety=args.safety, n_rc=args.nrc, pollution=args.pollution, **common)
    u0 = torch.empty((n, 3), dtype=torch.float64, device=dev)

    def plain_step():
        plan.set_geometry(x)
        plan.execute(f0, out=u0)

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()
    plan.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    plain_par = plan.params

    # ---- learned + batched: learned parameters, nrhs sets on the shared
    # geometry, binding and evaluation each replayed as a HIP graph on a side stream
    batch = se.Batch([dict(selector=se.SELECT_LEARNED, n_rhs=nrhs, **common)])
    bplan = batch.plans[0]
    fb = f if nrhs > 1 else f0
    ub = torch.empty_like(fb)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def batched_step():
        batch.set_geometry([x], stream=side)
        batch.execute([fb], [ub], stream=side)

    # the batch's autotuner (real-space blocking, FFT column bundles), part
    # of setting the batch up like plan creation, outside the timed region
    with torch.cuda.stream(side):
        batch.set_geometry([x], stream=side)
        tuned = batch.tune([fb], [ub], stream=side)[0] if args.tune else (0, 0, 0)
    side.synchronize()
    with torch.cuda.stream(side):
        for _ in range(max(1, args.warmup)):
            batched_step()
    side.synchronize()
    bplan.sync()
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        for _ in range(args.steps):
            batched_step()
    side.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    value = nrhs * n / (ms_per_step * 1e-3)
    plain_value = n / (plain_ms * 1e-3)
    par = bplan.params

    # live per-phase durations of the same kernels (eager launches with HIP
    # events on the launch stream; a replayed graph carries no events)
    bplan.set_timing(True)
    with torch.cuda.stream(side):
        for _ in range(args.steps):
            bplan.set_geometry(x, stream=side)
            bplan.execute(fb, out=ub, stream=side)
    side.synchronize()
    phases = bplan.phase_times()
    bplan.set_timing(False)
    slots = 2 if nrhs >= 2 else 1  # right-hand sides per chunk of the phases (stokeslet)
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()}
    dom = max((k for k in per_launch if k not in ("geometry",)), key=lambda k: per_launch[k])
    rl = roofline_for(dom, per_launch[dom], par, n, n, 3, True, slots=slots)
    roof = None
    if rl is not None:
        roof = {"kernel": dom, "bound": rl["bound"], "achieved": round(rl["achieved"], 4), "peak": rl["peak"],
                "unit": rl["unit"], "frac": round(rl["achieved"] / rl["peak"], 5),
                "traffic": measured_traffic(dom), "ms_per_launch": round(per_launch[dom], 4),
                "work_per_launch": rl["work_per_launch"]}
    # every phase against its binding roofline and against HBM: the
    # algorithmic bytes, and the counter-measured bytes where they were taken
    # on the current kernel source, over the live launch duration
    phase_frac = {}
    for k, v in per_launch.items():
        r = roofline_for(k, v, par, n, n, 3, True, slots=slots) if v > 0 else None
        if r is not None:
            e = {"bound": r["bound"], "frac": round(r["achieved"] / r["peak"], 5)}
            b = hbm_bytes(k, par, n, n, 3, True, slots=slots)
            if b:
                e["hbm_frac"] = round(b / (v * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)
            t = measured_traffic(k)
            if t:
                e["hbm_frac_measured"] = round(t / (v * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)
            phase_frac[k] = e

    if args.copy_calib_mib > 0:
        nel = args.copy_calib_mib * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)                  # runtime blit kernel
        torch.mul(a, 1.0, out=b)    # compiled elementwise kernel: reads and writes the size once
        torch.cuda.synchronize()
        del a, b

    cpu = None
    err_plain = err_batched = None
    if args.cpu_sample > 0:
        import oracle
        oracle.build(force=False)
        idx = np.sort(W.rng(args.seed + 1).choice(n, args.cpu_sample, replace=False))
        c0 = time.perf_counter()
        ref = oracle.ewald(3, "stokeslet", [1.0, 1.0, 1.0], s["x"], f=s["f"][0], targets=s["x"][idx],
                           self_src=idx)
        c1 = time.perf_counter()
        cores = os.cpu_count()
        try:
            cores = len(os.sched_getaffinity(0))
        except Exception:
            pass
        omp = os.environ.get("OMP_NUM_THREADS")
        if omp:
            cores = min(cores, int(omp))
        cpu = {"value": round(args.cpu_sample / (c1 - c0), 4), "unit": "targets/s", "cores": cores,
               "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
               "sample": "%d of %d targets (all %d sources), FP64 classical Ewald, xi_o=%.3f, %.1f s"
                         % (args.cpu_sample, n, n, ref["xi"], c1 - c0)}
        err_plain = oracle.rms_rel_error(u0.cpu().numpy()[idx], ref.total)
        ub0 = ub[0] if nrhs > 1 else ub
        err_batched = oracle.rms_rel_error(ub0.cpu().numpy()[idx], ref.total)

    def pdesc(p):
        return {"xi": round(p["xi"], 4), "rc": round(p["rc"], 5), "M": p["M"], "P": p["P"]}

    out = {
        "metric": "targets/sec at 1e-8 rms-rel err, N=1M TP stokeslet; learned+batched vs plain",
        "value": round(value, 1),
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "triply periodic stokeslet, unit cube, N=1e6 uniform sources = targets, "
                               "f~N(0,1)^3 zero mean, tol 1e-8 rms-rel, FP64; learned parameters, %d strength "
                               "sets on the shared geometry; binding and evaluation replayed as HIP graphs" % nrhs,
                   "form": "learned+batched", "n_rhs": nrhs, "learned": pdesc(par),
                   "launch_shape": {"real_tb": int(tuned[0]), "fft_cols": int(tuned[1]),
                                    "tile_items": int(tuned[2]), "autotuned": bool(args.tune)},
                   "plain": dict(pdesc(plain_par), safety=args.safety, n_rc=args.nrc or 400.0,
                                 pollution_rule=["h/1.05,P+4", "h/1.1,P+2"][args.pollution])},
        "plain": {"value": round(plain_value, 1), "ms_per_step": round(plain_ms, 4),
                  "err_rms_rel_sample": err_plain},
        "speedup_vs_plain": round(value / plain_value, 4),
        "err_rms_rel_sample": err_batched,
        "phases_ms": {k: round(v, 4) for k, v in per_launch.items()},
        "phases_roofline": phase_frac,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
