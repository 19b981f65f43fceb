"""Training data, training and evaluation of the learned parameter selector.

The selector is a small network (se_selector_* in the library) that maps a
problem's features (log10 N, box elongation, periodicity, kernel, log10 of
the rms-relative tolerance) to (xi, h, P, rc).  Its training records are
runs of the method itself:

* ``generate``: for each sampled problem, a reference (the direct Ewald sum,
  se_ewald_reference, for D = 3 and 0; the same method at a much tighter
  tolerance for D = 2 and 1, where the direct sum's Fourier integrals are too
  slow at large N), then candidate parameter sets from the analytic procedure
  of Sec. 4.6 with varied n_rc (Sec. 5.2) and safety factor, each also run
  with its window support lowered by 2 (the free-direction parameters then
  completed as the procedure does); each run records its parameters, the
  measured time of se_set_geometry + se_execute and the measured rms-relative
  error against the reference.
* ``labels``: per problem, the fastest run whose measured error is within
  ``margin`` times the tolerance.
* ``train``: se_selector_train on the labels, then se_selector_save.

Command line (GPU):
    python -m paper_2210_01255_amd.selector generate --seed 0 --first 0 --count 100 --out runs0.npz
    python -m paper_2210_01255_amd.selector train --runs runs0.npz runs1.npz --out weights.bin
    python -m paper_2210_01255_amd.selector evaluate --weights weights.bin --random 40
"""
from __future__ import annotations

import argparse
import ctypes
import math
import sys
import time

import numpy as np

from . import (KERNELS, MLP_IN, MLP_OUT, POLLUTION_FINE, POLLUTION_PAPER, PREC_FP64, SE_OK, SELECT_MANUAL, SEError,
               Plan, ewald_reference, lib, make_problem, se_params, se_train_cfg)

# Expected sources within rc for the uniform system, Table 3 (rows: stokeslet
# and rotlet, stresslet; columns D = 0..3): the candidates scale these.
NRC_TABLE = {0: (2500.0, 950.0, 450.0, 400.0), 1: (2500.0, 950.0, 450.0, 400.0), 2: (6000.0, 1600.0, 800.0, 800.0)}
NRC_SCALE = (0.06, 0.1, 0.15, 0.25, 0.4)
SAFETY_PERIODIC = (0.3, 1.0, 3.0, 10.0)
SAFETY_FREE = (0.3, 1.2, 5.0, 20.0)

FIELDS = ("problem", "N", "D", "kernel", "aspect", "box0", "box1", "box2", "tol", "n_rc", "safety", "pollution",
          "xi", "rc", "h", "P", "M0", "M1", "M2", "create_ms", "geom_ms", "exec_ms", "err", "ok", "dP", "ref")


def features(N, D, kernel, box, tol) -> np.ndarray:
    """Feature row through the library (se_selector_features)."""
    prob = make_problem(kernel=int(kernel), periodicity=int(D), box=tuple(float(b) for b in box), tol=float(tol),
                        n_src=int(N))
    x = (ctypes.c_float * MLP_IN)()
    st = lib.se_selector_features(ctypes.byref(prob), x)
    if st != SE_OK:
        raise SEError(st, "se_selector_features")
    return np.array(x[:], dtype=np.float32)


def targets_of(xi, h, P, rc, box) -> np.ndarray:
    """Network outputs of a parameter set: ln(xi Lc), ln(Lc/h), P, ln(xi rc)."""
    Lc = float(np.prod(box)) ** (1.0 / 3.0)
    return np.array([math.log(xi * Lc), math.log(Lc / h), float(P), math.log(xi * rc)], dtype=np.float32)


def sample_problem(g: np.random.Generator, n_min: float = 1e3):
    N = int(round(math.exp(g.uniform(math.log(n_min), math.log(1e6)))))
    D = int(g.integers(0, 4))
    kernel = int(g.integers(0, 3))
    box = np.ones(3)
    if g.random() < 0.5:
        box[int(g.integers(0, 3))] = g.uniform(1.0, 4.0)
    tol = 10.0 ** g.uniform(-10.0, -4.0)
    return N, D, kernel, box, tol


def _system(g, N, D, kernel, box):
    x = g.uniform(size=(N, 3)) * box[None, :]
    if kernel == KERNELS["stresslet"]:
        q = g.standard_normal((N, 3))
        nu = g.standard_normal((N, 3))
        nu /= np.linalg.norm(nu, axis=1, keepdims=True)
        Q = float(np.sum((q[:, :, None] * nu[:, None, :]) ** 2))
        return x, q, nu, Q
    f = g.standard_normal((N, 3))
    if D == 3 and kernel == KERNELS["stokeslet"]:
        f -= f.mean(axis=0, keepdims=True)
    return x, f, None, float(np.sum(f * f))


def candidates(D, kernel):
    """(n_rc, safety, pollution rule) sets; the finer pollution rule (h/1.1,
    P+2) is faster on this hardware in nearly every measured case, so the
    search spends its runs on n_rc and the safety factor."""
    base = NRC_TABLE[kernel][D]
    safeties = SAFETY_FREE if D == 0 else SAFETY_PERIODIC
    return [(s * base, c, POLLUTION_FINE) for s in NRC_SCALE for c in safeties]


def lowered_window(par, D):
    """Manual parameters of an analytic set with the window support lowered
    by 2: the same xi, rc and periodic grid (D = 0: the spacing), from which
    the free directions are completed."""
    m = se_params()
    m.struct_size = ctypes.sizeof(se_params)
    m.xi, m.rc, m.P = par["xi"], par["rc"], par["P"] - 2
    for i in range(D):
        m.M[i] = par["M"][i]
    if D == 0:
        m.h[0] = min(par["h"]) * (1.0 + 1e-12)
    return m


def _timed(plan, x, str_, nu, out, reps):
    import torch
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    plan.set_geometry(x, nu)
    plan.execute(str_, out=out)
    e0.record()
    plan.set_geometry(x, nu)
    e1.record()
    for _ in range(reps):
        plan.execute(str_, out=out)
    e2.record()
    e2.synchronize()
    return e0.elapsed_time(e1), e1.elapsed_time(e2) / reps


def generate(seed: int, first: int, count: int, out_path: str, max_seconds: float = 1e9, reps: int = 3, ids=None,
             n_min: float = 1e3):
    """Runs for problems first .. first+count-1 of the seeded problem stream
    (or for the listed problem ids)."""
    import torch
    dev = torch.device("cuda:0")
    t_start = time.time()
    rows = []
    pids = list(ids) if ids is not None else list(range(first, first + count))
    for k, pid in enumerate(pids):
        if time.time() - t_start > max_seconds:
            print("time budget reached before problem %d" % pid, flush=True)
            break
        g = np.random.default_rng([seed, pid])
        N, D, kernel, box, tol = sample_problem(g, n_min)
        x, s, nu, Q = _system(g, N, D, kernel, box)
        xd = torch.tensor(x, device=dev)
        sd = torch.tensor(s, device=dev)
        nud = torch.tensor(nu, device=dev) if nu is not None else None
        common = dict(kernel=kernel, periodicity=D, box=tuple(box), n_src=N, source_q=Q, precision=PREC_FP64)
        try:
            if D in (3, 0):
                ref = ewald_reference(kernel, D, tuple(box), xd, sd, nud)
                torch.cuda.synchronize()
                ref_kind = 1
            else:
                tol_ref = max(min(tol * 1e-3, 1e-11), 1e-13)
                ref_plan = Plan(tol=tol_ref, safety=10.0, **common)
                ref_plan.set_geometry(xd, nud)
                ref = ref_plan.execute(sd)
                ref_plan.sync()
                del ref_plan
                ref_kind = 0
        except SEError as e:
            print("problem %d N=%d D=%d k=%d tol=%.1e: no reference (%s)" % (pid, N, D, kernel, tol, e), flush=True)
            continue
        rnorm = torch.linalg.vector_norm(ref).item()
        out = torch.empty_like(ref)
        aspect = float(box.max() / box.min())
        best = None

        def run(row, make):
            nonlocal best
            try:
                t0 = time.time()
                plan = make()
                cms = 1e3 * (time.time() - t0)
                gms, ems = _timed(plan, xd, sd, nud, out, reps)
                plan.sync()
                err = (torch.linalg.vector_norm(out - ref).item() / rnorm)
                par = plan.params
                hmin = min(par["h"][i] for i in range(3) if (i < D or D == 0))
                row.update(xi=par["xi"], rc=par["rc"], h=hmin, P=par["P"], M0=par["M"][0], M1=par["M"][1],
                           M2=par["M"][2], create_ms=cms, geom_ms=gms, exec_ms=ems, err=err, ok=1)
                del plan
                if err <= tol and (best is None or gms + ems < best):
                    best = gms + ems
                return par
            except SEError:
                row.update(xi=0, rc=0, h=0, P=0, M0=0, M1=0, M2=0, create_ms=0, geom_ms=0, exec_ms=0, err=np.inf, ok=0)
                return None

        for (nrc, safety, pol) in candidates(D, kernel):
            base = dict(problem=pid, N=N, D=D, kernel=kernel, aspect=aspect, box0=box[0], box1=box[1], box2=box[2],
                        tol=tol, n_rc=nrc, safety=safety, pollution=pol, ref=ref_kind)
            row = dict(base, dP=0)
            par = run(row, lambda: Plan(tol=tol, n_rc=nrc, safety=safety, pollution=pol, **common))
            rows.append(row)
            if par is not None and par["P"] - 2 >= 4:
                row = dict(base, dP=2)
                m = lowered_window(par, D)
                rows.append(row)
                run(row, lambda: Plan(m, tol=tol, safety=safety, selector=SELECT_MANUAL, **common))
        print("problem %d N=%d D=%d k=%d aspect=%.2f tol=%.1e: best %s ms (%.0f s)" %
              (pid, N, D, kernel, aspect, tol, "%.3f" % best if best else "-", time.time() - t_start), flush=True)
        torch.cuda.empty_cache()
        if k % 25 == 24:
            _save_runs(rows, out_path)
    return _save_runs(rows, out_path)


def _save_runs(rows, out_path):
    arr = {k: np.array([r[k] for r in rows], dtype=np.float64) for k in FIELDS}
    np.savez_compressed(out_path, **arr)
    return arr


def evaluate(problems, seed=0, reps=3, plain_safety=10.0):
    """Plain (analytic, Table 3 n_rc, the paper's pollution rule, safety
    plain_safety) against learned parameters on each (N, D, kernel, box, tol):
    measured time of se_set_geometry + se_execute and rms-relative error
    on every target against the direct Ewald reference (se_ewald_reference,
    no grid or window; checked against the oracle to 1e-12).  Returns a list
    of dicts."""
    import torch
    from . import SELECT_LEARNED, ewald_reference
    dev = torch.device("cuda:0")
    rows = []
    for i, (N, D, kernel, box, tol) in enumerate(problems):
        g = np.random.default_rng([seed, 7919, i])
        box = np.asarray(box, dtype=np.float64)
        x, s, nu, Q = _system(g, int(N), D, kernel, box)
        xd, sd = torch.tensor(x, device=dev), torch.tensor(s, device=dev)
        nud = torch.tensor(nu, device=dev) if nu is not None else None
        common = dict(kernel=kernel, periodicity=D, box=tuple(box), n_src=int(N), source_q=Q, precision=PREC_FP64)
        t0 = time.perf_counter()
        ref = ewald_reference(kernel, D, tuple(box), xd, sd, nud)
        torch.cuda.synchronize()
        ref_s = time.perf_counter() - t0
        rnorm = torch.linalg.vector_norm(ref).item()
        out = torch.empty_like(ref)
        row = dict(N=int(N), D=D, kernel=kernel, aspect=float(box.max() / box.min()), tol=tol, ref_s=ref_s)
        for name, kw in (("plain", dict(safety=plain_safety, pollution=POLLUTION_PAPER)),
                         ("learned", dict(selector=SELECT_LEARNED))):
            plan = Plan(tol=tol, **kw, **common)
            gms, ems = _timed(plan, xd, sd, nud, out, reps)
            plan.sync()
            row[name + "_ms"] = gms + ems
            row[name + "_err"] = torch.linalg.vector_norm(out - ref).item() / rnorm
            row[name + "_M"] = list(plan.params["M"])
            row[name + "_P"] = plan.params["P"]
            if name == "learned":
                row["learned_msg"] = plan.message
            del plan
        print("eval %d N=%d D=%d k=%d aspect=%.2f tol=%.0e: plain %.3f ms err %.2e | learned %.3f ms err %.2e (%s)"
              " [reference %.1f s]" % (i, N, D, kernel, row["aspect"], tol, row["plain_ms"], row["plain_err"],
                                       row["learned_ms"], row["learned_err"], row["learned_msg"], ref_s), flush=True)
        rows.append(row)
        torch.cuda.empty_cache()
    return rows


METRIC_PROBLEMS = [(1_000_000, D, 0, (1.0, 1.0, 1.0), tol) for D in (3, 0) for tol in (1e-4, 1e-6, 1e-8, 1e-10)]


def load_runs(paths):
    parts = [np.load(p) for p in paths]
    return {k: np.concatenate([p[k] if k in p.files else np.zeros(len(p["problem"])) for p in parts])
            for k in FIELDS}


def labels(runs, margin=0.3):
    """(X, Y, problem ids): per problem the fastest run with err <= margin*tol."""
    X, Y, ids = [], [], []
    prob = runs["problem"].astype(np.int64)
    for pid in np.unique(prob):
        sel = np.nonzero((prob == pid) & (runs["ok"] > 0))[0]
        good = sel[runs["err"][sel] <= margin * runs["tol"][sel]]
        if good.size == 0:
            continue
        t = runs["geom_ms"][good] + runs["exec_ms"][good]
        i = good[int(np.argmin(t))]
        box = np.array([runs["box0"][i], runs["box1"][i], runs["box2"][i]])
        X.append(features(runs["N"][i], runs["D"][i], runs["kernel"][i], box, runs["tol"][i]))
        Y.append(targets_of(runs["xi"][i], runs["h"][i], runs["P"][i], runs["rc"][i], box))
        ids.append(pid)
    return np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32), np.array(ids)


def train(X, Y, epochs=150, batch=64, lr=1e-3, seed=1, device=0):
    """se_selector_train; returns the per-epoch loss."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    cfg = se_train_cfg()
    cfg.struct_size = ctypes.sizeof(se_train_cfg)
    cfg.epochs, cfg.batch, cfg.device = int(epochs), int(batch), int(device)
    cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = float(lr), 0.9, 0.999, 1e-8
    cfg.seed = int(seed)
    hist = np.zeros(int(epochs), dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    st = lib.se_selector_train(ctypes.byref(cfg), X.ctypes.data_as(fp), Y.ctypes.data_as(fp), len(X),
                               hist.ctypes.data_as(fp))
    if st != SE_OK:
        raise SEError(st, "se_selector_train")
    return hist


def predict(X):
    """Raw outputs for raw feature rows through se_selector_predict (GPU)."""
    import torch
    Xd = torch.tensor(np.asarray(X, dtype=np.float32), device="cuda:0")
    Yd = torch.empty((len(X), MLP_OUT), dtype=torch.float32, device="cuda:0")
    st = lib.se_selector_predict(ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Yd.data_ptr()), len(X),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != SE_OK:
        raise SEError(st, "se_selector_predict")
    return Yd.cpu().numpy()


def save(path):
    st = lib.se_selector_save(path.encode())
    if st != SE_OK:
        raise SEError(st, "se_selector_save")


def load(path):
    st = lib.se_selector_load(path.encode())
    if st != SE_OK:
        raise SEError(st, "se_selector_load")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--seed", type=int, default=0)
    g.add_argument("--first", type=int, default=0)
    g.add_argument("--count", type=int, default=10)
    g.add_argument("--max-seconds", type=float, default=1e9)
    g.add_argument("--ids", default=None, help="comma-separated problem ids, or @file holding them")
    g.add_argument("--out", required=True)
    g.add_argument("--n-min", type=float, default=1e3, help="smallest N of the log-uniform draw (largest 1e6)")
    t = sub.add_parser("train")
    t.add_argument("--runs", nargs="+", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=150)
    t.add_argument("--batch", type=int, default=64)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--margin", type=float, default=0.3)
    t.add_argument("--seed", type=int, default=1)
    ev = sub.add_parser("evaluate")
    ev.add_argument("--weights", default=None)
    ev.add_argument("--random", type=int, default=0, help="held-out random problems (seed 1) besides the N=1e6 set")
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        ids = None
        if a.ids:
            txt = open(a.ids[1:]).read() if a.ids.startswith("@") else a.ids
            ids = [int(v) for v in txt.replace("\n", ",").split(",") if v.strip()]
        generate(a.seed, a.first, a.count, a.out, a.max_seconds, ids=ids, n_min=a.n_min)
        return 0
    if a.cmd == "evaluate":
        if a.weights:
            load(a.weights)
        probs = list(METRIC_PROBLEMS)
        g = np.random.default_rng(1)
        probs += [sample_problem(g) for _ in range(a.random)]
        rows = evaluate(probs)
        tp = sum(r["plain_ms"] for r in rows)
        tl = sum(r["learned_ms"] for r in rows)
        bad = [r for r in rows if r["learned_err"] > r["tol"]]
        print("total plain %.1f ms, learned %.1f ms (x%.2f); learned above tol: %d of %d" %
              (tp, tl, tp / tl, len(bad), len(rows)), flush=True)
        return 0
    runs = load_runs(a.runs)
    X, Y, ids = labels(runs, a.margin)
    print("runs %d, labelled problems %d" % (len(runs["problem"]), len(X)), flush=True)
    hist = train(X, Y, a.epochs, a.batch, a.lr, a.seed)
    print("loss: first %.4g, last %.4g" % (hist[0], hist[-1]), flush=True)
    save(a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
