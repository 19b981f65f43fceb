"""Batches of independent systems (uneven N, periodicity 3/2/1/0, elongated
boxes) through se_batch_*: the eager pass, every HIP-graph replay and the
autotuned launch shapes against single-plan runs and the FP64 oracle.

Floating-point bar: the requested rms-relative tolerance against the oracle
(safety factor 10 as in the single-system parity tests); replays against the
eager pass within 1e-12 relative (only the order of the atomic additions in
spreading and gathering may differ between launches).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SAFETY = 10.0


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_2210_01255_amd as se
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    oracle.build(force=False)
    return se, oracle, torch


def _systems(seed, count, lo, hi, kernel="stokeslet"):
    """Uneven systems: N log-uniform in [lo, hi], D uniform in {3,2,1,0},
    one box axis stretched by a ~ U[1, 4]."""
    g = W.rng(seed)
    sizes = W.loguniform_sizes(g, count, lo, hi)
    out = []
    for i, n in enumerate(sizes):
        D = int(g.integers(0, 4))
        box = W.aspect_box(g)
        s = W.system(seed * 1000 + i, int(n), box=tuple(box), kernel=kernel, zero_mean=(D == 3),
                     layout="uniform")
        s["D"] = D
        out.append(s)
    return out


def _problem(s, kernel, tol):
    q = float(np.sum(s["f"] ** 2)) if kernel != "stresslet" else float(
        np.sum((s["q"][:, :, None] * s["nu"][:, None, :]) ** 2))
    return dict(kernel=kernel, periodicity=s["D"], box=tuple(s["box"]), tol=tol, n_src=len(s["x"]),
                source_q=q, safety=SAFETY)


def _dev(env, systems, key):
    _, _, torch = env
    return [torch.tensor(s[key], device="cuda:0") if key in s else None for s in systems]


def _oracle_ref(env, s, kernel, idx=None):
    _, oracle, _ = env
    D = s["D"]
    xi = 6.0 / float(np.max(s["box"][:D])) if D in (1, 2) else None
    tg = None if idx is None else s["x"][idx]
    r = oracle.ewald(D, kernel, s["box"], s["x"], f=s.get("f"), q=s.get("q"), nu=s.get("nu"),
                     targets=tg, self_src=idx, xi=xi)
    return r.total if D else r["direct"]


def test_batch_graph_replays_match_eager_and_oracle(env):
    se, oracle, torch = env
    tol = 1e-6
    systems = _systems(41, 8, 200, 1500)
    print("batch Ns", [len(s["x"]) for s in systems], "Ds", [s["D"] for s in systems], flush=True)
    b = se.Batch([_problem(s, "stokeslet", tol) for s in systems])
    x = _dev(env, systems, "x")
    f = _dev(env, systems, "f")
    outs = [torch.empty_like(t) for t in f]
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.set_geometry(x, stream=st)
        b.execute(f, outs, stream=st)  # eager pass (records the graph)
    st.synchronize()
    eager = [o.cpu().numpy() for o in outs]
    for s, u in zip(systems, eager):
        err = oracle.rms_rel_error(u, _oracle_ref(env, s, "stokeslet"))
        print("D=%d N=%d err %.3g" % (s["D"], len(s["x"]), err), flush=True)
        assert err <= tol

    for rep in range(4):
        # unrelated eager work and host synchronisation between the replays
        junk = torch.randn(1 << 16, device="cuda:0", dtype=torch.float64)
        (junk * 2.0).sum().item()
        for o in outs:
            o.fill_(float("nan"))
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            b.execute(f, outs, stream=st)  # graph replay
        st.synchronize()
        for u0, o in zip(eager, outs):
            u = o.cpu().numpy()
            assert np.all(np.isfinite(u)), "replay %d left unwritten outputs" % rep
            assert oracle.rms_rel_error(u, u0) <= 1e-12, rep

    # new output tensors: a fresh eager pass and a new graph
    outs2 = [torch.empty_like(t) for t in f]
    st.wait_stream(torch.cuda.current_stream())
    for _ in range(2):
        with torch.cuda.stream(st):
            b.execute(f, outs2, stream=st)
        st.synchronize()
        for u0, o in zip(eager, outs2):
            assert oracle.rms_rel_error(o.cpu().numpy(), u0) <= 1e-12

    # new positions bound in place: the recorded graph replays on them
    moved = []
    for s in systems:
        s2 = dict(s)
        s2["x"] = np.mod(s["x"] + 0.137 * s["box"][None, :], s["box"][None, :])
        moved.append(s2)
    x2 = _dev(env, moved, "x")
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.set_geometry(x2, stream=st)
        b.execute(f, outs2, stream=st)  # same pointers: graph replay
    st.synchronize()
    for s2, o, p in zip(moved, outs2, b.plans):
        single = se.Plan(**_problem(s2, "stokeslet", tol))
        single.set_geometry(torch.tensor(s2["x"], device="cuda:0"))
        u = single.execute(torch.tensor(s2["f"], device="cuda:0"))
        single.sync()
        assert oracle.rms_rel_error(o.cpu().numpy(), u.cpu().numpy()) <= 1e-12
    with torch.cuda.stream(st):
        b.set_geometry(x, stream=st)
    st.synchronize()

    # each member equals a single plan of the same problem
    for s, u0, p in zip(systems, eager, b.plans):
        single = se.Plan(**_problem(s, "stokeslet", tol))
        assert single.params == p.params
        xs = torch.tensor(s["x"], device="cuda:0")
        single.set_geometry(xs)
        u = single.execute(torch.tensor(s["f"], device="cuda:0"))
        single.sync()
        assert oracle.rms_rel_error(u.cpu().numpy(), u0) <= 1e-12
    b.close()


def test_batch_of_64_uneven_systems_with_tuning(env):
    """64 systems, N log-uniform in [1e3, 5e4], D uniform in {3,2,1,0}, box
    aspect in [1,4], tol 1e-6: autotuned shapes, graph replay; every member
    against the replayed eager pass, and on every target at the requested
    tolerance against the GPU direct Ewald reference (itself checked against
    the oracle to 1e-12 in test_gpu_reference.py)."""
    se, oracle, torch = env
    tol = 1e-6
    systems = _systems(64, 64, 1e3, 5e4)
    print("64 systems, total N", sum(len(s["x"]) for s in systems), flush=True)
    b = se.Batch([_problem(s, "stokeslet", tol) for s in systems])
    x = _dev(env, systems, "x")
    f = _dev(env, systems, "f")
    outs = [torch.empty_like(t) for t in f]
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.set_geometry(x, stream=st)
        b.execute(f, outs, stream=st)
    st.synchronize()
    before = [o.cpu().numpy() for o in outs]
    with torch.cuda.stream(st):
        shapes = b.tune(f, outs, stream=st)
    st.synchronize()
    print("tuned shapes", shapes, flush=True)
    assert all(0 <= tb <= 4 and fc in (0, 2, 4, 8, 16) and ti in (0, 4, 8, 16, 64) for tb, fc, ti in shapes)
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            b.execute(f, outs, stream=st)
        st.synchronize()
    # replayed graph against the same launches issued one system after another
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    with torch.cuda.stream(st):
        ev[0].record(st)
        for _ in range(5):
            b.execute(f, outs, stream=st)
        ev[1].record(st)
        for _ in range(5):
            for p, fi, oi in zip(b.plans, f, outs):
                p.execute(fi, out=oi, stream=st)
        ev[2].record(st)
    st.synchronize()
    print("64 systems: graph replay %.3f ms, one after another %.3f ms" %
          (ev[0].elapsed_time(ev[1]) / 5, ev[1].elapsed_time(ev[2]) / 5), flush=True)
    worst = 0.0
    for i, (s, o, u0) in enumerate(zip(systems, outs, before)):
        u = o.cpu().numpy()
        assert oracle.rms_rel_error(u, u0) <= 1e-12, i
        ref = se.ewald_reference("stokeslet", s["D"], tuple(s["box"]), x[i], f[i]).cpu().numpy()
        err = oracle.rms_rel_error(u, ref)
        worst = max(worst, err)
        print("sys %d D=%d N=%d box=%s all-target err %.3g" % (i, s["D"], len(s["x"]),
                                                               np.round(s["box"], 3).tolist(), err), flush=True)
        assert err <= tol, (i, err)
    print("64 systems: worst all-target err %.3g (tol %g)" % (worst, tol), flush=True)
    b.close()


def test_batch_merged_launches_cover_every_variant(env):
    """A batch whose merged phase launches mix every job variant: the four
    kernels, D = 3, 2, 1, 0, one to three right-hand sides (pairs and a
    single slot in one chunk), FP32 grids, the truncated-Gaussian window and
    separate targets.  Each member, eager and on graph replays, against a
    single plan of the same problem (1e-12 relative for FP64 grids; FP32
    grids within 1e-5, where the order of the atomic additions shows)."""
    se, oracle, torch = env
    specs = [
        dict(kernel="stokeslet", D=3, n=900, rhs=3),
        dict(kernel="rotlet", D=2, n=700, rhs=2),
        dict(kernel="stresslet", D=1, n=600, rhs=2),
        dict(kernel="stokeslet", D=0, n=500, rhs=1, fp32=True),
        dict(kernel="harmonic", D=3, n=400, rhs=2, window="tg"),
        dict(kernel="stokeslet", D=3, n=800, rhs=2, nt=300),
        dict(kernel="rotlet", D=1, n=650, rhs=3, fp32=True, window="tg"),
        dict(kernel="stresslet", D=0, n=450, rhs=1),
        dict(kernel="stokeslet", D=2, n=1200, rhs=2, fp32=True),
    ]
    probs, xs, nus, tgs, fs = [], [], [], [], []
    g = W.rng(77)
    for i, c in enumerate(specs):
        box = tuple(W.aspect_box(g))
        s = W.system(7700 + i, c["n"], box=box, kernel=c["kernel"], zero_mean=(c["D"] == 3), n_rhs=c["rhs"])
        key = "q" if c["kernel"] == "stresslet" else "f"
        fr = s[key] if c["rhs"] > 1 else s[key][0]
        nt = c.get("nt", 0)
        tol = 1e-5 if c.get("fp32") else 1e-8
        probs.append(dict(kernel=c["kernel"], periodicity=c["D"], box=box, tol=tol, n_src=c["n"], n_tgt=nt,
                          targets_are_sources=nt == 0, n_rhs=c["rhs"], source_q=float(np.sum(fr ** 2)) / c["rhs"],
                          precision=se.PREC_FP32 if c.get("fp32") else se.PREC_FP64,
                          window=c.get("window", "pkb")))
        xs.append(torch.tensor(s["x"], device="cuda:0"))
        nus.append(torch.tensor(s["nu"], device="cuda:0") if "nu" in s else None)
        tgs.append(torch.tensor(g.random((nt, 3)) * np.asarray(box)[None, :], device="cuda:0") if nt else None)
        fs.append(torch.tensor(fr, device="cuda:0"))
    b = se.Batch(probs)
    print("merged batch:", [(c["kernel"], c["D"], c["rhs"], p.params["M"], p.params["P"])
                            for c, p in zip(specs, b.plans)], flush=True)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.set_geometry(xs, nus, tgs, stream=st)
        outs = b.execute(fs, stream=st)  # eager pass (records the graph)
    st.synchronize()
    eager = [o.cpu().numpy() for o in outs]
    singles = []
    for c, pr, x, nu, tg, f in zip(specs, probs, xs, nus, tgs, fs):
        single = se.Plan(**pr)
        single.set_geometry(x, nu, tg)
        u = single.execute(f)
        single.sync()
        singles.append(u.cpu().numpy())
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            b.execute(fs, outs, stream=st)  # graph replay
        st.synchronize()
        for i, (c, o, u0, us) in enumerate(zip(specs, outs, eager, singles)):
            u = o.cpu().numpy()
            bar = 1e-5 if c.get("fp32") else 1e-12
            assert np.all(np.isfinite(u)), (rep, i)
            e1, e2 = oracle.rms_rel_error(u, u0), oracle.rms_rel_error(u, us)
            if rep == 0:
                print("member %d %s D=%d rhs=%d: replay vs eager %.2e, vs single plan %.2e" %
                      (i, c["kernel"], c["D"], c["rhs"], e1, e2), flush=True)
            assert e1 <= bar and e2 <= bar, (rep, i, e1, e2)
    b.close()


def test_batch_rejects_bad_arguments(env):
    se, _, torch = env
    with pytest.raises(se.SEError):
        se.Batch([dict(kernel="stokeslet", periodicity=5, n_src=10)])
    b = se.Batch([dict(kernel="stokeslet", periodicity=3, n_src=100, tol=1e-6, source_q=300.0)])
    f = torch.zeros(100, 3, dtype=torch.float64, device="cuda:0")
    with pytest.raises(se.SEError):
        b.execute([f])  # no geometry bound
    b.close()
