"""Summaries of rocprofv3 output for the benchmark workload (text for
profiles/, and the measured-traffic record bench.py reads).

    python -m paper_2210_01255_amd.profile_summary trace   KT_DIR          > kernel_trace.md
    python -m paper_2210_01255_amd.profile_summary traffic FETCH_DIR WRITE_DIR CALIB_MIB OUT.json > traffic.md
    python -m paper_2210_01255_amd.profile_summary counters DIR [DIR ...]   > counters.md

KT_DIR holds a `--kernel-trace` CSV (*kernel_trace.csv); FETCH_DIR / WRITE_DIR
hold `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of `bench.py --copy-calib-mib
CALIB_MIB`, whose last elementwise kernel reads and writes CALIB_MIB MiB of
FP64 and so calibrates each counter (scaled bytes = KiB * 1024 / factor);
DIR holds `--pmc` SQ counter runs.  Kernels are grouped by (name, grid size).
"""
from __future__ import annotations

import collections
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the benchmark phases whose dominant kernel is summarised: (phase, name
# pattern, instance) where instance picks the launch of the learned+batched
# form (largest grid among the kernel's launches)
PHASES = (("gather", r"^k_gather_rt<double, 6"), ("spread", r"^k_spread_rt<double, 6"),
          ("real_space", r"^k_real2<0, 2>"), ("fft_z_scale", r"^k_fft_z_scale<double, 0, 3"),
          ("fft_fwd_xy", r"^k_fft_x_r2c<double"), ("fft_inv_yx", r"^k_fft_x_c2r<double"))


def _name(raw: str) -> str:
    n = re.sub(r"^void ", "", raw)
    n = re.sub(r"\(anonymous namespace\)::", "", n)
    return n.split("(")[0].strip()


def _csvs(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _grid(r) -> int:
    if "Grid_Size" in r:
        return int(r["Grid_Size"])
    return int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])


def trace(kt_dir: str) -> str:
    calls = collections.defaultdict(list)
    for f in _csvs(kt_dir, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            key = (_name(r["Kernel_Name"]), _grid(r))
            calls[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    total = sum(sum(v) for v in calls.values())
    rows = sorted(calls.items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | grid (work items) | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|---:|"]
    for (name, grid), us in rows:
        if sum(us) < 1e-3 * total:
            continue
        out.append("| %s | %d | %d | %.1f | %.2f | %.1f |" % (name[:60], grid, len(us), sum(us) / len(us),
                                                              sum(us) * 1e-3, 100.0 * sum(us) / total))
    return "\n".join(out)


def _counters(dirs):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    last = {}  # counter -> (dispatch id, kernel, value) of the last elementwise kernel
    for d in dirs:
        for f in _csvs(d, "counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                key = (_name(r["Kernel_Name"]), _grid(r))
                c, v = r["Counter_Name"], float(r["Counter_Value"])
                vals[key][c].append(v)
                meta[key] = (r.get("VGPR_Count", ""), r.get("Scratch_Size", ""), r.get("LDS_Block_Size", ""))
                did = int(r.get("Dispatch_Id", 0) or 0)
                if "elementwise" in key[0] and (c not in last or did >= last[c][0]):
                    last[c] = (did, key, v)
    vals["__last_elementwise__"] = {c: [t[2]] for c, t in last.items()}
    return vals, meta


def _phase_keys(vals, phases=PHASES):
    keys = {}
    for phase, pat in phases:
        cand = [k for k in vals if isinstance(k, tuple) and re.search(pat, k[0])]
        if cand:
            keys[phase] = max(cand, key=lambda k: k[1])
    return keys


def _calib(vals, counter):
    """The calibration copy: the last elementwise kernel dispatched in the run."""
    v = vals.get("__last_elementwise__", {}).get(counter)
    return v[0] if v else None


def traffic(fetch_dir, write_dir, calib_mib, out_json):
    sys.path.insert(0, ROOT)
    import bench
    fv, _ = _counters([fetch_dir])
    wv, _ = _counters([write_dir])
    kib = float(calib_mib) * 1024.0
    ff = _calib(fv, "FETCH_SIZE") / kib
    wf = _calib(wv, "WRITE_SIZE") / kib
    rec = {"workload": "N = 1e6 stokeslet, tol 1e-8, FP64, learned+batched", "phases": {}}
    lines = ["Calibration: one elementwise kernel reads and writes %.0f KiB; the counters report FETCH %.1f KiB "
             "(factor %.4f) and WRITE %.1f KiB (factor %.4f)." % (kib, ff * kib, ff, wf * kib, wf), "",
             "| phase | kernel | FETCH KiB/launch | WRITE KiB/launch | scaled HBM MB/launch |",
             "|---|---|---:|---:|---:|"]
    # phases whose time is one kernel's (the FFT x/y phases are two kernels each)
    one = tuple(p for p in PHASES if p[0] in ("gather", "spread", "real_space", "fft_z_scale"))
    fk, wk = _phase_keys(fv, one), _phase_keys(wv, one)
    for phase, _ in one:
        if phase not in fk or phase not in wk:
            continue
        kf, kw = fk[phase], wk[phase]
        f = sum(fv[kf]["FETCH_SIZE"]) / len(fv[kf]["FETCH_SIZE"])
        w = sum(wv[kw]["WRITE_SIZE"]) / len(wv[kw]["WRITE_SIZE"])
        b = f * 1024.0 / ff + w * 1024.0 / wf
        rec["phases"][phase] = {"kernel": kf[0], "grid": kf[1], "source_sha": bench.source_digest(phase),
                                "fetch_kib": f, "write_kib": w, "fetch_factor": ff, "write_factor": wf,
                                "bytes_per_launch": b}
        lines.append("| %s | %s | %.0f | %.0f | %.1f |" % (phase, kf[0], f, w, b / 1e6))
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return "\n".join(lines)


def counters(dirs) -> str:
    vals, meta = _counters(dirs)
    keys = _phase_keys(vals)
    names = sorted({c for k in keys.values() for c in vals[k]})
    out = ["| counter | " + " | ".join("%s<br>`%s`" % (p, keys[p][0]) for p in keys) + " |",
           "|---|" + "---:|" * len(keys)]
    for c in names:
        cells = []
        for p in keys:
            v = vals[keys[p]].get(c)
            cells.append("%.4g" % (sum(v) / len(v)) if v else "")
        out.append("| %s | %s |" % (c, " | ".join(cells)))
    out.append("| VGPR / scratch / LDS | " + " | ".join("/".join(meta[keys[p]]) for p in keys) + " |")
    return "\n".join(out)


def main(argv=None):
    a = list(sys.argv[1:] if argv is None else argv)
    if not a:
        print(__doc__)
        return 2
    if a[0] == "trace":
        print(trace(a[1]))
    elif a[0] == "traffic":
        print(traffic(a[1], a[2], a[3], a[4]))
    elif a[0] == "counters":
        print(counters(a[1:]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main())
