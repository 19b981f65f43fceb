"""The rocprofv3 summary tool that writes profiles/: kernel-trace table,
counter table and the traffic record (calibrated by the copy kernel) from
small synthetic CSV files in rocprofv3's column layout."""
import csv
import json
import os

from paper_2210_01255_amd import profile_summary as PS


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_trace_and_traffic(tmp_path):
    kt = tmp_path / "kt" / "host" / "x_kernel_trace.csv"
    rows = [dict(Kernel_Name="void (anonymous namespace)::k_gather_rt<double, 6, false>(se_tile_args)",
                 Grid_Size_X=6094080, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=1000,
                 End_Timestamp=1000 + 4000000 + 1000 * i) for i in range(3)]
    rows += [dict(Kernel_Name="void (anonymous namespace)::k_spread_rt<double, 6, false>(se_tile_args)",
                  Grid_Size_X=6094080, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=0, End_Timestamp=3000000)]
    _write(str(kt), rows)
    table = PS.trace(str(tmp_path / "kt"))
    lines = table.splitlines()
    assert "k_gather_rt<double, 6, false> | 6094080 | 3 | 4001.0 |" in lines[2]
    assert "k_spread_rt<double, 6, false>" in lines[3]

    def pmc(d, counter, vals):
        r = []
        for i, (name, grid, v) in enumerate(vals):
            r.append(dict(Dispatch_Id=i + 1, Kernel_Name=name, Grid_Size=grid, Counter_Name=counter, Counter_Value=v,
                          VGPR_Count=8, Scratch_Size=0, LDS_Block_Size=0))
        _write(str(tmp_path / d / "h" / "c_counter_collection.csv"), r)
    ew = "void at::native::elementwise_kernel<128, 4>(int)"
    g6 = "void (anonymous namespace)::k_gather_rt<double, 6, false>(se_tile_args)"
    pmc("f", "FETCH_SIZE", [(ew, 1 << 22, 7.0), (g6, 6094080, 1000.0), (g6, 6094080, 1200.0), (ew, 1 << 20, 512.0)])
    pmc("w", "WRITE_SIZE", [(ew, 1 << 22, 9.0), (g6, 6094080, 300.0), (ew, 1 << 20, 1024.0)])
    out = tmp_path / "t.json"
    md = PS.traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1.0, str(out))
    rec = json.load(open(out))["phases"]["gather"]
    assert abs(rec["fetch_factor"] - 0.5) < 1e-12 and abs(rec["write_factor"] - 1.0) < 1e-12
    assert abs(rec["bytes_per_launch"] - (1100.0 * 1024 / 0.5 + 300.0 * 1024)) < 1e-6
    assert "| gather | k_gather_rt<double, 6, false> | 1100 | 300 |" in md
    cnt = PS.counters([str(tmp_path / "f")])
    assert "| FETCH_SIZE | 1100 |" in cnt
