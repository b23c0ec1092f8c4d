"""Host-side checks of the rocprofv3 summary helper used by bench.py for the roofline
traffic figure (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2412_09584_amd import rocprof_summary as RS  # noqa: E402


def _write_counter_csv(path, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w") as f:
        f.write(",".join(f'"{c}"' for c in cols) + "\n")
        for i, (name, grid, val) in enumerate(rows):
            f.write(f'"{i}","{i}","{grid}","{name}","X","{val}","0","1000"\n')


def test_traffic_scaling_and_staleness(tmp_path):
    # copy of 1 GiB reads as 0.5 GiB fetch / 1 GiB write; the kernel's last dispatch counts
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    k = "void bp::(anonymous namespace)::k_conv<bp::dev::EpiRelax, 16, 16, true>(bp::GeomSet, x)"
    _write_counter_csv(fetch, [("__amd_rocclr_copyBuffer", 4096, 2**19), (k, 64, 10.0), (k, 64, 1000.0)])
    _write_counter_csv(write, [("__amd_rocclr_copyBuffer", 4096, 2**20), (k, 64, 20.0), (k, 64, 3000.0)])
    out = tmp_path / "x_traffic.md"

    class A:
        pass
    a = A()
    a.fetch, a.write, a.kernel, a.grid, a.label = str(fetch), str(write), \
        "void k_conv<EpiRelax, 16, 16, true>", 64, "bwd_relax_L2"
    a.copy_bytes, a.title, a.cmd = float(2**30), "t", ["c"]
    a.stride, a.offset = 1, 0
    out.write_text(RS.report_traffic(a))
    rec = RS.read_traffic(str(out), "bwd_relax_L2")
    assert rec is not None
    assert abs(rec["fetch_bytes"] - 2 * 1000 * 1024) < 1e-6
    assert abs(rec["write_bytes"] - 3000 * 1024) < 1e-6
    assert RS.read_traffic(str(out), "adj_L1") is None          # another kernel
    txt = out.read_text().replace(RS.source_hash(), "0" * 64)   # other kernel sources
    out.write_text(txt)
    assert RS.read_traffic(str(out), "bwd_relax_L2") is None


def test_match_picks_one_launch_per_step():
    # two steps, each launching the same kernel and grid for two layers (A, B), after
    # tuning launches of the same kernel; the selection is aligned to the last dispatch
    k = "void bp::(anonymous namespace)::k_gemm<bp::dev::EpiAdj, 32, 256, 32, 4, 1, false, true>(bp::GeomSet, x)"
    ds = [{"name": k, "grid": 8, "ns": n, "value": 0.0}
          for n in (7, 7, 7, 1, 2, 3, 4)]       # tuning x3, then A1 B1 A2 B2
    first = RS._match(ds, "void k_gemm<EpiAdj, 32, 256, 32, 4, 1, false, true>", 8, 2, 0)
    second = RS._match(ds, "void k_gemm<EpiAdj, 32, 256, 32, 4, 1, false, true>", 8, 2, 1)
    assert [d["ns"] for d in first][-2:] == [1, 3]
    assert [d["ns"] for d in second][-2:] == [2, 4]
    assert [d["ns"] for d in RS._match(ds, "void k_gemm<EpiAdj, 32, 256, 32, 4, 1, false, true>", 8)] \
        == [7, 7, 7, 1, 2, 3, 4]


def test_committed_traffic_summaries_parse():
    d = os.path.join(ROOT, "profiles")
    for n in os.listdir(d):
        if n.endswith("_traffic.md"):
            txt = open(os.path.join(d, n)).read()
            i = txt.index("<!-- traffic: ")
            rec = json.loads(txt[i + 14: txt.index(" -->", i)])
            assert rec["bytes"] > 0 and len(rec["src_sha256"]) == 64
