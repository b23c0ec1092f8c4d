"""Summaries of rocprofv3 CSV output for the kernel profiles kept with the library.

Two reports, each printed as Markdown that records the command which produced the data:

``trace``   per-kernel totals from a ``--kernel-trace`` CSV, plus the average duration of
            one kernel (name + grid size) over its last N dispatches -- the launches of
            the timed steps when the traced command ends with them.
``counters`` per-kernel SQ counters of the last dispatch of each kernel and grid from
            ``--pmc`` runs (instruction counts, MFMA busy cycles, wave wait / activity
            cycles): MFMA busy % = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x
            SIMDs), the GRBM count being the sum over the XCDs.
``gaps``    the idle time between consecutive kernels inside each replay of the captured
            optimisation (a replay opens with the torch fills that reset its state).
``traffic`` HBM bytes of that kernel's last dispatch from a ``--pmc FETCH_SIZE`` run and
            a ``--pmc WRITE_SIZE`` run (KiB per dispatch), each scaled by what the same
            counter reads for a plain copy of known size in the same run (the largest
            ``copyBuffer`` dispatch: it reads and writes ``--copy-bytes`` bytes).  The
            report ends with a JSON comment that bench.py reads, together with a hash
            of the kernel sources, so the figure is dropped once the kernels change.

Usage::

    python -m paper_2412_09584_amd.rocprof_summary trace --csv T.csv --kernel NAME \\
        --grid G --last N --title ... --cmd ...
    python -m paper_2412_09584_amd.rocprof_summary traffic --fetch F.csv --write W.csv \\
        --kernel NAME --grid G --label LABEL --title ... --cmd ...
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """sha256 over the kernel sources (csrc/*.hip, csrc/*.h), in name order."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                    glob.glob(os.path.join(HERE, "csrc", "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    for pre in ("bp::(anonymous namespace)::", "bp::dev::"):
        name = name.replace(pre, "")
    name = name.split("(bp::GeomSet")[0].split("(const bp::")[0]
    return name.strip()


def _dispatches(path: str):
    """Rows of a kernel-trace or counter CSV folded to one record per dispatch."""
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            did = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
            d = out.get(did)
            if d is None:
                d = out[did] = {
                    "name": r["Kernel_Name"],
                    "grid": int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0),
                    "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                    "value": 0.0,
                }
            if "Counter_Value" in r:
                d["value"] += float(r["Counter_Value"])
    return list(out.values())


def _match(ds, kernel: str, grid: int, stride: int = 1, offset: int = 0):
    """Dispatches of one kernel and grid.  Where a step launches the same kernel and grid
    `stride` times (different layers of one shape class), keep the `offset`-th launch of
    each step, counting the steps back from the last dispatch."""
    sel = [d for d in ds if _short(d["name"]) == kernel and (grid <= 0 or d["grid"] == grid)]
    last = len(sel) - stride + offset
    return [d for p, d in enumerate(sel) if p <= last and (last - p) % stride == 0]


def _which(a) -> str:
    if a.stride <= 1:
        return ""
    return f", launch {a.offset + 1} of the {a.stride} of this kernel and grid per step"


def report_trace(a) -> str:
    ds = _dispatches(a.csv)
    tot = collections.defaultdict(lambda: [0, 0])
    for d in ds:
        t = tot[_short(d["name"])]
        t[0] += d["ns"]
        t[1] += 1
    allns = sum(v[0] for v in tot.values()) or 1
    sel = _match(ds, a.kernel, a.grid, a.stride, a.offset)[-a.last:]
    avg = sum(d["ns"] for d in sel) / max(len(sel), 1) / 1e6
    lines = [f"# {a.title}", "", "Command (TMPDIR=/tmp; <repo> is the repository root):", "",
             f"    {a.cmd}", "",
             f"Kernel `{a.kernel}` (grid {a.grid}{_which(a)}): average {avg:.4f} ms over its "
             f"last {len(sel)} dispatches (the timed steps).", "",
             "| total ms | calls | avg us | % | kernel |", "|---:|---:|---:|---:|---|"]
    for k, (ns, n) in sorted(tot.items(), key=lambda kv: -kv[1][0])[: a.top]:
        lines.append(f"| {ns / 1e6:.2f} | {n} | {ns / n / 1e3:.1f} | {100 * ns / allns:.1f} | `{k[:90]}` |")
    lines += ["", f"<!-- trace: {json.dumps({'kernel': a.kernel, 'grid': a.grid, 'stride': a.stride, 'offset': a.offset, 'avg_ms': avg, 'n': len(sel)})} -->"]
    return "\n".join(lines) + "\n"


def report_traffic(a) -> str:
    fd, wd = _dispatches(a.fetch), _dispatches(a.write)

    def calib(ds):
        cps = [d for d in ds if "copyBuffer" in d["name"]]
        if not cps:
            raise SystemExit("no copyBuffer dispatch for the calibration")
        big = max(cps, key=lambda d: d["value"])
        return big["value"] * 1024.0

    fc, wc = calib(fd), calib(wd)
    fs, ws = a.copy_bytes / fc, a.copy_bytes / wc
    fsel = _match(fd, a.kernel, a.grid, a.stride, a.offset)
    wsel = _match(wd, a.kernel, a.grid, a.stride, a.offset)
    if not fsel or not wsel:
        raise SystemExit(f"kernel {a.kernel!r} grid {a.grid} not found")
    fb, wb = fsel[-1]["value"] * 1024.0, wsel[-1]["value"] * 1024.0
    rec = {"label": a.label, "kernel": a.kernel, "grid": a.grid, "stride": a.stride,
           "offset": a.offset, "fetch_bytes": fb * fs,
           "write_bytes": wb * ws, "fetch_scale": fs, "write_scale": ws,
           "bytes": fb * fs + wb * ws, "src_sha256": source_hash()}
    lines = [f"# {a.title}", "", "Commands (one counter per run; TMPDIR=/tmp; <repo> is the "
             "repository root):", ""]
    lines += [f"    {c}" for c in a.cmd]
    lines += ["", f"Calibration: the {a.copy_bytes / 2**30:.0f} GiB device copy in the same run reads "
              f"FETCH_SIZE = {fc / 2**30:.3f} GiB and WRITE_SIZE = {wc / 2**30:.3f} GiB, so the "
              f"counters are scaled by {fs:.3f} (fetch) and {ws:.3f} (write).", "",
              f"Kernel `{a.kernel}` (grid {a.grid}{_which(a)}, `{a.label}`), last dispatch:", "",
              "| counter | raw GB | scaled GB |", "|---|---:|---:|",
              f"| FETCH_SIZE | {fb / 1e9:.3f} | {fb * fs / 1e9:.3f} |",
              f"| WRITE_SIZE | {wb / 1e9:.3f} | {wb * ws / 1e9:.3f} |",
              f"| total | {(fb + wb) / 1e9:.3f} | {(fb * fs + wb * ws) / 1e9:.3f} |", "",
              f"<!-- traffic: {json.dumps(rec)} -->"]
    return "\n".join(lines) + "\n"


def _counter_rows(paths):
    """{(short name, grid): {counter: value of the last dispatch}} over several CSVs."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (_short(r["Kernel_Name"]), int(r.get("Grid_Size") or 0))
                agg[key][r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return {k: {c: sorted(v)[-1][1] for c, v in cs.items()} for k, cs in agg.items()}


def report_counters(a) -> str:
    rows = _counter_rows(a.csv)
    lines = [f"# {a.title}", "", "Commands (TMPDIR=/tmp; <repo> is the repository root):", ""]
    lines += [f"    {c}" for c in a.cmd]
    lines += ["", f"Last dispatch of each kernel and grid; MFMA busy % = SQ_VALU_MFMA_BUSY_CYCLES / "
              f"(GRBM_GUI_ACTIVE / {a.xcds} XCDs x {a.simds} SIMDs); wave-cycle shares are of "
              "SQ_WAVE_CYCLES.", "",
              "| kernel | grid | GUI cycles / XCD | VALU insts | MFMA insts | VALU / MFMA | MFMA busy % "
              "| wait % | wait-issue % | VALU active % |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    order = sorted(rows.items(), key=lambda kv: -kv[1].get("GRBM_GUI_ACTIVE", 0))[: a.top]
    for (name, grid), c in order:
        gui = c.get("GRBM_GUI_ACTIVE", 0) / a.xcds
        valu, mfma = c.get("SQ_INSTS_VALU"), c.get("SQ_INSTS_MFMA")
        busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES")
        wc = c.get("SQ_WAVE_CYCLES")
        f = lambda v: "" if v is None else f"{v:.0f}"
        pct = lambda k: "" if not wc or k not in c else f"{100 * c[k] / wc:.1f}"
        util = "" if busy is None or not gui else f"{100 * busy / (gui * a.simds):.1f}"
        ratio = "" if not valu or not mfma else f"{valu / mfma:.2f}"
        lines.append(f"| `{name[:70]}` | {grid} | {gui:.0f} | {f(valu)} | {f(mfma)} | {ratio} | {util} | "
                     f"{pct('SQ_WAIT_ANY')} | {pct('SQ_WAIT_INST_ANY')} | {pct('SQ_ACTIVE_INST_VALU')} |")
    return "\n".join(lines) + "\n"


def report_gaps(a) -> str:
    with open(a.csv) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    st = [int(r["Start_Timestamp"]) for r in rows]
    en = [int(r["End_Timestamp"]) for r in rows]
    fill = ["FillFunctor" in r["Kernel_Name"] for r in rows]
    starts, i = [], 0
    while i < len(rows):          # a run of >= a.reset torch fills opens a replay
        j = i
        while j < len(rows) and fill[j]:
            j += 1
        if j - i >= a.reset:
            starts.append(i)
        i = max(j, i + 1)
    starts.append(len(rows))
    lines = [f"# {a.title}", "", "Command (TMPDIR=/tmp; <repo> is the repository root):", "",
             f"    {a.cmd}", "", "Windows that open with the optimiser's reset and hold at least "
             f"{a.min_kernels} kernels (the graph replays; warm-up and eager windows hold fewer "
             "or carry host gaps):", "",
             "| kernels | span ms | kernel busy ms | gaps ms | gaps % |", "|---:|---:|---:|---:|---:|"]
    for s, e in zip(starts[:-1], starts[1:]):
        e -= 1
        if e - s + 1 < a.min_kernels:
            continue
        span = en[e] - st[s]
        busy = sum(en[k] - st[k] for k in range(s, e + 1))
        gaps = sum(max(0, st[k + 1] - en[k]) for k in range(s, e))
        lines.append(f"| {e - s + 1} | {span / 1e6:.3f} | {busy / 1e6:.3f} | {gaps / 1e6:.3f} | "
                     f"{100 * gaps / max(span, 1):.2f} |")
    return "\n".join(lines) + "\n"


def read_traffic(path: str, label: str):
    """The traffic record of a summary, or None if missing, for another kernel, or taken
    from kernel sources other than the current ones."""
    try:
        with open(path) as f:
            txt = f.read()
    except OSError:
        return None
    key = "<!-- traffic: "
    i = txt.find(key)
    if i < 0:
        return None
    rec = json.loads(txt[i + len(key): txt.index(" -->", i)])
    if rec.get("label") != label or rec.get("src_sha256") != source_hash():
        return None
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int, default=0)
    t.add_argument("--last", type=int, default=20)
    t.add_argument("--top", type=int, default=25)
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    r = sub.add_parser("traffic")
    for q in (t, r):
        q.add_argument("--stride", type=int, default=1,
                       help="launches of this kernel and grid per step")
        q.add_argument("--offset", type=int, default=0,
                       help="which of them (0-based, in launch order)")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--grid", type=int, default=0)
    r.add_argument("--label", required=True)
    r.add_argument("--copy-bytes", type=float, default=float(2**30))
    r.add_argument("--title", required=True)
    r.add_argument("--cmd", action="append", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--csv", action="append", required=True)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--top", type=int, default=16)
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", action="append", required=True)
    g = sub.add_parser("gaps")
    g.add_argument("--csv", required=True)
    g.add_argument("--reset", type=int, default=7, help="torch fills that open a replay")
    g.add_argument("--min-kernels", type=int, default=300)
    g.add_argument("--title", required=True)
    g.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    rep = {"trace": report_trace, "traffic": report_traffic, "counters": report_counters,
           "gaps": report_gaps}[a.what]
    print(rep(a), end="")


if __name__ == "__main__":
    main()
