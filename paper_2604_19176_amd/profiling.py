"""Summaries of rocprofv3 CSV output for the library's kernels.

`python -m paper_2604_19176_amd.profiling stats <dir>/run_kernel_trace.csv`
prints, per kernel and launch grid (a run mixes batched and single-instance
calls), the number of dispatches and their average duration, next to
rocprofv3's own average over all of a kernel's dispatches.

`python -m paper_2604_19176_amd.profiling traffic <fetch.csv> <write.csv>
--kernel NAME [NAME ...] --calib-bytes BYTES` turns two `--pmc FETCH_SIZE` /
`--pmc WRITE_SIZE` counter-collection files into HBM bytes per launch of
each named kernel (one JSON object, entries under "kernels").  Each counter
(KiB per dispatch) is scaled by known/counted bytes of the calibration copy in
the same run: the library's streaming copy k_stream_copy with the largest
counter value (it reads and writes BYTES each).  The same factors for the
library's 8-byte scatter copy k_scatter_copy over BYTES (the scattered-store
pattern of the ring adjoint) are reported beside them.

`python -m paper_2604_19176_amd.profiling counters <csv> --kernel NAME ...`
prints, for each named kernel at its main launch grid, the mean of every
counter of a `--pmc` pass per dispatch.

With `--rdreq <csv>`, a third pass counting the L2-to-memory read requests by
size (`--pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum
TCC_EA0_RDREQ_sum`), the fetched bytes of each kernel are 32, 64 and 128 times
its requests of each size instead of the scaled FETCH_SIZE; the same sum for
k_stream_copy is reported against the bytes it is known to read.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict


def _short(name):
    base = name.split("(")[0]
    if base.startswith("void "):
        base = base[5:]
    return base[5:] if base.startswith("pat::") else base


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _grid(row):
    if "Grid_Size" in row:
        return int(row["Grid_Size"])
    return int(row["Grid_Size_X"]) * int(row["Grid_Size_Y"]) * int(row["Grid_Size_Z"])


def kernel_durations(trace_csv):
    """{(kernel, grid): {"n": dispatches, "avg_us": mean duration}} -- one entry
    per launch shape, since a run mixes batched, single-instance and tuning calls."""
    by = defaultdict(list)
    for r in _rows(trace_csv):
        by[(_short(r["Kernel_Name"]), _grid(r))].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return {k: {"n": len(v), "avg_us": sum(v) / len(v) / 1e3} for k, v in by.items()}


def stats_table(trace_csv, stats_csv=None, min_dispatches=5):
    kd = kernel_durations(trace_csv)
    allavg = {}
    if stats_csv and os.path.exists(stats_csv):
        for r in _rows(stats_csv):
            allavg[_short(r["Name"])] = float(r["AverageNs"]) / 1e3
    lines = ["| kernel | grid (work-items) | dispatches | avg us | rocprofv3 avg over all grids (us) |",
             "|---|---|---|---|---|"]
    rows = [(k, v) for k, v in kd.items() if v["n"] >= min_dispatches]
    for (name, grid), v in sorted(rows, key=lambda kv: -kv[1]["avg_us"] * kv[1]["n"]):
        a = allavg.get(name)
        lines.append("| %s | %d | %d | %.1f | %s |" % (name, grid, v["n"], v["avg_us"],
                                                    "%.1f" % a if a is not None else "-"))
    return "\n".join(lines)


def _main_grid(counts):
    """The largest launch grid with at least three dispatches ({grid: count}):
    the full-batch launches of bench.py's per-kernel timing, which run on one
    stream (its timed steps may run as two half-batches with half the grid,
    and its single-instance calls have smaller grids; with a cached tuning no
    candidate shapes run)."""
    many = [g for g, n in counts.items() if n >= 3]
    return max(many) if many else max(counts)


def _counter(path, kernel):
    """Mean counter value over the dispatches of `kernel` at its main grid
    (_main_grid)."""
    vals, calib = [], []
    for r in _rows(path):
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        if _short(name) == kernel:
            vals.append((_grid(r), v))
        elif _short(name) == "k_stream_copy":
            calib.append(v)
    if not vals:
        raise SystemExit("kernel %s not found in %s" % (kernel, path))
    count = defaultdict(int)
    for g, _ in vals:
        count[g] += 1
    gsel = _main_grid(count)
    kv = [v for g, v in vals if g == gsel]
    return sum(kv) / len(kv), (max(calib) if calib else None), len(kv)


def scatter_factors(fetch_csv, write_csv, calib_bytes):
    """Known/counted bytes of the 8-byte scatter copy (largest dispatch) for
    each counter, or None when the run has none.  It reads its source and a
    4-byte index per 8-byte element (1.5 x calib_bytes) and writes calib_bytes
    at scattered 8-byte addresses."""
    out = []
    for path, known in ((fetch_csv, 1.5 * calib_bytes), (write_csv, calib_bytes)):
        v = [float(r["Counter_Value"]) for r in _rows(path) if _short(r["Kernel_Name"]) == "k_scatter_copy"]
        out.append(known / (max(v) * 1024.0) if v and max(v) > 0 else None)
    return {"fetch_scale": out[0], "write_scale": out[1]}


RDREQ_SIZES = {"TCC_EA0_RDREQ_32B_sum": 32, "TCC_EA0_RDREQ_64B_sum": 64, "TCC_EA0_RDREQ_128B_sum": 128}


def read_bytes_by_size(path):
    """{(kernel, grid): [bytes of each dispatch]} from a request-size pass:
    32, 64 and 128 bytes per counted request of each size."""
    per = defaultdict(float)
    key = {}
    for r in _rows(path):
        size = RDREQ_SIZES.get(r["Counter_Name"])
        if size is None:
            continue
        d = (r["Dispatch_Id"], _short(r["Kernel_Name"]), _grid(r))
        per[d] += size * float(r["Counter_Value"])
        key[d] = (d[1], d[2])
    out = defaultdict(list)
    for d, v in per.items():
        out[key[d]].append(v)
    return out


def _select(by_grid):
    """The values at the main grid (as _counter)."""
    return by_grid[_main_grid({g: len(v) for g, v in by_grid.items()})]


def traffic(fetch_csv, write_csv, kernel, calib_bytes, rdreq=None):
    f_kib, f_cal, nf = _counter(fetch_csv, kernel)
    w_kib, w_cal, nw = _counter(write_csv, kernel)
    sf = calib_bytes / (f_cal * 1024.0) if f_cal else 1.0
    sw = calib_bytes / (w_cal * 1024.0) if w_cal else 1.0
    out = {
        "kernel": kernel,
        "fetch_kib_per_launch_raw": f_kib, "write_kib_per_launch_raw": w_kib,
        "fetch_scale": sf, "write_scale": sw,
        "fetch_bytes_per_launch": f_kib * 1024.0 * sf, "write_bytes_per_launch": w_kib * 1024.0 * sw,
        "dispatches": [nf, nw],
        "calib_bytes": calib_bytes,
        "calib_fetch_kib": f_cal, "calib_write_kib": w_cal,
    }
    if rdreq is not None:
        v = _select({g: b for (k, g), b in rdreq.items() if k == kernel})
        out["fetch_bytes_per_launch_scaled"] = out["fetch_bytes_per_launch"]
        out["fetch_bytes_per_launch"] = sum(v) / len(v)
        out["fetch_from"] = "request sizes"
    return out


# the device sources every kernel is compiled from
KERNEL_FILES = ("kernels.hip", "fft.hpp", "cfft.hpp", "pat_internal.hpp")


def source_hash(path):
    """Hash of the device sources' code (comments and whitespace removed, so
    that a comment edit keeps measured figures valid): `path` is the source
    directory or a file in it."""
    d = path if os.path.isdir(path) else os.path.dirname(os.path.abspath(path))
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def counter_means(path, kernels):
    """{kernel: {counter: mean per dispatch}} at each kernel's main grid (as _counter)."""
    by = defaultdict(lambda: defaultdict(list))  # kernel -> grid -> [(dispatch, counter, value)]
    for r in _rows(path):
        k = _short(r["Kernel_Name"])
        if k in kernels:
            by[k][_grid(r)].append((r["Dispatch_Id"], r["Counter_Name"], float(r["Counter_Value"])))
    out = {}
    for k in kernels:
        if k not in by:
            continue
        grids = {g: len({dsp for dsp, _, _ in v}) for g, v in by[k].items()}
        g = _main_grid(grids)
        acc = defaultdict(float)
        for dsp, c, v in by[k][g]:
            acc[c] += v
        out[k] = {c: v / grids[g] for c, v in acc.items()}
        out[k]["dispatches"] = grids[g]
        out[k]["grid"] = g
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace")
    s.add_argument("--stats-csv")
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--kernel", required=True, nargs="+")
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--batch", type=int, required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--rdreq")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True, nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.trace, a.stats_csv))
    elif a.cmd == "counters":
        json.dump(counter_means(a.csv, a.kernel), sys.stdout, indent=1)
        print()
    else:
        rd = read_bytes_by_size(a.rdreq) if a.rdreq else None
        d = {"batch": a.batch, "kernels_hash": source_hash(a.source), "calib_bytes": a.calib_bytes,
             "scatter_copy_factors": scatter_factors(a.fetch, a.write, a.calib_bytes),
             "kernels": {k: traffic(a.fetch, a.write, k, a.calib_bytes, rd) for k in a.kernel}}
        if rd is not None:
            cp = [v for (k, g), vs in rd.items() if k == "k_stream_copy" for v in vs]
            d["copy_read_bytes_by_size"] = max(cp) if cp else None
        json.dump(d, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
