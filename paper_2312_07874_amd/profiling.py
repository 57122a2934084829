"""Summaries of rocprofv3 output for the right-hand-side kernel K2.

Two commands, both reading the CSV files rocprofv3 writes with
``--output-format csv``:

  python -m paper_2312_07874_amd.profiling traffic WORKLOAD FETCH_CSV WRITE_CSV
      HBM bytes of K2 from a ``--pmc FETCH_SIZE`` and a ``--pmc WRITE_SIZE`` run
      of ``bench.py --workload WORKLOAD --steps 1 --warmup 0 --no-autotune
      --extra "" --no-batched --no-adjoint --calibrate-copy``.  The first four K2 dispatches
      of such a run are the four stage kernels of the timed RK4 step (right-hand
      side and stage combination, with fused stages also the next projection);
      their counters
      are averaged and scaled by what the same counters read on the closing
      1 GiB device-to-device copy.  The result goes into profiles/traffic.json
      with a hash of the kernel sources (bench.py reports it only while they
      are unchanged).

  python -m paper_2312_07874_amd.profiling counters CSV [CSV ...]
      Any ``--pmc`` counters of a ``--steps 1 --warmup 0 --no-autotune`` bench
      run: per counter, the mean over the four stage kernels of the timed RK4
      step and over the entropy-projection launches, as a markdown table.

  python -m paper_2312_07874_amd.profiling stats TRACE_CSV [KERNEL_PREFIX]
      Per-block-size launch count and average duration of a kernel from a
      ``--kernel-trace`` run (default prefix ``esd::k_rhs<``), as a markdown table.

No GPU is needed: this only reads files.
"""
from __future__ import annotations

import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
K2_PREFIX = "esd::k_rhs<"
COPY_BYTES = 1 << 30


def _rows(path):
    with open(path, newline="") as fh:
        yield from csv.DictReader(fh)


def _counter(path, counter):
    """[(dispatch id, kernel name, value)] of one counter, in dispatch order."""
    out = []
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    out.sort()
    return out


def _short(name):
    """Kernel name without return type and argument list."""
    name = name[5:] if name.startswith("void ") else name
    return name.split("(")[0]


def _is_k2(name):
    return _short(name).startswith(K2_PREFIX)


def _k2_and_copy(path, counter):
    rows = _counter(path, counter)
    k2 = [(d, n, v) for d, n, v in rows if _is_k2(n)]
    copies = [v for d, n, v in rows if "copyBuffer" in n]
    if len(k2) < 4 or not copies:
        raise SystemExit(f"{path}: need 4 K2 dispatches and the calibration copy, found {len(k2)} and {len(copies)}")
    return k2[:4], max(copies)


def traffic(workload, fetch_csv, write_csv):
    import bench                              # kernel_source_hash, the workloads
    from . import perfmodel as pm

    k2f, copy_f = _k2_and_copy(fetch_csv, "FETCH_SIZE")
    k2w, copy_w = _k2_and_copy(write_csv, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (copy_f * 1024.0)
    write_scale = COPY_BYTES / (copy_w * 1024.0)
    fk = [v for _, _, v in k2f]
    wk = [v for _, _, v in k2w]
    wl = bench.WORKLOADS[workload]()
    ne = int(wl.mesh().elem_vertex_ids.shape[0])
    rec = {
        "kernel": _short(k2f[0][1]),
        "launches": "the 4 stages of one RK4 step",
        "fetch_kib_per_stage": fk,
        "write_kib_per_stage": wk,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "read_bytes_per_launch": statistics.fmean(fk) * 1024.0 * fetch_scale,
        "write_bytes_per_launch": statistics.fmean(wk) * 1024.0 * write_scale,
        "algorithmic_bytes_per_launch": (pm.k2_next_bytes(wl.dim, wl.degree) if _short(k2f[0][1]).endswith("true>")
                                         else pm.k2_rk_bytes(wl.dim, wl.degree)) * ne,
    }
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    h = bench.kernel_source_hash()
    if t.get("kernel_source_sha256") != h:
        t = {"kernel_source_sha256": h, "kernel_sources": list(bench.KERNEL_SOURCES), "workloads": {}}
    t["workloads"][workload] = rec
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    meas = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    print(f"| {workload} | `{rec['kernel']}` | {statistics.fmean(fk):.1f} | {statistics.fmean(wk):.1f} | "
          f"{fetch_scale:.3f} / {write_scale:.3f} | {rec['read_bytes_per_launch'] / 1e6:.2f} MB | "
          f"{rec['write_bytes_per_launch'] / 1e6:.2f} MB | {rec['algorithmic_bytes_per_launch'] / 1e6:.2f} MB | "
          f"{meas / rec['algorithmic_bytes_per_launch']:.2f} |")


def counters(paths):
    k2, k1 = {}, {}
    names = {}
    for path in paths:
        seen = {}
        for r in sorted(_rows(path), key=lambda r: int(r["Dispatch_Id"])):
            name = _short(r["Kernel_Name"])
            c = r["Counter_Name"]
            v = float(r["Counter_Value"])
            if name.startswith(K2_PREFIX):
                n = seen.setdefault((c, "k2"), 0)
                if n < 4:
                    k2.setdefault(c, []).append(v)
                    names["k2"] = name
                seen[(c, "k2")] = n + 1
            elif name.startswith("esd::k_entropy_projection<") and name.endswith("false>"):
                k1.setdefault(c, []).append(v)
                names["k1"] = name
    print(f"| counter | `{names.get('k2', 'K2')}` (4 stages) | `{names.get('k1', 'K1')}` |")
    print("|---|---|---|")
    for c in k2:
        a = statistics.fmean(k2[c])
        b = statistics.fmean(k1[c]) if c in k1 else float("nan")
        print(f"| {c} | {a:.4g} | {b:.4g} |")


def stats(trace_csv, prefix=K2_PREFIX):
    by = {}
    for r in _rows(trace_csv):
        name = _short(r.get("Kernel_Name", ""))
        if not name.startswith(prefix):
            continue
        bs = int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0)
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        by.setdefault((name, bs), []).append(dur)
    print("| kernel | block | launches | average us |")
    print("|---|---|---|---|")
    for (name, bs), d in sorted(by.items()):
        print(f"| `{name}` | {bs} | {len(d)} | {statistics.fmean(d) / 1e3:.2f} |")


def main(argv):
    if len(argv) >= 4 and argv[0] == "traffic":
        sys.path.insert(0, ROOT)
        traffic(argv[1], argv[2], argv[3])
    elif len(argv) >= 2 and argv[0] == "counters":
        counters(argv[1:])
    elif len(argv) >= 2 and argv[0] == "stats":
        stats(argv[1], *(argv[2:3]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
