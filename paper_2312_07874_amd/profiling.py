"""The profiled command and summaries of its rocprofv3 output.

  python -m paper_2312_07874_amd.profiling run WORKLOAD [REPS] [--no-autotune]
      The command to profile: builds the plan of WORKLOAD (a name understood by
      workloads.named), projects its state, autotunes its block sizes (as the
      benchmark does; --no-autotune keeps the defaults, for counter runs),
      evaluates REPS residuals
      (esd_residual: per residual K1 of every degree bucket, the mixed-degree
      interface kernel of batched plans, K2 of every bucket), synchronises,
      and ends with a plain 1 GiB device-to-device copy whose counters
      calibrate the traffic counters.

  python -m paper_2312_07874_amd.profiling traffic WORKLOAD FETCH_CSV WRITE_CSV
      HBM bytes of K2 per residual from a ``--pmc FETCH_SIZE`` and a
      ``--pmc WRITE_SIZE`` run of the command above: the K2 dispatches (every
      bucket) summed per residual, averaged over the last 5 residuals (after
      the autotuner's trial launches), scaled by
      what the same counter reads for the copy.  The result goes into
      profiles/traffic.json with a hash of the kernel sources (bench.py reports
      it only while they are unchanged).

  python -m paper_2312_07874_amd.profiling counters CSV [CSV ...]
      Any ``--pmc`` counters of the command above: per counter, the mean per
      residual of K2 (every bucket summed) and of K1 over the last 5 residuals,
      as a markdown table.

  python -m paper_2312_07874_amd.profiling stats TRACE_CSV
      Launch count and average duration per kernel (and block size) from a
      ``--kernel-trace`` run, as a markdown table.

Only ``run`` needs a GPU; the others read files.
"""
from __future__ import annotations

import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("device.hpp", "physics.hpp", "kernels.hip", "plan.hpp")
K2_PREFIX = "esd::k_rhs<"
K1_PREFIX = "esd::k_entropy_projection<"
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    """sha256 over the sources the right-hand-side kernel is built from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_07874_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name: str):
    """HBM bytes of K2 per residual recorded in profiles/traffic.json, if they
    were taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    w = t.get("workloads", {}).get(name)
    return None if w is None else w["read_bytes_per_residual"] + w["write_bytes_per_residual"]


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


def _per_residual(rows, prefix):
    """Sums over each run of consecutive dispatches of kernels with the prefix
    (one run per residual: K1 of every bucket, then the interface kernels,
    then K2 of every bucket).  A run also ends where the dispatch ids jump,
    so that runs with counters taken on a subset of the kernels
    (--kernel-include-regex) still split per residual."""
    sums, cur, inside, last = [], 0.0, False, None
    for d, n, v in rows:
        if _short(n).startswith(prefix):
            if inside and last is not None and d != last + 1:
                sums.append(cur)
                cur = 0.0
            cur += v
            inside = True
            last = d
        elif inside:
            sums.append(cur)
            cur, inside = 0.0, False
    if inside:
        sums.append(cur)
    return sums


def _k2_and_copy(path, counter, last=5):
    """K2 sums of the last residuals (the run command's, after the autotuner's
    trial launches) and the copy's counter."""
    rows = _counter(path, counter)
    k2 = _per_residual([r for r in rows if "copyBuffer" not in r[1]], K2_PREFIX)[-last:]
    copies = [v for _, n, v in rows if "copyBuffer" in n]
    if not k2 or not copies:
        raise SystemExit(f"{path}: need K2 dispatches and the calibration copy")
    return k2, max(copies)


def traffic(workload, fetch_csv, write_csv):
    import workloads as wl

    from . import perfmodel as pm

    k2f, copy_f = _k2_and_copy(fetch_csv, "FETCH_SIZE")
    k2w, copy_w = _k2_and_copy(write_csv, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (copy_f * 1024.0)
    write_scale = COPY_BYTES / (copy_w * 1024.0)
    w = wl.named(workload)
    if hasattr(w, "meshes"):
        import numpy as np
        buckets = {}
        for d in w.degrees:
            for p, n in zip(*np.unique(d, return_counts=True)):
                buckets[int(p)] = buckets.get(int(p), 0) + int(n)
        dim, items = w.dim, sorted(buckets.items())
    else:
        dim, items = w.dim, [(w.degree, w.mesh().n_elements)]
    rec = {
        "kernel": "esd::k_rhs (every bucket of one residual)",
        "residuals": len(k2f),
        "fetch_kib_per_residual": k2f,
        "write_kib_per_residual": k2w,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "read_bytes_per_residual": statistics.fmean(k2f) * 1024.0 * fetch_scale,
        "write_bytes_per_residual": statistics.fmean(k2w) * 1024.0 * write_scale,
        "min_bytes_per_residual": sum(n * pm.min_bytes(dim, p) for p, n in items),
        "layout_bytes_k2_per_residual": sum(n * pm.k2_bytes(dim, p) for p, n in items),
    }
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    h = kernel_source_hash()
    if t.get("kernel_source_sha256") != h:
        t = {"kernel_source_sha256": h, "kernel_sources": list(KERNEL_SOURCES), "workloads": {}}
    t["workloads"][workload] = rec
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    meas = rec["read_bytes_per_residual"] + rec["write_bytes_per_residual"]
    # per degree bucket (one K2 instantiation each), last 5 residuals
    if len(items) > 1:
        import re
        per_f, per_w = {}, {}
        for rows, dst in ((_counter(fetch_csv, "FETCH_SIZE"), per_f), (_counter(write_csv, "WRITE_SIZE"), per_w)):
            for _, n, v in rows:
                m = re.match(r"esd::k_rhs<\d+, (\d+), ", _short(n))
                if m:
                    dst.setdefault(int(m.group(1)), []).append(v)
        print("| p | elements | K2 read MB | K2 write MB | layout MB | measured / layout |")
        print("|---|---|---|---|---|---|")
        for p, n in items:
            rb = statistics.fmean(per_f[p][-5:]) * 1024.0 * fetch_scale
            wb = statistics.fmean(per_w[p][-5:]) * 1024.0 * write_scale
            lb = n * pm.k2_bytes(dim, p)
            print(f"| {p} | {n} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | {lb / 1e6:.1f} | {(rb + wb) / lb:.2f} |")
        print()
    print("| workload | FETCH KiB | WRITE KiB | scale (fetch / write) | read | written | layout bytes | "
          "minimum bytes | measured / layout |")
    print("|---|---|---|---|---|---|---|---|---|")
    print(f"| {workload} | {statistics.fmean(k2f):.1f} | {statistics.fmean(k2w):.1f} | "
          f"{fetch_scale:.3f} / {write_scale:.3f} | {rec['read_bytes_per_residual'] / 1e6:.2f} MB | "
          f"{rec['write_bytes_per_residual'] / 1e6:.2f} MB | {rec['layout_bytes_k2_per_residual'] / 1e6:.2f} MB | "
          f"{rec['min_bytes_per_residual'] / 1e6:.2f} MB | {meas / rec['layout_bytes_k2_per_residual']:.2f} |")


def counters(paths):
    k2, k1 = {}, {}
    for path in paths:
        rows = list(_rows(path))
        for c in sorted({r["Counter_Name"] for r in rows}):
            sel = sorted(((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]))
                          for r in rows if r["Counter_Name"] == c and "copyBuffer" not in r["Kernel_Name"]))
            k2[c] = _per_residual(sel, K2_PREFIX)[-5:]
            k1[c] = _per_residual(sel, K1_PREFIX)[-5:]
    print("| counter | K2 per residual (every bucket) | K1 per residual |")
    print("|---|---|---|")
    for c in k2:
        a = statistics.fmean(k2[c]) if k2[c] else float("nan")
        b = statistics.fmean(k1[c]) if k1.get(c) else float("nan")
        print(f"| {c} | {a:.4g} | {b:.4g} |")


def stats(trace_csv):
    """Per kernel instantiation: the block size the plan ran with (the most
    launches; the autotuner's trial launches at other sizes aside), its launch
    count and average duration; then the per-residual sums of K1 (with the
    mixed-degree interface kernel) and K2 over the degree buckets; then every
    (kernel, block) pair."""
    import re

    by = {}
    for r in _rows(trace_csv):
        name = _short(r.get("Kernel_Name", ""))
        if not name.startswith("esd::"):
            continue
        bs = int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0)
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        by.setdefault((name, bs), []).append(dur)
    chosen = {}
    for (name, bs), d in by.items():
        if name not in chosen or len(d) > len(by[(name, chosen[name])]):
            chosen[name] = bs
    print("| kernel | block (most launches) | launches | average us |")
    print("|---|---|---|---|")
    k1 = k2 = mixed = 0.0

    def plain_k2(n):
        # k_rhs<dim, p, flux, NEXT, DENSE[, DET]>: the plain residual's right-hand side
        m = re.match(r"esd::k_rhs<\d+, \d+, \d+, (true|false), (true|false)(?:, (true|false))?>$", n)
        return bool(m) and m.group(1) == "false" and m.group(2) == "false" and m.group(3) in (None, "false")

    nbuckets = sum(1 for n in chosen if plain_k2(n))
    for name in sorted(chosen, key=lambda n: [int(x) if x.isdigit() else x for x in re.split(r"(\d+)", n)]):
        d = by[(name, chosen[name])]
        avg = statistics.fmean(d) / 1e3
        print(f"| `{name}` | {chosen[name]} | {len(d)} | {avg:.2f} |")
        # the plain residual's kernels: K1 without the projection-only variant,
        # K2 without the stage-combination variant (RK4)
        if name.startswith(K1_PREFIX) and name.endswith("false>"):
            k1 += avg
        elif name.startswith("esd::k_mixed_exterior<"):
            mixed += avg * nbuckets   # one launch per bucket and residual
        elif plain_k2(name):
            k2 += avg
    print()
    print(f"Per residual (sum over buckets of the averages above): K1 {k1 / 1e3:.3f} ms, mixed-degree "
          f"interface {mixed / 1e3:.3f} ms, K2 {k2 / 1e3:.3f} ms.")
    print()
    print("| kernel | block | launches | average us | total us |")
    print("|---|---|---|---|---|")
    for (name, bs), d in sorted(by.items()):
        print(f"| `{name}` | {bs} | {len(d)} | {statistics.fmean(d) / 1e3:.2f} | {sum(d) / 1e3:.1f} |")


def run(workload, reps=5, autotune=True):
    sys.path.insert(0, ROOT)
    import torch

    import workloads as wl

    import paper_2312_07874_amd as esd

    w = wl.named(workload)
    if hasattr(w, "meshes"):
        plan = esd.BatchedPlan(w.dim, [(m.elem_vertex_ids, m.elem_vertex_coords, d) for m, d in zip(w.meshes, w.degrees)],
                               w.warp, w.gamma, w.ecflux, w.dissipation)
        x = plan.node_coords().cpu().numpy()
        u = plan.project(torch.tensor(w.state(x), device="cuda").reshape(plan.nodal_shape).contiguous())
    else:
        plan = esd.Plan.from_workload(w)
        x = plan.node_coords().cpu().numpy()
        u = plan.project(torch.tensor(w.state(x), device="cuda").contiguous())
    print(f"[profiling] {workload}: plan built, state projected", flush=True)
    if autotune:
        plan.autotune(u)
        print(f"[profiling] {workload}: autotuned", flush=True)
    out = torch.empty_like(u)
    torch.cuda.synchronize()
    for i in range(reps):
        plan.residual(u, out)
        torch.cuda.synchronize()
        print(f"[profiling] {workload}: residual {i + 1} of {reps}", flush=True)
    plan.sync_status()
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[profiling] {workload}: calibration copy 1 GiB; blocks {plan.tuning()}", flush=True)


def main(argv):
    if len(argv) >= 2 and argv[0] == "run":
        pos = [a for a in argv[1:] if not a.startswith("--")]
        run(pos[0], int(pos[1]) if len(pos) > 1 else 5, "--no-autotune" not in argv)
    elif len(argv) >= 4 and argv[0] == "traffic":
        sys.path.insert(0, ROOT)
        traffic(argv[1], argv[2], argv[3])
    elif len(argv) >= 2 and argv[0] == "counters":
        counters(argv[1:])
    elif len(argv) >= 2 and argv[0] == "stats":
        stats(argv[1])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
