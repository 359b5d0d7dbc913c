"""HBM traffic of one loop from rocprofv3 hardware counters.

    python -m paper_1802_03749_amd.counters --loop edge --out profiles/<name>_traffic.json
    python -m paper_1802_03749_amd.counters --loop hex --out profiles/<name>_traffic.json
    python -m paper_1802_03749_amd.counters --loop batch --out profiles/<name>_gaps.json

The driver runs this same module in workload mode (--workload) under
rocprofv3 once per counter pass (FETCH_SIZE, then WRITE_SIZE: one counter
group per run), reads the per-dispatch counter CSVs and writes a JSON file
with the loop kernel's bytes per launch.  The driver itself never touches
the GPU; rocprofv3 starts the workload process directly.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) count the bytes the L2 caches
exchange with the memory fabric, which holds the 256 MB last-level cache
(MALL) in front of HBM, so they are HBM traffic plus MALL hits.  Each is
scaled by what it reads for kernels of known size run in the same process:
a 512 MiB device-to-device copy (512 MiB read, 512 MiB written), a 1 GiB
read-only reduction and a 1 GiB fill (written only).  The copy fixes the
scales; the reduction and the fill check that a read-only and a write-only
kernel are counted the same way (their ratios are reported).

The workload builds the benchmark's plan (the same options as bench.py's
headline) and runs it `--launches` times after the calibration kernels.
With --loop batch the workload is the 64-mesh batch's union time step
replayed from its captured graph, and the driver runs only a kernel trace:
it reports how much of each replayed step lies between the step's kernels.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 512 << 20
READ_BYTES = 1 << 30
FILL_BYTES = 1 << 30


def source_sha(loop: str) -> str:
    name = "kernels_lf2d.hip" if loop == "edge" else "kernels_hex.hip"
    with open(os.path.join(ROOT, "paper_1802_03749_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


# ------------------------------------------------------------ workload mode
def workload(args) -> int:
    import torch
    sys.path.insert(0, ROOT)
    from meshgen import hex_mesh, quad_mesh
    from paper_1802_03749_amd.edgeloop import EdgeFluxLoop
    from paper_1802_03749_amd.hexloop import HexLoop

    # calibration kernels of known size
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    r = torch.ones(READ_BYTES // 8, dtype=torch.float64, device="cuda")
    w = torch.empty(FILL_BYTES // 8, dtype=torch.float64, device="cuda")
    for _ in range(3):
        b.copy_(a)
        _ = r.sum()
        w.fill_(2.0)
    torch.cuda.synchronize()
    del a, b, r, w
    if args.loop == "batch":
        import numpy as np
        from meshgen import quad_batch
        from paper_1802_03749_amd.batched import BatchedSteps
        ms = quad_batch(64, c_min=5e3, c_max=5e5, size_seed=5)
        B = BatchedSteps(ms, np.array([1.0, 0.35, 0.05, 2.7]), mode="union", dtype=args.dtype)
        B.capture()
        for _ in range(args.launches):
            B.replay()
        torch.cuda.synchronize()
        B.check_errors()
        print(json.dumps({"tuned": {str(k): v[0] for k, v in B.tuned.items()},
                          "launches_per_step": B.launches_per_step()}), flush=True)
        B.close()
        return 0
    if args.loop == "edge":
        m = quad_mesh(args.nx, args.ny, seed=1)
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                         block_size=args.block_size, layout=args.layout,
                         point_reorder=args.point_order)
        kw = dict(schedule=args.schedule, elems_per_thread=args.ept, staging=args.staging,
                  tcmode=args.tcmode, block_colouring=args.bcol)
        if args.schedule == "dataflow":
            kw["gather"] = args.gather
        p = L.plan("hier", args.block_size, **kw)
    else:
        m = hex_mesh(args.n, seed=1)
        L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=args.block_size,
                    layout=args.layout, point_reorder=args.point_order)
        p = L.plan("hier", args.block_size, block_colouring="min", schedule=args.schedule,
                   tcmode=args.tcmode)
    for _ in range(args.launches):
        L.run(p)
    torch.cuda.synchronize()
    print(json.dumps({"plan": p.stats}), flush=True)
    L.close()
    return 0


# -------------------------------------------------------------- driver mode
def _kernel_key(name: str) -> str:
    """The kernel name without its trailing parameter list (names contain
    parentheses of their own, e.g. "(anonymous namespace)")."""
    name = name.strip()
    if not name.endswith(")"):
        return name
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        depth += {")": 1, "(": -1}.get(name[i], 0)
        if depth == 0:
            return name[:i].rstrip()
    return name


def _read_counters(outdir: str, counter: str):
    """{kernel name: [value per dispatch]} from the pass's CSV files."""
    per = {}
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter CSV under {outdir}")
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                per.setdefault(_kernel_key(row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
    return per


def _mean_of(per, pattern: str):
    vals = [v for k, vs in per.items() if re.search(pattern, k) for v in vs]
    if not vals:
        raise RuntimeError(f"no dispatch of a kernel matching {pattern!r}")
    return sum(vals) / len(vals), len(vals)


def _max_of(per, pattern: str):
    vals = [v for k, vs in per.items() if re.search(pattern, k) for v in vs]
    if not vals:
        raise RuntimeError(f"no dispatch of a kernel matching {pattern!r}")
    return max(vals)


def _kernel_stats(outdir: str):
    """Rows of rocprofv3's kernel statistics CSV (--stats)."""
    files = glob.glob(os.path.join(outdir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no kernel statistics CSV under {outdir}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def trace_pass(args, passthrough, base):
    """Kernel trace with statistics of the same workload; returns the
    command and {kernel: (calls, avg us, min us, max us)}."""
    outdir = os.path.join(base, "trace")
    cmd = ["timeout", "-s", "KILL", str(args.pass_timeout), "rocprofv3", "--kernel-trace",
           "--stats", "--output-format", "csv", "-d", outdir, "-o", "t", "--", sys.executable,
           "-m", "paper_1802_03749_amd.counters", "--workload", *passthrough]
    print("[counters]", " ".join(cmd), file=sys.stderr, flush=True)
    r = subprocess.run(cmd, cwd=ROOT, stdout=subprocess.PIPE, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"trace pass failed with status {r.returncode}")
    wl = {}
    for line in r.stdout.splitlines():   # the workload's one JSON line
        if line.startswith("{"):
            wl = json.loads(line)
    stats = {}
    for row in _kernel_stats(outdir):
        name = _kernel_key(row["Name"])
        stats[name] = (int(row["Calls"]), float(row["AverageNs"]) / 1e3,
                       float(row["MinNs"]) / 1e3, float(row["MaxNs"]) / 1e3)
    return " ".join(cmd[4:]), stats, wl


def step_gaps(outdir: str, per_step: int, n_steps: int, skip_steps: int = 2):
    """From the kernel trace of graph-replayed steps: a step is the edge-flux
    dispatch that opens it and the per_step - 1 dispatches after it; the
    step's span (first start to last end) against the sum of its kernels'
    durations gives the share of the step spent between kernels."""
    files = glob.glob(os.path.join(outdir, "**", "*kernel_trace.csv"), recursive=True)
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                             _kernel_key(r["Kernel_Name"])))
    rows.sort()
    names = [r[2] for r in rows]
    fpat = r"hier_dma_kernel|hier_flow_kernel|hier_kernel|gcol_kernel|atomic_kernel"
    flux = [i for i, k in enumerate(names) if re.search(fpat, k)]
    # a step may hold several flux launches (colour launches): a step opens
    # with a flux launch that follows a dispatch of another kernel; the
    # last n_steps such openings are the replays
    starts = [i for i in flux if i == 0 or not re.search(fpat, names[i - 1])]
    starts = starts[-n_steps:][skip_steps:]
    steps = [rows[i:i + per_step] for i in starts if i + per_step <= len(rows)]
    spans = [st[-1][1] - st[0][0] for st in steps]
    busy = [sum(e - b for b, e, _ in st) for st in steps]
    gaps = [sp - bu for sp, bu in zip(spans, busy)]
    # start to start of consecutive steps: includes the time between two
    # graph replays
    periods = [b[0][0] - a[0][0] for a, b in zip(steps, steps[1:])]
    n = len(steps)
    pbusy = busy[:len(periods)]
    return {"steps_analysed": n, "dispatches_per_step": per_step,
            "mean_period_us": sum(periods) / len(periods) / 1e3 if periods else None,
            "period_gap_share": (1 - sum(pbusy) / sum(periods)) if periods else None,
            "kernels_of_a_step": [k for _, _, k in steps[-1]] if steps else [],
            "mean_step_span_us": sum(spans) / n / 1e3 if n else None,
            "mean_kernel_time_us": sum(busy) / n / 1e3 if n else None,
            "mean_gap_us": sum(gaps) / n / 1e3 if n else None,
            "gap_share": (sum(gaps) / sum(spans)) if n else None,
            "all_dispatches": len(names)}


def driver(args, passthrough) -> int:
    base = os.path.abspath(args.workdir or tempfile.mkdtemp(prefix="counters_"))
    cmds, per = [], {}
    trace = None
    if args.loop == "batch":
        # the batch: kernel trace only, the gaps between the step's launches
        tcmd, stats, wl = trace_pass(args, passthrough, base)
        per_step = wl.get("launches_per_step", args.per_step)
        out = {"loop": "batch", "dtype": args.dtype, "trace_command": tcmd,
               "tuned": wl.get("tuned"), "launches_per_step": per_step,
               "kernels": {k: {"calls": v[0], "avg_us": v[1], "min_us": v[2], "max_us": v[3]}
                           for k, v in sorted(stats.items())},
               "gaps": step_gaps(os.path.join(base, "trace"), per_step, args.launches)}
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)
        return 0
    if args.trace:
        trace = trace_pass(args, passthrough, base)[:2]
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        outdir = os.path.join(base, counter.lower())
        cmd = ["timeout", "-s", "KILL", str(args.pass_timeout), "rocprofv3", "--pmc", counter,
               "--output-format", "csv", "-d", outdir, "-o", "p", "--", sys.executable, "-m",
               "paper_1802_03749_amd.counters", "--workload", *passthrough]
        print("[counters]", " ".join(cmd), file=sys.stderr, flush=True)
        r = subprocess.run(cmd, cwd=ROOT)
        if r.returncode != 0:
            print(f"[counters] pass {counter} failed with status {r.returncode}", file=sys.stderr)
            return r.returncode
        per[counter] = _read_counters(outdir, counter)
        cmds.append(" ".join(cmd[4:]))
    fetch, write = per["FETCH_SIZE"], per["WRITE_SIZE"]
    # the calibration dispatches are the largest of their kernels in the
    # workload (the same kernels also copy or fill smaller buffers)
    copy_f = _max_of(fetch, r"copyBuffer")
    copy_w = _max_of(write, r"copyBuffer")
    red_f = _max_of(fetch, r"reduce_kernel")
    fill_w = _max_of(write, r"FillFunctor")
    kib = 1024.0
    fetch_scale = COPY_BYTES / kib / copy_f
    write_scale = COPY_BYTES / kib / copy_w
    kpat = r"hier_dma_kernel|hier_flow_kernel|hier_kernel" if args.loop == "edge" \
        else r"hex_flow_kernel|hex_hier_kernel"
    lf, nl = _mean_of(fetch, kpat)
    lw, _ = _mean_of(write, kpat)
    kname = sorted(k for k in fetch if re.search(kpat, k))
    out = {
        "kernel": kname,
        "loop": args.loop,
        "kernel_source_sha256": source_sha(args.loop),
        "block_size": args.block_size, "layout": args.layout, "staging": args.staging,
        "schedule": args.schedule, "elems_per_thread": args.ept if args.loop == "edge" else 1,
        "tcmode": args.tcmode,
        "gather": args.gather if args.loop == "edge" and args.schedule == "dataflow" else "registers",
        "mesh": f"{args.nx}x{args.ny}" if args.loop == "edge" else f"{args.n}^3",
        "point_order": args.point_order,
        "fetch_kib_per_launch": lf, "write_kib_per_launch": lw, "launches_counted": nl,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "bytes_per_launch": (lf * fetch_scale + lw * write_scale) * kib,
        "calibration": {
            "copy_512MiB_fetch_kib": copy_f, "copy_512MiB_write_kib": copy_w,
            "read_only_1GiB_fetch_kib": red_f, "fill_1GiB_write_kib": fill_w,
            "read_only_scale": READ_BYTES / kib / red_f,
            "fill_scale": FILL_BYTES / kib / fill_w,
            "note": "scales from the copy; the read-only reduction and the fill check "
                    "that reads and writes of other kernels are counted alike"},
        "what_is_counted": "L2-to-fabric bytes (HBM plus last-level-cache hits), scaled",
        "commands": cmds,
    }
    if trace is not None:
        tcmd, stats = trace
        mine = {k: v for k, v in stats.items() if re.search(kpat, k)}
        out["trace"] = {"command": tcmd,
                        "kernels": {k: {"calls": v[0], "avg_us": v[1], "min_us": v[2],
                                        "max_us": v[3]} for k, v in sorted(mine.items())}}
        if mine:
            calls = sum(v[0] for v in mine.values())
            avg = sum(v[0] * v[1] for v in mine.values()) / calls
            out["trace"]["avg_us"] = avg
            out["trace"]["traffic_tbps"] = out["bytes_per_launch"] / (avg * 1e-6) / 1e12
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--out", default=None)
    ap.add_argument("--workdir", default=None, help="where rocprofv3 writes its CSV files")
    ap.add_argument("--pass-timeout", type=int, default=150)
    ap.add_argument("--loop", default="edge", choices=["edge", "hex", "batch"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--per-step", type=int, default=6,
                    help="batch: kernel launches of one replayed step")
    ap.add_argument("--nx", type=int, default=2400)
    ap.add_argument("--ny", type=int, default=1200)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--layout", default="aos", choices=["aos", "soa"])
    ap.add_argument("--staging", default="all", choices=["all", "inc"])
    ap.add_argument("--tcmode", default="barrier", choices=["barrier", "lds_atomic"])
    ap.add_argument("--schedule", default="dataflow", choices=["colour_launches", "dataflow"])
    ap.add_argument("--bcol", default="recolour", choices=["first_fit", "recolour", "min"])
    ap.add_argument("--ept", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--gather", default="lds_dma", choices=["registers", "lds_dma"])
    ap.add_argument("--point-order", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--trace", action="store_true",
                    help="also run a kernel-trace pass with statistics (average launch time)")
    args, _ = ap.parse_known_args()
    if args.workload:
        return workload(args)
    if not args.out:
        ap.error("--out is required")
    skip = {"--out", "--workdir", "--pass-timeout"}
    passthrough, argv, i = [], sys.argv[1:], 0
    while i < len(argv):
        if argv[i] in skip:
            i += 2
            continue
        if argv[i] == "--trace":
            i += 1
            continue
        passthrough.append(argv[i])
        i += 1
    return driver(args, passthrough)


if __name__ == "__main__":
    sys.exit(main())
