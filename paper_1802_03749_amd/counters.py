"""HBM traffic of one loop from rocprofv3 hardware counters.

    python -m paper_1802_03749_amd.counters --loop edge --out profiles/<name>_traffic.json
    python -m paper_1802_03749_amd.counters --loop hex --out profiles/<name>_traffic.json

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
    if args.loop == "edge":
        m = quad_mesh(args.nx, args.ny, seed=1)
        L = EdgeFluxLoop(m.x, m.q, m.adt, m.e2n, m.e2c, device=0, order="rcm+partition",
                         block_size=args.block_size, layout=args.layout)
        kw = dict(schedule=args.schedule, elems_per_thread=args.ept, staging=args.staging,
                  tcmode=args.tcmode, block_colouring=args.bcol)
        if args.schedule == "dataflow":
            kw["gather"] = args.gather
        p = L.plan("hier", args.block_size, **kw)
    else:
        m = hex_mesh(args.n, seed=1)
        L = HexLoop(m.x, m.v, m.e2n, device=0, order="rcm+partition", block_size=args.block_size,
                    layout=args.layout)
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
    return re.sub(r"\(.*$", "", name.strip())


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


def driver(args, passthrough) -> int:
    base = os.path.abspath(args.workdir or tempfile.mkdtemp(prefix="counters_"))
    cmds, per = [], {}
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
    copy_f, _ = _mean_of(fetch, r"copyBuffer")
    copy_w, _ = _mean_of(write, r"copyBuffer")
    red_f, _ = _mean_of(fetch, r"reduce_kernel")
    fill_w, _ = _mean_of(write, r"FillFunctor")
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
        "schedule": args.schedule, "elems_per_thread": args.ept, "tcmode": args.tcmode,
        "gather": args.gather if args.loop == "edge" and args.schedule == "dataflow" else "registers",
        "mesh": f"{args.nx}x{args.ny}" if args.loop == "edge" else f"{args.n}^3",
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
    ap.add_argument("--loop", default="edge", choices=["edge", "hex"])
    ap.add_argument("--nx", type=int, default=2400)
    ap.add_argument("--ny", type=int, default=1200)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--layout", default="aos", choices=["aos", "soa"])
    ap.add_argument("--staging", default="all", choices=["all", "inc"])
    ap.add_argument("--tcmode", default="barrier", choices=["barrier", "lds_atomic"])
    ap.add_argument("--schedule", default="dataflow", choices=["colour_launches", "dataflow"])
    ap.add_argument("--bcol", default="recolour", choices=["first_fit", "recolour", "min"])
    ap.add_argument("--ept", type=int, default=2, choices=[1, 2])
    ap.add_argument("--gather", default="registers", choices=["registers", "lds_dma"])
    ap.add_argument("--launches", type=int, default=20)
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
        passthrough.append(argv[i])
        i += 1
    return driver(args, passthrough)


if __name__ == "__main__":
    sys.exit(main())
