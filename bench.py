#!/usr/bin/env python3
"""Benchmark of the race-free indirect-increment edge loop on one MI355X.

One step = one execution of the whole loop (all of its kernel launches) over
the 2D edge-flux workload: a 2400 x 1200 jittered quad mesh (2.88M cells,
5,756,400 interior edges) in FP64, reordered (reverse Cuthill-McKee, then
block partitioning with block-signature point grouping) and run with the
two-layer (hierarchical) colouring, its block colours executed by default
as one dataflow launch (blocks in colour order, each waiting only for its
earlier-coloured neighbours; --schedule colour_launches runs one launch per
block colour as in the paper).  Inputs are seeded synthetic data
resident in HBM before timing starts; the plan is built once beforehand and
its build time is reported separately.

Prints one JSON line to stdout; progress goes to stderr.  Besides the
headline it reports: the global-colouring and atomics baselines on the same
GPU and mesh (each at its best of RCM / RCM + partition order and AoS /
SoA layout), the FP32-storage
variant, the 3D hexahedral element loop (128^3 elements) with its own
baselines, a batch of 64 meshes of uneven size (5k-500k cells) advanced by
full time steps as one union and one mesh at a time (eager and replayed
from a captured HIP graph), a plain device-copy bandwidth probe, and the
CPU oracle timed on the host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "edges/s and achieved HBM GB/s (% peak) vs atomics/global-colour, FP64 and FP32"
KERNEL_SRC = os.path.join(ROOT, "paper_1802_03749_amd", "csrc", "kernels_lf2d.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "edge_flux_2400x1200_traffic.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def time_steps(torch, run, steps: int, warmup: int, settle_s: float = 0.05) -> float:
    """Seconds per step over `steps` timed steps after `warmup` untimed (and,
    before those, untimed executions for about settle_s seconds)."""
    settle(torch, run, settle_s)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def settle(torch, run, seconds: float) -> None:
    """Untimed executions for about `seconds`, so that timing does not start
    on a GPU that idled through host-side setup (plan builds, uploads)."""
    until = time.perf_counter() + seconds
    while time.perf_counter() < until:
        for _ in range(20):
            run()
        torch.cuda.synchronize()


def copy_probe(torch, nbytes: int = 512 << 20, reps: int = 20):
    """Device-to-device copy of nbytes (read nbytes + write nbytes): the
    bandwidth a plain streaming kernel reaches on this GPU, and the
    reference kernel of known size for scaling HBM byte counters."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2 * nbytes / sec / 1e9, sec


def cold_sweep_seconds(torch, run, steps: int) -> float:
    """Seconds per sweep with the caches evicted: before every sweep a 1 GiB
    fill (four times the 256 MB last-level cache) runs on the same stream,
    and only the sweep's launches sit between the two events."""
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    run()
    torch.cuda.synchronize()
    for e0, e1 in evs:
        flush.fill_(1.0)
        e0.record()
        run()
        e1.record()
    torch.cuda.synchronize()
    ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    del flush
    return sum(ms) / len(ms) * 1e-3


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_sweep(torch, args, U):
    """The 1200 x 600 sweep (720k cells, 1.44M edges, FP64): order x strategy
    x block size.  Random-order hierarchical plans need more block colours
    than the limit of 256 and are reported as not run, as the paper did for
    such meshes (Section 3.1.5)."""
    from meshgen import quad_mesh
    from paper_1802_03749_amd import measure
    from paper_1802_03749_amd.edgeloop import EdgeFluxLoop
    nx, ny = 1200, 600
    C, N, E = measure.quad_counts(nx, ny)
    useful = measure.useful_bytes(N, C, E)
    mesh = quad_mesh(nx, ny, seed=1)
    steps, warm = max(args.steps // 2, 10), 2
    sizes = (128, 256, 384, 512, 640, 768, 896, 1024)
    out = {"mesh": f"{nx}x{ny}", "edges": E, "useful_bytes_per_step": useful,
           "steps_per_entry": steps, "entries": {}}
    ent = out["entries"]

    def timed(L, p):
        s = time_steps(torch, lambda: L.run(p), steps, warm)
        if U.um_plan_errors(p.handle) != 0:
            raise RuntimeError("a dataflow wait timed out in the sweep")
        return {"us_per_sweep": s * 1e6, "edges_per_s": E / s, "useful_gbps": useful / s / 1e9,
                "launches": p.stats["n_launches"], "block_colours": p.stats["n_block_colours"],
                "global_colours": p.stats["n_global_colours"],
                "sum_first_blocks": p.stats["n_sum_first_blocks"]}

    def hier_entries(L, order, S, plans):
        for name, kw in plans:
            try:
                ent[f"{order}/hier_{name}/S{S}"] = timed(L, L.plan("hier", S, **kw))
            except U.UmeshError as e:
                why = "colours" if e.status == U.UM_ERR_COLOURS else U.STATUS_NAMES.get(e.status)
                ent[f"{order}/hier_{name}/S{S}"] = {"not_run": why}

    cl = ("colour_launches", dict(schedule="colour_launches", block_colouring="recolour"))
    df = ("dataflow", dict(schedule="dataflow", elems_per_thread=2, block_colouring="recolour",
                           gather=args.gather))
    for order, lorder in (("random", "none"), ("rcm", "rcm")):
        L = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0, order=lorder,
                         block_size=512)
        for S in sizes:
            for strat in ("atomic", "global"):
                ent[f"{order}/{strat}/S{S}"] = timed(L, L.plan(strat, S))
            hier_entries(L, order, S, (cl,))
        L.close()
        log(f"sweep {order} done")
    for S in sizes:
        L = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0,
                         order="rcm+partition", block_size=S, point_reorder=args.point_order)
        for strat in ("atomic", "global"):
            ent[f"rcm+partition/{strat}/S{S}"] = timed(L, L.plan(strat, S))
        extra = ()
        if args.gather == "lds_dma":
            # every block loading its residuals early instead (none sums first)
            extra = (("dataflow_no_sum_first", dict(df[1], sum_first="never")),)
        hier_entries(L, "rcm+partition", S, (cl, df) + extra)
        L.close()
    log("sweep rcm+partition done")
    best = {}
    for k, v in ent.items():
        if "us_per_sweep" not in v:
            continue
        order, strat = k.split("/")[0], k.split("/")[1]
        key = f"{order}/{strat}"
        if key not in best or v["us_per_sweep"] < best[key]["us_per_sweep"]:
            best[key] = dict(v, block_size=int(k.rsplit("/S", 1)[1]))
    out["best"] = best
    return out


def tile_blocks(mesh, tx: int, ty: int) -> np.ndarray:
    """Hand-made geometric edge blocks (the paper's reuse upper bound): tiles
    of tx x ty cells of the natural grid; an interior edge belongs to the
    tile of its right cell (a cell takes its left and bottom edges)."""
    nat = mesh.cell_nat[mesh.e2c[:, 1]]
    i, j = nat % mesh.nx, nat // mesh.nx
    return ((j // ty) * ((mesh.nx + tx - 1) // tx) + i // tx).astype(np.int32)


def run_ablations(torch, mesh, S, args, useful, E):
    """One knob at a time around the headline configuration."""
    from paper_1802_03749_amd.edgeloop import EdgeFluxLoop
    steps, warm = max(args.steps // 4, 10), max(args.warmup // 4, 2)
    out = {}

    def entry(L, p):
        s = time_steps(torch, lambda: L.run(p), steps, warm)
        st = p.stats
        return {"us_per_sweep": s * 1e6, "useful_gbps": useful / s / 1e9,
                "pct_hbm_peak": 100 * useful / s / 1e9 / 8000.0, "launches": st["n_launches"],
                "block_colours": st["n_block_colours"], "global_colours": st["n_global_colours"],
                "reuse_factor": st["reuse_factor"]}

    base = dict(staging=args.staging, tcmode=args.tcmode, block_colouring=args.bcol,
                schedule=args.schedule, elems_per_thread=args.ept)
    if args.schedule == "dataflow":
        base["gather"] = args.gather
    tx = 16
    ty = max(S // (2 * tx), 1)
    parts = (("chunks_of_rcm", "rcm", {}),
             ("recursive_bisection", "rcm+partition", {}),
             (f"geometric_tiles_{tx}x{ty}", "rcm+user", {"edge_blocks": tile_blocks(mesh, tx, ty)}))
    for name, order, kw in parts:
        for layout in ("aos", "soa"):
            L = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0, order=order,
                             block_size=S, layout=layout, point_reorder=args.point_order, **kw)
            kw0 = dict(base)
            if layout == "soa" and "gather" in kw0:
                kw0["gather"] = "registers"   # the LDS-DMA gather reads AoS records
            out[f"hier_{name}_{layout}"] = entry(L, L.plan("hier", S, **kw0))
            if name == "recursive_bisection" and layout == args.layout:
                for knob, val in (("staging", "inc"), ("tcmode", "lds_atomic"),
                                  ("block_colouring", "first_fit"), ("block_colouring", "recolour"),
                                  ("schedule", "colour_launches"), ("schedule", "dataflow"),
                                  ("elems_per_thread", 1), ("elems_per_thread", 2),
                                  ("gather", "registers"), ("gather", "lds_dma"),
                                  ("wave_colour_groups", True), ("xcd_groups", 8),
                                  ("sum_first", "always")):
                    if base.get(knob) == val:
                        continue
                    o = dict(base); o[knob] = val
                    if o["schedule"] != "dataflow":
                        o.pop("gather", None)
                    elif "gather" not in o:
                        o["gather"] = args.gather
                    try:
                        out[f"hier_partition_{knob}_{val}"] = entry(L, L.plan("hier", S, **o))
                    except Exception as e:  # an unsupported combination
                        out[f"hier_partition_{knob}_{val}"] = {"error": str(e)}
            L.close()
            if name == "recursive_bisection" and layout == args.layout:
                # the other point order (a property of the renumbered mesh)
                po = 1 if args.point_order != 1 else 2
                L = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0,
                                 order=order, block_size=S, layout=layout, point_reorder=po)
                out[f"hier_partition_point_order_{po}"] = entry(L, L.plan("hier", S, **base))
                L.close()
            log(f"ablation {name} {layout} done")
    for order in ("none", "rcm", "gps", "rcm+partition"):
        for layout in ("aos", "soa"):
            L = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0, order=order,
                             block_size=S, layout=layout)
            out[f"global_{order}_{layout}"] = entry(L, L.plan("global", 256))
            out[f"atomic_{order}_{layout}"] = entry(L, L.plan("atomic", 256))
            L.close()
        log(f"ablation global/atomic {order} done")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--nx", type=int, default=2400)
    ap.add_argument("--ny", type=int, default=1200)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--layout", default="aos", choices=["aos", "soa"])
    ap.add_argument("--staging", default="all", choices=["all", "inc"])
    ap.add_argument("--tcmode", default="barrier", choices=["barrier", "lds_atomic"])
    ap.add_argument("--schedule", default="dataflow", choices=["colour_launches", "dataflow"])
    ap.add_argument("--bcol", default="recolour", choices=["first_fit", "recolour"])
    ap.add_argument("--ept", type=int, default=2, choices=[1, 2],
                    help="edges per lane (the workgroup has block_size / ept lanes)")
    ap.add_argument("--point-order", type=int, default=2, choices=[1, 2, 3],
                    help="1: the paper's block-signature order of points; 2: smallest "
                         "accessing block first; 3: accessing blocks from the largest down")
    ap.add_argument("--hex-point-order", type=int, default=3, choices=[1, 2, 3],
                    help="point order of the hex loop's hierarchical plans")
    ap.add_argument("--gather", default="lds_dma", choices=["registers", "lds_dma"],
                    help="dataflow gather: through registers, or loads that write LDS directly")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="host time spent timing the CPU oracle (0 = skip)")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the global-colour and atomics baselines")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32 variant, the 3D hex workload and the batch")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batch of 64 meshes")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the ablation matrix (partitioner, order, layout, staging, colour "
                         "rounds, block colouring, schedule, gather, wave-pure colour groups)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 1200x600 order x strategy x block-size sweep")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch

    sys.path.insert(0, ROOT)
    from meshgen import hex_mesh, quad_mesh
    from paper_1802_03749_amd import measure
    from paper_1802_03749_amd import umesh as U
    from paper_1802_03749_amd.edgeloop import EdgeFluxLoop
    from paper_1802_03749_amd.hexloop import HexLoop

    U.lib()  # fails loudly if the HIP library is not built
    dev = torch.cuda.get_device_properties(0)
    log(f"device {dev.name} {dev.gcnArchName} CUs={dev.multi_processor_count}")
    copy_gbps, _ = copy_probe(torch)
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write of 512 MiB)")
    nx, ny, S = args.nx, args.ny, args.block_size
    C, N, E = measure.quad_counts(nx, ny)
    t = time.perf_counter()
    mesh = quad_mesh(nx, ny, seed=1)
    log(f"mesh {nx}x{ny}: C={C} N={N} E={E} generated in {time.perf_counter() - t:.1f}s")

    # ---- hierarchical colouring on the reordered + partitioned mesh
    t = time.perf_counter()
    hier = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0,
                        order="rcm+partition", block_size=S, layout=args.layout,
                        point_reorder=args.point_order)
    reorder_s = time.perf_counter() - t
    hopts = dict(staging=args.staging, tcmode=args.tcmode, block_colouring=args.bcol,
                 elems_per_thread=args.ept)
    if args.schedule == "dataflow":
        hopts["gather"] = args.gather
    plan = hier.plan("hier", S, schedule=args.schedule, **hopts)
    st = plan.stats
    log(f"reorder {reorder_s:.1f}s, plan {st['build_seconds']:.2f}s: blocks={st['n_blocks']} "
        f"block colours={st['n_block_colours']} thread colours<={st['max_thread_colours']} "
        f"reuse={st['reuse_factor']:.3f} lds={st['lds_bytes_max']} launches={st['n_launches']}")
    run = lambda: hier.run(plan)
    settle(torch, run, 0.3)
    sec = time_steps(torch, run, args.steps, args.warmup)
    if U.um_plan_errors(plan.handle) != 0:
        log("a dataflow wait timed out: the timed results are invalid")
        return 3
    log(f"hier ({args.schedule}): {sec * 1e6:.1f} us/step")

    # roofline: the timed region above was bracketed by HIP events on the
    # stream the library launches on (torch's current stream); its launches
    # run back to back, so the average launch takes sec / launches_per_step
    useful = measure.useful_bytes(N, C, E)
    launches_per_step = st["n_launches"]
    avg_launch_s = sec / launches_per_step
    bytes_per_launch = useful / launches_per_step
    achieved, frac = measure.roofline(bytes_per_launch, avg_launch_s)
    # per-launch durations from event pairs the library records around every
    # launch (a second pass; the extra event packets between launches make
    # these slightly longer, so they are a diagnostic only)
    U.um_plan_set_timing(plan.handle, True)
    for _ in range(args.steps):
        run()
    kern_ms, n_launch = U.um_plan_timing(plan.handle)
    U.um_plan_set_timing(plan.handle, False)
    torch.cuda.synchronize()
    log(f"avg launch {avg_launch_s * 1e6:.1f} us ({launches_per_step} per step), achieved "
        f"{achieved:.0f} GB/s ({100 * frac:.1f}% of peak); per-launch events: "
        f"{kern_ms / n_launch * 1e3:.1f} us")

    # the same plan with cold caches: a 1 GiB fill before every sweep, only
    # the sweep between the events
    cold_s = cold_sweep_seconds(torch, run, args.steps)
    cold_achieved, cold_frac = measure.roofline(useful / launches_per_step,
                                                cold_s / launches_per_step)
    log(f"cold caches: {cold_s * 1e6:.1f} us/step, {cold_achieved:.0f} GB/s "
        f"({100 * cold_frac:.1f}% of peak)")

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if (tr.get("kernel_source_sha256") == kernel_hash() and tr.get("block_size") == S
                and tr.get("layout") == args.layout and tr.get("staging") == args.staging
                and tr.get("schedule") == args.schedule
                and tr.get("elems_per_thread", 1) == args.ept
                and tr.get("gather", "registers") == (args.gather if args.schedule == "dataflow"
                                                      else "registers")
                and tr.get("point_order", 1) == args.point_order):
            traffic = tr.get("bytes_per_launch")

    variants = {}
    other = "colour_launches" if args.schedule == "dataflow" else "dataflow"
    o2 = dict(hopts)
    if other == "dataflow":
        o2["gather"] = args.gather
    else:
        o2.pop("gather", None)
    p2 = hier.plan("hier", S, schedule=other, **o2)
    s2 = time_steps(torch, lambda: hier.run(p2), args.steps, args.warmup)
    variants[f"fp64_{other}"] = {"edges_per_s": E / s2, "ms_per_step": s2 * 1e3,
                                 "useful_gbps": useful / s2 / 1e9,
                                 "launches": p2.stats["n_launches"]}
    log(f"hier ({other}): {s2 * 1e6:.1f} us/step")
    # LDS atomics instead of thread-colour rounds (an extension; the order of
    # additions inside a block is then not fixed)
    if args.tcmode != "lds_atomic":
        o4 = dict(hopts); o4["tcmode"] = "lds_atomic"
        p4 = hier.plan("hier", S, schedule=args.schedule, **o4)
        s4 = time_steps(torch, lambda: hier.run(p4), args.steps, args.warmup)
        variants[f"fp64_{args.schedule}_lds_atomic"] = {
            "edges_per_s": E / s4, "ms_per_step": s4 * 1e3, "useful_gbps": useful / s4 / 1e9,
            "pct_hbm_peak": 100 * useful / s4 / 1e9 / measure.HBM_PEAK_GBPS,
            "launches": p4.stats["n_launches"]}
        log(f"hier ({args.schedule}, lds atomics): {s4 * 1e6:.1f} us/step")
    # the other number of edges per lane (the paper's kernels use one)
    o5 = dict(hopts); o5["elems_per_thread"] = 3 - args.ept
    p5 = hier.plan("hier", S, schedule=args.schedule, **o5)
    s5 = time_steps(torch, lambda: hier.run(p5), args.steps, args.warmup)
    variants[f"fp64_{args.schedule}_{3 - args.ept}_edges_per_lane"] = {
        "edges_per_s": E / s5, "ms_per_step": s5 * 1e3, "useful_gbps": useful / s5 / 1e9,
        "launches": p5.stats["n_launches"]}
    log(f"hier ({args.schedule}, {3 - args.ept} edge(s) per lane): {s5 * 1e6:.1f} us/step")
    # the other gather of the dataflow schedule
    if args.schedule == "dataflow":
        og = "registers" if args.gather == "lds_dma" else "lds_dma"
        o6 = dict(hopts); o6["gather"] = og
        p6 = hier.plan("hier", S, schedule=args.schedule, **o6)
        s6 = time_steps(torch, lambda: hier.run(p6), args.steps, args.warmup)
        variants[f"fp64_{args.schedule}_gather_{og}"] = {
            "edges_per_s": E / s6, "ms_per_step": s6 * 1e3, "useful_gbps": useful / s6 / 1e9,
            "pct_hbm_peak": 100 * useful / s6 / 1e9 / measure.HBM_PEAK_GBPS,
            "launches": p6.stats["n_launches"]}
        log(f"hier ({args.schedule}, gather {og}): {s6 * 1e6:.1f} us/step")
        # the headline plan's launches captured in one HIP graph and replayed
    graph = U.HipGraph(lambda stream: hier.run(plan, stream=stream))
    s3 = time_steps(torch, graph.replay, args.steps, args.warmup)
    variants[f"fp64_{args.schedule}_graph"] = {"edges_per_s": E / s3, "ms_per_step": s3 * 1e3,
                                               "useful_gbps": useful / s3 / 1e9,
                                               "launches": st["n_launches"]}
    log(f"hier ({args.schedule}, graph replay): {s3 * 1e6:.1f} us/step")
    graph.close()
    hier.close()

    # ---- baselines on the same GPU and mesh, each in its best order and
    # layout (the atomics are much faster on SoA data, global colouring on the
    # partition order)
    baselines = {}
    if not args.no_baselines:
        tried = {"global_colour": {}, "atomics": {}}
        for order in ("rcm", "rcm+partition"):
            for layout in ("aos", "soa"):
                base = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0,
                                    order=order, block_size=S, layout=layout)
                for name, strat in (("global_colour", "global"), ("atomics", "atomic")):
                    p = base.plan(strat, 256)
                    s = time_steps(torch, lambda: base.run(p), args.steps, args.warmup)
                    tried[name][f"{order}/{layout}"] = {
                        "order": order, "layout": layout, "edges_per_s": E / s,
                        "ms_per_step": s * 1e3, "useful_gbps": useful / s / 1e9,
                        "launches": p.stats["n_launches"], "hier_speedup": s / sec}
                base.close()
        for name, runs in tried.items():
            best = min(runs.values(), key=lambda r: r["ms_per_step"])
            baselines[name] = dict(best, configurations=runs)
            log(f"{name}: best {best['ms_per_step'] * 1e3:.1f} us/step ({best['order']}, "
                f"{best['layout']}); hierarchical {best['hier_speedup']:.2f}x faster")

    extras = {}
    if not args.no_extras:
        # FP32 storage of x, q, adt (res stays FP64)
        f32 = EdgeFluxLoop(mesh.x, mesh.q, mesh.adt, mesh.e2n, mesh.e2c, device=0,
                           order="rcm+partition", block_size=S, layout=args.layout, dtype="f32")
        useful32 = measure.useful_bytes(N, C, E, real_bytes=4)
        p = f32.plan("hier", S, schedule=args.schedule, **hopts)
        s = time_steps(torch, lambda: f32.run(p), args.steps, args.warmup)
        extras["edge_flux_fp32"] = {"edges_per_s": E / s, "ms_per_step": s * 1e3,
                                    "useful_bytes_per_step": useful32,
                                    "useful_gbps": useful32 / s / 1e9,
                                    "pct_hbm_peak": 100 * useful32 / s / 1e9 / measure.HBM_PEAK_GBPS,
                                    "speedup_vs_fp64": sec / s}
        log(f"fp32 hier: {s * 1e6:.1f} us/step ({useful32 / s / 1e9:.0f} GB/s useful)")
        f32.close()
        # 3D hexahedral element loop, 128^3 elements
        hm = hex_mesh(128, seed=1)
        hb = 96 * hm.n_nodes + 32 * hm.n_elems   # x, v once, force twice, int32 map
        hx = {"elements": hm.n_elems, "nodes": hm.n_nodes, "useful_bytes_per_step": hb}
        # hierarchical in the headline layout (dataflow schedule at 256
        # elements per block; one launch per block colour at 512 as a
        # variant), points ordered by --hex-point-order; the baselines in
        # their best layout (atomics run far faster on SoA data)
        for order, strat, hS, layouts in (("rcm+partition", "hier", 256, (args.layout,)),
                                          ("rcm+partition", "hier_colour_launches", 512,
                                           (args.layout,)),
                                          ("rcm", "global", 256, ("aos", "soa")),
                                          ("rcm", "atomic", 256, ("aos", "soa"))):
            runs = {}
            for lay in layouts:
                H = HexLoop(hm.x, hm.v, hm.e2n, device=0, order=order, block_size=hS,
                            layout=lay, point_reorder=args.hex_point_order)
                if strat == "hier":
                    p = H.plan("hier", hS, block_colouring="min", schedule="dataflow")
                elif strat == "hier_colour_launches":
                    p = H.plan("hier", hS, block_colouring="min")
                else:
                    p = H.plan(strat, hS)
                s = time_steps(torch, lambda: H.run(p), max(args.steps // 2, 1), args.warmup)
                if U.um_plan_errors(p.handle) != 0:
                    log("a hex dataflow wait timed out: the timed results are invalid")
                    return 3
                runs[lay] = {"order": order, "layout": lay, "block_size": hS,
                             "point_order": args.hex_point_order if "hier" in strat else None,
                             "elements_per_s": hm.n_elems / s, "ms_per_step": s * 1e3,
                             "useful_gbps": hb / s / 1e9, "launches": p.stats["n_launches"],
                             "block_colours": p.stats["n_block_colours"]}
                if strat == "hier":
                    p2 = H.plan("hier", hS, block_colouring="min", tcmode="lds_atomic",
                                schedule="dataflow")
                    s2 = time_steps(torch, lambda: H.run(p2), max(args.steps // 2, 1),
                                    args.warmup)
                    hx["hier_lds_atomic"] = {"order": order, "layout": lay, "block_size": hS,
                                             "elements_per_s": hm.n_elems / s2,
                                             "ms_per_step": s2 * 1e3,
                                             "useful_gbps": hb / s2 / 1e9,
                                             "launches": p2.stats["n_launches"]}
                    log(f"hex hier lds atomics: {s2 * 1e6:.1f} us/step")
                H.close()
            best = min(runs.values(), key=lambda r: r["ms_per_step"])
            hx[strat] = dict(best, configurations=runs) if len(runs) > 1 else best
            log(f"hex {strat}: {best['ms_per_step'] * 1e3:.1f} us/step "
                f"({best['useful_gbps']:.0f} GB/s, {best['layout']})")
        extras["hex_hourglass_128cubed"] = hx
        # one full explicit time step on the benchmark mesh: cell adt, edge
        # flux (the headline plan's options), far-field boundary flux, update
        # with the sum of squares
        from paper_1802_03749_amd.timestep import TimeStep2D
        qinf = np.array([1.0, 0.35, 0.05, 2.7])
        tsx = {}
        for dt, rb in (("f64", 8), ("f32", 4)):
            ts = TimeStep2D(mesh.x, mesh.q, mesh.e2n, mesh.e2c, mesh.b2n, mesh.b2c, mesh.c2n,
                            qinf, device=0, block_size=S, layout=args.layout, dtype=dt)
            # the four loops as such, then the update fused with the next
            # step's adt (one pass over q fewer; the step's algorithmic
            # bytes are counted for the four loops in both cases)
            for fused in (False, True):
                ts.build_plans(flux_block_size=S, staging=args.staging, tcmode=args.tcmode,
                               block_colouring=args.bcol, schedule=args.schedule,
                               elems_per_thread=args.ept, fuse_adt=fused,
                               gather=args.gather if args.schedule == "dataflow" else "registers")
                s = time_steps(torch, ts.step, max(args.steps // 4, 1), args.warmup)
                sb = measure.step_useful_bytes(N, C, E, ts.B, rb)
                name = dt + ("_fused_update_adt" if fused else "")
                loops = ("flux", "bres", "upa") if fused else ("adt", "flux", "bres", "upd")
                tsx[name] = {"ms_per_step": s * 1e3, "cells_per_s": C / s,
                             "useful_bytes_per_step": sb, "useful_gbps": sb / s / 1e9,
                             "launches": sum(ts.plans[k].stats["n_launches"] for k in loops)}
                log(f"time step {name}: {s * 1e6:.1f} us/step ({sb / s / 1e9:.0f} GB/s useful)")
            ts.close()
        extras["time_step_2400x1200"] = tsx

    if not args.no_extras and not args.no_batched:
        # 64 meshes of log-uniform size 5k-500k cells, one full time step
        # (adt, edge flux, boundary flux, update + sum of squares) per mesh
        from meshgen import quad_batch
        from paper_1802_03749_amd.batched import BatchedSteps
        t = time.perf_counter()
        ms = quad_batch(64, c_min=5e3, c_max=5e5, size_seed=5)
        qinf = np.array([1.0, 0.35, 0.05, 2.7])
        bx = {"meshes": len(ms), "cells": int(sum(m.q.shape[0] for m in ms)),
              "interior_edges": int(sum(m.e2n.shape[0] for m in ms)),
              "boundary_edges": int(sum(m.b2n.shape[0] for m in ms))}
        log(f"batch of {len(ms)} meshes: {bx['cells']} cells, generated in "
            f"{time.perf_counter() - t:.1f}s")
        bsteps = max(args.steps // 20, 5)
        for dt in ("f64", "f32"):
            for mode in ("union", "sequential"):
                t = time.perf_counter()
                B = BatchedSteps(ms, qinf, mode=mode, dtype=dt)
                setup = time.perf_counter() - t
                eager = time_steps(torch, B.step, bsteps, 2)
                B.capture()
                graph = time_steps(torch, B.replay, bsteps, 2)
                launches = B.launches_per_step()
                bx[f"{mode}_{dt}"] = {
                    "ms_per_step_eager": eager * 1e3, "ms_per_step_graph": graph * 1e3,
                    "edges_per_s_graph": bx["interior_edges"] / graph,
                    "cells_per_s_graph": bx["cells"] / graph,
                    "launches_per_step": launches, "setup_seconds": setup,
                    "tuned": {str(k): v[0] for k, v in B.tuned.items()}}
                log(f"batched {mode} {dt}: eager {eager * 1e3:.3f} ms, graph {graph * 1e3:.3f} ms "
                    f"per step, {launches} launches")
                B.close()
            bx[f"union_speedup_vs_sequential_graph_{dt}"] = (
                bx[f"sequential_{dt}"]["ms_per_step_graph"] / bx[f"union_{dt}"]["ms_per_step_graph"])
        extras["batched_64_meshes"] = bx

    ablations = None if args.no_ablations else run_ablations(torch, mesh, S, args, useful, E)
    sweep = None if args.no_sweep else run_sweep(torch, args, U)

    # ---- CPU baseline: the oracle's sequential loop on the host
    cpu = None
    if args.cpu_seconds > 0:
        from oracle import native
        native.lib()
        budget = args.cpu_seconds / 2

        def timed_sweeps(fn):
            t0, n = time.perf_counter(), 0
            while True:
                fn()
                n += 1
                el = time.perf_counter() - t0
                if el >= budget and n >= 2:
                    return n, el
        sweeps, el = timed_sweeps(lambda: native.edge_loop(mesh.e2n, mesh.e2c, mesh.x, mesh.q,
                                                            mesh.adt))
        nproc = os.cpu_count()
        model = cpu_model()
        cpu = {"value": E * sweeps / el, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"{sweeps} full sequential sweeps of the same {nx}x{ny} mesh "
                         f"({E} edges) in user numbering, {el:.1f}s on 1 host core",
               "nproc": nproc, "cpu_model": model}
        log(f"cpu oracle (1 core): {cpu['value']:.3g} edges/s")
        groups = native.colour_groups(mesh.e2c)
        threads = native.omp_threads()
        sweeps2, el2 = timed_sweeps(lambda: native.edge_loop_coloured(
            groups, mesh.e2n, mesh.e2c, mesh.x, mesh.q, mesh.adt))
        cpu["all_cores"] = {
            "value": E * sweeps2 / el2, "unit": "edges/s", "cores": threads,
            "kind": "oracle, colour-parallel",
            "sample": f"{sweeps2} full sweeps of the same mesh, {groups[0]} global edge colours, "
                      f"one OpenMP parallel loop per colour on {threads} threads, {el2:.1f}s"}
        log(f"cpu oracle ({threads} threads): {cpu['all_cores']['value']:.3g} edges/s")

    out = {
        "metric": METRIC,
        "value": E / sec,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D quad edge-flux loop (central Euler flux + scalar Lax-Friedrichs "
                        f"dissipation), {nx}x{ny} cells, jitter 0.2h, seed 1, FP64",
            "cells": C, "nodes": N, "edges": E,
            "strategy": "hierarchical two-layer colouring",
            "order": "rcm+partition+point-reorder",
            "point_order": {1: "block signature", 2: "smallest block first",
                            3: "blocks from the largest down"}[args.point_order],
            "block_size": S, "layout": args.layout, "staging": args.staging,
            "tcmode": args.tcmode, "schedule": args.schedule, "block_colouring": args.bcol,
            "edges_per_lane": args.ept,
            "gather": args.gather if args.schedule == "dataflow" else "registers",
            "parallelism": "none (one GPU)",
        },
        "useful_gbps": useful / sec / 1e9,
        "useful_bytes_per_step": useful,
        "pct_hbm_peak_step": 100 * useful / sec / 1e9 / measure.HBM_PEAK_GBPS,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": measure.HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": frac, "traffic": traffic,
                     "kernel": ("hier_kernel" if args.schedule != "dataflow" else
                                "hier_dma_kernel" if args.gather == "lds_dma" else
                                "hier_flow_kernel"),
                     "launches_per_step": launches_per_step,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "avg_launch_us_event_pairs": kern_ms / n_launch * 1e3,
                     "bytes_per_launch": bytes_per_launch},
        "roofline_cold": {"bound": "hbm", "achieved": cold_achieved,
                          "peak": measure.HBM_PEAK_GBPS, "unit": "GB/s", "frac": cold_frac,
                          "us_per_step": cold_s * 1e6,
                          "how": "1 GiB fill before every sweep, events around the sweep only"},
        "cpu_baseline": cpu,
        "baselines": baselines,
        "variants": variants,
        "extras": extras,
        "ablations": ablations,
        "sweep_1200x600": sweep,
        "plan": {k: st[k] for k in ("n_blocks", "n_block_colours", "max_thread_colours",
                                     "avg_thread_colours", "reuse_factor", "lds_bytes_max",
                                     "staged_points", "plan_device_bytes", "build_seconds")},
        "reorder_seconds": reorder_s,
        "device_copy_gbps": copy_gbps,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
