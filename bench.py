#!/usr/bin/env python3
"""Benchmark of closest-hit ray intersection with Catmull-Clark patch scenes.

Workload (default): 1,000,000 patches (2000 seeded displaced tori / apple tori,
25 % Gregory, leaf depth 10), 1920x1080 pinhole primary rays plus one secondary
ray per pixel (cosine-weighted bounce from seeded surface points).  Synthetic,
seeded, generated on the host and resident in HBM before timing starts.

Patches are subdivided in their local frames (Sec. 3.4; --world-frames for world
coordinates).  A step is one pass over all primary and all secondary rays.
Variants: "plain" (one launch per ray class, default launch parameters),
"batched" (both classes as two batches of one launch, autotuned), the same in
world coordinates, and "learned_batched" (learned child order); `value` is the
fastest batched variant that passes the oracle gate.  W warm-up steps,
then K steps timed with HIP events recorded on the stream the kernels run on.
Prints one JSON line.  The CPU baseline times the FP64 oracle on a bounded seeded
sample of the same rays on the host cores and reports the parity of that sample.
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
sys.path.insert(0, ROOT)

METRIC = "MRays/s primary+diffuse at 1M patches: plain vs learned-order batched, oracle-exact"

# Algorithmic 32-bit VALU operations per counted unit of work: the fewest gfx950
# vector operations the arithmetic needs (add, sub, mul, fma, 2- or 3-operand
# min/max, compare, select, bit op, and the midpoint (a+b)/2 as one add with the
# /2 output modifier: 1 each; a division: 1).  Derived from the method's
# arithmetic, not from the compiled code; each entry below names its parts.
OPS_PER_UNIT = {
    "ray": 25,         # ray setup (validity, reciprocals) and the hit write
    "node": 58,        # BVH node: two slab tests (25 each), ordering, stack push
    "cand": 12,        # candidate patch: anchored origin
    "split": 276,      # Alg. 3 step: 72 midpoints, two boxes (96), two slab tests (50), choice (22), 36 selects
    "backtrack": 6,    # count-trailing-zeros, path and trail update
    "greg": 622,       # Alg. 2 on a domain: extreme blends, displacement, crop of the lower grid
    "leaf": 30,        # leaf record: compare, (u, v) from the path code
    "crop": 502,       # Bezier grid recompute after backtracking (crop to the domain)
}
# Smallest seeded sample, per ray class, on which a variant's hits are gated against the oracle.
MIN_GATE_RAYS = 131072
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # CUs x SIMDs x lanes x clock: 39.32 T lane-op/s
COUNTERS = ("node", "cand", "split", "backtrack", "greg", "leaf", "crop", "cand_greg")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# What the intersection kernel's machine code is built from: its source, the headers
# it includes, and the build script that holds its compiler flags.
KERNEL_SOURCES = ("paper_1811_03510_amd/csrc/trace.hip", "paper_1811_03510_amd/csrc/patch_math.h",
                  "paper_1811_03510_amd/csrc/ccs_internal.h", "paper_1811_03510_amd/csrc/policy.h",
                  "paper_1811_03510_amd/csrc/ray_valid.h", "include/ccs.h", "paper_1811_03510_amd/build.py")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_ops(cnt: np.ndarray) -> float:
    tot = cnt.astype(np.float64).sum(axis=0)
    ops = OPS_PER_UNIT["ray"] * cnt.shape[0]
    for k, name in enumerate(COUNTERS):
        ops += OPS_PER_UNIT.get(name, 0) * tot[k]
    return float(ops)


def roofline_record(ops_per_launch: float, launch_ms: float, kernel: str) -> dict:
    """VALU roofline of one intersection launch: algorithmic lane-ops per launch over
    the launch's measured duration, against 256 CUs x 64 lanes x 2.4 GHz."""
    achieved = ops_per_launch / (launch_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / PEAK_VALU_TOPS, 4), "traffic": None, "kernel": kernel,
            "kernel_avg_ms": round(launch_ms, 4), "ops_per_launch": ops_per_launch}


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch of `kernel` measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE),
    scaled by the copy-kernel calibration, when recorded for the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "intersect_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_hash") != source_hash() or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def _counter_means(csv_dir: str, counter: str) -> dict:
    """Mean value of `counter` per kernel name over the dispatches in a rocprofv3
    --pmc CSV folder, and the largest single reading per kernel name."""
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), max(v)) for k, v in vals.items()}


def write_traffic_record(fetch_dir: str, write_dir: str, calib_mib: int) -> dict:
    """profiles/intersect_traffic.json from a FETCH_SIZE and a WRITE_SIZE pass of
    `bench.py --only batched ... --copy-calibration calib_mib`: the intersection
    kernel's mean readings (KiB per dispatch), each scaled by known bytes over what
    the same counter reads for the calibration's copy (FETCH) and fill (WRITE)."""
    fetch, write = _counter_means(fetch_dir, "FETCH_SIZE"), _counter_means(write_dir, "WRITE_SIZE")
    kib = calib_mib * 1024.0

    def pick(d, key):
        hits = [v for k, v in d.items() if key in k]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel matching {key!r}, found {sorted(d)}")
        return hits[0]
    k_fetch, k_write = pick(fetch, "k_trace<false, false>")[0], pick(write, "k_trace<false, false>")[0]
    fetch_scale = kib / pick(fetch, "copyBuffer")[1]
    write_scale = kib / pick(write, "elementwise")[1]
    rec = {"source_hash": source_hash(), "kernel": "k_trace<false, false>",
           "workload": "instanced1m batched, patch-local frames (2073600 + 2073600 rays)",
           "fetch_kib": round(k_fetch, 1), "write_kib": round(k_write, 1),
           "fetch_scale": round(fetch_scale, 3), "write_scale": round(write_scale, 3),
           "bytes_per_launch": int(round((k_fetch * fetch_scale + k_write * write_scale) * 1024))}
    with open(os.path.join(ROOT, "profiles", "intersect_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["instanced1m", "torus512", "anim512", "combined8m"],
                    default="instanced1m",
                    help="anim512: the 512-patch torus animated over 16 frames, every frame refit and all "
                         "frames' uneven ray batches in one launch, the frame loop replayed as a HIP graph; "
                         "combined8m: 8M patches, 8 animation frames, 3840x2160 primary rays and 3 diffuse "
                         "bounces generated from the hits, closest-first and learned order")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-counters", action="store_true", help="skip the counted launch (roofline)")
    ap.add_argument("--launch", default="",
                    help="waves_per_cu,fetch_min,traverse_min,grid_min,traverse_steps (default: library's)")
    ap.add_argument("--only", choices=["", "plain", "batched", "learned", "single"], default="",
                    help="time one variant only (a profiler run then sees one launch shape)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batched variant with the given/default launch instead of the tuned one")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--world-frames", action="store_true",
                    help="subdivide in world coordinates instead of patch-local frames (Sec. 3.4)")
    ap.add_argument("--policy-rays", type=int, default=12 << 20,
                    help="secondary rays on the 512-patch torus whose records train the ordering network "
                         "(12 x 2^20 rays give about 10M labelled records)")
    ap.add_argument("--policy-steps", type=int, default=4000, help="Adam steps of the ordering network")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized device buffer once (a plain copy kernel of known size that "
                         "scales the profiler's FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no benchmark: write profiles/intersect_traffic.json from the rocprofv3 CSV folders of a "
                         "FETCH_SIZE and a WRITE_SIZE pass run with --copy-calibration (its MIB is required)")
    args = ap.parse_args()
    if args.write_traffic:
        if not args.copy_calibration:
            raise SystemExit("--write-traffic needs the --copy-calibration MIB the passes ran with")
        print(json.dumps(write_traffic_record(*args.write_traffic, args.copy_calibration)))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: every ray is independent, so N GPUs "
                                   "would each run this same benchmark on 1/N of the rays; use --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_1811_03510_amd import ccs, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del src, dst
    if args.workload == "anim512":
        return bench_animation(args, torch, ccs, scenes)
    if args.workload == "combined8m":
        return bench_combined(args, torch, ccs, scenes)
    t0 = time.time()
    w = scenes.config2() if args.workload == "instanced1m" else scenes.config1()
    gen_s = time.time() - t0
    log(f"workload {w.name}: {w.cp.shape[0]} patches, {len(w.primary)} + {len(w.diffuse)} rays "
        f"(generated in {gen_s:.1f} s)")
    t0 = time.time()
    scene = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth,
                      local_frames=not args.world_frames)
    torch.cuda.synchronize()
    create_s = time.time() - t0
    if args.launch:
        scene.set_launch(*[int(x) for x in args.launch.split(",")])
    launch = scene.get_launch()
    info = scene.info()
    log(f"scene: {info['n_nodes']} nodes, BVH depth {info['bvh_depth']}, {info['device_bytes'] / 2**20:.1f} MiB, "
        f"create {create_s:.2f} s (host BVH {info['build_seconds']:.2f} s)")

    prim = torch.from_numpy(w.primary).cuda()
    diff = torch.from_numpy(w.diffuse).cuda()
    n_p, n_d = prim.shape[0], diff.shape[0]
    hp = torch.empty((n_p, 4), dtype=torch.float32, device="cuda")
    hd = torch.empty((n_d, 4), dtype=torch.float32, device="cuda")
    hbp, hbd = torch.empty_like(hp), torch.empty_like(hd)
    stream = torch.cuda.current_stream()
    batches = [(0, prim, hbp), (0, diff, hbd)]

    def plain_step(evs=None):
        if evs:
            evs[0].record(stream)
        scene.intersect(prim, hp)
        if evs:
            evs[1].record(stream)
        scene.intersect(diff, hd)
        if evs:
            evs[2].record(stream)

    def batched_step(evs=None):
        if evs:
            evs[0].record(stream)
        scene.intersect_batched(batches)
        if evs:
            evs[1].record(stream)

    def timed(step, n_events):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(n_events)] for _ in range(args.steps)]
        for k in range(args.steps):
            step(events[k])
        torch.cuda.synchronize()
        laps = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(n_events - 1)] for e in events])
        return laps, events[0][0].elapsed_time(events[-1][-1]) / args.steps

    def cls(n, t, hits):
        return {"rays": n, "ms_median": float(np.median(t)), "ms_p10": float(np.percentile(t, 10)),
                "ms_p90": float(np.percentile(t, 90)), "mrays_per_s": n / np.median(t) / 1e3,
                "hit_fraction": float((ccs.hit_ids(hits) != ccs.NO_HIT).mean())}

    variants = {}
    if args.only in ("", "plain"):
        laps, ms = timed(plain_step, 3)
        tp, td = laps[:, 0], laps[:, 1]
        hits_p, hits_d = hp.cpu().numpy(), hd.cpu().numpy()
        variants["plain"] = {
            "ms_per_step": ms, "mrays_per_s": (n_p + n_d) / (ms * 1e-3) / 1e6, "launch": dict(launch),
            "launches_per_step": 2, "kernel_ms": float(np.mean(laps)),
            "per_class": {"primary": cls(n_p, tp, hits_p), "diffuse": cls(n_d, td, hits_d)}}
        log(f"plain: {ms:.3f} ms/step, primary {np.median(tp):.3f} ms, secondary {np.median(td):.3f} ms "
            f"-> {variants['plain']['mrays_per_s']:.1f} MRays/s")
    if args.only in ("", "batched"):
        if args.autotune:
            from paper_1811_03510_amd import autotune
            t0 = time.time()
            tuned = autotune.tuned(scene, batches, name=w.name, log=log if args.verbose else None)
            log(f"autotuned launch {tuned} in {time.time() - t0:.1f} s")
        laps, ms = timed(batched_step, 2)
        hits_p, hits_d = hbp.cpu().numpy(), hbd.cpu().numpy()
        variants["batched"] = {
            "ms_per_step": ms, "mrays_per_s": (n_p + n_d) / (ms * 1e-3) / 1e6, "launch": scene.get_launch(),
            "launches_per_step": 1, "kernel_ms": float(np.mean(laps)), "autotuned": bool(args.autotune),
            "ms_median": float(np.median(laps)), "ms_p10": float(np.percentile(laps, 10)),
            "ms_p90": float(np.percentile(laps, 90))}
        if "plain" in variants:
            variants["batched"]["bitwise_equal_to_plain"] = bool(
                np.array_equal(hits_p.view(np.uint32), hp.cpu().numpy().view(np.uint32))
                and np.array_equal(hits_d.view(np.uint32), hd.cpu().numpy().view(np.uint32)))
        log(f"batched: {ms:.3f} ms/step -> {variants['batched']['mrays_per_s']:.1f} MRays/s "
            f"(launch {variants['batched']['launch']})")
    world_hits = None
    if args.only == "" and not args.world_frames:
        # the same launch with subdivision in world coordinates, for the Sec. 3.4 comparison
        wsc = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth)
        wsc.set_launch(**{k: v for k, v in scene.get_launch().items() if k != "waves_per_cu"})
        wh = [torch.empty_like(hp), torch.empty_like(hd)]
        wb = [(0, prim, wh[0]), (0, diff, wh[1])]

        def world_step(evs=None):
            if evs:
                evs[0].record(stream)
            wsc.intersect_batched(wb)
            if evs:
                evs[1].record(stream)

        laps, ms = timed(world_step, 2)
        world_hits = (wh[0].cpu().numpy(), wh[1].cpu().numpy())
        variants["batched_world_frames"] = {
            "ms_per_step": ms, "mrays_per_s": (n_p + n_d) / (ms * 1e-3) / 1e6, "launches_per_step": 1,
            "kernel_ms": float(np.mean(laps)), "note": "closest-first, both classes in one launch, world frame"}
        log(f"batched, world frame: {ms:.3f} ms/step -> {variants['batched_world_frames']['mrays_per_s']:.1f} MRays/s")
        del wsc, wh, wb
    single_hits = None
    if args.only in ("", "single"):
        # the ablation of Sec. 3.3's two-box test: each step tests only the current
        # domain's box (same launch parameters as the batched variant)
        ssc = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth,
                        local_frames=not args.world_frames, single_box=True)
        ssc.set_launch(**{k: v for k, v in scene.get_launch().items() if k != "waves_per_cu"})
        sh = [torch.empty_like(hp), torch.empty_like(hd)]
        sb = [(0, prim, sh[0]), (0, diff, sh[1])]

        def single_step(evs=None):
            if evs:
                evs[0].record(stream)
            ssc.intersect_batched(sb)
            if evs:
                evs[1].record(stream)

        laps, ms = timed(single_step, 2)
        single_hits = (sh[0].cpu().numpy(), sh[1].cpu().numpy())
        v = {"ms_per_step": ms, "mrays_per_s": (n_p + n_d) / (ms * 1e-3) / 1e6, "launches_per_step": 1,
             "kernel_ms": float(np.mean(laps)),
             "note": "ablation (Sec. 3.3): each step tests only the current domain's box; closest-first "
                     "variant's launch parameters, both classes in one launch"}
        if not args.no_counters:
            _, sc_p = ssc.intersect_counted(prim)
            _, sc_d = ssc.intersect_counted(diff)
            sc_p, sc_d = sc_p.cpu().numpy(), sc_d.cpu().numpy()
            v["work_per_ray"] = {c: {"primary": float(sc_p[:, k].mean()), "diffuse": float(sc_d[:, k].mean())}
                                 for k, c in enumerate(COUNTERS)}
        variants["batched_single_box"] = v
        log(f"batched, single box per step: {ms:.3f} ms/step -> {v['mrays_per_s']:.1f} MRays/s")
        del ssc, sh, sb
    bounce = None
    if args.only == "":
        # secondary rays as the 1M configuration states them: one cosine bounce per primary
        # hit, generated on the GPU from that launch's hits (seeded uniforms); rays of
        # missed pixels are inactive and are not counted
        u = torch.from_numpy(scenes.uniform(scenes.substream(scenes.STREAM_BOUNCE, 7), 2 * n_p)
                             .astype(np.float32)).cuda()
        hit_rows = (hbp[:, 0] < float("inf")).nonzero().squeeze(1)
        brays = scene.bounce(prim[hit_rows].contiguous(), hbp[hit_rows].contiguous(), u[:2 * hit_rows.numel()]
                             .reshape(-1, 2).contiguous())
        bh = torch.empty((brays.shape[0], 4), dtype=torch.float32, device="cuda")
        hp2 = torch.empty_like(hp)
        bb = [(0, prim, hp2), (0, brays, bh)]

        def bounce_step(evs=None):
            if evs:
                evs[0].record(stream)
            scene.intersect_batched(bb)
            if evs:
                evs[1].record(stream)

        laps, ms = timed(bounce_step, 2)
        nb = brays.shape[0]
        bh_only = torch.empty_like(bh)

        def bounce_only_step(evs=None):
            if evs:
                evs[0].record(stream)
            scene.intersect(brays, bh_only)
            if evs:
                evs[1].record(stream)

        laps_b, _ = timed(bounce_only_step, 2)
        variants["batched_bounce"] = {
            "ms_per_step": ms, "mrays_per_s": (n_p + nb) / (ms * 1e-3) / 1e6, "launches_per_step": 1,
            "kernel_ms": float(np.mean(laps)), "rays": {"primary": n_p, "bounce": nb},
            "bounce_hit_fraction": float((bh[:, 0] < float("inf")).float().mean().item()) if nb else 0.0,
            "per_class": {"bounce": cls(nb, laps_b[:, 0], bh_only.cpu().numpy())},
            "note": "closest-first; the configuration's own secondary rays: one cosine bounce per primary hit "
                    "(ccs_bounce on the GPU's hits), primary and bounce rays in one launch; per_class.bounce "
                    "times the bounce rays alone in a launch of their own"}
        bounce = (brays.cpu().numpy(), bh.cpu().numpy(), hp2.cpu().numpy())
        log(f"batched with real bounces ({nb} bounce rays): {ms:.3f} ms/step -> "
            f"{variants['batched_bounce']['mrays_per_s']:.1f} MRays/s; bounce rays alone "
            f"{variants['batched_bounce']['per_class']['bounce']['mrays_per_s']:.1f} MRays/s")
    learned_hits = None
    if args.only in ("", "learned"):
        policy, pstats = train_policy(args, torch, ccs, scenes)
        scene.set_policy(policy)
        hlp, hld = torch.empty_like(hp), torch.empty_like(hd)
        lbatches = [(0, prim, hlp), (0, diff, hld)]

        def learned_step(evs=None):
            if evs:
                evs[0].record(stream)
            scene.intersect_batched(lbatches)
            if evs:
                evs[1].record(stream)

        if args.autotune:
            from paper_1811_03510_amd import autotune
            tuned = autotune.tuned(scene, lbatches, name=w.name, learned=True, log=log if args.verbose else None)
            log(f"autotuned learned launch {tuned}")
        laps, ms = timed(learned_step, 2)
        learned_hits = (hlp.cpu().numpy(), hld.cpu().numpy())
        v = {"ms_per_step": ms, "mrays_per_s": (n_p + n_d) / (ms * 1e-3) / 1e6, "launch": scene.get_launch(),
             "launches_per_step": 1, "kernel_ms": float(np.mean(laps)), "autotuned": bool(args.autotune),
             "ms_median": float(np.median(laps)), "policy": pstats}
        if "batched" in variants:
            v["identical_to_closest_first"] = {
                "primary": float(np.mean(np.all(learned_hits[0].view(np.uint32) == hits_p.view(np.uint32), axis=1))),
                "diffuse": float(np.mean(np.all(learned_hits[1].view(np.uint32) == hits_d.view(np.uint32), axis=1)))}
        if not args.no_counters:
            _, lc_p = scene.intersect_counted(prim)
            _, lc_d = scene.intersect_counted(diff)
            lc_p, lc_d = lc_p.cpu().numpy(), lc_d.cpu().numpy()
            v["work_per_ray"] = {c: {"primary": float(lc_p[:, k].mean()), "diffuse": float(lc_d[:, k].mean())}
                                 for k, c in enumerate(COUNTERS)}
        scene.set_policy(None)
        variants["learned_batched"] = v
        log(f"learned batched: {ms:.3f} ms/step -> {v['mrays_per_s']:.1f} MRays/s; {pstats}")
    # ------------------------------------------------------------ oracle gate
    # Every timed variant's hits are gated against the FP64 oracle on seeded samples
    # (closest-first: the batched launch's hits, bit-identical to the plain launches';
    # world frames: against the world-frame oracle; bounce: the configuration's own
    # secondary rays; learned order).  A variant that fails reports no MRays/s, and
    # any failure withholds the headline value and ends the run with status 1.
    cpu = None
    parity = None
    gates = {}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.parity import gate
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        threads = min(threads, os.cpu_count() or threads)
        t0 = time.time()
        osc = oracle.Scene(w.cp, w.types, w.leaf_depth, local_frames=not args.world_frames)
        obuild = time.time() - t0
        calib = scenes.sample_indices(n_p, 1024, seed=91)
        t0 = time.time()
        osc.intersect(w.primary[calib], nthreads=threads)
        osc.intersect(w.diffuse[calib], nthreads=threads)
        per_ray = (time.time() - t0) / (2 * len(calib))
        k = int(min(max(MIN_GATE_RAYS, args.cpu_seconds / max(per_ray, 1e-9) / 2), n_p, n_d))
        sel_p = scenes.sample_indices(n_p, k, seed=92)
        sel_d = scenes.sample_indices(n_d, k, seed=93)
        t0 = time.time()
        op = osc.intersect(w.primary[sel_p], nthreads=threads)
        od = osc.intersect(w.diffuse[sel_d], nthreads=threads)
        osec = time.time() - t0
        cpu = {"value": round(2 * k / osec / 1e6, 4), "unit": "MRays/s", "cores": threads, "kind": "oracle",
               "per_core": round(2 * k / osec / 1e6 / threads, 5), "cpu_model": cpu_model(),
               "sample": (f"all {n_p} primary + {n_d} secondary rays of the workload" if k >= max(n_p, n_d) else
                          f"{k} primary + {k} secondary rays (seeded subset of the same {n_p}+{n_d} rays)")
                         + f", {osec:.1f} s; oracle BVH build {obuild:.1f} s excluded"}

        def summary(r):
            return {"rays": r["n"], "same_hit_and_patch": r["id_rate"], "strict": r["match_rate"],
                    "excused": r["excused"], "ok": r["ok"], "hard_examples": r["hard"][:3]}

        if "batched" in variants or "plain" in variants:
            # the closest-first hits (the batched launch's when it ran: bit-identical to the
            # plain launches', which bench reports as bitwise_equal_to_plain)
            cf_hits = (hits_p, hits_d)
            rp = gate(cf_hits[0][sel_p], op, w.primary[sel_p], osc, w.diameter, w.leaf_depth, label="primary")
            rd = gate(cf_hits[1][sel_d], od, w.diffuse[sel_d], osc, w.diameter, w.leaf_depth, label="diffuse")
            parity = {"primary": summary(rp), "diffuse": summary(rd)}
            ok_cf = rp["ok"] and rd["ok"]
            if "batched" in variants:
                gates["batched"] = ok_cf
            if "plain" in variants:  # gated directly, or through its bitwise equality with the batched hits
                gates["plain"] = ok_cf and variants.get("batched", {}).get("bitwise_equal_to_plain", True)
        if bounce is not None:
            sel_b = scenes.sample_indices(len(bounce[0]), min(len(bounce[0]), MIN_GATE_RAYS), seed=94)
            ob = osc.intersect(bounce[0][sel_b], nthreads=threads)
            rb = gate(bounce[1][sel_b], ob, bounce[0][sel_b], osc, w.diameter, w.leaf_depth, label="bounce")
            stride = max(1, len(sel_p) // MIN_GATE_RAYS)  # a spread subset of the primary sample
            sel_bp = sel_p[::stride]
            rbp = gate(bounce[2][sel_bp], {kk: vv[::stride] for kk, vv in op.items()}, w.primary[sel_bp], osc,
                       w.diameter, w.leaf_depth, label="bounce-launch primary")
            variants["batched_bounce"]["parity_sample"] = {"bounce": summary(rb), "primary": summary(rbp)}
            gates["batched_bounce"] = rb["ok"] and rbp["ok"]
        if single_hits is not None:
            # against the oracle's own single-box mode (a Gregory leaf tested by its own bound)
            ss_p = scenes.sample_indices(n_p, min(n_p, 65536), seed=97)
            ss_d = scenes.sample_indices(n_d, min(n_d, 65536), seed=98)
            osp = osc.intersect_single_box(w.primary[ss_p], nthreads=threads)
            osd = osc.intersect_single_box(w.diffuse[ss_d], nthreads=threads)
            sp_ = gate(single_hits[0][ss_p], osp, w.primary[ss_p], osc, w.diameter, w.leaf_depth, label="1box-primary")
            sd_ = gate(single_hits[1][ss_d], osd, w.diffuse[ss_d], osc, w.diameter, w.leaf_depth, label="1box-diffuse")
            variants["batched_single_box"]["parity_sample"] = {"primary": summary(sp_), "diffuse": summary(sd_)}
            gates["batched_single_box"] = sp_["ok"] and sd_["ok"]
        if learned_hits is not None:
            lp_ = gate(learned_hits[0][sel_p], op, w.primary[sel_p], osc, w.diameter, w.leaf_depth, label="l-primary")
            ld_ = gate(learned_hits[1][sel_d], od, w.diffuse[sel_d], osc, w.diameter, w.leaf_depth, label="l-diffuse")
            variants["learned_batched"]["parity_sample"] = {"primary": summary(lp_), "diffuse": summary(ld_)}
            gates["learned_batched"] = lp_["ok"] and ld_["ok"]
        del osc
        if world_hits is not None:
            osw = oracle.Scene(w.cp, w.types, w.leaf_depth, local_frames=False)
            sw_p = scenes.sample_indices(n_p, MIN_GATE_RAYS, seed=95)
            sw_d = scenes.sample_indices(n_d, MIN_GATE_RAYS, seed=96)
            ow_p = osw.intersect(w.primary[sw_p], nthreads=threads)
            ow_d = osw.intersect(w.diffuse[sw_d], nthreads=threads)
            rwp = gate(world_hits[0][sw_p], ow_p, w.primary[sw_p], osw, w.diameter, w.leaf_depth,
                       label="world primary")
            rwd = gate(world_hits[1][sw_d], ow_d, w.diffuse[sw_d], osw, w.diameter, w.leaf_depth,
                       label="world diffuse")
            variants["batched_world_frames"]["parity_sample"] = {"primary": summary(rwp), "diffuse": summary(rwd)}
            gates["batched_world_frames"] = rwp["ok"] and rwd["ok"]
            del osw
        log(f"cpu baseline: {cpu['value']} MRays/s on {threads} threads; gates {gates}; parity {parity}")
        for v, ok in gates.items():
            variants[v]["gate_ok"] = ok
            if not ok:
                variants[v]["mrays_per_s"] = None
                print(f"bench: PARITY FAILED for variant {v}", file=sys.stderr, flush=True)

    # headline: the faster of closest-first and learned order among the variants that
    # passed the gate; without the oracle only closest-first is reported
    cands = [v for v in ("batched", "plain") if v in variants][:1]
    if "learned_batched" in variants and gates.get("learned_batched"):
        cands.append("learned_batched")
    cands = [v for v in cands if variants[v]["mrays_per_s"] is not None]
    head = max(cands, key=lambda v: variants[v]["mrays_per_s"]) if cands else None
    failed = [v for v, ok in gates.items() if not ok]
    value = None if (failed or head is None) else variants[head]["mrays_per_s"]
    ms_step = variants[head]["ms_per_step"] if head else None

    roofline = None
    work = None
    if not args.no_counters and head is not None:
        if head == "learned_batched":
            scene.set_policy(policy)
        _, cp_ = scene.intersect_counted(prim)
        _, cd_ = scene.intersect_counted(diff)
        torch.cuda.synchronize()
        scene.set_policy(None)
        cp_, cd_ = cp_.cpu().numpy(), cd_.cpu().numpy()
        ops_p, ops_d = algorithmic_ops(cp_), algorithmic_ops(cd_)
        per_launch = variants[head]["launches_per_step"]
        launch_ms = variants[head]["kernel_ms"]
        ops_launch = (ops_p + ops_d) / per_launch
        achieved = ops_launch / (launch_ms * 1e-3) / 1e12
        kname = "k_trace<false, true>" if head == "learned_batched" else "k_trace<false, false>"
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 2),
                    "unit": "TOP/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                    "traffic": traffic_from_profiles(kname),
                    "kernel": kname, "kernel_avg_ms": round(launch_ms, 4),
                    "ops_per_launch": ops_launch,
                    "ops_per_ray": {"primary": ops_p / n_p, "diffuse": ops_d / n_d}}
        work = {c: {"primary": float(cp_[:, k].mean()), "diffuse": float(cd_[:, k].mean())}
                for k, c in enumerate(COUNTERS)}

    out = {
        "metric": METRIC,
        "value": None if value is None else round(value, 3),
        "unit": "MRays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None if ms_step is None else round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": (f"{w.name}: {w.cp.shape[0]} patches "
                                f"({int(w.types.sum())} Gregory), {n_p} primary + {n_d} secondary rays per step"),
                   "variant": {None: "none passed the oracle gate",
                               "plain": "closest-first order, one launch per ray class",
                               "batched": "closest-first order, both ray classes in one autotuned launch",
                               "learned_batched": "learned child order, both ray classes in one autotuned launch"
                               }[head],
                   "launch": variants[head]["launch"] if head else None,
                   "frames": "world" if args.world_frames else "patch-local (Sec. 3.4)",
                   "leaf_depth": w.leaf_depth,
                   "secondary_rays": "stand-in: one cosine-weighted ray per pixel from a seeded surface point; "
                                     "variants.batched_bounce has the configuration's own bounce per primary hit"},
        "variants": variants,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "parity_ok": None if not gates else not failed,
        "gate_failed": failed,
        "work_per_ray": work,
        "scene": {"create_s": round(create_s, 3), "bvh_build_s": round(info["build_seconds"], 3),
                  "bvh_depth": info["bvh_depth"], "device_mib": round(info["device_bytes"] / 2**20, 1)},
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)
    if failed:
        sys.exit(1)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def train_policy(args, torch, ccs, scenes):
    """Ordering network trained on records of secondary rays of the 512-patch torus
    (GPU: record, Adam in bfloat16); returns (params on the GPU, statistics)."""
    t0 = time.time()
    c1 = scenes.config1()
    rays = scenes.policy_training_rays(args.policy_rays)
    gen_s = time.time() - t0
    g1 = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                   local_frames=not args.world_frames)

    def records(r_np):
        # in chunks of 2^20 rays: a ray gives L rows before the unlabelled ones are dropped
        fs, ys = [], []
        for b in range(0, len(r_np), 1 << 20):
            r = torch.from_numpy(r_np[b:b + (1 << 20)]).cuda()
            f, y = g1.record(r, g1.intersect(r))
            keep = (y != ccs.NO_LABEL).nonzero().squeeze(1)
            fs.append(f[keep].contiguous())
            ys.append(y[keep].contiguous())
            del f, y, r
        return torch.cat(fs), torch.cat(ys)

    f, y = records(rays)
    th = torch.from_numpy(scenes.mlp_init()).cuda()
    torch.cuda.synchronize()
    t1 = time.time()
    hist = ccs.policy_train(th, f, y, steps=args.policy_steps, batch=8192, lr=3e-3, seed=1, bf16=True)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    fe, ye = records(c1.diffuse)  # held out: the torus workload's own secondary rays
    z = ccs.policy_infer(th, fe).cpu().numpy()
    ye, fe12 = ye.cpu().numpy(), fe[:, 12].cpu().numpy()
    hist = hist.cpu().numpy()
    return th, {"train_rays": len(rays), "records": int(f.shape[0]), "steps": args.policy_steps, "batch": 8192,
                "train_s": round(train_s, 3), "ray_gen_s": round(gen_s, 2),
                "loss_first": float(hist[:20].mean()), "loss_last": float(hist[-100:].mean()),
                "heldout_records": int(len(ye)),
                "u_half_accuracy": {"closest_first": float(((fe12 > 0).astype(int) == (ye >> 1)).mean()),
                                    "learned": float(((np.argmax(z, axis=1) >> 1) == (ye >> 1)).mean())},
                "grandchild_accuracy": float((np.argmax(z, axis=1) == ye).mean())}


def bench_animation(args, torch, ccs, scenes):
    """Batched animation playback: per step, refit all frames and intersect every
    frame's rays in one launch; the step is captured once as a HIP graph and replayed."""
    from paper_1811_03510_amd import autotune
    t0 = time.time()
    a = scenes.config3()
    gen_s = time.time() - t0
    nf = len(a.frames)
    n_rays = sum(len(r) for r in a.rays)
    log(f"workload {a.name}: {a.cp0.shape[0]} patches, {nf} frames, {n_rays} rays "
        f"({[len(r) for r in a.rays]}), generated in {gen_s:.1f} s")
    scene = ccs.Scene(torch.from_numpy(a.cp0).cuda(), torch.from_numpy(a.types).cuda(), a.leaf_depth,
                      local_frames=not args.world_frames)
    scene.set_frames(nf)
    cps = [torch.from_numpy(c).cuda() for c in a.frames]
    rays = [torch.from_numpy(r).cuda() for r in a.rays]
    hits = [torch.empty((r.shape[0], 4), dtype=torch.float32, device="cuda") for r in rays]
    batches = [(f, rays[f], hits[f]) for f in range(nf)]

    def frame_loop():
        for f in range(nf):
            scene.refit_frame(f, cps[f])
        scene.intersect_batched(batches)

    frame_loop()
    torch.cuda.synchronize()
    tuned = autotune.tuned(scene, batches, name=a.name, log=log if args.verbose else None) if args.autotune else None
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        frame_loop()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        frame_loop()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        graph.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    laps = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    value = n_rays / (ms * 1e-3) / 1e6
    log(f"animation: {ms:.3f} ms per replay of {nf} refits + one launch -> {value:.1f} MRays/s")
    roofline = None
    if not args.no_counters:
        # the intersection launch of the replay, timed eagerly on the refit frames, and
        # its algorithmic work from the counting kernel on the same batches
        kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for e0, e1 in kev:
            e0.record()
            scene.intersect_batched(batches)
            e1.record()
        _, cnt = scene.intersect_batched(batches, counted=True)
        torch.cuda.synchronize()
        kms = float(np.median([e0.elapsed_time(e1) for e0, e1 in kev]))
        roofline = roofline_record(algorithmic_ops(cnt.cpu().numpy()), kms, "k_trace<false, false>")
        log(f"animation intersect launch {kms:.3f} ms, roofline {roofline['frac']}")

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.parity import gate
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        threads = min(threads, os.cpu_count() or threads)
        per_frame = 4096
        osec, ok, worst, nsamp = 0.0, True, 1.0, 0
        for f in range(nf):
            osc = oracle.Scene(a.frames[f], a.types, a.leaf_depth, local_frames=not args.world_frames)
            sel = scenes.sample_indices(len(a.rays[f]), min(per_frame, len(a.rays[f])), seed=200 + f)
            t0 = time.time()
            o = osc.intersect(a.rays[f][sel], nthreads=threads)
            osec += time.time() - t0
            nsamp += len(sel)
            r = gate(hits[f].cpu().numpy()[sel], o, a.rays[f][sel], osc, a.diameter, a.leaf_depth,
                     label=f"frame{f}")
            ok, worst = ok and r["ok"], min(worst, r["id_rate"])
        cpu = {"value": round(nsamp / osec / 1e6, 4), "unit": "MRays/s", "cores": threads, "kind": "oracle",
               "sample": f"{per_frame} seeded rays per frame of the {nf} frames (oracle BVH builds excluded)"}
        parity = {"frames": nf, "rays": nsamp, "ok": ok, "worst_frame_same_hit_and_patch": worst}
        log(f"cpu baseline {cpu['value']} MRays/s; parity {parity}")
    print(json.dumps({
        "metric": "MRays/s batched animation playback (refit + intersect per frame, HIP graph replay)",
        "value": round(value, 3), "unit": "MRays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded)",
        "config": {"workload": f"{a.name}: {a.cp0.shape[0]} patches, {nf} frames, {n_rays} rays "
                               f"(half primary, half secondary per frame)",
                   "frames": "world" if args.world_frames else "patch-local (Sec. 3.4)",
                   "launch": scene.get_launch(), "autotuned": tuned is not None, "leaf_depth": a.leaf_depth,
                   "ms_median": float(np.median(laps))},
        "roofline": roofline, "cpu_baseline": cpu, "parity_sample": parity, "source_hash": source_hash()}),
        flush=True)


def bench_combined(args, torch, ccs, scenes):
    """8M patches over 8 frames: per step every frame is refit, then one launch
    intersects the primary rays of all frames, and each of 3 bounce levels
    generates secondary rays from the previous level's hits (per frame), compacts
    them to the active ones (a bounce of a missed ray is inactive) and intersects
    those in one launch.  Closest-first and learned order are timed."""
    from paper_1811_03510_amd import autotune
    t0 = time.time()
    w = scenes.config5()
    log(f"workload {w.name}: {w.cp.shape[0]} patches ({int(w.types.sum())} Gregory), {len(w.primary)} primary "
        f"rays, {w.n_frames} frames, {w.bounces} bounces; generated in {time.time() - t0:.1f} s")
    t0 = time.time()
    scene = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth,
                      local_frames=not args.world_frames)
    scene.set_frames(w.n_frames)
    cps = []
    for f in range(w.n_frames):
        cps.append(torch.from_numpy(w.frame(f)).cuda())
        scene.refit_frame(f, cps[-1])
    torch.cuda.synchronize()
    info = scene.info()
    log(f"scene + frames ready in {time.time() - t0:.1f} s: BVH depth {info['bvh_depth']}, "
        f"{info['device_bytes'] / 2**30:.2f} GiB")
    F, B, n = w.n_frames, w.bounces, len(w.primary)
    prim = torch.from_numpy(w.primary).cuda()
    # level b > 0 of frame f: the bounce rays of level b - 1's active rays (bounced[f]), their
    # active ones compacted to rays[b][f][:m] with their indices (ccs_compact_rays), and hits
    rays = [[prim] * F] + [[torch.empty_like(prim) for _ in range(F)] for _ in range(B)]
    hits = [[torch.empty((n, 4), dtype=torch.float32, device="cuda") for _ in range(F)] for _ in range(B + 1)]
    bounced = [torch.empty_like(prim) for _ in range(F)]
    index = [[torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(F)] for _ in range(B)]
    work = [torch.empty(ccs.compact_work_words(n), dtype=torch.int32, device="cuda") for _ in range(F)]
    unif = [[torch.from_numpy(w.bounce_uniforms(f, b, n).reshape(n, 2)).cuda() for f in range(F)] for b in range(B)]
    ray_bytes = sum(t.numel() * 4 for lvl in rays[1:] for t in lvl) + prim.numel() * 4 + sum(
        t.numel() * 4 for t in bounced) + sum(t.numel() * 4 for lvl in index for t in lvl)
    hit_bytes = sum(t.numel() * 4 for lvl in hits for t in lvl)
    stream = torch.cuda.current_stream()
    counts = [[n] * F for _ in range(B + 1)]  # active rays per level and frame (the last step's)

    def batches(b):
        return [(f, rays[b][f][:counts[b][f]], hits[b][f][:counts[b][f]]) for f in range(F)]

    def step(evs=None):
        for f in range(F):
            scene.refit_frame(f, cps[f])
        for b in range(B + 1):
            if b > 0:
                for f in range(F):
                    m = counts[b - 1][f]
                    scene.bounce(rays[b - 1][f][:m], hits[b - 1][f][:m], unif[b - 1][f][:m], out=bounced[f][:m],
                                 frame=f)
                    ccs.compact_rays(bounced[f][:m], out=rays[b][f], index=index[b - 1][f], work=work[f])
                # the launch needs the level's sizes: one read of the F counts
                counts[b] = [int(c) for c in torch.stack([wk[0] for wk in work]).cpu()]
            if evs:
                evs[b].record(stream)
            scene.intersect_batched(batches(b))
            if evs:
                evs[b + 1 + B].record(stream)

    def run(label):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * B + 2)] for _ in range(args.steps)]
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for k in range(args.steps):
            step(evs[k])
        z.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(z) / args.steps
        lvl = [float(np.median([e[b].elapsed_time(e[b + 1 + B]) for e in evs])) for b in range(B + 1)]
        # rays traced: every primary ray, and the active bounce rays (those of pixels whose
        # previous ray hit; the compaction drops the others); the same every step
        live = [int(sum(c)) for c in counts]
        total = sum(live)
        active = [float((hits[b][0][:counts[b][0], 0] < float("inf")).float().mean().item()) for b in range(B + 1)]
        res = {"ms_per_step": ms, "mrays_per_s": total / (ms * 1e-3) / 1e6, "launch": scene.get_launch(),
               "rays_per_step": total, "rays_per_level": live,
               "bounce_rays_before_compaction_per_level": [0] + [int(sum(c)) for c in counts[:B]],
               "intersect_ms_per_level": lvl,
               "mrays_per_s_per_level": [k / (t * 1e-3) / 1e6 for k, t in zip(live, lvl)],
               "hit_fraction_frame0_per_level": active}
        log(f"{label}: {ms:.1f} ms/step -> {res['mrays_per_s']:.1f} MRays/s; levels {[round(t, 2) for t in lvl]} ms")
        return res

    def level_ops():
        """Algorithmic work of each level's launch (counting kernel, same batches as the
        last timed step)."""
        ops = []
        for b in range(B + 1):
            _, cnt = scene.intersect_batched(batches(b), counted=True)
            ops.append(algorithmic_ops(cnt.cpu().numpy()))
            del cnt
        return ops

    def with_roofline(res, kname):
        if not args.no_counters:
            ops = level_ops()
            tot_ms = sum(res["intersect_ms_per_level"])
            res["roofline"] = roofline_record(sum(ops) / (B + 1), tot_ms / (B + 1), kname)
            res["roofline"]["per_level_frac"] = [round(o / (t * 1e-3) / 1e12 / PEAK_VALU_TOPS, 4)
                                                 for o, t in zip(ops, res["intersect_ms_per_level"])]
        return res

    variants = {}
    b0 = [(f, rays[0][f], hits[0][f]) for f in range(F)]
    if args.autotune:
        autotune.tuned(scene, b0, name=w.name)
    gate_frames, per_level = (0, F - 1), 8192

    def take_samples():
        """Seeded samples of the traced rays of every level of the gated frames, with their
        hits (the last step's): rays and hits as host arrays."""
        out = {}
        for f in gate_frames:
            for b in range(B + 1):
                m = counts[b][f]
                k = torch.from_numpy(scenes.sample_indices(m, min(per_level, m), seed=700 + 10 * f + b)).cuda()
                out[(f, b)] = (rays[b][f][:m][k].cpu().numpy(), hits[b][f][:m][k].cpu().numpy())
        return out

    variants["batched"] = with_roofline(run("closest-first"), "k_trace<false, false>")
    gated = {"batched": take_samples()}
    if info["bvh_depth"] < 37:
        policy, pstats = train_policy(args, torch, ccs, scenes)
        scene.set_policy(policy)
        if args.autotune:
            autotune.tuned(scene, b0, name=w.name, learned=True)
        variants["learned_batched"] = with_roofline(run("learned order"), "k_trace<false, true>")
        variants["learned_batched"]["policy"] = pstats
        gated["learned_batched"] = take_samples()
        scene.set_policy(None)
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        import oracle
        from oracle.parity import gate
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        threads = min(threads, os.cpu_count() or threads)
        parity, osec, nsamp = {}, 0.0, 0
        for f in gate_frames:
            t0 = time.time()
            # the oracle's scene from the very arrays the frame was refit with
            osc = oracle.Scene(cps[f].cpu().numpy(), w.types, w.leaf_depth, local_frames=not args.world_frames)
            log(f"oracle scene of frame {f} in {time.time() - t0:.1f} s")
            for vname, smp in gated.items():
                for b in range(B + 1):
                    r, h = smp[(f, b)]
                    t0 = time.time()
                    o = osc.intersect(r, nthreads=threads)
                    if vname == "batched":
                        osec += time.time() - t0
                        nsamp += len(r)
                    g = gate(h, o, r, osc, w.diameter, w.leaf_depth, label=f"{vname}-frame{f}-level{b}")
                    parity[f"{vname}_frame{f}_level{b}"] = {
                        "rays": g["n"], "hits": g["hits"], "same_hit_and_patch": g["id_rate"],
                        "strict": g["match_rate"], "excused": g["excused"], "ok": g["ok"], "hard_examples": g["hard"][:3]}
            del osc
        cpu = {"value": round(nsamp / osec / 1e6, 4), "unit": "MRays/s", "cores": threads, "kind": "oracle",
               "sample": f"{per_level} seeded rays of every level (of its traced rays) of frames 0 and {F - 1}, "
                         f"closest-first variant's rays (oracle BVH builds excluded)"}
        log(f"cpu baseline {cpu['value']} MRays/s; parity " +
            ", ".join(f"{k}: {v['same_hit_and_patch']:.6f} ({'ok' if v['ok'] else 'FAILED'})" for k, v in parity.items()))
    head = "batched"
    failed = sorted(k for k, v in (parity or {}).items() if not v["ok"])
    if failed:
        log(f"oracle gate failed for {failed}: no throughput is reported")
    print(json.dumps({
        "metric": "MRays/s combined run: 8M patches, 8 frames, primary + 3 diffuse bounces",
        "value": None if failed else round(variants[head]["mrays_per_s"], 3), "unit": "MRays/s", "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(variants[head]["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded)",
        "config": {"workload": f"{w.name}: {w.cp.shape[0]} patches, {F} frames, {n} primary rays + {B} bounces "
                               f"per frame ({variants[head]['rays_per_step']} rays traced per step: every "
                               f"primary ray and, per bounce level, the active bounces of the previous level's "
                               f"rays, compacted; a bounce of a missed ray is inactive)",
                   "leaf_depth": w.leaf_depth,
                   "frames": "world" if args.world_frames else "patch-local (Sec. 3.4)",
                   "variant": "closest-first order, batched over frames"},
        "variants": variants, "roofline": variants[head].get("roofline"), "cpu_baseline": cpu, "parity_sample": parity,
        "parity_ok": None if parity is None else not failed, "gate_failed": failed,
        "device_memory_gib": {"scene_all_frames": round(info["device_bytes"] / 2**30, 3),
                              "frame_control_points": round(sum(c.numel() * 4 for c in cps) / 2**30, 3),
                              "rays": round(ray_bytes / 2**30, 3), "hits": round(hit_bytes / 2**30, 3)},
        "source_hash": source_hash()}), flush=True)
    if failed:
        sys.exit(1)


if __name__ == "__main__":
    main()
