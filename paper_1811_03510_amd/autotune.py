"""Launch-parameter autotuner for the persistent intersect kernel.

The kernel's results never depend on its launch parameters (ray-to-lane
assignment and phase order change only the schedule), so the tuner is free to
pick whatever runs fastest.  It searches, by coordinate descent from the
library defaults:

  waves_per_cu     resident waves per compute unit (0 = as many as fit)
  fetch_min        free lanes a wave waits for before it refills from the queue
                   (the queue chunk: a refill takes exactly that many rays or more)
  traverse_min     lanes in BVH traversal that trigger a traversal phase
  grid_min         lanes waiting for a grid recompute that trigger that phase
  traverse_steps   BVH nodes a lane visits per traversal phase
  decide_min       lanes waiting for the ordering network that trigger it
                   (searched only when the scene has a learned order)

timing the caller's workload (a list of batches for one ccs_intersect_batched
call) with HIP events, median of a few repetitions.  The fastest settings seen
are then timed again side by side with the library defaults, which they replace
only when faster by more than 0.5 %.  The winner is cached in a JSON file keyed
by GPU architecture, library source hash and a workload key.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
from pathlib import Path

DEFAULT = dict(waves_per_cu=0, fetch_min=16, traverse_min=1, grid_min=8, traverse_steps=3, decide_min=8)
SPACE = dict(
    waves_per_cu=[0, 4, 8],
    fetch_min=[4, 8, 16, 24, 32, 48],
    traverse_min=[1, 2, 8],
    grid_min=[4, 8, 16, 24, 32],
    traverse_steps=[1, 2, 3, 4, 8],
    decide_min=[1, 4, 8, 16, 32],
)


def _cache_path() -> Path:
    return Path(os.environ.get("CCS_AUTOTUNE_CACHE", Path.home() / ".cache" / "ccs_autotune.json"))


def library_hash() -> str:
    here = Path(__file__).resolve().parent / "csrc"
    h = hashlib.sha256()
    for p in sorted(here.glob("*")):
        if p.suffix in (".hip", ".h", ".cpp"):
            h.update(p.read_bytes())
    return h.hexdigest()[:16]


def workload_key(scene, batches) -> str:
    """Scene size and depth, batch frames and sizes, and a hash of a few rays."""
    import torch
    info = scene.info()
    h = hashlib.sha256()
    h.update(repr((info["n_patches"], info["leaf_depth"], info["n_frames"])).encode())
    for f, rays, _ in batches:
        h.update(repr((int(f), int(rays.shape[0]))).encode())
        if rays.shape[0]:
            idx = torch.linspace(0, rays.shape[0] - 1, 16, device=rays.device).long()
            h.update(rays[idx].cpu().numpy().tobytes())
    return h.hexdigest()[:16]


def time_launch(scene, batches, reps: int = 3) -> float:
    """Median milliseconds of one batched launch of ``batches``."""
    import torch
    scene.intersect_batched(batches)  # warm-up
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        scene.intersect_batched(batches)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def confirm(scene, batches, cands: list, rounds: int = 5, log=None, prefer: dict | None = None,
            margin: float = 0.005) -> tuple[dict, float]:
    """The fastest of ``cands`` by the median of ``rounds`` timings each, taken
    round-robin so that clock drift affects every candidate alike.  ``prefer`` (one
    of ``cands``) is kept unless another candidate is faster by more than ``margin``
    (a fraction of its time), so that noise alone does not move the choice."""
    times = [[] for _ in cands]
    for _ in range(rounds):
        for i, p in enumerate(cands):
            scene.set_launch(**p)
            times[i].append(time_launch(scene, batches, 1))
    med = [statistics.median(t) for t in times]
    k = min(range(len(cands)), key=lambda i: med[i])
    if prefer in cands:
        j = cands.index(prefer)
        if med[k] > med[j] * (1.0 - margin):
            k = j
    if log:
        for p, m in zip(cands, med):
            log(f"autotune confirm {p} -> {m:.3f} ms")
    scene.set_launch(**cands[k])
    return dict(cands[k]), med[k]


# Settings that won on the benchmark workloads, always timed in the confirmation
# round (a descent step can miss one when a timing is noisy).
PRESETS = (
    dict(DEFAULT, fetch_min=16, traverse_min=1, grid_min=16, traverse_steps=2),
    dict(DEFAULT, fetch_min=16, traverse_min=2, grid_min=4, traverse_steps=3),
    dict(DEFAULT, fetch_min=24, traverse_min=8, grid_min=16, traverse_steps=4),
)


def tune(scene, batches, reps: int = 5, sweeps: int = 2, log=None, space=None,
         learned: bool = False, finalists: int = 4) -> tuple[dict, float, list]:
    """Coordinate descent over ``space`` from DEFAULT, then the ``finalists``
    fastest settings seen, DEFAULT and PRESETS timed again side by side (confirm).
    Returns (params, ms, trials)."""
    space = dict(space or SPACE)
    if not learned:
        space.pop("decide_min", None)
    best = dict(DEFAULT)
    trials = []
    seen = {}

    def run(p):
        key = tuple(sorted(p.items()))
        if key not in seen:
            scene.set_launch(**p)
            seen[key] = time_launch(scene, batches, reps)
            trials.append((dict(p), seen[key]))
            if log:
                log(f"autotune {p} -> {seen[key]:.3f} ms")
        return seen[key]

    best_ms = run(best)
    for _ in range(sweeps):
        improved = False
        for name, values in space.items():
            for v in values:
                cand = dict(best, **{name: v})
                ms = run(cand)
                if ms < best_ms * 0.995:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    if finalists > 1:
        ranked = sorted(seen.items(), key=lambda kv: kv[1])[:finalists]
        cands = [dict(k) for k, _ in ranked]
        for extra in (dict(DEFAULT),) + tuple(dict(p) for p in PRESETS):
            if extra not in cands:
                cands.append(extra)
        best, best_ms = confirm(scene, batches, cands, rounds=15, log=log, prefer=dict(DEFAULT))
    scene.set_launch(**best)
    return best, best_ms, trials


def tuned(scene, batches, name: str = "", reps: int = 3, log=None, retune: bool = False,
          learned: bool = False) -> dict:
    """Launch parameters for this (arch, library, workload): from the cache, else
    tuned now and stored.  The scene is left configured with them."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    key = f"{arch}|{library_hash()}|{name}|{'learned' if learned else 'plain'}|{workload_key(scene, batches)}"
    path = _cache_path()
    cache = {}
    if path.exists():
        try:
            cache = json.loads(path.read_text())
        except (OSError, json.JSONDecodeError):
            cache = {}
    if key in cache and not retune:
        p = cache[key]["params"]
        scene.set_launch(**p)
        if log:
            log(f"autotune cache hit {p}")
        return p
    p, ms, trials = tune(scene, batches, reps=reps, log=log, learned=learned)
    cache[key] = {"params": p, "ms": ms, "trials": len(trials)}
    try:
        path.parent.mkdir(parents=True, exist_ok=True)
        tmp = path.with_suffix(".tmp")
        tmp.write_text(json.dumps(cache, indent=1, sort_keys=True))
        tmp.replace(path)
    except OSError:
        pass
    return p
