"""Autotuner for the batched persistent pass.

Tries workgroup size, tile size, grid size and in-run point sorting for one
(tree, instances, precision, spreading mode) signature, times each candidate
plan with events on the current stream (graph replays, after a warm-up
replay), and keeps the fastest.  Results are cached in a JSON file keyed by
the device name and the workload signature, so a later run with the same
shapes skips the search.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, Iterable, List, Optional, Sequence

import torch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "octrack", "tune.json")


@dataclass(frozen=True)
class Candidate:
    block: int
    tile: int
    grid: int = 0          # 0: as many workgroups as fit on the chip
    sort_points: bool = True

    def label(self) -> str:
        return f"b{self.block}_t{self.tile}_g{self.grid}_{'sort' if self.sort_points else 'nosort'}"


def default_candidates(n_points: int, uniform_ops: bool = True) -> List[Candidate]:
    sorts = (True, False) if uniform_ops else (False,)
    out = []
    # small runs are latency bound: narrow workgroups keep every CU busy
    blocks = (64, 128, 256, 512) if n_points < 2 * 256 * 512 else (256, 512)
    for sort in sorts:
        for block in blocks:
            for mult in (1, 2, 4, 8):
                tile = block * mult
                if tile > max(block, n_points) or (sort and mult == 8) or (not sort and mult == 1):
                    continue
                out.append(Candidate(block, tile, 0, sort))
    return out


def signature(tree, offsets: Sequence[int], ops: Sequence[int], dtype, mode: str) -> str:
    """Device name + everything that changes the kernel's work."""
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    h = hashlib.sha256()
    h.update(str([int(v) for v in offsets]).encode())
    h.update(str([int(v) for v in ops]).encode())
    return "|".join([dev, f"leaves={tree.n_leaves}", f"l={tree.l_min}-{tree.l_max}",
                     f"periodic={int(tree.periodic)}", f"points={int(offsets[-1])}",
                     f"inst={len(offsets) - 1}", str(dtype).replace("torch.", ""), mode, h.hexdigest()[:12]])


def load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str, key: str, entry: dict) -> None:
    d = load_cache(path)
    d[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(plan, pos, field, force, ids, vel, fout, reps: int = 5) -> float:
    """Average milliseconds per replay of a plan."""
    plan.run(pos, field=field, force=force, ids=ids, vel=vel, field_out=fout)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.run(pos, field=field, force=force, ids=ids, vel=vel, field_out=fout)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(tree, offsets: Sequence[int], ops: Sequence[int], pos, field=None, force=None, dtype=torch.float32,
         mode: str = "fixed", candidates: Optional[Iterable[Candidate]] = None, reps: int = 5,
         cache_path: Optional[str] = DEFAULT_CACHE, use_cache: bool = True, log=None):
    """Return (best Candidate, {label: ms}).  `pos`, `field`, `force` are
    the run's device tensors (the timing uses them)."""
    import paper_2605_20565_amd as ot

    key = signature(tree, offsets, ops, dtype, mode)
    if cache_path and use_cache:
        hit = load_cache(cache_path).get(key)
        if hit:
            return Candidate(**hit["best"]), hit.get("timings_ms", {})
    n = int(offsets[-1])
    live = [o for i, o in enumerate(ops) if offsets[i + 1] > offsets[i] and o]
    uniform = len(set(live)) <= 1
    cands = list(candidates) if candidates is not None else default_candidates(n, uniform)
    dev = pos.device
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    vel = torch.empty((n, 3), dtype=dtype, device=dev)
    fout = torch.empty((tree.n_leaves, 3), dtype=dtype, device=dev)
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for c in cands:
        if c.sort_points and not uniform:
            continue
        t0 = time.perf_counter()
        plan = ot.BatchPlan(tree, offsets, ops, dtype=dtype, mode=mode, block=c.block, tile=c.tile, grid=c.grid,
                            sort_points=c.sort_points)
        ms = time_plan(plan, pos, field, force, ids, vel, fout, reps)
        plan.close()
        timings[c.label()] = round(ms, 4)
        if log:
            log(f"[tune] {c.label()}: {ms:.3f} ms ({time.perf_counter() - t0:.1f}s)")
        if ms < best_ms:
            best, best_ms = c, ms
    if best is None:
        raise RuntimeError("no tuning candidate could run")
    if cache_path:
        store_cache(cache_path, key, {"best": asdict(best), "ms": round(best_ms, 4), "timings_ms": timings})
    return best, timings
