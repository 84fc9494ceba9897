"""Schedule autotuner for batched simulation.

A batch plan has two schedule choices that change which workgroup computes an
output pixel but not the arithmetic done for it: the blur work-item height
(16 or 8 output rows; 8 gives twice as many items for small frames) and whether
each stage is launched persistently (as many workgroups as the device holds,
striding over the item list) or with one workgroup per item.  The tuner times
every candidate on the real batch (graph-free, events on the stream, median of
a few launches) and keeps the fastest per batch signature: precision, basis
shape and the multiset of frame shapes.  Results are cached in memory and,
when a path is given (argument or P2S_TUNE_CACHE), in a JSON file.
"""
from __future__ import annotations

import collections
import json
import os
from typing import Dict, List, Optional, Sequence

CANDIDATES: List[Dict[str, int]] = [
    {"blur_tile_rows": 16, "persistent": 1},
    {"blur_tile_rows": 16, "persistent": 0},
    {"blur_tile_rows": 8, "persistent": 1},
    {"blur_tile_rows": 8, "persistent": 0},
]

_memory: Dict[str, dict] = {}


def signature(shapes: Sequence[Sequence[int]], precision: str, K: int, P: int) -> str:
    counts = collections.Counter(tuple(int(v) for v in s) for s in shapes)
    body = ";".join(f"{c}x{h}x{w}*{n}" for (c, h, w), n in sorted(counts.items()))
    return f"{precision}|K{K}|P{P}|{body}"


def _load(path: Optional[str]) -> dict:
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _store(path: Optional[str], table: dict) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(sim, images, d_over_r0s, seeds, precision="bf16", outs=None, ws=None, reps: int = 3,
         cache_path: Optional[str] = None, candidates=None) -> dict:
    """Best schedule options for this batch, e.g. {"blur_tile_rows": 16,
    "persistent": 1}; also records each candidate's median time (us)."""
    import torch

    from . import p2s

    cache_path = cache_path or os.environ.get("P2S_TUNE_CACHE")
    shapes = [tuple(im.shape) for im in images]
    key = signature(shapes, precision, sim.basis.K, sim.basis.P)
    table = _load(cache_path)
    if key in _memory:
        return dict(_memory[key]["best"])
    if key in table:
        _memory[key] = table[key]
        return dict(table[key]["best"])
    if outs is None:
        outs = [torch.empty_like(im) for im in images]
    if ws is None:
        ws = sim.batch_workspace(shapes)
    timings = []
    stream = torch.cuda.current_stream()
    for opt in candidates or CANDIDATES:
        b = p2s.Batch(images, outs, d_over_r0s, seeds, sim.basis, sim.net, precision, ws, sim.n_zernike,
                      sim.corr_len_px, sim.q_sampling, **opt)
        b.upload()
        b.launch()                                  # warm-up
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.launch()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        torch.cuda.synchronize()
        b.close()
        ts.sort()
        timings.append((ts[len(ts) // 2], opt))
    best_t, best = min(timings, key=lambda t: t[0])
    rec = {"best": dict(best), "us": {f"rows{o['blur_tile_rows']}_p{o['persistent']}": t for t, o in timings}}
    _memory[key] = rec
    if cache_path:
        table = _load(cache_path)
        table[key] = rec
        _store(cache_path, table)
    return dict(best)


def last_timings(shapes, precision, K, P) -> Optional[dict]:
    rec = _memory.get(signature(shapes, precision, K, P))
    return None if rec is None else dict(rec["us"])
