"""Autotuner of the batched kernel.

Searches the schedule (grid-barrier persistent kernel, or workgroup regions), block
size, and for the persistent kernel the evaluate-ahead mode and the size below which
a circuit is stamped inside one workgroup (colour-phase fusion), timing each
candidate with HIP graph replays of one batched step; the winner is cached in a JSON file keyed by the
batch signature (sorted circuit sizes and colour counts) and the GPU architecture."""
from __future__ import annotations

import hashlib
import json
import os

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune", "batch_tune.json")
BLOCKS = (128, 256)
LOCAL = (0, 64, 256, 1024, 4096)
EAHEAD = (-1, 0)
REGION_BLOCKS = (128, 192, 256)


def candidates():
    for block in BLOCKS:
        for local in LOCAL:
            for ea in EAHEAD:
                yield dict(schedule="persistent", block=block, eval_ahead=ea, local_max_dev=local)
    for block in REGION_BLOCKS:
        yield dict(schedule="region", block=block, eval_ahead=-1, local_max_dev=0)


def _apply(batch, cfg, W, L, VTH0):
    batch.set_launch(cfg["block"], cfg["eval_ahead"], cfg["local_max_dev"], cfg.get("schedule", "persistent"))
    batch.set_params(W, L, VTH0)


def signature(batch) -> str:
    import torch
    sizes = sorted((c.n_dev, c.n_colors or 0) for c in batch.circuits)
    arch = torch.cuda.get_device_properties(0).gcnArchName
    h = hashlib.sha256(json.dumps([arch, sizes]).encode()).hexdigest()[:24]
    return f"{arch}:{h}"


def _time(torch, fn, reps=8):
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(batch, W, L, VTH0, x, ag0, A, b, cache_path: str | None = DEFAULT_CACHE, reps: int = 8,
         log=None) -> dict:
    """Pick (schedule, block, eval_ahead, local_max_dev) for this batch; leaves it
    configured."""
    import torch
    key = signature(batch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except Exception:
            cache = {}
    if key in cache and "schedule" in cache[key]:
        best = cache[key]
        _apply(batch, best, W, L, VTH0)
        return dict(best, cached=True)
    results = []
    for cfg in candidates():
        try:
            _apply(batch, cfg, W, L, VTH0)
            ms = _time(torch, lambda: batch.eval_stamp(x, ag0, None, A, b), reps)
            batch.check()
        except Exception as e:   # configuration not supported on this device
            if log:
                log(f"  tune skip {cfg}: {e}")
            continue
        results.append(dict(cfg, ms=ms))
        if log:
            log(f"  tune {cfg['schedule']:10s} block={cfg['block']:4d} local={cfg['local_max_dev']:5d} "
                f"ea={cfg['eval_ahead']:2d}: {ms * 1e3:9.1f} us")
    best = min(results, key=lambda r: r["ms"])
    _apply(batch, best, W, L, VTH0)
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[key] = best
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dict(best, cached=False, tried=len(results))
