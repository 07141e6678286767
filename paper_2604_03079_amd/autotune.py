"""Autotuner of the batched persistent kernel.

Searches block size, the evaluate-ahead mode and the size below which a circuit is
stamped inside one workgroup (colour-phase fusion), timing each candidate with HIP
graph replays of one batched step; the winner is cached in a JSON file keyed by the
batch signature (sorted circuit sizes and colour counts) and the GPU architecture."""
from __future__ import annotations

import hashlib
import json
import os

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune", "batch_tune.json")
BLOCKS = (128, 256)
LOCAL = (0, 64, 256, 1024, 4096)
EAHEAD = (-1, 0)


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
    """Pick (block, eval_ahead, local_max_dev) for this batch; leaves it configured."""
    import torch
    key = signature(batch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except Exception:
            cache = {}
    if key in cache:
        best = cache[key]
        batch.set_launch(best["block"], best["eval_ahead"], best["local_max_dev"])
        batch.set_params(W, L, VTH0)
        return dict(best, cached=True)
    results = []
    for block in BLOCKS:
        for local in LOCAL:
            for ea in EAHEAD:
                try:
                    batch.set_launch(block, ea, local)
                    batch.set_params(W, L, VTH0)
                    ms = _time(torch, lambda: batch.eval_stamp(x, ag0, None, A, b), reps)
                    batch.check()
                except Exception as e:   # configuration not supported on this device
                    if log:
                        log(f"  tune skip block={block} local={local} ea={ea}: {e}")
                    continue
                results.append(dict(block=block, eval_ahead=ea, local_max_dev=local, ms=ms))
                if log:
                    log(f"  tune block={block:4d} local={local:5d} ea={ea:2d}: {ms * 1e3:9.1f} us")
    best = min(results, key=lambda r: r["ms"])
    batch.set_launch(best["block"], best["eval_ahead"], best["local_max_dev"])
    batch.set_params(W, L, VTH0)
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache[key] = best
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dict(best, cached=False, tried=len(results))
