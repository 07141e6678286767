"""Autotuner of the batched kernel: a caller of the library's cs_batch_tune.

The search itself (candidate schedules, block sizes, evaluate-ahead modes and
colour-phase fusion sizes, each timed by HIP graph replays of one batched step) and
its cache file (keyed by the GPU architecture and the batch signature) live in the
library, so that C callers tune the same way."""
from __future__ import annotations

import os

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune", "batch_tune.txt")


def tune(batch, W, L, VTH0, x, ag0, A, b, cache_path: str | None = DEFAULT_CACHE, reps: int = 8,
         log=None) -> dict:
    """Pick (schedule, block, eval_ahead, local_max_dev) for this batch; leaves it
    configured with its parameters set."""
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    best = batch.tune(W, L, VTH0, x, ag0, A, b, reps=reps, cache_path=cache_path)
    if log:
        log(f"  tuned: {best['schedule']} block={best['block']} local={best['local_max_dev']} "
            f"ea={best['eval_ahead']}: {best['ms'] * 1e3:.1f} us ({'cached' if best['cached'] else str(best['tried']) + ' timed'})")
    return best
