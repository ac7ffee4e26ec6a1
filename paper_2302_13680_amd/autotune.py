"""Autotuner of the batched solver's lanes-per-node width, with a JSON cache.

For every distinct (n, N, precision) among a batch's contexts the library's
smg_tune_lanes times the finest-level half-sweep for each admissible
power-of-two width.  The batched kernels are compiled for one samples-per-lane
count JM = max_i JM_i(W_i) for all instances, with JM_i(W) = v ceil(N_i / (v W))
and v = 2 samples per access when every instance is FP32 with even N (else 1),
so a narrow width for a large-N instance slows every instance; the choice for
each instance is therefore the fastest width with JM_i(W) <= max_i JM_i(64), the
smallest JM the batch allows.  Timings are cached by key
"n x N : precision : device name" in a JSON file so that later runs reuse them.
"""
from __future__ import annotations

import json
import os

from . import binding


def _key(ctx, device_name: str) -> str:
    prec = "f32" if ctx.precision == binding.SMG_F32 else "f64"
    return f"{ctx.n}x{ctx.N}:{prec}:{device_name}"


def tune(contexts, cache_path: str | None = None, device_name: str = "gfx950"):
    """Return one lane width per context (tuned or from the cache) and the table."""
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    v = 2 if all(c.precision == binding.SMG_F32 and c.N % 2 == 0 for c in contexts) else 1

    def jm(N, w):
        return v * -(-N // (v * w))

    jm_cap = max(jm(ctx.N, 64) for ctx in contexts)
    lanes = []
    for ctx in contexts:
        key = _key(ctx, device_name)
        if key not in cache:
            best, table = binding.tune_lanes(ctx)
            cache[key] = {"best": best, "us": {str(k): v for k, v in table.items()}}
        table = {int(w): us for w, us in cache[key]["us"].items() if jm(ctx.N, int(w)) <= jm_cap}
        lanes.append(min(table, key=table.get) if table else int(cache[key]["best"]))
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return lanes, cache
