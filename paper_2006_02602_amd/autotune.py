"""Autotuner of the batched form's launch shape.

What the batched kernel leaves open, per cavity size, is the tile shape
(the element type's wide tile, or its narrow one for narrow cavities, where
a wide tile would leave lanes idle: FP64 64 x 8 or 32 x 16, FP32 32 x 8 or
16 x 16) and the number of k planes per work item (kc), and, for
the whole batch, the number of persistent blocks.  For each distinct cube
edge the tuner times a small batch of that edge over every (tile, kc)
candidate with HIP events and keeps the fastest; then it times the whole
batch over the candidate block counts.  Results can be cached in a JSON file
keyed by device architecture, element type and edge.
"""
import json
import os

import torch

from . import BATCH_TILE_WIDTHS, Batch, Grid, Params

KC_CANDIDATES = (4, 8, 16, 32, 0)        # 0 = whole columns (the cavity height per item)
BLOCK_CANDIDATES = (256, 512, 768, 1024)
CACHE_VERSION = 2                        # bump when the tile shapes change


def ti_candidates(dtype):
    """Tile widths the tuner tries for element type dtype (wide, narrow)."""
    return BATCH_TILE_WIDTHS[dtype]


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, cache):
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)


def tune_shapes(edges, dtype, steps=4, reps=3, probe_members=6, cache_path=None):
    """{edge: (ti, kc)} for every distinct edge in `edges` (FP32 or FP64
    cubes): the tile width and k-chunk length that step a small batch of
    that edge fastest."""
    cache = _load(cache_path)
    out = {}
    for e in sorted(set(edges)):
        key = "v%d:%s:dtype%d:edge%d" % (CACHE_VERSION, _arch(), dtype, e)
        if key in cache and "ti" in cache[key]:
            out[e] = (cache[key]["ti"], cache[key]["kc"])
            continue
        g = Grid.cube(e, dtype)
        best, best_ms, timings = None, None, {}
        for ti in ti_candidates(dtype):
            for kc in KC_CANDIDATES:
                if kc > e:
                    continue
                b = Batch([(g, Params(Ra=1e4), kc, ti)] * probe_members).init(range(probe_members))
                ms = _time(lambda: b.step(steps), reps)
                timings["ti%d:kc%d" % (ti, kc)] = ms
                if best_ms is None or ms < best_ms:
                    best, best_ms = (ti, kc), ms
                del b
        out[e] = best
        cache[key] = {"ti": best[0], "kc": best[1], "ms_per_%d_steps" % steps: timings}
    _save(cache_path, cache)
    return out


def tune_blocks(batch, steps=4, reps=3):
    """Fastest persistent block count for a built batch."""
    best, best_ms, timings = None, None, {}
    for nb in BLOCK_CANDIDATES:
        ms = _time(lambda: batch.step(steps, nblocks=nb), reps)
        timings[nb] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = nb, ms
    return best, timings
