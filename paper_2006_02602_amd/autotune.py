"""Autotuner of the batched form's launch shape.

What the batched kernel leaves open, per cavity size, is the tile shape
(the element type's wide tile, or its narrow one for narrow cavities, where
a wide tile would leave lanes idle: FP64 64 x 8 or 32 x 16, FP32 32 x 8 or
16 x 16) and the number of k planes per work item (kc), and, for
the whole batch, the number of persistent blocks.  Two tuners time
candidates with HIP events and keep the fastest:

- tune_batch (what the batched workload uses) tunes a built batch in place:
  members that share a key (a cube edge) share a (tile, kc), chosen by
  coordinate descent over the whole batch, then the block count;
- tune_shapes tunes each distinct edge alone, on a small batch of that edge,
  and tune_blocks the block count of a built batch.

Results can be cached in a JSON file keyed by device architecture, element
type and edge (or the batch's mix of edges).
"""
import json
import os

import torch

from . import BATCH_TILE_WIDTHS, Batch, Grid, Params

KC_CANDIDATES = (4, 8, 16, 32, 0)        # 0 = whole columns (the cavity height per item)
BLOCK_CANDIDATES = (256, 512, 768, 1024)
CACHE_VERSION = 3                        # bump when the tile shapes or batch kernels change


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


def tune_batch(batch, keys, dtype, steps=8, reps=3, passes=2, cache_path=None):
    """({key: (ti, kc)}, nblocks, timings) for a built batch whose member m
    has shape key keys[m] (its cube edge, say), tuned on the whole batch:
    members of one key share a (tile width, kc); starting from the wide tile
    with whole columns for every key, each key in turn takes the candidate
    that steps the whole batch fastest with the others held (coordinate
    descent, `passes` rounds) at the block count that is fastest for the
    starting shapes; the block count is tuned again at the end.
    Tuning in the full mix matters: alone, a small cavity wants short k
    chunks for parallelism, while in a batch the other members supply it and
    short chunks only add work items, each paying its start-up (the centre
    cell's star for the rescale, the k-queue prologue).  keys should
    identify a member's grid (the cache is keyed by the multiset of keys).
    The batch is stepped while tuning and left with the chosen work list."""
    distinct = sorted(set(keys))
    ckey = "v%d:%s:dtype%d:batch:%s" % (CACHE_VERSION, _arch(), dtype,
                                        ",".join("%s*%d" % (k, keys.count(k)) for k in distinct))
    cache = _load(cache_path)
    depth = {k: min(batch.grids[m].nk for m in range(len(keys)) if keys[m] == k) for k in distinct}
    if ckey in cache:
        shape = {k: tuple(cache[ckey]["shape"][str(k)]) for k in distinct}
        batch.retile([(shape[k][1], shape[k][0]) for k in keys])
        return shape, cache[ckey]["blocks"], cache[ckey]["timings"]
    shape = {k: (ti_candidates(dtype)[0], 0) for k in distinct}
    timings = {}
    batch.retile([(shape[k][1], shape[k][0]) for k in keys])
    nb0, _ = tune_blocks(batch, steps, reps)

    def trial(sh):
        batch.retile([(sh[k][1], sh[k][0]) for k in keys])
        return _time(lambda: batch.step(steps, nblocks=nb0), reps)

    best_ms = trial(shape)
    for _ in range(passes):
        changed = False
        for k in distinct:
            for ti in ti_candidates(dtype):
                for kc in KC_CANDIDATES:
                    if kc >= depth[k] or (ti, kc) == shape[k]:
                        continue
                    cand = dict(shape)
                    cand[k] = (ti, kc)
                    ms = trial(cand)
                    timings["%s:ti%d:kc%d" % (k, ti, kc)] = ms
                    if ms < best_ms:
                        shape, best_ms, changed = cand, ms, True
        if not changed:
            break
    batch.retile([(shape[k][1], shape[k][0]) for k in keys])
    nb, tb = tune_blocks(batch, steps, reps)
    timings["blocks"] = {str(b): v for b, v in tb.items()}
    cache[ckey] = {"shape": {str(k): list(v) for k, v in shape.items()}, "blocks": nb, "timings": timings}
    _save(cache_path, cache)
    return shape, nb, timings


def tune_blocks(batch, steps=4, reps=3):
    """Fastest persistent block count for a built batch."""
    best, best_ms, timings = None, None, {}
    for nb in BLOCK_CANDIDATES:
        ms = _time(lambda: batch.step(steps, nblocks=nb), reps)
        timings[nb] = ms
        if best_ms is None or ms < best_ms:
            best, best_ms = nb, ms
    return best, timings
