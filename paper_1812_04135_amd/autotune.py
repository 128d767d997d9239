"""Strip-row autotuner of the batched run.

The batched kernel marches each box along y in strips; a strip block is the
unit of work one workgroup takes from the queue.  Short strips give more
items (better balance, shorter dependency waits) but pay the march start-up
(four planes loaded and one face flux computed before the first row) more
often.  The best length depends on the box widths (1..4 waves per row), the
mix of sizes and the precision, so it is measured: coordinate sweeps over
the four width classes (repeated from the result while they change it, at
most `passes`), each candidate timed on whole runs of the caller's batch (HIP events on the launch stream, best of `reps`), on a scratch copy
of the state so the caller's state is not advanced.  Results are cached in a
JSON file keyed by device, precision, form and the batch's width/height
histogram.
"""
from __future__ import annotations

import json
import os

CANDIDATES = (8, 16, 24, 32, 48, 64, 96, 128, 256)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rsst_gfx950_tiles.json")


def width_class(nx: int) -> int:
    return (int(nx) + 63) // 64 - 1


def batch_key(batch) -> str:
    """Device, precision, form and, per width class, the box count and the
    median height rounded to 16 rows."""
    import torch

    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    parts = []
    for c in range(4):
        hs = sorted(int(s[1]) for s in batch.shapes if width_class(s[2]) == c)
        if hs:
            parts.append(f"w{c}:{len(hs)}x{16 * round(hs[len(hs) // 2] / 16)}")
    form = batch.cfgs[0].get("form", "pvs")
    return f"{dev}|{batch.prec}|{form}|" + ",".join(parts)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time_run(batch, U, nsteps, reps, stream):
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    batch.run(U, nsteps, st)  # capture (first use of these tiles) and warm up
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        batch.run(U, nsteps, st)
        b.record(st)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune(batch, U, nsteps: int = 20, candidates=CANDIDATES, reps: int = 2, cache: str | None = DEFAULT_CACHE,
         stream=None, retune: bool = False, log=None, passes: int = 2):
    """Pick strip rows for `batch` (a paper_1812_04135_amd.Batch) and set them.

    U is the packed state of the batch; it is only read (runs go to a
    scratch copy).  Returns (strip_rows, ms of an nsteps run, from_cache)."""
    import torch

    key = batch_key(batch)
    db = _load(cache) if cache else {}
    if not retune and key in db:
        tiles = [int(x) for x in db[key]["strip_rows"]]
        batch.set_tiles(tiles)
        return tiles, float(db[key]["ms"]), True
    nsteps = max(1, min(int(nsteps), batch.max_steps))
    present = sorted({width_class(s[2]) for s in batch.shapes})
    # the runs below advance the per-box times and may latch flags: keep the
    # batch's record and put it back afterwards
    from . import rsst_batch_poll_raw, rsst_batch_set_times
    times0 = batch.times(stream)
    flags0 = rsst_batch_poll_raw(batch.h)
    scratch = torch.empty_like(U)
    tiles = list(batch.tiles())
    times = {}

    def measure(t):
        tt = tuple(t)
        if tt not in times:
            batch.set_tiles(list(t))
            scratch.copy_(U)
            times[tt] = _time_run(batch, scratch, nsteps, reps, stream)
            if log:
                log(f"[autotune] strip rows {list(t)}: {times[tt]:.3f} ms / {nsteps} steps")
        return times[tt]

    best = measure(tiles)
    # the width classes share the GPU, so one class's best length depends on
    # the others': sweep again from the result until a pass changes nothing
    for _ in range(max(1, int(passes))):
        start = list(tiles)
        for c in present:
            for cand in candidates:
                t = list(tiles)
                t[c] = cand
                ms = measure(t)
                if ms < best:
                    best, tiles = ms, t
        if tiles == start:
            break
    batch.set_tiles(tiles)
    del scratch
    rsst_batch_set_times(batch.h, times0, flags0, stream)
    if cache:
        db = _load(cache)
        db[key] = {"strip_rows": tiles, "ms": best, "nsteps": nsteps}
        os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return tiles, best, False
