"""Autotuner for the persistent batched launch.

The batch plan (csrc/ldp_batch.hip) cuts every image into work items of whole
cell rows and runs them on resident workgroups.  How that is done is a small
set of choices (ldp_tune): the workgroup size, and per image size class the
number of cell rows one work item covers and the minimum code rows of one
lane task (short tasks give more parallelism inside an item, long ones
amortise the three-row prologue of each task).  This module times candidate
choices on the caller's own device-resident batch by coordinate descent and
keeps the winners in a JSON cache keyed by GPU architecture, k, cell grid and
a coarse signature of the image size distribution.

Timings are taken on a warmed-up device (the clocks ramp up under sustained
load), each as the best of a few rounds, and the leading candidates are timed
again interleaved before the winner is chosen, so the order in which
candidates are tried does not decide the result.
"""
import json
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "tuned.json")

THREADS = tuple(range(128, 1025, 64))  # whole waves
ROWS_PER_TASK = (4, 8, 16, 32)


def arch():
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def size_signature(Hs, Ws):
    """Coarse size-distribution signature: a single size, or pixel-count
    quantiles rounded to powers of two."""
    Hs = np.asarray(Hs)
    Ws = np.asarray(Ws)
    if len(Hs) and (Hs == Hs[0]).all() and (Ws == Ws[0]).all():
        return "%dx%d" % (int(Hs[0]), int(Ws[0]))
    px = Hs.astype(np.int64) * Ws
    q = [int(2 ** round(np.log2(max(1, v)))) for v in np.quantile(px, [0.1, 0.5, 0.9])]
    return "mix:%d/%d/%d" % tuple(q)


def key(Hs, Ws, k, cells, flags=0, windows=False):
    """Cache key: architecture, k, cell grid (or window size, with "|win"),
    size signature, and the ldp_*_ex flags when set (the variants weigh
    arithmetic against memory traffic differently, so their best split
    differs)."""
    base = "%s|k%d|%dx%d|%s" % (arch(), k, cells[0], cells[1], size_signature(Hs, Ws))
    if windows:
        base += "|win"
    return base if not flags else base + "|f%d" % flags


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(Hs, Ws, k, cells, path=CACHE, flags=0, windows=False):
    """Cached tune dict for this batch shape (and flags; window plans when
    `windows`, with cells = the window size), or None."""
    return load_cache(path).get(key(Hs, Ws, k, cells, flags, windows), {}).get("tune")


def default_classes(Hs, Ws, cells_y):
    """Size classes for a batch: one class for a single size, else small /
    medium / large split at pixel-count quantiles."""
    px = np.asarray(Hs, dtype=np.int64) * np.asarray(Ws, dtype=np.int64)
    if len(px) == 0 or (px == px[0]).all():
        return [dict(cell_rows_per_item=1, rows_per_task=8)]
    b1, b2 = (int(v) for v in np.quantile(px, [1 / 3, 2 / 3]))
    return [dict(max_pixels=b1, cell_rows_per_item=min(cells_y, 4), rows_per_task=4),
            dict(max_pixels=b2, cell_rows_per_item=2, rows_per_task=8),
            dict(cell_rows_per_item=1, rows_per_task=8)]


def _plan(binding, n, pixels, k, cells, tune, flags, max_width):
    """A batch plan: over the cell grid, or over windows of cells[0] x cells[1]
    code pixels when max_width (the widest image) is given."""
    if max_width:
        return binding.BatchPlan(n, pixels, k, cells[0], cells[1], tune, flags=flags,
                                 windows=True, max_width=max_width)
    return binding.BatchPlan(n, pixels, k, cells[0], cells[1], tune, flags=flags)


def _time_plan(binding, descs, n, pixels, k, cells, tune, reps=8, rounds=3, flags=0,
               max_width=0):
    """Best mean launch time (ms) over `rounds` rounds of `reps` launches."""
    import torch
    plan = _plan(binding, n, pixels, k, cells, tune, flags, max_width)
    try:
        plan.set(descs)
        for _ in range(2):
            plan.run()
        torch.cuda.synchronize()
        best = float("inf")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for _ in range(rounds):
            e0.record()
            for _ in range(reps):
                plan.run()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / reps)
        return best
    finally:
        plan.close()


def _warm_up(binding, descs, n, pixels, k, cells, tune, seconds=0.3, flags=0, max_width=0):
    """Keep the device busy with this batch for about `seconds`."""
    import torch
    plan = _plan(binding, n, pixels, k, cells, tune, flags, max_width)
    try:
        plan.set(descs)
        t_end = time.time() + seconds
        while time.time() < t_end:
            for _ in range(10):
                plan.run()
            torch.cuda.synchronize()
    finally:
        plan.close()


def tune_batch(descs, Hs, Ws, k, cells, budget_s=60.0, verbose=False, flags=0, windows=False,
               start=None):
    """Coordinate descent over ldp_tune for the device-resident batch `descs`
    (a ctypes ImageDesc array) and ldp_*_ex `flags`; with `windows`, for a
    window plan of cells[0] x cells[1] code pixels.  `start` is the first
    candidate (default: 256 threads, default classes).  Returns (best tune
    dict, best ms)."""
    from . import binding
    n = len(descs)
    pixels = int((np.asarray(Hs, dtype=np.int64) * np.asarray(Ws, dtype=np.int64)).sum())
    mw = int(np.asarray(Ws).max()) if windows else 0
    t_end = time.time() + budget_s
    best = start or dict(block_threads=256, classes=default_classes(Hs, Ws, cells[0]))
    _warm_up(binding, descs, n, pixels, k, cells, best, flags=flags, max_width=mw)
    best_ms = _time_plan(binding, descs, n, pixels, k, cells, best, flags=flags, max_width=mw)
    seen = {json.dumps(best, sort_keys=True): best_ms}

    def attempt(cand):
        nonlocal best, best_ms
        s = json.dumps(cand, sort_keys=True)
        if s in seen or time.time() > t_end:
            return
        try:
            ms = _time_plan(binding, descs, n, pixels, k, cells, cand, flags=flags, max_width=mw)
        except binding.LdpError:
            return
        seen[s] = ms
        if verbose:
            print("  %.4f ms %s" % (ms, s), flush=True)
        if ms < best_ms:
            best, best_ms = cand, ms

    for _ in range(2):  # two sweeps of coordinate descent
        for th in THREADS:
            attempt(dict(best, block_threads=th))
        for ci in range(len(best["classes"])):
            cpis = sorted({1, 2, 4, cells[0]} & set(range(1, cells[0] + 1)))
            for cpi in cpis:
                cls = [dict(c) for c in best["classes"]]
                cls[ci]["cell_rows_per_item"] = cpi
                attempt(dict(best, classes=cls))
            for rpt in ROWS_PER_TASK:
                cls = [dict(c) for c in best["classes"]]
                cls[ci]["rows_per_task"] = rpt
                attempt(dict(best, classes=cls))

    # time the leading candidates again, interleaved, and keep the best
    lead = sorted(seen.items(), key=lambda kv: kv[1])[:4]
    again = {s: float("inf") for s, _ in lead}
    for _ in range(3):
        for s in again:
            ms = _time_plan(binding, descs, n, pixels, k, cells, json.loads(s), flags=flags,
                            max_width=mw)
            again[s] = min(again[s], ms)
    s_best = min(again, key=again.get)
    if verbose:
        for s, ms in sorted(again.items(), key=lambda kv: kv[1]):
            print("  again %.4f ms %s" % (ms, s), flush=True)
    return json.loads(s_best), again[s_best]


def save(Hs, Ws, k, cells, tune, ms, path=CACHE, note="", flags=0, windows=False):
    cache = load_cache(path)
    cache[key(Hs, Ws, k, cells, flags, windows)] = {"tune": tune, "ms": round(ms, 4),
                                                     "note": note}
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
