"""Launch-parameter autotuner for seeding.

The tunable parameters (godiet_seed_opts: the short/long read threshold, the lookup grid
and the long-read grid) change only how work is mapped onto the GPU, never the result.
tune() times every candidate on the caller's index and read batch with HIP events,
checks that every candidate produced byte-identical anchors, and keeps the fastest.
Results are cached in a JSON file keyed by GPU architecture, k, w, pattern, index size
class and the batch's read-length profile, so a later batch of the same shape reuses
them without timing.
"""
import hashlib
import itertools
import json
import os

import numpy as np

from .api import TUNING_KEYS
from .plan import SeedPlan

DEFAULT_GRID = {
    "long_records": [64, 192, 768],
    "lookup_blocks": [2048, 8192, 32768],
    "long_blocks": [256, 1024, 4096],
}


def candidates(grid):
    """Every combination of the grid's values, in the grid's key order."""
    bad = set(grid) - set(TUNING_KEYS)
    if bad:
        raise ValueError("unknown launch parameters: %s" % ", ".join(sorted(bad)))
    keys = list(grid)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(grid[k] for k in keys))]


def _cache_path(path):
    if path:
        return path
    base = os.environ.get("GODIET_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "godiet", "autotune.json")
    return base


def shape_key(index, reads, pattern, k, w):
    """Key describing what the best launch parameters depend on."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    offs = reads.offsets.cpu().numpy()
    lens = np.diff(offs)
    # read-length profile: counts per power-of-two length class, in 1/8 of the batch
    cls = np.bincount(np.clip(np.log2(np.maximum(lens, 1)).astype(int), 0, 24), minlength=25)
    prof = tuple(int(round(8 * c / max(lens.size, 1))) for c in cls)
    size_cls = int(np.log2(max(index.n, 1)))
    return "%s|k%d|w%d|%s|n2^%d|%s" % (arch, k, w, pattern, size_cls, ",".join(map(str, prof)))


def _digest(plan):
    a, off, sh = plan.outputs()
    h = hashlib.sha256()
    h.update(a.cpu().numpy().tobytes())
    h.update(off.cpu().numpy().tobytes())
    h.update(sh.cpu().numpy().tobytes())
    return h.hexdigest()


def tune(index, reads, pattern, k, w, grid=None, reps=3, cache=None, use_cache=True, **seed_kw):
    """Return (best tuning dict, report list).  report rows: (tuning, ms per pass)."""
    import torch
    grid = grid or DEFAULT_GRID
    path = _cache_path(cache)
    key = shape_key(index, reads, pattern, k, w)
    table = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        if key in table:
            return dict(table[key]["tuning"]), []
    cands = candidates(grid)
    report, ref_digest, capacity = [], None, None
    for cand in cands:
        plan = SeedPlan(index, reads, pattern, k, w, tuning=cand, capacity=capacity, **seed_kw)
        capacity = plan.capacity
        plan.run()
        plan.check()
        dg = _digest(plan)
        if ref_digest is None:
            ref_digest = dg
        elif dg != ref_digest:
            raise RuntimeError("tuning candidate %r changed the anchors" % (cand,))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        report.append((cand, e0.elapsed_time(e1) / reps))
        del plan
    best = min(report, key=lambda r: r[1])[0]
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            table[key] = {"tuning": best, "ms": min(r[1] for r in report)}
            with open(path, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best, report
