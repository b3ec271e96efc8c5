"""Digests of full-size outputs, shared by the script that records the oracle's results
(tests/golden/make_fullsize.py) and the GPU tests that check the library against them.

A digest holds the record count, a SHA-256 over the whole output in a fixed byte form,
and per-part counts and short digests (64 key ranges of the index, 64 read-id ranges of
the anchors, 64 query ranges of the lookups) so that a mismatch names where it is.  This
module only hashes and partitions arrays; it computes nothing of the method.

Byte forms: index keys and values as little-endian uint64 (32-bit values widened);
anchors as uint32 rows (read_id, qpos, rpos, strand); per-read anchor offsets as uint64;
shifts as uint8; lookup results as uint32.
"""
import hashlib

import numpy as np

PARTS = 64


def _h(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()


def index_digest(keys, vals):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals = np.ascontiguousarray(vals).astype(np.uint64)
    bounds = np.searchsorted(keys, np.array([i << 58 for i in range(PARTS)], dtype=np.uint64))
    bounds = np.append(bounds, keys.size)
    parts = [[int(bounds[i + 1] - bounds[i]), _h(keys[bounds[i]:bounds[i + 1]],
                                                 vals[bounds[i]:bounds[i + 1]])[:16]]
             for i in range(PARTS)]
    return dict(n=int(keys.size), sha256=_h(keys, vals), parts=parts)


def anchors_digest(anchors, read_off, shift):
    a = np.ascontiguousarray(anchors, dtype=np.uint32).reshape(-1, 4)
    off = np.ascontiguousarray(read_off).astype(np.uint64)
    sh = np.ascontiguousarray(shift).astype(np.uint8)
    n_reads = off.size - 1
    cut = [i * n_reads // PARTS for i in range(PARTS + 1)]
    parts = []
    for i in range(PARTS):
        lo, hi = int(off[cut[i]]), int(off[cut[i + 1]])
        parts.append([hi - lo, _h(a[lo:hi], off[cut[i]:cut[i + 1] + 1] - off[cut[i]],
                                  sh[cut[i]:cut[i + 1]])[:16]])
    return dict(n=int(a.shape[0]), sha256=_h(a, off, sh),
                shift_hist=np.bincount(sh, minlength=1).tolist(), parts=parts)


def lookup_digest(lb, occ):
    lb = np.ascontiguousarray(lb).astype(np.uint32)
    occ = np.ascontiguousarray(occ).astype(np.uint32)
    n = lb.size
    cut = [i * n // PARTS for i in range(PARTS + 1)]
    parts = [[int(occ[cut[i]:cut[i + 1]].astype(np.uint64).sum()),
              _h(lb[cut[i]:cut[i + 1]], occ[cut[i]:cut[i + 1]])[:16]] for i in range(PARTS)]
    return dict(n=int(n), found=int(np.count_nonzero(occ)),
                occ_sum=int(occ.astype(np.uint64).sum()), sha256=_h(lb, occ), parts=parts)


def votes_digest(n_win, rows):
    """rows: (n, 5) int64 (read, strand, votes, flags, loc) of every output winner in read
    order; n_win: winners per read."""
    nw = np.ascontiguousarray(n_win).astype(np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.int64).reshape(-1, 5)
    off = np.zeros(nw.size + 1, np.int64)
    off[1:] = np.cumsum(nw)
    n_reads = nw.size
    cut = [i * n_reads // PARTS for i in range(PARTS + 1)]
    parts = [[int(off[cut[i + 1]] - off[cut[i]]), _h(rows[off[cut[i]]:off[cut[i + 1]]],
                                                       nw[cut[i]:cut[i + 1]])[:16]]
             for i in range(PARTS)]
    return dict(n=int(rows.shape[0]), sha256=_h(rows, nw),
                rescued=int((rows[:, 3] & 1).sum()), parts=parts)


def lookup_queries(read_keys, n_total=500_000_000, absent_frac=0.2, seed=404):
    """Lookup workload: n_total queries, the first (1 - absent_frac) drawn uniformly with
    replacement from read_keys (seed 404), the rest random 64-bit keys (seed 304; one
    present in the index by chance is simply found)."""
    import datagen
    rng = np.random.default_rng(seed)
    n_abs = int(round(n_total * absent_frac))
    n_pres = n_total - n_abs
    q = np.empty(n_total, np.uint64)
    idx = rng.integers(0, read_keys.size, size=n_pres)
    np.take(np.ascontiguousarray(read_keys, dtype=np.uint64), idx, out=q[:n_pres])
    del idx
    q[n_pres:] = datagen.absent_keys(n_abs)
    return q


def diff_parts(got, want):
    """Indices of the parts whose count or digest differ."""
    return [i for i, (g, w) in enumerate(zip(got["parts"], want["parts"])) if g != w]


def pairs_digest(per_pair):
    """Per-pair outputs (one row per pair, any fixed width of uint32) of the
    seed-matching experiment."""
    a = np.ascontiguousarray(per_pair).astype(np.uint32)
    a = a.reshape(a.shape[0], -1) if a.ndim > 1 else a.reshape(-1, 1)
    n = a.shape[0]
    cut = [i * n // PARTS for i in range(PARTS + 1)]
    parts = [[int(a[cut[i]:cut[i + 1]].astype(np.uint64).sum()), _h(a[cut[i]:cut[i + 1]])[:16]]
             for i in range(PARTS)]
    return dict(n=int(n), sha256=_h(a), parts=parts)
