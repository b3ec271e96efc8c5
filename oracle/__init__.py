"""Plain CPU oracle of the Genome-on-Diet sparsified-seeding hot path (arXiv 2211.08157).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the GPU library never does, and the two share no
code (they meet only in the seeded inputs of ``datagen``).

The arithmetic lives in ``godiet_oracle.c`` (plain C, one sequence at a time, every
k-mer code and window minimum recomputed from its definition).  This module only builds
that file with gcc, loads it with ctypes and marshals numpy arrays.

Sequences are given as one base code per byte (A=0, C=1, G=2, T=3) with n_seq+1 offsets.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "godiet_oracle.c")
_LIB = os.path.join(_HERE, "libgodiet_oracle.so")

ECAP = -2


def build(force=True):
    """Compile the oracle with gcc (-O2, no intrinsics)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("GODIET_ORACLE_LIB")
        if override:
            # a separately built copy (tests/oracle_mutants.py loads planted-mistake builds)
            L = ctypes.CDLL(override)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
        L.gdo_mix64.argtypes = [u64]
        L.gdo_mix64.restype = u64
        L.gdo_kept_count.argtypes = [u64, ctypes.c_char_p, u32]
        L.gdo_kept_count.restype = u64
        L.gdo_sparsify.argtypes = [P, P, u32, ctypes.c_char_p, P, P, P, P]
        L.gdo_sparsify.restype = i64
        L.gdo_sketch.argtypes = [P, P, u32, ctypes.c_char_p, P, i32, i32, P, P, P, u64]
        L.gdo_sketch.restype = i64
        L.gdo_index_build.argtypes = [P, P, u32, ctypes.c_char_p, i32, i32, i32, P, P, u64]
        L.gdo_index_build.restype = i64
        L.gdo_lookup.argtypes = [P, u64, P, u64, P, P]
        L.gdo_lookup.restype = None
        L.gdo_seed.argtypes = [P, P, u64, P, P, u32, ctypes.c_char_p, i32, i32, i32, u32, u32,
                               P, u64, P, P]
        L.gdo_seed.restype = i64
        L.gdo_contain.argtypes = [P, P, u64, P, P, u32, ctypes.c_char_p, i32, i32, i32, u32, u32,
                                  u32, P, P]
        L.gdo_contain.restype = i64
        L.gdo_vote.argtypes = [P, P, u32, u32, u32, u32, P, P]
        L.gdo_vote.restype = i64
        L.gdo_wang64.argtypes = [u64, i32]
        L.gdo_wang64.restype = u64
        L.gdo_set_hash.argtypes = [i32]
        L.gdo_seed_match.argtypes = [P, P, P, P, u32, ctypes.c_char_p, i32, i32, P]
        L.gdo_seed_match.restype = i32
        L.gdo_edit_distance.argtypes = [P, u64, P, u64]
        L.gdo_edit_distance.restype = u64
        L.gdo_accepted.argtypes = [P, P, P, u32, u32, P]
        L.gdo_accepted.restype = None
        L.gdo_set_hash.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _codes(codes, offsets):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if codes.size and codes.max() > 4:
        raise ValueError("base codes must be 0..3, or 4 for the ambiguous base N")
    return codes, offsets


def _check(r, what):
    if r < 0:
        raise RuntimeError("oracle %s failed with code %d" % (what, r))
    return r


def mix64(z):
    return int(lib().gdo_mix64(int(z) & (2**64 - 1)))


def kept_count(length, pattern, shift=0):
    return int(lib().gdo_kept_count(int(length), pattern.encode(), int(shift)))


def sparsify(codes, offsets, pattern, shifts=None):
    """Returns (patterned codes, patterned offsets, original coordinate of each kept base)."""
    codes, offsets = _codes(codes, offsets)
    n_seq = offsets.size - 1
    sh = None if shifts is None else np.ascontiguousarray(shifts, dtype=np.uint32)
    out = np.zeros(max(codes.size, 1), np.uint8)
    oofs = np.zeros(n_seq + 1, np.uint64)
    orig = np.zeros(max(codes.size, 1), np.uint64)
    n = _check(lib().gdo_sparsify(_ptr(codes), _ptr(offsets), n_seq, pattern.encode(), _ptr(sh),
                                  _ptr(out), _ptr(oofs), _ptr(orig)), "sparsify")
    return out[:n].copy(), oofs, orig[:n].copy()


def sketch(codes, offsets, pattern, k, w, shifts=None):
    """Minimizers of every sequence: (keys u64, vals u64 = pos<<1|strand, offsets[n_seq+1])."""
    codes, offsets = _codes(codes, offsets)
    n_seq = offsets.size - 1
    sh = None if shifts is None else np.ascontiguousarray(shifts, dtype=np.uint32)
    cap = max(codes.size, 1)
    keys = np.zeros(cap, np.uint64)
    vals = np.zeros(cap, np.uint64)
    mz = np.zeros(n_seq + 1, np.uint64)
    n = _check(lib().gdo_sketch(_ptr(codes), _ptr(offsets), n_seq, pattern.encode(), _ptr(sh),
                                k, w, _ptr(keys), _ptr(vals), _ptr(mz), cap), "sketch")
    return keys[:n].copy(), vals[:n].copy(), mz


def index_build(codes, offsets, pattern, k, w, val_bits=32):
    """Sorted seed index: (keys u64, vals u64) sorted by (key, val)."""
    codes, offsets = _codes(codes, offsets)
    n_seq = offsets.size - 1
    cap = max(codes.size, 1)
    keys = np.zeros(cap, np.uint64)
    vals = np.zeros(cap, np.uint64)
    n = _check(lib().gdo_index_build(_ptr(codes), _ptr(offsets), n_seq, pattern.encode(), k, w,
                                     val_bits, _ptr(keys), _ptr(vals), cap), "index_build")
    return keys[:n].copy(), vals[:n].copy()


def chunk_margin(pattern, k, w):
    """Original bases on each side of a chunk that decide its minimizers: a k-mer at kept
    position i is selected through the windows starting at i - w + 1 .. i, whose k-mers
    cover kept positions i - w + 1 .. i + w + k - 2; w + k kept bases lie within
    ceil((w + k) / x) + 1 periods.  A whole number of periods, so a chunk keeps the
    sequence's pattern phase."""
    p, x = len(pattern), pattern.count("1")
    return p * (-(-(w + k) // x) + 2)


def index_build_chunked(codes, pattern, k, w, threads, n_chunks=None):
    """The seed index of ONE sequence built chunk by chunk on `threads` threads (harness
    around index_build; the arithmetic is the oracle's): chunk c covers original
    positions [a_c, b_c) (multiples of the period), is indexed as a sequence of its own
    with chunk_margin() bases of context on both sides, and keeps the records whose
    position lies in [a_c, b_c).  The sorted chunks are then merged by key ranges on the
    threads (every chunk holds smaller positions than the next, so a stable sort by key
    of the chunks in order is the (key, value) order).  32-bit values."""
    from concurrent.futures import ThreadPoolExecutor
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    L = codes.size
    p = len(pattern)
    h = chunk_margin(pattern, k, w)
    n_chunks = n_chunks or 4 * threads
    step = max(p, -(-L // n_chunks) // p * p)
    bounds = list(range(0, L, step)) + [L]

    def one(c):
        a, b = bounds[c], bounds[c + 1]
        lo, hi = max(0, a - h), min(L, b + h)
        ik, iv = index_build(codes[lo:hi], np.array([0, hi - lo], np.int64), pattern, k, w)
        iv = iv + np.uint64(2 * lo)
        pos = iv >> np.uint64(1)
        keep = (pos >= np.uint64(a)) & (pos < np.uint64(b))
        return ik[keep], iv[keep]

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, range(len(bounds) - 1)))
    # key-range merge: cut points from one chunk's keys, each range sorted on a thread
    cuts = np.unique(np.quantile(np.concatenate([pk[::max(1, pk.size // 64)] for pk, _ in parts]
                                                + [np.zeros(1, np.uint64)]).astype(np.float64),
                                 np.linspace(0, 1, threads + 1)[1:-1]).astype(np.uint64))
    ranges = [[np.searchsorted(pk, cuts) for pk, _ in parts]]

    def merge(r):
        ks, vs = [], []
        for (pk, pv), idx in zip(parts, ranges[0]):
            lo = idx[r - 1] if r > 0 else 0
            hi = idx[r] if r < idx.size else pk.size
            ks.append(pk[lo:hi])
            vs.append(pv[lo:hi])
        kk = np.concatenate(ks)
        vv = np.concatenate(vs)
        order = np.argsort(kk, kind="stable")
        return kk[order], vv[order]

    with ThreadPoolExecutor(max_workers=threads) as ex:
        out = list(ex.map(merge, range(cuts.size + 1)))
    return np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out])


def lookup(keys, queries):
    """(lb, occ) of every query in the sorted key array."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    q = np.ascontiguousarray(queries, dtype=np.uint64)
    lb = np.zeros(q.size, np.uint64)
    occ = np.zeros(q.size, np.uint64)
    lib().gdo_lookup(_ptr(keys), keys.size, _ptr(q), q.size, _ptr(lb), _ptr(occ))
    return lb, occ


def seed(ikeys, ivals, codes, offsets, pattern, k, w, shift_mode=-1, align_t=0, max_occ=0,
         capacity=None):
    """Pattern alignment + compressed seeding.  Returns (anchors (n,4) uint32 rows of
    read_id, qpos, rpos, strand; read_off[n_reads+1]; shift[n_reads])."""
    ikeys = np.ascontiguousarray(ikeys, dtype=np.uint64)
    ivals = np.ascontiguousarray(ivals, dtype=np.uint64)
    codes, offsets = _codes(codes, offsets)
    n_reads = offsets.size - 1
    cap = capacity if capacity is not None else max(1024, 4 * codes.size)
    while True:
        anchors = np.zeros((cap, 4), np.uint32)
        roff = np.zeros(n_reads + 1, np.uint64)
        shift = np.zeros(max(n_reads, 1), np.uint32)
        n = lib().gdo_seed(_ptr(ikeys), _ptr(ivals), ikeys.size, _ptr(codes), _ptr(offsets),
                           n_reads, pattern.encode(), k, w, shift_mode, align_t, max_occ,
                           _ptr(anchors), cap, _ptr(roff), _ptr(shift))
        if n == ECAP and capacity is None:
            cap *= 4
            continue
        _check(n, "seed")
        return anchors[:n].copy(), roff, shift[:n_reads].copy()


def contain(ikeys, ivals, codes, offsets, pattern, k, w, n_genomes, shift_mode=-1, align_t=0,
            max_occ=0):
    """Per-genome shared distinct minimizer counts: (counts[n_genomes], sizes[n_genomes])."""
    ikeys = np.ascontiguousarray(ikeys, dtype=np.uint64)
    ivals = np.ascontiguousarray(ivals, dtype=np.uint64)
    codes, offsets = _codes(codes, offsets)
    counts = np.zeros(n_genomes, np.uint32)
    sizes = np.zeros(n_genomes, np.uint32)
    _check(lib().gdo_contain(_ptr(ikeys), _ptr(ivals), ikeys.size, _ptr(codes), _ptr(offsets),
                             offsets.size - 1, pattern.encode(), k, w, shift_mode, align_t,
                             max_occ, n_genomes, _ptr(counts), _ptr(sizes)), "contain")
    return counts, sizes


def vote(anchors, read_off, max_dist, min_votes, max_win):
    """Location voting (Illumina form) with rescue.  anchors: (n, 4) uint32 rows of
    (read_id, qpos, rpos, strand) grouped by read; read_off[n_reads+1].  Returns (rows
    (n_reads, max_win, 4) int64 of (strand, votes, flags, loc), n_win[n_reads])."""
    a = np.ascontiguousarray(anchors, dtype=np.uint32).reshape(-1, 4)
    off = np.ascontiguousarray(read_off, dtype=np.uint64)
    n_reads = off.size - 1
    out = np.zeros((max(n_reads, 1), max_win, 4), np.int64)
    nw = np.zeros(max(n_reads, 1), np.uint32)
    _check(lib().gdo_vote(_ptr(a), _ptr(off), n_reads, int(max_dist), int(min_votes),
                          int(max_win), _ptr(out), _ptr(nw)), "vote")
    return out[:n_reads], nw[:n_reads]


def wang64(key, k):
    return int(lib().gdo_wang64(int(key) & (2**64 - 1), int(k)))


class use_hash:
    """Context manager selecting the k-mer hash of the oracle's sketches:
    with oracle.use_hash("wang"): ..."""

    def __init__(self, name):
        self.kind = {"splitmix64": 0, "wang": 1}[name]

    def __enter__(self):
        _check(lib().gdo_set_hash(self.kind), "set_hash")
        return self

    def __exit__(self, *exc):
        lib().gdo_set_hash(0)
        return False


FIG4_ALGORITHMS = ("all", "minimizers", "spaced", "god")


def seed_match(codes_a, offs_a, codes_b, offs_b, pattern, k, w):
    """Seed matching of pairs (sequence i of a = original, of b = mutated copy): uint32
    array (n_pairs, 4, 2) of (matched seeds of the copy, seeds of the copy) for the
    algorithms FIG4_ALGORITHMS."""
    ca, oa = _codes(codes_a, offs_a)
    cb, ob = _codes(codes_b, offs_b)
    n = oa.size - 1
    if ob.size - 1 != n:
        raise ValueError("both batches need the same number of sequences")
    out = np.zeros((max(n, 1), 4, 2), np.uint32)
    _check(lib().gdo_seed_match(_ptr(ca), _ptr(oa), _ptr(cb), _ptr(ob), n, pattern.encode(),
                                k, w, _ptr(out)), "seed_match")
    return out[:n]


def edit_distance(a, b):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    return int(lib().gdo_edit_distance(_ptr(a), a.size, _ptr(b), b.size))


def accepted(dist, matched, total, max_e):
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    m = np.ascontiguousarray(matched, dtype=np.uint32)
    t = np.ascontiguousarray(total, dtype=np.uint32)
    out = np.zeros(max_e + 1, np.uint32)
    lib().gdo_accepted(_ptr(d), _ptr(m), _ptr(t), d.size, max_e, _ptr(out))
    return out
