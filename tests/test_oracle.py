"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published generator outputs, hand-worked examples, closed forms, brute-force
enumeration (tests/brute.py), library routines (numpy sort/searchsorted, Python sets)
and invariants of the definitions (window coverage, the opening identity, strand
symmetry, the expected minimizer density, recovery of the true pattern phase)."""
import os
import zlib

import numpy as np
import pytest

import brute
import datagen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
BASES = {"A": 0, "C": 1, "G": 2, "T": 3}


def codes_of(text):
    return np.array([BASES[c] for c in text], np.uint8)


def one(seq):
    return np.array([0, len(seq)], np.uint64)


# ---------------------------------------------------------------- hash (splitmix64)

def published_vectors():
    out = []
    with open(os.path.join(GOLD, "splitmix64_published.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            seed = int(parts[0], 0)
            out.append((seed, [int(v, 0) for v in parts[1:]]))
    return out


def test_mix64_matches_published_splitmix64():
    for seed, outs in published_vectors():
        state = seed
        for expected in outs:
            state = (state + GAMMA) & M64
            assert oracle.mix64(state) == expected
            assert brute.mix64(state) == expected


def test_mix64_zero_is_fixed_point():
    # every shift-xor and multiply maps 0 to 0: poly-A k-mers always hash to 0
    assert oracle.mix64(0) == 0


# ---------------------------------------------------------------- sparsification

def closed_form_kept(L, pattern, a):
    p, x = len(pattern), pattern.count("1")
    rem = sum(1 for t in range(L % p) if pattern[(t - a) % p] == "1")
    return (L // p) * x + rem


@pytest.mark.parametrize("pattern", ["1", "10", "110", "101", "100", "1110", "11100",
                                     "101001", "1001010011", "0001"])
def test_kept_count_closed_form(pattern):
    for L in list(range(0, 40)) + [1000, 1001, 123457]:
        for a in range(len(pattern)):
            assert oracle.kept_count(L, pattern, a) == closed_form_kept(L, pattern, a)


def test_ceil_form_on_leading_ones_patterns():
    # sparsified length = ceil(L * x / p) holds at shift 0 when the pattern's ones
    # come first; it fails in general ('101' at L = 2 keeps 1 base, ceil gives 2)
    for pattern in ["10", "110", "100", "1110", "1"]:
        p, x = len(pattern), pattern.count("1")
        for L in range(0, 200):
            assert oracle.kept_count(L, pattern, 0) == -(-L * x // p)
    assert oracle.kept_count(2, "101", 0) == 1


def test_sparsify_10_is_every_other_base():
    rng = np.random.default_rng(7)
    s = rng.integers(0, 4, 1001, dtype=np.uint8)
    pc, po, orig = oracle.sparsify(s, one(s), "10")
    assert np.array_equal(pc, s[0::2])
    assert np.array_equal(orig, np.arange(0, 1001, 2))
    pc1, _, orig1 = oracle.sparsify(s, one(s), "10", shifts=[1])
    assert np.array_equal(pc1, s[1::2])
    assert np.array_equal(orig1, np.arange(1, 1001, 2))


def test_sparsify_batch_restarts_phase_per_sequence():
    rng = np.random.default_rng(8)
    lens = [5, 0, 7, 3, 12]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    s = rng.integers(0, 4, offs[-1], dtype=np.uint8)
    shifts = [0, 1, 2, 1, 0]
    pc, po, orig = oracle.sparsify(s, offs, "110", shifts=shifts)
    expect = []
    for i, L in enumerate(lens):
        kp = brute.kept_positions(L, "110", shifts[i])
        expect += [int(s[offs[i] + j]) for j in kp]
        assert po[i + 1] - po[i] == len(kp)
    assert pc.tolist() == expect


# ---------------------------------------------------------------- minimizers

def load_hand_cases():
    cases = []
    with open(os.path.join(GOLD, "hand_minimizers.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split("|")
            seq, pat, shift, k, w = lhs.split()
            recs = []
            for tok in rhs.split():
                hc, val = tok.split(":")
                c = int(hc[2:-1])
                recs.append((brute.mix64(c), int(val)))
            cases.append((seq, pat, int(shift), int(k), int(w), recs))
    return cases


@pytest.mark.parametrize("case", load_hand_cases(), ids=lambda c: "%s-%s-%d" % c[:3])
def test_hand_worked_examples(case):
    seq, pat, shift, k, w, recs = case
    s = codes_of(seq)
    keys, vals, mz = oracle.sketch(s, one(s), pat, k, w, shifts=[shift])
    assert list(zip(keys.tolist(), vals.tolist())) == recs
    assert mz.tolist() == [0, len(recs)]


SWEEP = [("1", 1, 1), ("10", 3, 2), ("110", 4, 3), ("101", 5, 4), ("100", 2, 5), ("1110", 8, 10),
         ("11100", 15, 11), ("101001", 21, 5), ("1001010011", 28, 2), ("1", 32, 40), ("10", 1, 2),
         ("110", 2, 1), ("1", 4, 7), ("10", 6, 3), ("1101", 11, 11)]


@pytest.mark.parametrize("pattern,k,w", SWEEP)
def test_sketch_matches_brute_force(pattern, k, w):
    rng = np.random.default_rng(zlib.crc32(("%s/%d/%d" % (pattern, k, w)).encode()))
    for trial in range(6):
        L = int(rng.integers(0, 260))
        if trial == 0:
            s = np.zeros(L, np.uint8)                  # poly-A: hash-0 ties everywhere
        elif trial == 1:
            s = np.tile(np.array([0, 3], np.uint8), L // 2 + 1)[:L]   # ATAT...: palindromes
        elif trial == 2:
            s = np.tile(rng.integers(0, 4, 3, dtype=np.uint8), L // 3 + 1)[:L]
        else:
            s = rng.integers(0, 4, L, dtype=np.uint8)
        for a in range(len(pattern)):
            keys, vals, mz = oracle.sketch(s, one(s), pattern, k, w, shifts=[a])
            got = list(zip(keys.tolist(), vals.tolist()))
            assert got == brute.sketch(s.tolist(), pattern, a, k, w), (pattern, k, w, a, L)


def test_sketch_batch_equals_per_sequence():
    rng = np.random.default_rng(11)
    lens = [0, 1, 30, 31, 200, 5, 64]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    s = rng.integers(0, 4, offs[-1], dtype=np.uint8)
    shifts = [i % 3 for i in range(len(lens))]
    keys, vals, mz = oracle.sketch(s, offs, "110", 5, 4, shifts=shifts)
    for i in range(len(lens)):
        seg = s[offs[i]:offs[i + 1]]
        exp = brute.sketch(seg.tolist(), "110", shifts[i], 5, 4)
        got = list(zip(keys[mz[i]:mz[i + 1]].tolist(), vals[mz[i]:mz[i + 1]].tolist()))
        assert got == exp


def _patterned_hashes(s, pattern, a, k):
    """Hashes of all patterned k-mers computed by brute force (None for palindromes)."""
    kept = brute.kept_positions(len(s), pattern, a)
    ps = [int(s[j]) for j in kept]
    hs = []
    for i in range(len(ps) - k + 1):
        f = brute.numeral(ps[i:i + k])
        r = brute.numeral([3 - b for b in reversed(ps[i:i + k])])
        hs.append(None if f == r else brute.mix64(min(f, r)))
    return kept, hs


@pytest.mark.parametrize("pattern,k,w", [("10", 15, 10), ("110", 7, 5), ("1", 5, 11)])
def test_window_coverage_and_opening_identity(pattern, k, w):
    rng = np.random.default_rng(12)
    s = rng.integers(0, 4, 3000, dtype=np.uint8)
    keys, vals, _ = oracle.sketch(s, one(s), pattern, k, w)
    kept, hs = _patterned_hashes(s, pattern, 0, k)
    pos_to_i = {o: i for i, o in enumerate(kept)}
    sel = {pos_to_i[int(v) >> 1] for v in vals}
    n = len(hs)
    # coverage: every full window's minimum is attained by a selected k-mer
    for st in range(n - w + 1):
        m = min(h for h in hs[st:st + w] if h is not None)
        assert any(hs[i] == m and i in sel for i in range(st, st + w))
    # opening: selected  <=>  hash equals the max over containing windows of their minima
    for i in range(n):
        if hs[i] is None:
            assert i not in sel
            continue
        wins = range(max(0, i - w + 1), min(i, n - w) + 1)
        opened = max(min(h for h in hs[st:st + w] if h is not None) for st in wins)
        assert (hs[i] == opened) == (i in sel)


@pytest.mark.parametrize("pattern,L", [("1", 2000), ("10", 2001)])
def test_strand_symmetry(pattern, L):
    # with '1' (or '10' on odd L) the kept set maps onto itself under reversal, so the
    # sketch of the reverse complement is the mirror image with flipped strands
    rng = np.random.default_rng(13)
    s = rng.integers(0, 4, L, dtype=np.uint8)
    k, w = 15, 10
    rcs = datagen.revcomp(s)
    k1, v1, _ = oracle.sketch(s, one(s), pattern, k, w)
    k2, v2, _ = oracle.sketch(rcs, one(rcs), pattern, k, w)
    span = (k - 1) * len(pattern) + 1
    mirrored = sorted(((int(kk), ((L - span - (int(v) >> 1)) << 1) | (1 - (int(v) & 1)))
                       for kk, v in zip(k1, v1)), key=lambda t: t[1])
    assert mirrored == list(zip(k2.tolist(), v2.tolist()))


def test_density_and_sparsified_index_size():
    s = datagen.random_genome(1_000_000, 1)
    k, w = 15, 10
    keys, _, _ = oracle.sketch(s, one(s), "10", k, w)
    nk = 500_000 - k + 1
    assert abs(keys.size / (nk * 2.0 / (w + 1)) - 1.0) < 0.02
    full, _, _ = oracle.sketch(s, one(s), "1", k, w)
    # the index shrinks by about the pattern's weight ratio x/p
    assert abs(keys.size / full.size - 0.5) < 0.02


# ---------------------------------------------------------------- index and lookup

@pytest.mark.parametrize("val_bits", [32, 64])
def test_index_is_sorted_sketch(val_bits):
    rng = np.random.default_rng(14)
    lens = [5000, 0, 17, 3000, 1]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    s = rng.integers(0, 4, offs[-1], dtype=np.uint8)
    s[100:400] = s[2000:2300]          # a repeat, so equal keys occur
    ik, iv = oracle.index_build(s, offs, "10", 9, 5, val_bits=val_bits)
    keys, vals, mz = oracle.sketch(s, offs, "10", 9, 5)
    seq = np.repeat(np.arange(len(lens)), np.diff(mz.astype(np.int64)))
    pos, strand = vals >> np.uint64(1), vals & np.uint64(1)
    if val_bits == 32:
        gv = ((offs[seq] + pos) << np.uint64(1)) | strand
    else:
        gv = (seq.astype(np.uint64) << np.uint64(32)) | vals
    order = np.lexsort((gv, keys))
    assert np.array_equal(ik, keys[order]) and np.array_equal(iv, gv[order])
    assert len(np.unique(ik)) < len(ik)


@pytest.mark.parametrize("pattern,k,w", [("10", 15, 10), ("110", 21, 11), ("1", 9, 5),
                                           ("1001010011", 11, 7)])
def test_chunked_index_equals_whole(pattern, k, w):
    # the CPU baseline's many-thread index: chunks with a margin of context, merged by
    # key ranges, equal the index of the whole sequence (chunk edges land everywhere:
    # 37 chunks, a repeat copied across a chunk edge, low-complexity runs)
    rng = np.random.default_rng(16)
    s = rng.integers(0, 4, 60_000, dtype=np.uint8)
    s[10_000:12_000] = s[30_000:32_000]
    s[40_000:40_300] = 0
    ik, iv = oracle.index_build(s, np.array([0, s.size], np.int64), pattern, k, w)
    for threads, chunks in ((3, 37), (4, None), (1, 1)):
        ck, cv = oracle.index_build_chunked(s, pattern, k, w, threads, chunks)
        assert np.array_equal(ck, ik) and np.array_equal(cv, iv), (threads, chunks)


def test_lookup_matches_searchsorted():
    rng = np.random.default_rng(15)
    keys = np.sort(rng.integers(0, 1000, 5000).astype(np.uint64))
    q = np.concatenate([rng.integers(0, 1100, 3000).astype(np.uint64),
                        np.array([0, 999, 1000, 2**64 - 1], np.uint64)])
    lb, occ = oracle.lookup(keys, q)
    assert np.array_equal(lb, np.searchsorted(keys, q, "left"))
    assert np.array_equal(occ, np.searchsorted(keys, q, "right") - np.searchsorted(keys, q, "left"))
    e_lb, e_occ = oracle.lookup(np.zeros(0, np.uint64), q[:3])
    assert e_lb.tolist() == [0, 0, 0] and e_occ.tolist() == [0, 0, 0]


# ---------------------------------------------------------------- pattern alignment, seeding

@pytest.mark.parametrize("pattern,k,w,t,max_occ", [("10", 7, 4, 0, 0), ("110", 5, 3, 0, 0),
                                                     ("101", 6, 2, 3, 0), ("1", 5, 3, 0, 0),
                                                     ("100", 4, 2, 0, 3), ("10", 4, 3, 2, 2),
                                                     ("110", 3, 2, 1, 0)])
def test_seed_matches_brute_force(pattern, k, w, t, max_occ):
    rng = np.random.default_rng(16)
    ref = rng.integers(0, 4, 600, dtype=np.uint8)
    ref[300:360] = ref[50:110]
    ik, iv = oracle.index_build(ref, one(ref), pattern, k, w)
    index = list(zip(ik.tolist(), iv.tolist()))
    reads, lens = [], [40, 0, 3, 77, 25, 60]
    for L in lens:
        st = int(rng.integers(0, 600 - L))
        r = ref[st:st + L].copy()
        if L > 10:
            r[5] = (r[5] + 1) % 4
        if rng.integers(0, 2):
            r = datagen.revcomp(r)
        reads.append(r)
    reads.append(rng.integers(0, 4, 50, dtype=np.uint8))
    offs = np.concatenate([[0], np.cumsum([len(r) for r in reads])]).astype(np.uint64)
    codes = np.concatenate(reads)
    for mode in (-1, 0, len(pattern) - 1):
        a, roff, sh = oracle.seed(ik, iv, codes, offs, pattern, k, w, shift_mode=mode,
                                  align_t=t, max_occ=max_occ)
        exp, exp_sh = brute.seed(index, [r.tolist() for r in reads], pattern, k, w,
                                 shift_mode=mode, t=t, max_occ=max_occ)
        assert [tuple(x) for x in a.tolist()] == exp
        assert sh.tolist() == exp_sh
        assert roff[-1] == len(exp)
        # anchors are in lexicographic (read, qpos, rpos, strand) order by construction
        assert [tuple(x) for x in a.tolist()] == sorted(exp)


def test_pattern_alignment_recovers_true_phase_and_anchor():
    # error-free reads of an i.i.d. reference: the chosen shift is the read's true phase
    # and every read minimizer hits its true location (forward: rpos = g + qpos;
    # reverse: rpos = g + L - qpos - span, strand 1)
    ref = datagen.random_genome(200_000, 21)
    k, w, L = 15, 10, 150
    for pattern in ["10", "110", "100"]:
        p = len(pattern)
        # reflection centre c of the pattern: P[t] == P[(c - t) mod p] for every t; a
        # reverse-strand read from g then carries the phase a = g + L - 1 - c (mod p)
        c = [c for c in range(p) if all(pattern[t] == pattern[(c - t) % p] for t in range(p))][0]
        ik, iv = oracle.index_build(ref, one(ref), pattern, k, w)
        codes, offs, st, sd = datagen.fixed_reads(ref, 60, L, 22, sub=0.0)
        anchors, roff, sh = oracle.seed(ik, iv, codes, offs, pattern, k, w)
        for r in range(60):
            g, strand = int(st[r]), int(sd[r])
            true_a = (-g) % p if strand == 0 else (g + L - 1 - c) % p
            assert sh[r] == true_a, (pattern, r)
            read = codes[offs[r]:offs[r + 1]]
            mk, mv, _ = oracle.sketch(read, one(read), pattern, k, w, shifts=[true_a])
            kept = brute.kept_positions(L, pattern, true_a)
            rows = anchors[roff[r]:roff[r + 1]]
            hits = {(int(q), int(rp), int(s)) for _, q, rp, s in rows}
            assert mv.size > 0
            for v in mv.tolist():
                q = v >> 1
                i = kept.index(q)
                span = kept[i + k - 1] - q + 1
                rp = g + q if strand == 0 else g + L - q - span
                assert (q, rp, strand) in hits


def test_pattern_alignment_tie_and_no_hit_rules():
    # no read minimizer in the index: all scores 0, shift 0
    ref = datagen.random_genome(5000, 31)
    ik, iv = oracle.index_build(ref, one(ref), "110", 11, 5)
    other = datagen.random_genome(300, 32)
    _, _, sh = oracle.seed(ik, iv, other, one(other), "110", 11, 5)
    assert sh.tolist() == [0]


# ---------------------------------------------------------------- containment

def test_contain_matches_python_sets():
    rng = np.random.default_rng(17)
    lens = [3000, 2000, 4000]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    db = rng.integers(0, 4, offs[-1], dtype=np.uint8)
    db[offs[1] + 100:offs[1] + 700] = db[200:800]     # genome 1 shares a block with 0
    k, w, pat = 9, 5, "10"
    ik, iv = oracle.index_build(db, offs, pat, k, w, val_bits=64)
    reads, ro, _ = datagen.sample_from_genomes(db, offs.astype(np.int64), 40, 2, 100, 33, sub=0.0)
    counts, sizes = oracle.contain(ik, iv, reads, ro, pat, k, w, 3)
    _, _, sh = oracle.seed(ik, iv & np.uint64(0xFFFFFFFF), reads, ro, pat, k, w)
    sample = set()
    for r in range(ro.size - 1):
        sample |= {kv[0] for kv in brute.sketch(reads[ro[r]:ro[r + 1]].tolist(), pat, int(sh[r]), k, w)}
    for g in range(3):
        hg = {int(kk) for kk, vv in zip(ik, iv) if int(vv) >> 32 == g}
        assert sizes[g] == len(hg)
        assert counts[g] == len(hg & sample)


# ---------------------------------------------------------------- location voting

def hand_vote_cases():
    cases, cur = [], None
    with open(os.path.join(GOLD, "hand_votes.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "case":
                cur = dict(D=int(line[1]), V=int(line[2]), cap=int(line[3]), anchors=[], expect=[])
                cases.append(cur)
            elif line[0] == "reads":
                cur["reads"] = int(line[1])
            elif line[0] == "anchor":
                cur["anchors"].append([int(v) for v in line[1:]])
            elif line[0] == "expect":
                cur["expect"].append([int(v) for v in line[1:]])
    return cases


def anchors_and_offsets(rows, n_reads):
    a = np.array(rows, np.uint32).reshape(-1, 4)
    counts = np.bincount(a[:, 0], minlength=n_reads) if a.size else np.zeros(n_reads, int)
    off = np.zeros(n_reads + 1, np.uint64)
    off[1:] = np.cumsum(counts)
    return a, off


def test_vote_hand_worked_cases():
    for c in hand_vote_cases():
        a, off = anchors_and_offsets(c["anchors"], c["reads"])
        rows, nw = oracle.vote(a, off, c["D"], c["V"], c["cap"])
        got = [[r] + list(rows[r, i]) for r in range(c["reads"]) for i in range(nw[r])]
        want = [[e[0], e[1], e[2], e[3], e[4]] for e in c["expect"]]
        assert got == want


def brute_votes(rows, D, V, cap):
    """Candidates by repeated minimum over the unsorted anchors of one read (no sort):
    the next temporary location is the smallest location beyond the previous one + D;
    its votes are counted over all anchors of its strand."""
    locs = {0: [], 1: []}
    for q, r, st in rows:
        locs[st].append(r + q if st else r - q)
    cands = []
    for st in (0, 1):
        rest = list(locs[st])
        lo = None
        while True:
            left = [x for x in rest if lo is None or x > lo + D]
            if not left:
                break
            lo = min(left)
            votes = sum(1 for x in locs[st] if lo <= x <= lo + D)
            cands.append((st, lo, votes))
    wins = sorted([c for c in cands if c[2] >= V], key=lambda c: (-c[2], c[0], c[1]))[:cap]
    if wins:
        return [(st, v, 0, lo) for st, lo, v in wins]
    if not cands:
        return []
    best = max(c[2] for c in cands)
    st, lo, v = min(c for c in cands if c[2] == best)
    return [(st, v, 1, lo)]


@pytest.mark.parametrize("D,V,cap", [(0, 1, 4), (3, 2, 2), (10, 3, 8), (50, 1, 1), (5, 100, 3)])
def test_vote_matches_repeated_minimum_brute_force(D, V, cap):
    rng = np.random.default_rng(7 + D + V)
    reads = []
    for r in range(300):
        m = int(rng.integers(0, 25))
        base = int(rng.integers(100, 10_000))
        rows = []
        for _ in range(m):
            q = int(rng.integers(0, 150))
            st = int(rng.integers(0, 2))
            if rng.random() < 0.6:          # on a true diagonal, with small indel drift
                r_ = (base + q if st == 0 else base - q) + int(rng.integers(-2, 3))
            else:
                r_ = int(rng.integers(200, 20_000))
            rows.append((q, max(r_, 0), st))
        rows.sort()                          # (qpos, rpos) order, as the seeder emits them
        reads.append(rows)
    flat = [[i, q, r_, st] for i, rows in enumerate(reads) for q, r_, st in rows]
    a, off = anchors_and_offsets(flat, len(reads))
    out, nw = oracle.vote(a, off, D, V, cap)
    for i, rows in enumerate(reads):
        want = brute_votes(rows, D, V, cap)
        got = [tuple(int(v) for v in out[i, j]) for j in range(nw[i])]
        assert got == want, (i, rows)


def test_vote_ignores_anchor_order_and_counts_exact_reads():
    rng = np.random.default_rng(11)
    rows = [[0, q, 5000 + q, 0] for q in range(0, 150, 7)] + [[0, 3, 90_000, 1]]
    a, off = anchors_and_offsets(rows, 1)
    out, nw = oracle.vote(a, off, 8, 3, 4)
    assert nw[0] == 1 and list(out[0, 0]) == [0, len(rows) - 1, 0, 5000]
    perm = a[rng.permutation(len(rows))]
    out2, nw2 = oracle.vote(perm, off, 8, 3, 4)
    assert np.array_equal(out, out2) and np.array_equal(nw, nw2)


# ---------------------------------------------------------------- Wang's hash (paper form)

@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_wang_hash_permutes_the_code_space(k):
    n = 4 ** k
    out = {oracle.wang64(x, k) for x in range(n)}
    assert out == set(range(n))


def test_wang_hash_matches_the_shift_and_add_form():
    rng = np.random.default_rng(5)
    for k in (4, 11, 15, 21, 31, 32):
        for x in rng.integers(0, 4 ** k if k < 32 else 2**63, 200, dtype=np.uint64):
            assert oracle.wang64(int(x), k) == brute.wang64(int(x), k)


@pytest.mark.parametrize("pattern,k,w", [("10", 5, 4), ("110", 4, 3), ("1", 7, 5), ("101001", 3, 6)])
def test_wang_sketch_matches_brute_force(pattern, k, w):
    rng = np.random.default_rng(len(pattern) * 7 + k)
    for _ in range(20):
        seq = rng.integers(0, 4, int(rng.integers(0, 90)), dtype=np.uint8)
        for shift in range(len(pattern)):
            with oracle.use_hash("wang"):
                keys, vals, _ = oracle.sketch(seq, one(seq), pattern, k, w,
                                              shifts=np.array([shift], np.uint32))
            want = brute.sketch(list(seq), pattern, shift, k, w, hash="wang")
            assert list(zip(keys.tolist(), vals.tolist())) == want


# ---------------------------------------------------------------- ambiguous bases (N)

def with_ns(rng, L, runs=2, singles=3):
    s = rng.integers(0, 4, L, dtype=np.uint8)
    for _ in range(singles if L else 0):
        s[int(rng.integers(0, L))] = 4
    for _ in range(runs if L > 10 else 0):
        a = int(rng.integers(0, L - 5))
        s[a:a + int(rng.integers(1, 12))] = 4
    return s


@pytest.mark.parametrize("pattern,k,w", [("1", 5, 4), ("10", 4, 3), ("110", 3, 5), ("101001", 3, 2),
                                         ("1", 2, 1), ("100", 6, 7)])
def test_n_sketch_matches_brute_force(pattern, k, w):
    # brute force: a k-mer holding an N is no k-mer, a window over any N is no window
    rng = np.random.default_rng(k * 31 + w)
    for _ in range(25):
        seq = with_ns(rng, int(rng.integers(0, 120)))
        for shift in range(len(pattern)):
            keys, vals, _ = oracle.sketch(seq, one(seq), pattern, k, w,
                                          shifts=np.array([shift], np.uint32))
            want = brute.sketch(list(seq), pattern, shift, k, w)
            assert list(zip(keys.tolist(), vals.tolist())) == want


def test_n_at_a_dropped_position_changes_nothing():
    rng = np.random.default_rng(40)
    seq = rng.integers(0, 4, 3000, dtype=np.uint8)
    for pattern, shift in [("10", 0), ("10", 1), ("110", 2), ("1001", 1)]:
        dropped = [j for j in range(seq.size) if pattern[(j - shift) % len(pattern)] == "0"]
        s2 = seq.copy()
        s2[rng.choice(dropped, 200, replace=False)] = 4
        sh = np.array([shift], np.uint32)
        a = oracle.sketch(seq, one(seq), pattern, 11, 7, shifts=sh)
        b = oracle.sketch(s2, one(s2), pattern, 11, 7, shifts=sh)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_kept_n_splits_the_sequence_in_two():
    # X + N + Y with the N kept sketches as X, then Y alone under the phase Y has in place
    rng = np.random.default_rng(41)
    for pattern, k, w in [("10", 9, 5), ("110", 7, 4), ("1", 8, 6), ("1011", 5, 3)]:
        p = len(pattern)
        for _ in range(20):
            L1 = int(rng.integers(0, 200))
            a = int(rng.integers(0, p))
            if pattern[(L1 - a) % p] != "1":
                continue
            x = rng.integers(0, 4, L1, dtype=np.uint8)
            y = rng.integers(0, 4, int(rng.integers(0, 200)), dtype=np.uint8)
            xy = np.concatenate([x, [4], y]).astype(np.uint8)
            got = oracle.sketch(xy, one(xy), pattern, k, w, shifts=np.array([a], np.uint32))
            kx, vx, _ = oracle.sketch(x, one(x), pattern, k, w, shifts=np.array([a], np.uint32))
            ay = (a - L1 - 1) % p
            ky, vy, _ = oracle.sketch(y, one(y), pattern, k, w, shifts=np.array([ay], np.uint32))
            assert np.array_equal(got[0], np.concatenate([kx, ky]))
            assert np.array_equal(got[1], np.concatenate([vx, vy + (np.uint64(L1 + 1) << 1)]))


def test_all_n_and_short_runs_give_nothing():
    s = np.full(500, 4, np.uint8)
    s[::7] = 1                                  # runs of one base between Ns
    for pattern in ("1", "10"):
        keys, _, mz = oracle.sketch(s, one(s), pattern, 3, 2)
        assert keys.size == 0 and mz.tolist() == [0, 0]


@pytest.mark.parametrize("pattern,k,w", [("10", 5, 3), ("110", 4, 2), ("1", 6, 4)])
def test_n_seed_matches_brute_force(pattern, k, w):
    rng = np.random.default_rng(17)
    ref = with_ns(rng, 700, runs=3, singles=10)
    ik, iv = oracle.index_build(ref, one(ref), pattern, k, w)
    index = list(zip(ik.tolist(), iv.tolist()))
    reads = []
    for L in (60, 45, 0, 90, 30):
        st = int(rng.integers(0, 700 - L))
        r = ref[st:st + L].copy()
        if L > 20:
            r[int(rng.integers(0, L))] = 4
        reads.append(r)
    offs = np.concatenate([[0], np.cumsum([len(r) for r in reads])]).astype(np.uint64)
    codes = np.concatenate(reads)
    a, _, sh = oracle.seed(ik, iv, codes, offs, pattern, k, w)
    exp, exp_sh = brute.seed(index, [r.tolist() for r in reads], pattern, k, w)
    assert [tuple(x) for x in a.tolist()] == exp and sh.tolist() == exp_sh
    assert len(exp) > 20


# ---------------------------------------------------------------- seed-matching experiment

def test_edit_distance_matches_recursion():
    rng = np.random.default_rng(50)
    for _ in range(300):
        a = rng.integers(0, 4, int(rng.integers(0, 8)), dtype=np.uint8)
        b = rng.integers(0, 4, int(rng.integers(0, 8)), dtype=np.uint8)
        assert oracle.edit_distance(a, b) == brute.edit_distance(tuple(a), tuple(b))


def test_edit_distance_properties():
    rng = np.random.default_rng(51)
    for _ in range(40):
        a = rng.integers(0, 4, int(rng.integers(0, 300)), dtype=np.uint8)
        b = rng.integers(0, 4, int(rng.integers(0, 300)), dtype=np.uint8)
        c = rng.integers(0, 4, int(rng.integers(0, 300)), dtype=np.uint8)
        dab = oracle.edit_distance(a, b)
        assert oracle.edit_distance(a, a) == 0
        assert dab == oracle.edit_distance(b, a)
        assert abs(a.size - b.size) <= dab <= max(a.size, b.size)
        assert oracle.edit_distance(a, c) <= dab + oracle.edit_distance(b, c)
        if a.size:
            i = int(rng.integers(0, a.size))
            assert oracle.edit_distance(a, np.delete(a, i)) == 1
            s = a.copy()
            s[i] = (s[i] + 1) % 4
            assert oracle.edit_distance(a, s) == 1
            m = a.copy()
            pos = rng.choice(a.size, min(a.size, 30), replace=False)
            m[pos] = (m[pos] + rng.integers(1, 4, pos.size)) % 4
            assert oracle.edit_distance(a, m) <= pos.size      # at most the Hamming distance


FIG4 = [("110", 8, 6), ("10", 8, 6), ("101001", 8, 6), ("100", 8, 6), ("10", 13, 9),
        ("1110110110111", 13, 9), ("111001011001010111", 18, 12), ("10", 21, 11)]


@pytest.mark.parametrize("pattern,k,w", FIG4)
def test_seed_match_matches_brute_force(pattern, k, w):
    rng = np.random.default_rng(k * 7 + len(pattern))
    pairs = []
    for L in (0, k - 1, k, 60, 200, 200):
        a = rng.integers(0, 4, L, dtype=np.uint8)
        b = a.copy()
        if L:
            pos = rng.choice(L, int(rng.integers(0, L // 3 + 1)), replace=False)
            b[pos] = (b[pos] + rng.integers(1, 4, pos.size)) % 4
        pairs.append((a, b))
    ca, oa = datagen.concat([(a, [0, a.size]) for a, _ in pairs])
    cb, ob = datagen.concat([(b, [0, b.size]) for _, b in pairs])
    got = oracle.seed_match(ca, oa, cb, ob, pattern, k, w)
    for i, (a, b) in enumerate(pairs):
        for g, alg in enumerate(oracle.FIG4_ALGORITHMS):
            assert tuple(got[i, g]) == brute.seed_match(a, b, alg, pattern, k, w), (i, alg)


def test_seed_match_identity_and_reductions():
    rng = np.random.default_rng(52)
    a = rng.integers(0, 4, 1000, dtype=np.uint8)
    b = a.copy()
    b[rng.choice(1000, 150, replace=False)] = rng.integers(0, 4, 150)
    o = [0, 1000]
    same = oracle.seed_match(a, o, a, o, "101001", 8, 6)[0]
    assert np.array_equal(same[:, 0], same[:, 1])             # every seed matches itself
    assert same[0, 1] == same[2, 1] == 1000 - 8 + 1            # all and spaced: every start
    one = oracle.seed_match(a, o, b, o, "1", 8, 6)[0]
    assert np.array_equal(one[0], one[2])                     # spaced with '1' = all seeds
    assert np.array_equal(one[1], one[3])                     # GoD with '1' = minimizers


def test_accepted_pairs_by_definition():
    from fractions import Fraction
    rng = np.random.default_rng(53)
    n = 300
    dist = rng.integers(0, 60, n).astype(np.uint32)
    total = rng.integers(0, 50, n).astype(np.uint32)
    matched = (total * rng.random(n)).astype(np.uint32)
    got = oracle.accepted(dist, matched, total, 70)
    rate = [Fraction(int(m), int(t)) if t else Fraction(0) for m, t in zip(matched, total)]
    for E in range(71):
        close = [rate[i] for i in range(n) if dist[i] <= E]
        want = sum(1 for r in rate if r >= min(close)) if close else 0
        assert got[E] == want
    assert got[-1] == n                                       # every pair is close enough



# ---------------------------------------------------------------- patterns longer than 64

def long_pattern(seed, p, density):
    rng = np.random.default_rng(seed)
    bits = rng.random(p) < density
    bits[int(rng.integers(0, p))] = True
    return "".join("1" if b else "0" for b in bits)


LONG = [long_pattern(1, 65, 0.5), long_pattern(2, 100, 0.7), long_pattern(3, 129, 0.1),
        long_pattern(4, 200, 0.5), "1" * 256, "0" * 255 + "1"]


@pytest.mark.parametrize("pattern", LONG)
def test_long_pattern_kept_count(pattern):
    p = len(pattern)
    rng = np.random.default_rng(p)
    for L in [0, 1, p - 1, p, p + 1, 3 * p + 7, 5000] + rng.integers(0, 3000, 10).tolist():
        for a in [0, 1, p // 2, p - 1]:
            assert oracle.kept_count(L, pattern, a) == closed_form_kept(L, pattern, a)


@pytest.mark.parametrize("pattern,k,w", [(LONG[0], 7, 5), (LONG[1], 11, 3), (LONG[2], 3, 2),
                                         (LONG[3], 9, 9), (LONG[4], 15, 4)])
def test_long_pattern_sketch_matches_brute_force(pattern, k, w):
    p = len(pattern)
    rng = np.random.default_rng(p + k)
    for L in (0, 50, 700, 1500):
        s = rng.integers(0, 4, L, dtype=np.uint8)
        for a in sorted({0, 1, p // 3, p - 1, int(rng.integers(0, p))}):
            keys, vals, _ = oracle.sketch(s, one(s), pattern, k, w, shifts=[a])
            assert list(zip(keys.tolist(), vals.tolist())) == brute.sketch(s.tolist(), pattern,
                                                                          a, k, w)


def test_pattern_of_257_is_rejected():
    assert oracle.kept_count(10, "1" * 257, 0) == 2**64 - 1
    with pytest.raises(RuntimeError):
        oracle.sketch(np.zeros(5, np.uint8), [0, 5], "1" * 257, 3, 2)
