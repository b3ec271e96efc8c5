"""Brute-force reference for tiny inputs, written from the definitions with Python
strings, sets and list slicing (shares nothing with the C oracle or the GPU library).

It enumerates every window explicitly and marks every k-mer attaining its minimum; k-mer
codes are read as base-4 numerals with int(text, 4); the reverse complement is built by
reversing and complementing the base list."""

MASK = (1 << 64) - 1


def mix64(z):
    # splitmix64 output function; pinned separately against the published generator
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


N = 4                                      # code of the ambiguous base


def wang64(key, k):
    # Thomas Wang's 64-bit integer hash in its published shift-and-add form, each step
    # reduced to the 2k-bit code space (the oracle writes the same steps as products)
    m = (1 << (2 * k)) - 1 if k < 32 else MASK
    key = ((~key & MASK) + (key << 21)) & m
    key = key ^ (key >> 24)
    key = ((key + (key << 3)) + (key << 8)) & m
    key = key ^ (key >> 14)
    key = ((key + (key << 2)) + (key << 4)) & m
    key = key ^ (key >> 28)
    key = (key + (key << 31)) & m
    return key


def kept_positions(length, pattern, shift):
    p = len(pattern)
    return [j for j in range(length) if pattern[(j - shift) % p] == "1"]


def numeral(bases):
    return int("".join("0123"[b] for b in bases), 4) if bases else 0


def sketch(seq, pattern, shift, k, w, hash="splitmix64"):
    """List of (key, val = orig << 1 | strand) in ascending k-mer order."""
    hf = (lambda c: wang64(c, k)) if hash == "wang" else mix64
    kept = kept_positions(len(seq), pattern, shift)
    ps = [int(seq[j]) for j in kept]
    ent = []
    for i in range(len(ps) - k + 1):
        kmer = ps[i:i + k]
        if N in kmer:                      # no k-mer holds the ambiguous base
            ent.append(None)
            continue
        f = numeral(kmer)
        r = numeral([3 - b for b in reversed(kmer)])
        ent.append(None if f == r else (hf(min(f, r)), 1 if r < f else 0))
    chosen = set()
    for s in range(len(ent) - w + 1):
        if N in ps[s:s + w + k - 1]:       # a window never spans an N
            continue
        hs = [e[0] for e in ent[s:s + w] if e is not None]
        if not hs:
            continue
        m = min(hs)
        for i in range(s, s + w):
            if ent[i] is not None and ent[i][0] == m:
                chosen.add(i)
    return [(ent[i][0], (kept[i] << 1) | ent[i][1]) for i in sorted(chosen)]


def occ(index_keys, q):
    return sum(1 for x in index_keys if x == q)


def align(seq, pattern, k, w, index_keys, t=0, max_occ=0):
    p = len(pattern)
    if p == 1:
        return 0
    ms = [sketch(seq, pattern, s, k, w) for s in range(p)]
    nstar = min(len(m) for m in ms)
    if t > 0:
        nstar = min(nstar, t)
    scores = []
    for m in ms:
        sc = 0
        for key, _ in m[:nstar]:
            o = occ(index_keys, key)
            if max_occ == 0 or o < max_occ:
                sc += o
        scores.append(sc)
    best = max(scores)
    return scores.index(best) if best > 0 else 0


def seed(index, reads, pattern, k, w, shift_mode=-1, t=0, max_occ=0):
    """index: list of (key, val) sorted; reads: list of code lists.
    Returns (anchors list of tuples, shifts)."""
    keys = [kv[0] for kv in index]
    out, shifts = [], []
    for r, seq in enumerate(reads):
        a = shift_mode if shift_mode >= 0 else align(seq, pattern, k, w, keys, t, max_occ)
        shifts.append(a)
        for key, val in sketch(seq, pattern, a, k, w):
            hits = [iv for ik, iv in index if ik == key]
            if max_occ and len(hits) >= max_occ:
                continue
            for iv in sorted(hits):
                out.append((r, val >> 1, iv >> 1, (val ^ iv) & 1))
    return out, shifts


def canonical(bases):
    return min(numeral(bases), numeral([3 - b for b in reversed(bases)]))


def fig4_seeds(seq, alg, pattern, k, w):
    """Seed identities of one sequence for the seed-matching experiment: all k-mers,
    minimizers, spaced seeds (pattern repeated to span k) or Genome-on-Diet minimizers."""
    seq = [int(b) for b in seq]
    if alg == "all":
        return [canonical(seq[i:i + k]) for i in range(len(seq) - k + 1)]
    if alg == "spaced":
        mask = [pattern[j % len(pattern)] == "1" for j in range(k)]
        return [canonical([seq[i + j] for j in range(k) if mask[j]])
                for i in range(len(seq) - k + 1)]
    return [key for key, _ in sketch(seq, "1" if alg == "minimizers" else pattern, 0, k, w)]


def seed_match(orig, copy, alg, pattern, k, w):
    stored = set(fig4_seeds(orig, alg, pattern, k, w))
    seeds = fig4_seeds(copy, alg, pattern, k, w)
    return sum(1 for s in seeds if s in stored), len(seeds)


def edit_distance(a, b):
    """Levenshtein distance by plain recursion with memoisation (tiny inputs only)."""
    from functools import lru_cache

    @lru_cache(maxsize=None)
    def d(i, j):
        if i == 0:
            return j
        if j == 0:
            return i
        return min(d(i - 1, j) + 1, d(i, j - 1) + 1, d(i - 1, j - 1) + (a[i - 1] != b[j - 1]))

    return d(len(a), len(b))
