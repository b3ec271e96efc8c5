"""GPU parity on windows whose hashes tie in their high 32 bits.

For w = 3..17 the sketch selects minimizers on the hashes' high words first and falls back
to the full hashes when two consecutive selected positions share the high word with
different hashes.  Random inputs essentially never produce such a tie (about one window
in 10^9), so these inputs are built to: two 21-mers that overlap by 5 bases and whose
canonical codes hash to equal high words (found by a birthday search over 2^19 x 2^19
candidates), with the smallest such high word, so that both attain the high-word minimum
of the window that holds them.  They are placed inside one tile, across a tile boundary
(the first in the chunk before a tile's owned range, the second in it) and at a
sequence's start; every output is compared with the oracle, which compares full hashes.

The hash below is only the input search's own splitmix64 (it is checked against the
oracle's); the expected outputs come from the oracle alone."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
K = 21
OVERLAP = 5
FREE = K - OVERLAP            # 16 free bases on each side: the two starts are 16 apart
M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def mix(z):
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
    return z ^ (z >> np.uint64(31))


def canon(bases):
    """Canonical 2k-bit codes of rows of k base codes (first base most significant)."""
    w = np.uint64(4) ** np.arange(K - 1, -1, -1, dtype=np.uint64)
    fwd = (bases.astype(np.uint64) * w).sum(axis=1, dtype=np.uint64)
    rc = ((3 - bases[:, ::-1]).astype(np.uint64) * w).sum(axis=1, dtype=np.uint64)
    return np.minimum(fwd, rc)


def colliding_37mer():
    """A 37-base sequence whose 21-mers at offsets 0 and 16 have different canonical codes
    with equal hash high words, the smallest such high word found."""
    rng = np.random.default_rng(2024)
    n = 1 << 19
    ov = rng.integers(0, 4, OVERLAP, dtype=np.uint8)
    a = rng.integers(0, 4, (n, FREE), dtype=np.uint8)
    b = rng.integers(0, 4, (n, FREE), dtype=np.uint8)
    ca = canon(np.concatenate([a, np.broadcast_to(ov, (n, OVERLAP))], axis=1))
    cb = canon(np.concatenate([np.broadcast_to(ov, (n, OVERLAP)), b], axis=1))
    ha, hb = mix(ca), mix(cb)
    hia, hib = ha >> np.uint64(32), hb >> np.uint64(32)
    common, ia, ib = np.intersect1d(hia, hib, return_indices=True)
    ok = (ca[ia] != cb[ib]) & (ha[ia] != hb[ib])
    assert ok.any(), "no high-word collision found"
    j = int(np.argmin(np.where(ok, common, M64)))
    seq = np.concatenate([a[ia[j]], ov, b[ib[j]]]).astype(np.uint8)
    return seq, int(ha[ia[j]]), int(hb[ib[j]])


@pytest.fixture(scope="module")
def tie():
    seq, h1, h2 = colliding_37mer()
    # the search's hash is the oracle's
    for c in (0, 1, 12345, 2**41 + 7):
        assert int(mix(np.array([c], np.uint64))[0]) == oracle.mix64(c)
    assert h1 >> 32 == h2 >> 32 and h1 != h2
    return seq


def place(length, spots, tie, step, seed):
    """Random bases with the tie's bases written at every spot (for pattern step 2 they go
    to the kept even positions)."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 4, length, dtype=np.uint8)
    for p in spots:
        s[p:p + step * tie.size:step] = tie
    return s


@pytest.mark.parametrize("pattern,w", [("1", 17), ("1", 17 - 1), ("10", 17)])
def test_high_word_ties_match_oracle(gpu, tie, pattern, w):
    step = len(pattern)
    T = 512 * 16 - 2 * 16          # positions a tile owns when w <= 17 (512 lanes x 16)
    # patterned positions: inside tile 0, just before tile 1's owned range (the second
    # k-mer inside it), deep in tile 2, and as a sequence of its own
    spots_np = [100, T - 8, 2 * T + 1000]
    seq = place(3 * T * step + 500, [p * step for p in spots_np], tie, step, 7)
    alone = tie if step == 1 else place(2 * tie.size, [0], tie, 2, 8)
    codes = np.concatenate([seq, alone])
    offs = np.array([0, seq.size, codes.size], np.int64)
    keys, vals, mz = gpu.sketch(gpu.to_device(codes, offs), pattern, K, w)
    ek, ev, em = oracle.sketch(codes, offs, pattern, K, w)
    assert np.array_equal(mz.cpu().numpy(), em.astype(np.int64))
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ek)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32).astype(np.uint64), ev)
    # the tie is real: in the lone sequence's window only the smaller hash is selected
    if step == 1 and w == 17:
        lone = ek[em[1]:em[2]]
        assert lone.size == 1
    ix = gpu.index_build(gpu.to_device(codes, offs), pattern, K, w)
    ik, iv = oracle.index_build(codes, offs, pattern, K, w)
    assert np.array_equal(ix.keys.cpu().numpy().view(np.uint64), ik)
    assert np.array_equal(ix.vals.cpu().numpy().view(np.uint32).astype(np.uint64), iv)
