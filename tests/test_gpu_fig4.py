"""Seed-matching experiment (Section 2.1.1, Fig. 4) on the GPU against the oracle,
bit-exact: per-pair matched/total seed counts of the four algorithms, Levenshtein
distances, and accepted pairs per edit-distance threshold."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

FIG4 = [("110", 8, 6), ("10", 8, 6), ("101001", 8, 6), ("100", 8, 6), ("10", 13, 9),
        ("1110110110111", 13, 9), ("10", 18, 12), ("111001011001010111", 18, 12),
        ("10", 21, 11), ("111101101101011101111", 21, 11), ("1", 32, 3), ("1", 2, 40)]


def pairs(seed, lens, rate=0.3):
    rng = np.random.default_rng(seed)
    a, b = [], []
    for L in lens:
        x = rng.integers(0, 4, L, dtype=np.uint8)
        y = x.copy()
        hit = rng.random(L) < rate * rng.random()
        y[hit] = (y[hit] + rng.integers(1, 4, int(hit.sum()), dtype=np.uint8)) % 4
        a.append((x, [0, L]))
        b.append((y, [0, L]))
    return datagen.concat(a), datagen.concat(b)


LENS = [0, 1, 7, 8, 9, 40, 63, 64, 65, 128, 500, 999, 1000, 1000, 1000, 1023, 1024, 300]


@pytest.mark.parametrize("pattern,k,w", FIG4)
def test_seed_match_matches_oracle(gpu, pattern, k, w):
    (ca, oa), (cb, ob) = pairs(k * 11 + len(pattern), LENS)
    got = gpu.seed_match(gpu.to_device(ca, oa), gpu.to_device(cb, ob), pattern, k, w)
    want = oracle.seed_match(ca, oa, cb, ob, pattern, k, w)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)


def test_seed_match_wang_hash(gpu):
    (ca, oa), (cb, ob) = pairs(7, LENS)
    got = gpu.seed_match(gpu.to_device(ca, oa), gpu.to_device(cb, ob), "110", 8, 6, hash="wang")
    with oracle.use_hash("wang"):
        want = oracle.seed_match(ca, oa, cb, ob, "110", 8, 6)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)


def test_edit_distance_matches_oracle(gpu):
    rng = np.random.default_rng(8)
    a_l, b_l = [], []
    for la, lb in [(0, 0), (0, 5), (5, 0), (1, 1), (63, 64), (64, 64), (65, 64), (128, 1),
                   (1024, 1024), (1024, 900), (700, 1100), (1000, 1000), (33, 2000)]:
        x = rng.integers(0, 4, la, dtype=np.uint8)
        y = rng.integers(0, 4, lb, dtype=np.uint8)
        if la == lb and la:                                # a close copy as well
            y = x.copy()
            hit = rng.random(la) < 0.05
            y[hit] = (y[hit] + 1) % 4
        a_l.append((x, [0, la]))
        b_l.append((y, [0, lb]))
    (ca, oa), (cb, ob) = datagen.concat(a_l), datagen.concat(b_l)
    got = gpu.edit_distance(gpu.to_device(ca, oa), gpu.to_device(cb, ob)).cpu().numpy()
    want = [oracle.edit_distance(ca[oa[i]:oa[i + 1]], cb[ob[i]:ob[i + 1]])
            for i in range(oa.size - 1)]
    assert got.tolist() == want


def test_edit_distance_many_substitution_pairs(gpu):
    o, oo, c, co, nsub = datagen.workload_fig4(n_pairs=600, seed=9)
    got = gpu.edit_distance(gpu.to_device(o, oo), gpu.to_device(c, co)).cpu().numpy()
    want = [oracle.edit_distance(o[oo[i]:oo[i + 1]], c[co[i]:co[i + 1]]) for i in range(600)]
    assert got.tolist() == want
    assert (got <= nsub).all()


def test_accepted_pairs_matches_oracle(gpu):
    import torch
    rng = np.random.default_rng(10)
    for n, max_e in [(1, 0), (1000, 50), (20_000, 700), (5, 3000)]:
        dist = rng.integers(0, max(max_e, 1) + 20, n).astype(np.uint32)
        total = rng.integers(0, 1000, (n, 4)).astype(np.uint32)
        matched = (total * rng.random((n, 4))).astype(np.uint32)
        counts = np.stack([matched, total], axis=2).astype(np.uint32)      # (n, 4, 2)
        d = torch.from_numpy(dist.view(np.int32)).cuda()
        cnt = torch.from_numpy(counts.reshape(-1).view(np.int32)).cuda()
        for g in range(4):
            got = gpu.accepted_pairs(d, cnt, g, max_e).cpu().numpy().view(np.uint32)
            want = oracle.accepted(dist, matched[:, g], total[:, g], max_e)
            assert np.array_equal(got, want), (n, max_e, g)


def test_fig4_workload_sample_matches_oracle(gpu):
    # the benchmark's input shape (1,000-base pairs over the whole range of differences)
    o, oo, c, co, _ = datagen.workload_fig4(n_pairs=3000, seed=11)
    so, sc = gpu.to_device(o, oo), gpu.to_device(c, co)
    for pattern, k, w in [("10", 8, 6), ("1110110110111", 13, 9)]:
        got = gpu.seed_match(so, sc, pattern, k, w).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.seed_match(o, oo, c, co, pattern, k, w))
    dist = gpu.edit_distance(so, sc)
    want = np.array([oracle.edit_distance(o[oo[i]:oo[i + 1]], c[co[i]:co[i + 1]])
                     for i in range(0, 3000, 10)])
    assert np.array_equal(dist.cpu().numpy()[::10], want)


def test_pair_longer_than_1024_is_rejected(gpu):
    (ca, oa), (cb, ob) = pairs(12, [10, 1025])
    with pytest.raises(ValueError):
        gpu.seed_match(gpu.to_device(ca, oa), gpu.to_device(cb, ob), "10", 8, 6)
    with pytest.raises(ValueError):
        gpu.edit_distance(gpu.to_device(ca, oa), gpu.to_device(cb, ob))
