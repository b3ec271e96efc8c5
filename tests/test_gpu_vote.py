"""Location voting on the GPU equals the oracle: on the oracle's own anchors of the tiny
workload and of a mixed short/long-read batch, end to end after GPU seeding, on
synthetic anchor sets built to exercise clusters, both strands, reads swept by a wave
(more than 256 anchors), empty reads, every parameter edge (D = 0, V = 0, caps 1 and 16),
and the status bits for a too-small capacity and anchors not grouped by read; with each
of the ways of sorting the locations (adaptive, batch digit sort, per-read merge of the
presorted runs, per-read heapsort)."""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu


def oracle_rows(out, nw):
    return np.array([[r, *out[r, j]] for r in range(nw.size) for j in range(nw[r])],
                    np.int64).reshape(-1, 5)


def gpu_vote(gpu, anchors_np, off_np, D, V, cap, capacity=None, sort="adaptive"):
    a = torch.from_numpy(np.ascontiguousarray(anchors_np, np.uint32).view(np.int32)).cuda()
    o = torch.from_numpy(np.asarray(off_np, np.int64)).cuda()
    w, nw = gpu.vote(a, o, D, V, cap, capacity=capacity, sort=sort)
    return gpu.winners_rows(w, nw)


def synthetic(seed, n_reads, long_every=0):
    rng = np.random.default_rng(seed)
    rows, off = [], [0]
    for r in range(n_reads):
        m = int(rng.integers(0, 30))
        if long_every and r % long_every == 0:
            m = int(rng.integers(257, 3000))
        base = int(rng.integers(1000, 1 << 30))
        read = []
        for _ in range(m):
            q = int(rng.integers(0, 20_000))
            st = int(rng.integers(0, 2))
            if rng.random() < 0.7:
                rp = (base + q if st == 0 else base - q) + int(rng.integers(-3, 4))
            else:
                rp = int(rng.integers(0, (1 << 31) - 1))
            read.append((q, max(rp, 0), st))
        read.sort()
        rows += [[r, q, rp, st] for q, rp, st in read]
        off.append(len(rows))
    return np.array(rows, np.uint32).reshape(-1, 4), np.array(off, np.uint64)


@pytest.mark.parametrize("D,V,cap", [(16, 3, 4), (0, 1, 1), (5, 0, 16), (100, 3, 4),
                                     (1000, 2, 2)])
def test_vote_on_synthetic_anchors(gpu, D, V, cap):
    a, off = synthetic(3 + D, 4000, long_every=97)
    want = oracle_rows(*oracle.vote(a, off, D, V, cap))
    for sort in ("adaptive", "radix", "merge", "heap"):
        got = gpu_vote(gpu, a, off, D, V, cap, sort=sort)
        assert np.array_equal(got, want), sort


def test_vote_on_oracle_anchors_of_tiny_workload(gpu):
    d = datagen.workload_tiny()
    ek, ev = oracle.index_build(d["ref"], d["ref_offsets"], "10", d["k"], d["w"])
    a, off, _ = oracle.seed(ek, ev, d["reads"], d["read_offsets"], "10", d["k"], d["w"])
    for D, V, cap in ((16, 3, 4), (4, 2, 8)):
        want = oracle_rows(*oracle.vote(a, off, D, V, cap))
        assert np.array_equal(gpu_vote(gpu, a, off, D, V, cap), want)


def test_vote_end_to_end_after_gpu_seeding_mixed_batch(gpu):
    ref = datagen.add_repeats(datagen.random_genome(2_000_000, 71), 271)
    roffs = np.array([0, ref.size], np.int64)
    rng = np.random.default_rng(72)
    short = datagen.fixed_reads(ref, 3000, 150, 73, sub=0.005, ins=0.0005, dele=0.0005)
    hifi = datagen.variable_reads(ref, datagen.hifi_lengths(10, rng), 74, 0.005, 0.0025, 0.0025)
    ont = datagen.variable_reads(ref, datagen.ont_lengths(10, rng), 75, 0.04, 0.02, 0.02)
    codes, offs = datagen.concat([short[:2], hifi[:2], ont[:2]])
    ix = gpu.index_build(gpu.to_device(ref, roffs), "10", 15, 10)
    a, off, _ = gpu.seed(ix, gpu.to_device(codes, offs), "10", 15, 10)
    ek, ev = oracle.index_build(ref, roffs, "10", 15, 10)
    ea, eoff, _ = oracle.seed(ek, ev, codes, offs, "10", 15, 10)
    want = oracle_rows(*oracle.vote(ea, eoff, 100, 3, 4))
    for sort in ("adaptive", "radix", "merge", "heap"):
        w, nw = gpu.vote(a, off, 100, 3, 4, sort=sort)
        assert np.array_equal(gpu.winners_rows(w, nw), want), sort
    assert (np.diff(eoff.astype(np.int64)) > 256).any()     # some reads took the wave path


def test_vote_empty_and_status(gpu):
    # no anchors at all, and reads without anchors
    off = np.zeros(5, np.uint64)
    got = gpu_vote(gpu, np.zeros((0, 4), np.uint32), off, 10, 2, 4)
    assert got.shape[0] == 0
    a, off = synthetic(5, 50)
    with pytest.raises(ValueError):                          # capacity below the count
        gpu_vote(gpu, a, off, 10, 2, 4, capacity=int(off[-1]) - 1)
    first = int(np.nonzero(np.diff(off.astype(np.int64)) > 0)[0][0])
    bad = a.copy()
    bad[int(off[first]), 0] = first + 1                      # one anchor claims the next read
    with pytest.raises(ValueError):
        gpu_vote(gpu, bad, off, 10, 2, 4)


def test_vote_sorts_on_reads_with_many_locations(gpu):
    # reads beyond one 4,096-key LDS chunk: the adaptive sort's merge passes run
    rng = np.random.default_rng(31)
    rows, off = [], [0]
    for r, m in enumerate([0, 4095, 4096, 4097, 9000, 20_000, 3, 300, 257, 8192, 12_345]):
        base = int(rng.integers(1000, 1 << 29))
        read = []
        for _ in range(m):
            q = int(rng.integers(0, 1 << 20))
            st = int(rng.integers(0, 2))
            rp = (base + q if st == 0 else base - q) + int(rng.integers(-50, 50)) \
                if rng.random() < 0.5 else int(rng.integers(0, (1 << 31) - 1))
            read.append((q, max(rp, 0), st))
        read.sort()
        rows += [[r, q, rp, st] for q, rp, st in read]
        off.append(len(rows))
    a = np.array(rows, np.uint32).reshape(-1, 4)
    off = np.array(off, np.uint64)
    want = oracle_rows(*oracle.vote(a, off, 100, 3, 4))
    for sort in ("adaptive", "radix", "merge", "heap"):
        assert np.array_equal(gpu_vote(gpu, a, off, 100, 3, 4, sort=sort), want), sort
