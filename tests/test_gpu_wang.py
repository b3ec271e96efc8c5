"""GPU parity of the alternative k-mer hash (Thomas Wang's 64-bit integer hash reduced to
the 2k-bit code space, the hash of the minimap2-style sketching the paper modifies,
Section 3.1): sketch, index build, seeding and containment with hash="wang" against the
oracle run with the same hash, bit-exact."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def dev(gd, codes, offsets):
    return gd.to_device(codes, offsets)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def ragged_batch(seed, lens):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return rng.integers(0, 4, int(offs[-1]), dtype=np.uint8), offs


LENS = [0, 1, 5, 20, 21, 22, 40, 100, 4100, 0, 3, 9000, 151, 150, 37]


@pytest.mark.parametrize("pattern,k,w", [("10", 21, 11), ("110", 21, 11), ("1", 15, 10),
                                         ("1", 32, 2), ("10", 2, 3), ("1", 19, 19),
                                         ("1", 6, 256), ("101001", 13, 5)])
def test_wang_sketch_matches_oracle(gpu, pattern, k, w):
    codes, offs = ragged_batch(21, LENS)
    codes[4200:4400] = 0
    codes[5000:5300] = np.tile(np.array([0, 3], np.uint8), 150)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 5) % len(pattern)
    for sh in (None, shifts):
        keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), pattern, k, w, shift=sh, hash="wang")
        with oracle.use_hash("wang"):
            ek, ev, em = oracle.sketch(codes, offs, pattern, k, w, shifts=sh)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


def test_wang_differs_from_default_hash(gpu):
    codes, offs = ragged_batch(22, [5000])
    k1, _, _ = gpu.sketch(dev(gpu, codes, offs), "10", 15, 10)
    k2, _, _ = gpu.sketch(dev(gpu, codes, offs), "10", 15, 10, hash="wang")
    assert not np.array_equal(u64(k1), u64(k2))


@pytest.mark.parametrize("pattern,k,w,kw", [("10", 15, 10, {}), ("110", 13, 7, {"align_t": 3}),
                                            ("1", 15, 10, {"max_occ": 2})])
def test_wang_index_and_seed_match_oracle(gpu, pattern, k, w, kw):
    d = datagen.workload_tiny()
    ref, roffs = d["ref"], d["ref_offsets"]
    ix = gpu.index_build(dev(gpu, ref, roffs), pattern, k, w, hash="wang")
    with oracle.use_hash("wang"):
        ek, ev = oracle.index_build(ref, roffs, pattern, k, w)
        assert np.array_equal(u64(ix.keys), ek)
        assert np.array_equal(u32(ix.vals).astype(np.uint64), ev)
        reads, offs = d["reads"], d["read_offsets"]
        a, off, sh = gpu.seed(ix, dev(gpu, reads, offs), pattern, k, w, hash="wang", **kw)
        ea, eoff, esh = oracle.seed(ek, ev, reads, offs, pattern, k, w,
                                    align_t=kw.get("align_t", 0), max_occ=kw.get("max_occ", 0))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    assert ea.shape[0] > 1000


def test_wang_containment_matches_oracle(gpu):
    codes, offs = datagen.genome_db(12, 61, min_len=30_000, max_len=90_000)
    reads, ro, _ = datagen.sample_from_genomes(codes, offs, 2000, 4, 150, 62, sub=0.01)
    ix = gpu.index_build(dev(gpu, codes, offs), "10", 15, 10, val_bits=64, hash="wang")
    c, s = gpu.contain(ix, dev(gpu, reads, ro), "10", 15, 10, 12, hash="wang")
    with oracle.use_hash("wang"):
        ek, ev = oracle.index_build(codes, offs, "10", 15, 10, val_bits=64)
        ec, es = oracle.contain(ek, ev, reads, ro, "10", 15, 10, 12)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u32(s), es)
    assert np.array_equal(u32(c), ec)
    assert (ec > 0).sum() >= 4
