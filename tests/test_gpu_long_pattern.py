"""Patterns longer than 64 characters (the paper allows any length; Section 3.1 step 1) on
the GPU against the oracle, bit-exact: sparsification with per-sequence shifts (with and
without ambiguous bases), sketches, index build, seeding with pattern alignment over
every shift, and the seed-matching experiment's spaced seeds."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def unpack(packed, n):
    b = np.asarray(packed, np.uint8)
    out = np.stack([(b >> s) & 3 for s in (0, 2, 4, 6)], axis=1).reshape(-1)
    return out[:n]


def make_pattern(seed, p, density):
    rng = np.random.default_rng(seed)
    bits = rng.random(p) < density
    bits[int(rng.integers(0, p))] = True
    return "".join("1" if b else "0" for b in bits)


LONG = [make_pattern(21, 65, 0.5), make_pattern(22, 100, 0.8), make_pattern(23, 150, 0.1),
        make_pattern(24, 256, 0.5), "1" * 256, "0" * 200 + "1", "1" + "0" * 127 + "1" * 128]
LENS = [0, 1, 5, 64, 65, 100, 257, 4100, 0, 3, 9000, 151, 150, 30_000]


def batch(seed):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(LENS)]).astype(np.int64)
    return rng.integers(0, 4, int(offs[-1]), dtype=np.uint8), offs


@pytest.mark.parametrize("pattern", LONG)
def test_sparsify_long_pattern(gpu, pattern):
    codes, offs = batch(1)
    p = len(pattern)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 37) % p
    for sh in (None, shifts):
        out, po = gpu.sparsify(gpu.to_device(codes, offs), pattern, shift=sh)
        ec, eo, _ = oracle.sparsify(codes, offs, pattern, shifts=sh)
        assert np.array_equal(po.cpu().numpy(), eo.astype(np.int64))
        assert np.array_equal(unpack(out.cpu().numpy(), ec.size), ec)
    gapped = datagen.add_gaps(codes, 2, n_runs=3, run_len=(5, 300), n_single=100)
    out, po, pn = gpu.sparsify(gpu.to_device(gapped, offs), pattern, shift=shifts, with_nmask=True)
    ec, eo, _ = oracle.sparsify(gapped, offs, pattern, shifts=shifts)
    isn = np.unpackbits(pn.cpu().numpy(), bitorder="little")[:ec.size].astype(bool)
    assert np.array_equal(isn, ec == 4)
    assert np.array_equal(unpack(out.cpu().numpy(), ec.size)[~isn], ec[~isn])


@pytest.mark.parametrize("pattern,k,w", [(LONG[0], 21, 11), (LONG[1], 15, 10), (LONG[2], 5, 3),
                                         (LONG[3], 31, 17), (LONG[4], 21, 40), (LONG[6], 13, 7)])
def test_sketch_long_pattern(gpu, pattern, k, w):
    codes, offs = batch(3)
    p = len(pattern)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 53) % p
    dev = gpu.to_device(codes, offs)
    for sh in (None, shifts):
        keys, vals, mz = gpu.sketch(dev, pattern, k, w, shift=sh)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w, shifts=sh)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


@pytest.mark.parametrize("pattern,k,w", [(LONG[0], 15, 10), (LONG[1], 13, 7)])
def test_index_and_seed_long_pattern(gpu, pattern, k, w):
    d = datagen.workload_tiny()
    ref, roffs = d["ref"], d["ref_offsets"]
    reads, offs = d["reads"][:300 * 150], d["read_offsets"][:301]
    ix = gpu.index_build(gpu.to_device(ref, roffs), pattern, k, w)
    ek, ev = oracle.index_build(ref, roffs, pattern, k, w)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u32(ix.vals).astype(np.uint64), ev)
    for kw in ({}, {"shift_mode": len(pattern) - 1}, {"align_t": 5}):
        a, off, sh = gpu.seed(ix, gpu.to_device(reads, offs), pattern, k, w, **kw)
        ea, eoff, esh = oracle.seed(ek, ev, reads, offs, pattern, k, w,
                                    shift_mode=kw.get("shift_mode", -1),
                                    align_t=kw.get("align_t", 0))
        assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
        assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
        assert np.array_equal(u32(a).reshape(-1, 4), ea)


def test_seed_match_long_pattern(gpu):
    o, oo, c, co, _ = datagen.workload_fig4(n_pairs=200, seed=12)
    for pattern, k, w in [(LONG[0], 21, 11), (LONG[3], 8, 6)]:
        got = gpu.seed_match(gpu.to_device(o, oo), gpu.to_device(c, co), pattern, k, w)
        want = oracle.seed_match(o, oo, c, co, pattern, k, w)
        assert np.array_equal(u32(got), want)
