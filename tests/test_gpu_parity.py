"""GPU parity: every entry point of the HIP library against the CPU oracle, bit-exact,
on seeded synthetic inputs (tiny sweeps with ragged and empty sequences, sizes spanning
many sketch tiles, the 1 Mbp / 2,000-read workload in full)."""
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


def unpack(packed, n):
    b = np.asarray(packed, np.uint8)
    out = np.stack([(b >> s) & 3 for s in (0, 2, 4, 6)], axis=1).reshape(-1)
    return out[:n]


def ragged_batch(seed, lens):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return rng.integers(0, 4, int(offs[-1]), dtype=np.uint8), offs


LENS = [0, 1, 5, 20, 21, 22, 40, 100, 4100, 0, 3, 9000, 151, 150, 37]


@pytest.mark.parametrize("pattern", ["1", "10", "01", "110", "101", "1001010011", "0001", "1" * 64,
                                     "10" * 32])
def test_sparsify_matches_oracle(gpu, pattern):
    codes, offs = ragged_batch(1, LENS)
    p = len(pattern)
    shifts = np.arange(len(LENS), dtype=np.uint32) % p
    for sh in (None, shifts):
        out, po = gpu.sparsify(dev(gpu, codes, offs), pattern, shift=sh)
        ec, eo, _ = oracle.sparsify(codes, offs, pattern, shifts=sh)
        assert np.array_equal(po.cpu().numpy(), eo.astype(np.int64))
        got = unpack(out.cpu().numpy(), ec.size)
        assert np.array_equal(got, ec)


@pytest.mark.parametrize("n_seq", [70_000, 4_300_000])
def test_sparsify_many_sequences(gpu, n_seq):
    # sequence counts past one workgroup's scan (two launches) and past 4M (three launches)
    rng = np.random.default_rng(n_seq)
    lens = rng.integers(0, 9, n_seq)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    codes = rng.integers(0, 4, int(offs[-1]), dtype=np.uint8)
    shifts = rng.integers(0, 3, n_seq).astype(np.uint32)
    out, po = gpu.sparsify(dev(gpu, codes, offs), "110", shift=shifts)
    ec, eo, _ = oracle.sparsify(codes, offs, "110", shifts=shifts)
    assert np.array_equal(po.cpu().numpy(), eo.astype(np.int64))
    assert np.array_equal(unpack(out.cpu().numpy(), ec.size), ec)


def test_sketch_many_tiny_sequences(gpu):
    # more sequences per tile than the tile's sequence cache holds (it is then bypassed)
    rng = np.random.default_rng(77)
    lens = rng.integers(0, 13, 70_000)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    codes = rng.integers(0, 4, int(offs[-1]), dtype=np.uint8)
    for pattern, k, w in [("1", 3, 2), ("10", 3, 1)]:
        keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), pattern, k, w)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


SKETCH_CASES = [("10", 15, 10), ("10", 21, 11), ("110", 21, 11), ("1", 15, 12), ("1", 19, 19),
                ("1", 28, 40), ("101001", 13, 5), ("1", 4, 1), ("10", 2, 3), ("1", 32, 2),
                ("1110", 31, 17), ("100", 8, 6), ("1" * 64, 21, 11), ("1", 6, 256),
                ("01", 21, 11)]


@pytest.mark.parametrize("pattern,k,w", SKETCH_CASES)
def test_sketch_matches_oracle(gpu, pattern, k, w):
    codes, offs = ragged_batch(2, LENS)
    codes[4200:4400] = 0                       # poly-A run: hash-0 ties
    codes[5000:5300] = np.tile(np.array([0, 3], np.uint8), 150)   # palindromic 2-mers
    p = len(pattern)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 7) % p
    for sh in (None, shifts):
        keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), pattern, k, w, shift=sh)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w, shifts=sh)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


@pytest.mark.parametrize("w", list(range(1, 19)))
def test_sketch_every_small_window(gpu, w):
    # w 2..17 use the register selection path, the others the LDS doubling path
    codes, offs = ragged_batch(12, [30_000, 0, 7, 60, 150, 151, 2000, 40])
    codes[10_000:10_400] = 0
    for pattern, k in [("10", 13), ("1", 8)]:
        keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), pattern, k, w)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


def test_sketch_many_tiles_and_reads(gpu):
    # one long sequence spanning hundreds of tiles plus 3,000 short reads in one batch
    ref = datagen.random_genome(600_000, 3)
    rc, ro, _, _ = datagen.fixed_reads(ref, 3000, 150, 4, sub=0.01)
    codes, offs = datagen.concat([(ref, np.array([0, ref.size])), (rc, ro)])
    for pattern, k, w in [("10", 21, 11), ("110", 15, 10)]:
        keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), pattern, k, w)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


@pytest.mark.parametrize("w", [1, 2, 4])
def test_index_64bit_values_dense_windows(gpu, w):
    # with w = 1 every k-mer is a minimizer: more records per tile than the exchange array
    # can stage at 16 bytes each, so those tiles write their records directly
    codes, offs = ragged_batch(13, [40_000, 0, 9, 151, 12_000])
    for pattern, k in [("1", 11), ("10", 9)]:
        ix = gpu.index_build(dev(gpu, codes, offs), pattern, k, w, val_bits=64)
        ek, ev = oracle.index_build(codes, offs, pattern, k, w, val_bits=64)
        assert np.array_equal(u64(ix.keys), ek)
        assert np.array_equal(u64(ix.vals), ev)


@pytest.mark.parametrize("w", [1, 11])
def test_sketch_capacity_short_writes_prefix_only(gpu, w):
    # an output buffer shorter than the sketch: the first `capacity` records are written,
    # nothing past them, the capacity status is raised and mz_offsets hold the full count
    import ctypes
    import torch
    from paper_2211_08157_amd import api
    codes, offs = ragged_batch(14, [30_000, 5, 2_000, 151])
    ek, ev, em = oracle.sketch(codes, offs, "1", 15, w)
    seqs = dev(gpu, codes, offs)
    cap = int(ek.size) * 2 // 3 + 5
    pad = 4096
    keys = torch.full((cap + pad,), -1, dtype=torch.int64, device="cuda")
    vals = torch.full((cap + pad,), -1, dtype=torch.int32, device="cuda")
    mz = torch.zeros(len(offs), dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(api.workspace_size(api.OP_SKETCH, seqs, "1", 15, w), dtype=torch.uint8,
                     device="cuda")
    prm = api._params("1", 15, w)
    s = seqs.c()
    api._check(api.lib().godiet_sketch(ctypes.byref(s), ctypes.byref(prm), None, api._ptr(keys),
                                       api._ptr(vals), api._ptr(mz), cap, api._ptr(ws),
                                       ws.numel(), api._ptr(st), api._stream()), "godiet_sketch")
    torch.cuda.synchronize()
    assert int(st.item()) & api.STATUS_CAPACITY
    assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
    assert np.array_equal(u64(keys)[:cap], ek[:cap])
    assert np.array_equal(u32(vals)[:cap].astype(np.uint64), ev[:cap])
    assert (keys[cap:] == -1).all() and (vals[cap:] == -1).all()


def test_sketch_empty_batch_and_no_sequences(gpu):
    codes, offs = ragged_batch(5, [0, 0, 3])
    keys, vals, mz = gpu.sketch(dev(gpu, codes, offs), "10", 15, 10)
    assert keys.numel() == 0 and mz.cpu().tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("val_bits", [32, 64])
def test_index_build_matches_oracle(gpu, val_bits):
    codes, offs = ragged_batch(6, [200_000, 0, 17, 150_000, 5, 80_000])
    codes[1000:6000] = codes[100_000:105_000]          # repeats -> equal keys
    codes[300_000:300_500] = 0
    for pattern, k, w in [("10", 15, 10), ("1", 21, 11), ("110", 9, 4)]:
        ix = gpu.index_build(dev(gpu, codes, offs), pattern, k, w, val_bits=val_bits)
        ek, ev = oracle.index_build(codes, offs, pattern, k, w, val_bits=val_bits)
        assert ix.n == ek.size
        assert np.array_equal(u64(ix.keys), ek)
        gv = u32(ix.vals).astype(np.uint64) if val_bits == 32 else u64(ix.vals)
        assert np.array_equal(gv, ev)


def test_index_build_large_buckets(gpu):
    # a low-complexity reference: huge runs of equal hashes exercise the LDS bitonic
    # path and the global-memory fallback for buckets beyond LDS capacity
    rng = np.random.default_rng(9)
    unit = rng.integers(0, 4, 7, dtype=np.uint8)
    codes = np.tile(unit, 60_000)
    codes[::997] = rng.integers(0, 4, codes[::997].size, dtype=np.uint8)
    offs = np.array([0, codes.size], np.int64)
    ix = gpu.index_build(dev(gpu, codes, offs), "1", 11, 5)
    ek, ev = oracle.index_build(codes, offs, "1", 11, 5)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u32(ix.vals).astype(np.uint64), ev)


# index capacities from 2^24 records take the two-level scatter (a coarse pass by the top
# 8 bits of the digit, then a fine pass inside each coarse digit); a large capacity over a
# small reference reaches it with few records per digit, many empty chunks and digits
TWO_LEVEL_CAPACITY = (1 << 24) + 12345


@pytest.mark.parametrize("val_bits", [32, 64])
def test_index_build_two_level_scatter(gpu, val_bits):
    codes, offs = ragged_batch(11, [3_000_000, 1, 2_500_000, 0, 999_999])
    codes[5000:405_000] = codes[1_000_000:1_400_000]   # a 400 kbp repeat: equal keys
    for pattern, k, w in [("10", 21, 11), ("1", 15, 5)]:
        ix = gpu.index_build(dev(gpu, codes, offs), pattern, k, w, val_bits=val_bits,
                             capacity=TWO_LEVEL_CAPACITY)
        ek, ev = oracle.index_build(codes, offs, pattern, k, w, val_bits=val_bits)
        assert ix.n == ek.size
        assert np.array_equal(u64(ix.keys), ek)
        gv = u32(ix.vals).astype(np.uint64) if val_bits == 32 else u64(ix.vals)
        assert np.array_equal(gv, ev)


def test_index_build_two_level_long_runs(gpu):
    # equal hashes by the thousand through the two-level scatter
    rng = np.random.default_rng(19)
    unit = rng.integers(0, 4, 7, dtype=np.uint8)
    codes = np.tile(unit, 300_000)
    codes[::997] = rng.integers(0, 4, codes[::997].size, dtype=np.uint8)
    offs = np.array([0, codes.size], np.int64)
    ix = gpu.index_build(dev(gpu, codes, offs), "1", 11, 5, capacity=TWO_LEVEL_CAPACITY)
    ek, ev = oracle.index_build(codes, offs, "1", 11, 5)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u32(ix.vals).astype(np.uint64), ev)


def _seed_compare(gpu, ref, roffs, reads, offs, pattern, k, w, **kw):
    ix = gpu.index_build(dev(gpu, ref, roffs), pattern, k, w)
    ek, ev = oracle.index_build(ref, roffs, pattern, k, w)
    a, off, sh = gpu.seed(ix, dev(gpu, reads, offs), pattern, k, w, **kw)
    ea, eoff, esh = oracle.seed(ek, ev, reads, offs, pattern, k, w,
                                shift_mode=kw.get("shift_mode", -1), align_t=kw.get("align_t", 0),
                                max_occ=kw.get("max_occ", 0))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    return ea


def test_seed_many_short_reads(gpu):
    # 100,000 reads of 0-40 bases (many without a single window) against 200 kbp, and a
    # reference of 70,000 tiny sequences for the 64-bit index: more sequences per tile
    # and per sparsify workgroup than the sequence cache holds
    ref = datagen.random_genome(200_000, 61)
    rng = np.random.default_rng(62)
    lens = rng.integers(0, 41, 100_000)
    starts = rng.integers(0, ref.size - 41, lens.size)
    reads = np.concatenate([ref[s:s + n] for s, n in zip(starts, lens)]).astype(np.uint8)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ea = _seed_compare(gpu, ref, np.array([0, ref.size], np.int64), reads, offs, "10", 9, 5)
    assert ea.shape[0] > 50_000
    tl = rng.integers(0, 13, 70_000)
    toffs = np.concatenate([[0], np.cumsum(tl)]).astype(np.int64)
    tcodes = rng.integers(0, 4, int(toffs[-1]), dtype=np.uint8)
    ix = gpu.index_build(dev(gpu, tcodes, toffs), "1", 5, 3, val_bits=64)
    ek, ev = oracle.index_build(tcodes, toffs, "1", 5, 3, val_bits=64)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u64(ix.vals), ev)


def test_seed_tiny_workload_full(gpu):
    d = datagen.workload_tiny()
    ea = _seed_compare(gpu, d["ref"], d["ref_offsets"], d["reads"], d["read_offsets"], "10", 15, 10)
    assert ea.shape[0] > 10_000


@pytest.mark.parametrize("pattern,k,w,kw", [
    ("110", 13, 7, {}), ("101", 11, 5, {"align_t": 3}), ("10", 15, 10, {"max_occ": 2}),
    ("10", 15, 10, {"shift_mode": 1}), ("1", 15, 10, {}), ("1001", 9, 4, {"align_t": 1})])
def test_seed_options_match_oracle(gpu, pattern, k, w, kw):
    ref = datagen.add_repeats(datagen.random_genome(300_000, 7), 207, frac=0.2, seg_len=2000,
                              copies=5)
    reads = [datagen.fixed_reads(ref, 500, 150, 8, sub=0.01)[:2],
             datagen.variable_reads(ref, [1, 30, 2000, 9000, 0 + 5], 9, 0.02, 0.01, 0.01)[:2]]
    codes, offs = datagen.concat(reads)
    _seed_compare(gpu, ref, np.array([0, ref.size]), codes, offs, pattern, k, w, **kw)


def test_seed_deterministic(gpu):
    d = datagen.workload_tiny()
    ix = gpu.index_build(dev(gpu, d["ref"], d["ref_offsets"]), "10", 15, 10)
    r = dev(gpu, d["reads"], d["read_offsets"])
    a1, o1, s1 = gpu.seed(ix, r, "10", 15, 10)
    a2, o2, s2 = gpu.seed(ix, r, "10", 15, 10)
    assert np.array_equal(a1.cpu().numpy(), a2.cpu().numpy())
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())


def test_capacity_status_and_retry(gpu):
    import torch
    d = datagen.workload_tiny()
    ix = gpu.index_build(dev(gpu, d["ref"], d["ref_offsets"]), "10", 15, 10, capacity=1000)
    ek, _ = oracle.index_build(d["ref"], d["ref_offsets"], "10", 15, 10)
    assert ix.n == ek.size          # the wrapper read the required count and retried
    a, off, _ = gpu.seed(ix, dev(gpu, d["reads"], d["read_offsets"]), "10", 15, 10, capacity=10)
    assert a.shape[0] == int(off[-1].item()) > 10
    torch.cuda.synchronize()


def test_seed_waits_for_an_index_built_on_another_stream(gpu):
    # the index is built on a side stream while seeding sketches the reads on the main
    # stream and waits on the index event before its lookups
    import torch
    d = datagen.workload_tiny()
    ref = dev(gpu, d["ref"], d["ref_offsets"])
    reads = dev(gpu, d["reads"], d["read_offsets"])
    ek, ev = oracle.index_build(d["ref"], d["ref_offsets"], "10", 15, 10)
    ea, eoff, esh = oracle.seed(ek, ev, d["reads"], d["read_offsets"], "10", 15, 10)
    side = torch.cuda.Stream()
    ready = torch.cuda.Event()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(side):
            ix = gpu.index_build(ref, "10", 15, 10)
            ix = gpu.rmi_train(ix, root="mlp", log2_leaves=12)
            ready.record(side)
        a, off, sh = gpu.seed(ix, reads, "10", 15, 10, index_ready=ready)
        torch.cuda.synchronize()
        assert np.array_equal(u32(a).reshape(-1, 4), ea)
        assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
        assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
