"""Ambiguous bases (N) on the GPU against the oracle, bit-exact: the device text packer,
the N mask of sparsified sequences, and sketch / index build / seeding / containment on
batches with assembly-gap runs and isolated Ns (an N among the kept bases ends a run of
patterned bases, Section 3.6.1)."""
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


def bits(mask_bytes, n):
    return np.unpackbits(np.asarray(mask_bytes, np.uint8), bitorder="little")[:n].astype(bool)


def gapped_batch(seed, lens, runs=2, singles=30):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    codes = rng.integers(0, 4, int(offs[-1]), dtype=np.uint8)
    return datagen.add_gaps(codes, seed + 1, n_runs=runs, run_len=(5, 400), n_single=singles), offs


LENS = [0, 1, 5, 20, 21, 40, 100, 4100, 0, 3, 9000, 151, 150, 37, 30_000]


@pytest.mark.parametrize("n", [0, 1, 15, 16, 63, 64, 65, 1000, 100_003])
def test_pack_ascii_matches_host_mapping(gpu, n):
    rng = np.random.default_rng(n)
    alphabet = np.frombuffer(b"ACGTUacgtuNnRY-*x\0", np.uint8)
    text = alphabet[rng.integers(0, alphabet.size, n)] if n else np.zeros(0, np.uint8)
    s = gpu.to_device_ascii(text, [0, n])
    lower = text | 0x20
    want = np.full(n, 4, np.uint8)
    for ch, v in ((b"a", 0), (b"c", 1), (b"g", 2), (b"t", 3), (b"u", 3)):
        want[lower == ch[0]] = v
    got = unpack(s.bases.cpu().numpy(), n)
    isn = bits(s.nmask.cpu().numpy(), n)
    assert np.array_equal(isn, want == 4)
    assert np.array_equal(got[~isn], want[~isn]) and not got[isn].any()
    # padding: zero codes and clear bits up to the packed size
    nb = gpu.lib().godiet_pack_bytes(n)
    assert not unpack(s.bases.cpu().numpy()[:nb], nb * 4)[n:].any()
    assert not bits(s.nmask.cpu().numpy()[:nb // 2], nb * 2)[n:].any()


@pytest.mark.parametrize("pattern", ["1", "10", "01", "110", "1001010011", "1" * 64])
def test_sparsify_carries_the_n_mask(gpu, pattern):
    codes, offs = gapped_batch(3, LENS)
    p = len(pattern)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 3) % p
    for sh in (None, shifts):
        out, po, pn = gpu.sparsify(gpu.to_device(codes, offs), pattern, shift=sh, with_nmask=True)
        ec, eo, _ = oracle.sparsify(codes, offs, pattern, shifts=sh)
        assert np.array_equal(po.cpu().numpy(), eo.astype(np.int64))
        got = unpack(out.cpu().numpy(), ec.size)
        isn = bits(pn.cpu().numpy(), ec.size)
        assert np.array_equal(isn, ec == 4)
        assert np.array_equal(got[~isn], ec[~isn])


@pytest.mark.parametrize("pattern", ["10", "110"])
def test_n_mask_of_many_tiny_sequences(gpu, pattern):
    # more sequences per sparsify workgroup and per sketch tile than the sequence cache holds
    rng = np.random.default_rng(91)
    codes, offs = gapped_batch(90, rng.integers(0, 13, 70_000), runs=20, singles=20_000)
    shifts = rng.integers(0, len(pattern), 70_000).astype(np.uint32)
    out, po, pn = gpu.sparsify(gpu.to_device(codes, offs), pattern, shift=shifts, with_nmask=True)
    ec, eo, _ = oracle.sparsify(codes, offs, pattern, shifts=shifts)
    assert np.array_equal(po.cpu().numpy(), eo.astype(np.int64))
    isn = bits(pn.cpu().numpy(), ec.size)
    assert np.array_equal(isn, ec == 4)
    assert np.array_equal(unpack(out.cpu().numpy(), ec.size)[~isn], ec[~isn])
    keys, vals, mz = gpu.sketch(gpu.to_device(codes, offs), pattern, 3, 2)
    ek, ev, em = oracle.sketch(codes, offs, pattern, 3, 2)
    assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
    assert np.array_equal(u64(keys), ek)
    assert np.array_equal(u32(vals).astype(np.uint64), ev)


CASES = [("10", 21, 11), ("110", 21, 11), ("1", 15, 10), ("1", 16, 5), ("10", 2, 3),
         ("1", 19, 19), ("1", 28, 40), ("101001", 13, 5), ("1", 6, 256), ("1", 4, 1),
         ("1110", 31, 17), ("1", 32, 2)]


@pytest.mark.parametrize("pattern,k,w", CASES)
def test_sketch_with_ns_matches_oracle(gpu, pattern, k, w):
    codes, offs = gapped_batch(4, LENS, runs=6, singles=200)
    codes[9000:9400] = 4                              # an N run across a tile boundary
    codes[20_000:20_050] = np.tile(np.array([4, 4, 0, 1, 2], np.uint8), 10)   # short runs
    p = len(pattern)
    shifts = (np.arange(len(LENS), dtype=np.uint32) * 7) % p
    dev = gpu.to_device(codes, offs)
    for sh in (None, shifts):
        keys, vals, mz = gpu.sketch(dev, pattern, k, w, shift=sh)
        ek, ev, em = oracle.sketch(codes, offs, pattern, k, w, shifts=sh)
        assert np.array_equal(mz.cpu().numpy().view(np.uint64), em)
        assert np.array_equal(u64(keys), ek)
        assert np.array_equal(u32(vals).astype(np.uint64), ev)


def test_ascii_upload_equals_code_upload(gpu):
    codes, offs = gapped_batch(5, [5000, 0, 300, 12_000], runs=3, singles=50)
    a = gpu.sketch(gpu.to_device(codes, offs), "10", 15, 10, hash="wang")
    b = gpu.sketch(gpu.to_device_ascii(datagen.to_text(codes, seed=6), offs), "10", 15, 10,
                   hash="wang")
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    # a batch without N gives the same minimizers with or without an (empty) N mask
    clean = np.where(codes == 4, 1, codes).astype(np.uint8)
    c = gpu.sketch(gpu.to_device(clean, offs), "110", 15, 10)
    d = gpu.sketch(gpu.to_device_ascii(datagen.to_text(clean), offs), "110", 15, 10)
    for x, y in zip(c, d):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("val_bits", [32, 64])
def test_index_build_with_gaps_matches_oracle(gpu, val_bits):
    genome = datagen.random_genome(3_000_000, 70)
    ref = datagen.add_gaps(genome, 71, n_runs=20, run_len=(1000, 60_000), n_single=3000)
    offs = np.array([0, 1_000_000, 1_000_000, 2_200_000, 3_000_000], np.int64)
    for pattern, k, w in [("10", 21, 11), ("110", 15, 10), ("1", 19, 40)]:
        ix = gpu.index_build(gpu.to_device(ref, offs), pattern, k, w, val_bits=val_bits)
        ek, ev = oracle.index_build(ref, offs, pattern, k, w, val_bits=val_bits)
        assert ix.n == ek.size
        assert np.array_equal(u64(ix.keys), ek)
        gv = u32(ix.vals).astype(np.uint64) if val_bits == 32 else u64(ix.vals)
        assert np.array_equal(gv, ev)


@pytest.mark.parametrize("pattern,k,w,kw", [("10", 15, 10, {}), ("110", 13, 7, {"align_t": 3}),
                                            ("1", 15, 10, {"max_occ": 2})])
def test_seed_with_ns_matches_oracle(gpu, pattern, k, w, kw):
    d = datagen.workload_tiny()
    ref = datagen.add_gaps(d["ref"], 72, n_runs=4, run_len=(500, 5000), n_single=500)
    roffs = d["ref_offsets"]
    reads = datagen.add_gaps(d["reads"], 73, n_single=d["reads"].size // 300)
    offs = d["read_offsets"]
    ix = gpu.index_build(gpu.to_device(ref, roffs), pattern, k, w)
    ek, ev = oracle.index_build(ref, roffs, pattern, k, w)
    assert np.array_equal(u64(ix.keys), ek)
    a, off, sh = gpu.seed(ix, gpu.to_device(reads, offs), pattern, k, w, **kw)
    ea, eoff, esh = oracle.seed(ek, ev, reads, offs, pattern, k, w, align_t=kw.get("align_t", 0),
                                max_occ=kw.get("max_occ", 0))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    assert ea.shape[0] > 1000


def test_containment_with_ns_matches_oracle(gpu):
    codes, offs = datagen.genome_db(10, 74, min_len=30_000, max_len=90_000)
    codes = datagen.add_gaps(codes, 75, n_runs=10, run_len=(50, 3000), n_single=400)
    reads, ro, _ = datagen.sample_from_genomes(codes, offs, 2000, 4, 150, 76, sub=0.01)
    ix = gpu.index_build(gpu.to_device(codes, offs), "10", 15, 10, val_bits=64)
    c, s = gpu.contain(ix, gpu.to_device(reads, ro), "10", 15, 10, 10)
    ek, ev = oracle.index_build(codes, offs, "10", 15, 10, val_bits=64)
    ec, es = oracle.contain(ek, ev, reads, ro, "10", 15, 10, 10)
    assert np.array_equal(u64(ix.keys), ek)
    assert np.array_equal(u32(s), es) and np.array_equal(u32(c), ec)
