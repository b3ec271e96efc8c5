"""Hash-table form of the seed index (the paper's hash -> location-list table): seeding
and containment through the table equal binary search and the oracle, on a repeat-rich
reference (long runs of equal keys), for keys absent from the index, with every read
option, for the empty index, and with a table built for other keys (refused when too small
for the index, ignored when of the same size)."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def setup(gpu):
    ref = datagen.add_repeats(datagen.random_genome(2_000_000, 81), 281, frac=0.3, seg_len=2000,
                              copies=12, divergence=0.005)
    offs = np.array([0, ref.size], np.int64)
    ix = gpu.index_build(gpu.to_device(ref, offs), "10", 15, 10)
    ek, ev = oracle.index_build(ref, offs, "10", 15, 10)
    codes, ro, _, _ = datagen.fixed_reads(ref, 4000, 150, 82, sub=0.01)
    return ref, offs, ix, ek, ev, codes, ro


@pytest.mark.parametrize("shift_mode,t,max_occ", [(-1, 0, 0), (-1, 3, 0), (-1, 0, 5), (1, 0, 0)])
def test_seed_through_table_equals_oracle(gpu, setup, shift_mode, t, max_occ):
    ref, offs, ix, ek, ev, codes, ro = setup
    tix = gpu.table_build(ix)
    reads = gpu.to_device(codes, ro)
    a_t, off_t, sh_t = gpu.seed(tix, reads, "10", 15, 10, shift_mode=shift_mode, align_t=t,
                                max_occ=max_occ)
    a_b, off_b, sh_b = gpu.seed(ix, reads, "10", 15, 10, shift_mode=shift_mode, align_t=t,
                                max_occ=max_occ)
    ea, eoff, esh = oracle.seed(ek, ev, codes, ro, "10", 15, 10, shift_mode=shift_mode,
                                align_t=t, max_occ=max_occ)
    assert np.array_equal(u32(a_t).reshape(-1, 4), ea)
    assert np.array_equal(u32(a_b).reshape(-1, 4), ea)
    assert np.array_equal(off_t.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh_t.cpu().numpy().astype(np.uint32), esh)


def test_table_from_other_keys_is_ignored_and_empty_index(gpu, setup):
    from paper_2211_08157_amd import api
    ref, offs, ix, ek, ev, codes, ro = setup
    reads = gpu.to_device(codes, ro)
    ea, _, _ = oracle.seed(ek, ev, codes, ro, "10", 15, 10)
    # a table of another index: smaller than this index needs, refused on the host
    other = gpu.index_build(gpu.to_device(ref[:300_000], [0, 300_000]), "10", 15, 10)
    with pytest.raises(api.GodietError):
        gpu.seed(ix.with_table(gpu.table_build(other).table), reads, "10", 15, 10)
    # a table of other keys with the same count: its key fingerprint differs, so seeding
    # searches the sorted keys instead
    shifted = api.DeviceIndex(ix.keys + 1, ix.vals, ix.n, 32)
    mixed = ix.with_table(gpu.table_build(shifted).table)
    a, _, _ = gpu.seed(mixed, reads, "10", 15, 10)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    empty = gpu.index_build(gpu.to_device(ref[:5], [0, 5]), "10", 15, 10)
    assert empty.n == 0
    a, off, _ = gpu.seed(gpu.table_build(empty), reads, "10", 15, 10)
    assert a.shape[0] == 0 and int(off[-1].item()) == 0


def test_contain_through_table_equals_oracle(gpu):
    codes, offs = datagen.genome_db(12, 91, min_len=50_000, max_len=200_000)
    rc, ro, _ = datagen.sample_from_genomes(codes, offs, 3000, 4, 150, 92)
    ix = gpu.index_build(gpu.to_device(codes, offs), "10", 15, 10, val_bits=64)
    ek, ev = oracle.index_build(codes, offs, "10", 15, 10, val_bits=64)
    c, sz = gpu.contain(gpu.table_build(ix), gpu.to_device(rc, ro), "10", 15, 10, 12)
    ec, esz = oracle.contain(ek, ev, rc, ro, "10", 15, 10, 12)
    assert np.array_equal(u32(c), ec) and np.array_equal(u32(sz), esz)


def test_saved_index_seeds_identically(gpu, setup, tmp_path):
    ref, offs, ix, ek, ev, codes, ro = setup
    full = gpu.table_build(gpu.rmi_train(ix, root="mlp", log2_leaves=12))
    p = str(tmp_path / "index.bin")
    gpu.save_index(p, full, "10", 15, 10)
    back, head = gpu.load_index(p)
    assert (head["pattern"], head["k"], head["w"], head["n"]) == ("10", 15, 10, ix.n)
    reads = gpu.to_device(codes, ro)
    ea, _, _ = oracle.seed(ek, ev, codes, ro, "10", 15, 10)
    for variant in (back, back.with_table(None), back.with_rmi(None).with_table(None)):
        a, _, _ = gpu.seed(variant, reads, "10", 15, 10)
        assert np.array_equal(u32(a).reshape(-1, 4), ea)
