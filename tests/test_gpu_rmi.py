"""Learned index: lookups and seeding through the two-stage model are identical to plain
binary search and to the oracle, for present keys, absent keys, the array ends, runs of
equal keys, a corrupted model (errors zeroed, slopes scrambled) and a model trained on
another index."""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def ref_index(gpu):
    ref = datagen.add_repeats(datagen.random_genome(2_000_000, 41), 241, frac=0.2, seg_len=3000,
                              copies=8)
    offs = np.array([0, ref.size], np.int64)
    ek, ev = oracle.index_build(ref, offs, "10", 15, 10)
    ix = gpu.index_build(gpu.to_device(ref, offs), "10", 15, 10)
    assert np.array_equal(ix.keys.cpu().numpy().view(np.uint64), ek)
    return ref, offs, ek, ev, ix


def queries_from(ek):
    rng = np.random.default_rng(42)
    present = ek[rng.integers(0, ek.size, 20_000)]
    absent = rng.integers(0, 2**64, 20_000, dtype=np.uint64)
    edges = np.array([0, 1, 2**64 - 1, 2**64 - 2, ek[0], ek[-1], ek[0] - np.uint64(1),
                      ek[-1] + np.uint64(1)], np.uint64)
    near = np.concatenate([present[:5000] + np.uint64(1), present[:5000] - np.uint64(1)])
    return np.concatenate([present, absent, edges, near])


@pytest.mark.parametrize("root,leaves", [("mlp", 18), ("linear", 18), ("mlp", 10), ("linear", 4)])
def test_rmi_lookup_equals_binary_search(gpu, ref_index, root, leaves):
    ref, offs, ek, ev, ix = ref_index
    q = queries_from(ek)
    qt = torch.from_numpy(q.view(np.int64)).cuda()
    m = gpu.rmi_train(ix, root=root, log2_leaves=leaves)
    lb_b, occ_b = gpu.lookup(ix, qt)
    lb_r, occ_r = gpu.lookup(m, qt)
    elb, eocc = oracle.lookup(ek, q)
    assert np.array_equal(u32(lb_b).astype(np.uint64), elb)
    assert np.array_equal(u32(occ_b).astype(np.uint64), eocc)
    assert np.array_equal(u32(lb_r), u32(lb_b))
    assert np.array_equal(u32(occ_r), u32(occ_b))


@pytest.mark.parametrize("root", ["mlp", "linear"])
def test_rmi_training_is_deterministic(gpu, ref_index, root):
    # every leaf's base is the first key routed to it or past it, whatever order the
    # claims land in: two trainings give the same bytes and the bases never decrease
    ref, offs, ek, ev, ix = ref_index
    a = gpu.rmi_train(ix, root=root, log2_leaves=18).rmi.cpu().numpy()
    b = gpu.rmi_train(ix, root=root, log2_leaves=18).rmi.cpu().numpy()
    assert np.array_equal(a, b)
    base = a[320:].view(np.uint32).reshape(-1, 4)[:, 1]     # header 320 B, 16-B leaves
    assert base.size == 1 << 18 and base[0] == 0
    assert np.all(np.diff(base.astype(np.int64)) >= 0) and base[-1] <= ek.size


def test_rmi_corrupted_model_falls_back(gpu, ref_index):
    ref, offs, ek, ev, ix = ref_index
    q = queries_from(ek)
    qt = torch.from_numpy(q.view(np.int64)).cuda()
    m = gpu.rmi_train(ix, root="mlp", log2_leaves=12)
    words = m.rmi.view(torch.int32)                 # header 320 B, then 16-B leaves
    leaves = words[80:].view(-1, 4)                 # khi, base, slope, icpt|err_lo|err_hi
    leaves[:, 3] = leaves[:, 3] & 0xFFFF            # both errors 0
    leaves[::3, 2] = 0x3f800000                     # slope = 1.0: wild predictions
    leaves[1::5, 1] = 0x7FFFFFFF                    # base far past the end
    lb_r, occ_r = gpu.lookup(m, qt)
    elb, eocc = oracle.lookup(ek, q)
    assert np.array_equal(u32(lb_r).astype(np.uint64), elb)
    assert np.array_equal(u32(occ_r).astype(np.uint64), eocc)


def test_rmi_trained_on_other_index_is_ignored(gpu, ref_index):
    ref, offs, ek, ev, ix = ref_index
    other = gpu.index_build(gpu.to_device(ref[:500_000], [0, 500_000]), "10", 15, 10)
    m = gpu.rmi_train(other, root="mlp", log2_leaves=12)
    mixed = ix.with_rmi(m.rmi)
    q = queries_from(ek)
    lb_r, occ_r = gpu.lookup(mixed, torch.from_numpy(q.view(np.int64)).cuda())
    elb, eocc = oracle.lookup(ek, q)
    assert np.array_equal(u32(lb_r).astype(np.uint64), elb)


def test_seed_with_rmi_matches_oracle(gpu, ref_index):
    ref, offs, ek, ev, ix = ref_index
    codes, ro, _, _ = datagen.fixed_reads(ref, 3000, 150, 43, sub=0.01)
    reads = gpu.to_device(codes, ro)
    m = gpu.rmi_train(ix, root="mlp", log2_leaves=14)
    a_r, off_r, sh_r = gpu.seed(m, reads, "10", 15, 10)
    a_b, off_b, sh_b = gpu.seed(ix, reads, "10", 15, 10)
    ea, eoff, esh = oracle.seed(ek, ev, codes, ro, "10", 15, 10)
    assert np.array_equal(u32(a_r).reshape(-1, 4), ea)
    assert np.array_equal(u32(a_b).reshape(-1, 4), ea)
    assert np.array_equal(sh_r.cpu().numpy().astype(np.uint32), esh)


def test_rmi_empty_and_tiny_index(gpu):
    for n_ref in (0, 30, 400):
        ref = datagen.random_genome(max(n_ref, 1), 44)[:n_ref]
        offs = np.array([0, n_ref], np.int64)
        ix = gpu.index_build(gpu.to_device(ref, offs), "1", 11, 3)
        ek, _ = oracle.index_build(ref, offs, "1", 11, 3)
        m = gpu.rmi_train(ix, root="mlp", log2_leaves=6)
        q = np.concatenate([ek, np.array([0, 5, 2**64 - 1], np.uint64)])
        lb, occ = gpu.lookup(m, torch.from_numpy(q.view(np.int64)).cuda())
        elb, eocc = oracle.lookup(ek, q)
        assert np.array_equal(u32(lb).astype(np.uint64), elb)
        assert np.array_equal(u32(occ).astype(np.uint64), eocc)
