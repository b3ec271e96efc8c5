"""Containment counts (per-genome shared distinct minimizers) on the GPU against the
oracle: a small multi-genome database with shared blocks, reads from a few genomes,
alignment options, the learned-index lookups, and more genomes than the LDS histogram
holds."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def db(gpu):
    codes, offs = datagen.genome_db(24, 51, min_len=40_000, max_len=160_000)
    reads, ro, src = datagen.sample_from_genomes(codes, offs, 4000, 5, 150, 52, sub=0.01)
    ek, ev = oracle.index_build(codes, offs, "10", 15, 10, val_bits=64)
    ix = gpu.index_build(gpu.to_device(codes, offs), "10", 15, 10, val_bits=64)
    assert np.array_equal(ix.keys.cpu().numpy().view(np.uint64), ek)
    assert np.array_equal(ix.vals.cpu().numpy().view(np.uint64), ev)
    return codes, offs, reads, ro, ek, ev, ix


@pytest.mark.parametrize("kw", [{}, {"max_occ": 2}, {"shift_mode": 1}, {"align_t": 3}])
def test_contain_matches_oracle(gpu, db, kw):
    codes, offs, reads, ro, ek, ev, ix = db
    c, s = gpu.contain(ix, gpu.to_device(reads, ro), "10", 15, 10, 24, **kw)
    ec, es = oracle.contain(ek, ev, reads, ro, "10", 15, 10, 24,
                            shift_mode=kw.get("shift_mode", -1), align_t=kw.get("align_t", 0),
                            max_occ=kw.get("max_occ", 0))
    assert np.array_equal(u32(s), es)
    assert np.array_equal(u32(c), ec)
    assert (ec > 0).sum() >= 5


def test_contain_with_learned_index(gpu, db):
    codes, offs, reads, ro, ek, ev, ix = db
    m = gpu.rmi_train(ix, root="mlp", log2_leaves=12)
    c, s = gpu.contain(m, gpu.to_device(reads, ro), "10", 15, 10, 24)
    ec, es = oracle.contain(ek, ev, reads, ro, "10", 15, 10, 24)
    assert np.array_equal(u32(c), ec) and np.array_equal(u32(s), es)


def test_contain_many_genomes(gpu):
    codes, offs = datagen.genome_db(5000, 53, min_len=300, max_len=900, shared_frac=0.1)
    reads, ro, _ = datagen.sample_from_genomes(codes, offs, 3000, 40, 100, 54, sub=0.0)
    ek, ev = oracle.index_build(codes, offs, "1", 11, 5, val_bits=64)
    ix = gpu.index_build(gpu.to_device(codes, offs), "1", 11, 5, val_bits=64)
    c, s = gpu.contain(ix, gpu.to_device(reads, ro), "1", 11, 5, 5000)
    ec, es = oracle.contain(ek, ev, reads, ro, "1", 11, 5, 5000)
    assert np.array_equal(u32(s), es) and np.array_equal(u32(c), ec)
