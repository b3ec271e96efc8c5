"""Uneven-length batching: one seeding pass over a mixed batch of short, HiFi-like and
ONT-like reads equals the oracle and the per-class runs; the pass captured into a HIP
graph and replayed (with other GPU work in between) reproduces the eager outputs; every
autotuner candidate gives identical anchors."""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu
PAT, K, W = "10", 15, 10


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def mixed(gpu):
    ref = datagen.add_repeats(datagen.random_genome(3_000_000, 61), 261, frac=0.1, seg_len=4000,
                              copies=6)
    roffs = np.array([0, ref.size], np.int64)
    rng = np.random.default_rng(62)
    short = datagen.fixed_reads(ref, 2000, 150, 63, sub=0.005, ins=0.0005, dele=0.0005)
    hifi = datagen.variable_reads(ref, datagen.hifi_lengths(20, rng), 64, 0.005, 0.0025, 0.0025)
    ont = datagen.variable_reads(ref, datagen.ont_lengths(20, rng), 65, 0.04, 0.02, 0.02)
    classes = [short[:2], hifi[:2], ont[:2]]
    codes, offs = datagen.concat(classes)
    ix = gpu.index_build(gpu.to_device(ref, roffs), PAT, K, W)
    ek, ev = oracle.index_build(ref, roffs, PAT, K, W)
    return ref, ix, ek, ev, classes, codes, offs


def test_mixed_batch_matches_oracle(gpu, mixed):
    ref, ix, ek, ev, classes, codes, offs = mixed
    a, off, sh = gpu.seed(ix, gpu.to_device(codes, offs), PAT, K, W)
    ea, eoff, esh = oracle.seed(ek, ev, codes, offs, PAT, K, W)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)


def test_mixed_batch_equals_per_class_runs(gpu, mixed):
    ref, ix, ek, ev, classes, codes, offs = mixed
    a, off, sh = gpu.seed(ix, gpu.to_device(codes, offs), PAT, K, W)
    parts, base = [], 0
    for c_codes, c_offs in classes:
        pa, _, _ = gpu.seed(ix, gpu.to_device(c_codes, c_offs), PAT, K, W)
        pa = u32(pa).reshape(-1, 4).copy()
        pa[:, 0] += base
        parts.append(pa)
        base += len(c_offs) - 1
    assert np.array_equal(u32(a).reshape(-1, 4), np.concatenate(parts))


def test_graph_replay_matches_eager(gpu, mixed):
    from paper_2211_08157_amd.plan import SeedPlan
    ref, ix, ek, ev, classes, codes, offs = mixed
    reads = gpu.to_device(codes, offs)
    plan = SeedPlan(ix, reads, PAT, K, W)
    plan.run()
    plan.check()
    eager = [t.cpu().numpy().copy() for t in plan.outputs()]
    plan.capture()
    other = gpu.to_device(*classes[0])
    for i in range(3):
        plan.anchors.fill_(-1)
        plan.read_off.fill_(-1)
        gpu.seed(ix, other, PAT, K, W)            # eager work between replays
        torch.cuda.synchronize()
        plan.replay()
        plan.check()
        got = [t.cpu().numpy() for t in plan.outputs()]
        for g, e in zip(got, eager):
            assert np.array_equal(g, e), "replay %d differs" % i


def test_autotune_candidates_agree(gpu, mixed, tmp_path):
    from paper_2211_08157_amd import autotune
    ref, ix, ek, ev, classes, codes, offs = mixed
    reads = gpu.to_device(codes, offs)
    grid = {"long_records": [32, 4096], "lookup_blocks": [64, 8192], "long_blocks": [1, 7, 512]}
    cache = str(tmp_path / "tune.json")
    best, report = autotune.tune(ix, reads, PAT, K, W, grid=grid, reps=1, cache=cache)
    assert len(report) == 12 and best in [r[0] for r in report]
    again, rep2 = autotune.tune(ix, reads, PAT, K, W, grid=grid, reps=1, cache=cache)
    assert again == best and rep2 == []
    a, _, _ = gpu.seed(ix, reads, PAT, K, W, tuning=best)
    ea, _, _ = oracle.seed(ek, ev, codes, offs, PAT, K, W)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)


def test_batch_with_huge_reads_matches_oracle(gpu, mixed):
    # reads above 16,384 minimizer records take the workgroup-per-read path
    ref, ix, ek, ev, classes, codes, offs = mixed
    huge = datagen.variable_reads(ref, [400_000, 150, 250_000, 30_000, 150], 66, 0.01, 0.005,
                                  0.005)
    hc, ho = datagen.concat([classes[0], huge[:2]])
    a, off, sh = gpu.seed(ix, gpu.to_device(hc, ho), PAT, K, W)
    ea, eoff, esh = oracle.seed(ek, ev, hc, ho, PAT, K, W)
    assert np.array_equal(u32(a).reshape(-1, 4), ea)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), eoff)
    assert np.array_equal(sh.cpu().numpy().astype(np.uint32), esh)
