"""Full-size parity: the library on the workloads at their real sizes, checked bit-exact
against digests of the oracle's complete outputs on the same seeded inputs
(tests/golden/fullsize_oracle.json, written by tests/golden/make_fullsize.py, which calls
only the oracle).  Each digest covers every output element; its per-part digests name the
part that differs when a check fails.

  * Illumina-like 100 Mbp reference, 1M x 150 bp reads, '10', k21 w11: the benchmark's
    own preallocated step (index build + seeding), with binary search and with the
    learned index, then location voting on its anchors (D 16, V 3, 4 winners); the same
    with assembly gaps (about 5 % N) in the reference and N calls in the reads;
  * 1 Gbp reference with one mixed batch of 2M short + 20k HiFi-like + 20k ONT-like reads,
    '10' and '110': index build, then one HIP-graph-captured seeding pass with launch
    parameters from the autotuner, then location voting (D 100, V 3, 4 winners);
  * 500M lookups (80 % drawn from that batch's read minimizers, 20 % random keys) in the
    1 Gbp '10' index (about 83M keys) and the unsparsified '11' index (about 167M keys):
    learned index (MLP and linear roots, 2^18 leaves; 2^22 leaves on '11') equals binary
    search equals the oracle; every result also satisfies the lower-bound property;
  * 1,000-genome containment database with 10M reads: 64-bit-value index and per-genome
    shared-minimizer counts, with binary search and with the learned index;
  * the seed-matching experiment on 100,000 pairs of 1,000 bases: edit distances, seed
    counts of four settings and their accepted-pairs curves.
"""
import json
import os

import numpy as np
import pytest
import torch

import datagen
import fullsize

pytestmark = pytest.mark.gpu
K, W = 21, 11
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_oracle.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def want(golden, key):
    if key not in golden:
        pytest.fail("no oracle digest for %s in %s" % (key, GOLDEN))
    return golden[key]


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def host_vals(t):
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a.view(np.uint64)


def assert_digest(got, exp, what):
    bad = fullsize.diff_parts(got, exp)
    assert got["n"] == exp["n"] and got["sha256"] == exp["sha256"], (
        "%s differs from the oracle: n %d vs %d, differing parts %s"
        % (what, got["n"], exp["n"], bad[:16]))


@pytest.mark.timeout(900)
def test_illumina_100mbp_benchmark_step(gpu, golden):
    import bench
    exp = want(golden, "illumina-100Mbp/10")
    d = datagen.workload_illumina()
    s = bench.Session(gpu, gpu.to_device(d["ref"], d["ref_offsets"]),
                      gpu.to_device(d["reads"], d["read_offsets"]), d["ref_offsets"],
                      d["read_offsets"], "10", K, W)
    del d
    # binary search, learned index, and the learned-index step with index construction on
    # a second stream overlapping the read sketches
    for learned, overlap in ((False, False), (True, False), (True, True)):
        s.overlap = overlap
        s.step("learned_index" if learned else "binary_search")
        s.check()
        n = s.n_index
        got = fullsize.index_digest(host_u64(s.ikeys[:n]), host_vals(s.ivals[:n]))
        assert_digest(got, exp["index"], "index")
        na = s.n_anchors
        a = s.anchors[:4 * na].cpu().numpy().view(np.uint32)
        got = fullsize.anchors_digest(a, host_u64(s.roff), s.shift.cpu().numpy())
        assert_digest(got, exp["anchors"], "anchors (learned index %s, overlap %s)"
                      % (learned, overlap))
    s.overlap = False
    check_votes(gpu, s.anchors[:4 * s.n_anchors].view(-1, 4), s.roff, exp["votes"])


@pytest.mark.timeout(900)
def test_illumina_gapped_100mbp_benchmark_step(gpu, golden):
    # the same step on the workload with assembly gaps and N calls (N-aware path)
    import bench
    exp = want(golden, "illumina-gapped-100Mbp/10")
    d = datagen.workload_gapped()
    s = bench.Session(gpu, gpu.to_device(d["ref"], d["ref_offsets"]),
                      gpu.to_device(d["reads"], d["read_offsets"]), d["ref_offsets"],
                      d["read_offsets"], "10", K, W)
    del d
    assert s.ref.nmask is not None and s.reads.nmask is not None
    for mode in ("binary_search", "learned_index"):
        s.step(mode)
        s.check()
        n = s.n_index
        got = fullsize.index_digest(host_u64(s.ikeys[:n]), host_vals(s.ivals[:n]))
        assert_digest(got, exp["index"], "index")
        na = s.n_anchors
        a = s.anchors[:4 * na].cpu().numpy().view(np.uint32)
        got = fullsize.anchors_digest(a, host_u64(s.roff), s.shift.cpu().numpy())
        assert_digest(got, exp["anchors"], "anchors (%s)" % mode)
    check_votes(gpu, s.anchors[:4 * s.n_anchors].view(-1, 4), s.roff, exp["votes"])


@pytest.mark.timeout(900)
def test_fig4_100k_pairs(gpu, golden):
    # seed-matching experiment at full size: 100,000 pairs of 1,000 bases
    exp = want(golden, "fig4-100k")
    o, oo, c, co, _ = datagen.workload_fig4()
    so, sc = gpu.to_device(o, oo), gpu.to_device(c, co)
    dist = gpu.edit_distance(so, sc)
    got = fullsize.pairs_digest(dist.cpu().numpy().view(np.uint32))
    assert_digest(got, exp["dist"], "edit distances")
    max_e = exp["max_e"]
    for setting, ent in exp["settings"].items():
        pattern, k, w = setting.split("/")
        counts = gpu.seed_match(so, sc, pattern, int(k), int(w))
        got = fullsize.pairs_digest(counts.cpu().numpy().view(np.uint32).reshape(-1, 8))
        assert_digest(got, ent["counts"], "seed counts " + setting)
        flat = counts.reshape(-1)
        for alg, curve in ent["accepted"].items():
            acc = gpu.accepted_pairs(dist, flat, alg, max_e).cpu().numpy()
            assert acc.tolist() == curve, (setting, alg)


def check_votes(gpu, anchors, read_off, exp, sorts=("adaptive",)):
    for sort in sorts:
        w, nw = gpu.vote(anchors, read_off, exp["D"], exp["V"], exp["cap"], sort=sort)
        got = fullsize.votes_digest(nw.cpu().numpy().view(np.uint32), gpu.winners_rows(w, nw))
        assert_digest(got, exp, "location votes (%s sort)" % sort)


@pytest.fixture(scope="module")
def uneven(gpu):
    d = datagen.workload_uneven()
    ref = gpu.to_device(d["ref"], d["ref_offsets"])
    reads = gpu.to_device(d["reads"], d["read_offsets"])
    return dict(ref=ref, reads=reads)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("pattern", ["10", "110"])
def test_uneven_1gbp_graph_captured_autotuned(gpu, golden, uneven, pattern, tmp_path):
    from paper_2211_08157_amd import autotune
    from paper_2211_08157_amd.plan import SeedPlan
    exp = want(golden, "uneven-1Gbp/" + pattern)
    ix = gpu.index_build(uneven["ref"], pattern, K, W)
    got = fullsize.index_digest(host_u64(ix.keys), host_vals(ix.vals))
    assert_digest(got, exp["index"], "index")
    # a small grid: every candidate's anchors are compared by the tuner itself
    grid = {"long_records": [64, 192], "lookup_blocks": [8192], "long_blocks": [1024]}
    tuning, report = autotune.tune(ix, uneven["reads"], pattern, K, W, grid=grid, reps=1,
                                   cache=str(tmp_path / "tune.json"))
    assert len(report) == 2
    plan = SeedPlan(ix, uneven["reads"], pattern, K, W, tuning=tuning)
    plan.capture()
    plan.status.zero_()
    plan.replay()
    plan.check()
    a, off, sh = plan.outputs()
    got = fullsize.anchors_digest(a.cpu().numpy().view(np.uint32), host_u64(off),
                                  sh.cpu().numpy())
    assert_digest(got, exp["anchors"], "anchors")
    # the batch digit sort of tens of millions of anchors takes the two-level scatter
    check_votes(gpu, a, off, exp["votes"], sorts=("adaptive", "radix"))


@pytest.mark.timeout(900)
def test_uneven_1gbp_benchmark_step(gpu, golden, uneven):
    # the benchmark's headline step on the mixed batch, as it times it: index build, then
    # learned-index training (or nothing, or the hash table), then seeding with launch
    # parameters from the autotuner; every mode, and the step replayed as one HIP graph
    import bench
    from paper_2211_08157_amd import autotune
    exp = want(golden, "uneven-1Gbp/10")
    d = datagen.workload_uneven()
    ix = gpu.index_build(uneven["ref"], "10", K, W)
    leaves = bench.leaves_for(ix.n)
    tuning, _ = autotune.tune(gpu.rmi_train(ix, root="mlp", log2_leaves=leaves), uneven["reads"],
                              "10", K, W, grid=bench.TUNE_GRID, reps=1, use_cache=False)
    del ix
    s = bench.Session(gpu, uneven["ref"], uneven["reads"], d["ref_offsets"], d["read_offsets"],
                      "10", K, W, log2_leaves=leaves, tuning=tuning)
    del d
    for mode in bench.STEP_MODES:
        s.step(mode)
        s.check()
        n = s.n_index
        got = fullsize.index_digest(host_u64(s.ikeys[:n]), host_vals(s.ivals[:n]))
        assert_digest(got, exp["index"], "index")
        a = s.anchors[:4 * s.n_anchors].cpu().numpy().view(np.uint32)
        got = fullsize.anchors_digest(a, host_u64(s.roff), s.shift.cpu().numpy())
        assert_digest(got, exp["anchors"], "anchors (%s)" % mode)
    bench.graph_step(torch, s, "learned_index", 2)
    a = s.anchors[:4 * s.n_anchors].cpu().numpy().view(np.uint32)
    got = fullsize.anchors_digest(a, host_u64(s.roff), s.shift.cpu().numpy())
    assert_digest(got, exp["anchors"], "anchors (graph-replayed step)")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("pattern", ["10", "11"])
def test_learned_index_500m_lookups_1gbp(gpu, golden, uneven, pattern):
    ent = want(golden, "lookups-1Gbp/" + pattern)
    exp = ent["lookups"]
    ix = gpu.index_build(uneven["ref"], pattern, K, W)
    if "index_keys" in ent:
        assert ix.n == ent["index_keys"]
    rk, _, _ = gpu.sketch(uneven["reads"], pattern, K, W)
    q = fullsize.lookup_queries(host_u64(rk))
    del rk
    qd = torch.from_numpy(q.view(np.int64)).cuda()
    del q
    lb0, occ0 = gpu.lookup(ix, qd)
    # both roots at 2^18 leaves; the unsparsified array also at about 40 keys per leaf
    models = [("mlp", 18), ("linear", 18)] + ([("mlp", 22)] if pattern == "11" else [])
    for root, leaves in models:
        lb1, occ1 = gpu.lookup(gpu.rmi_train(ix, root=root, log2_leaves=leaves), qd)
        assert torch.equal(lb0, lb1) and torch.equal(occ0, occ1), (root, leaves)
        del lb1, occ1
    # lower-bound property of every result: keys[lb-1] < q <= keys[lb], and the run
    # [lb, lb+occ) holds exactly the keys equal to q (keys compared as unsigned)
    keys = ix.keys
    n = ix.n
    flip = torch.tensor(-2**63, dtype=torch.int64, device=qd.device)
    ks = keys ^ flip
    qs = qd ^ flip
    lb = lb0.to(torch.int64)
    occ = occ0.to(torch.int64)
    assert bool(((lb >= 0) & (lb + occ <= n)).all())
    prev = ks[(lb - 1).clamp(min=0)]
    assert bool(((lb == 0) | (prev < qs)).all())
    at = ks[lb.clamp(max=n - 1)]
    assert bool(((lb == n) | (at >= qs)).all())
    assert bool(((occ == 0) | (at == qs)).all())
    last = ks[(lb + occ - 1).clamp(min=0, max=n - 1)]
    assert bool(((occ == 0) | (last == qs)).all())
    after = ks[(lb + occ).clamp(max=n - 1)]
    assert bool(((lb + occ == n) | (after != qs)).all())
    del prev, at, last, after, lb, occ, ks, qs
    got = fullsize.lookup_digest(lb0.cpu().numpy().view(np.uint32),
                                 occ0.cpu().numpy().view(np.uint32))
    assert got["n"] == 500_000_000
    assert got["found"] == exp["found"] and got["occ_sum"] == exp["occ_sum"]
    assert_digest(got, exp, "lookups")


@pytest.mark.timeout(900)
def test_containment_1000_genomes(gpu, golden):
    exp = want(golden, "containment-1000/10")
    d = datagen.workload_containment()
    ng = d["ref_offsets"].size - 1
    ref = gpu.to_device(d["ref"], d["ref_offsets"])
    reads = gpu.to_device(d["reads"], d["read_offsets"])
    del d
    ix = gpu.index_build(ref, "10", K, W, val_bits=64)
    del ref
    got = fullsize.index_digest(host_u64(ix.keys), host_vals(ix.vals))
    assert_digest(got, exp["index"], "index")
    want_counts = np.array(exp["counts"], np.uint32)
    want_sizes = np.array(exp["sizes"], np.uint32)
    for index in (ix, gpu.rmi_train(ix, root="mlp", log2_leaves=18)):
        counts, sizes = gpu.contain(index, reads, "10", K, W, ng)
        c = counts.cpu().numpy().view(np.uint32)
        s = sizes.cpu().numpy().view(np.uint32)
        assert np.array_equal(s, want_sizes)
        assert np.array_equal(c, want_counts), np.nonzero(c != want_counts)[0][:10]
