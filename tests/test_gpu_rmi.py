"""Learned index: lookups and seeding through the two-stage model are identical to plain
binary search and to the oracle, for present keys, absent keys, the array ends, runs of
equal keys, a corrupted model (errors zeroed, slopes scrambled) and a model trained on
another index."""
from fractions import Fraction

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
    # every leaf's start is the first key routed to it or past it, written by the one lane
    # where the (monotone) routing steps up to it: two trainings give the same bytes;
    # every leaf's base position (its first key plus the fitted intercept) lies inside
    # the keys
    ref, offs, ek, ev, ix = ref_index
    a = gpu.rmi_train(ix, root=root, log2_leaves=18).rmi.cpu().numpy()
    b = gpu.rmi_train(ix, root=root, log2_leaves=18).rmi.cpu().numpy()
    assert np.array_equal(a, b)
    leaves = a[576:].view(np.uint32).reshape(-1, 4)         # header 576 B, 16-B leaves
    assert leaves.shape[0] == 1 << 18 and np.all(leaves[:, 1] <= ek.size)
    slope = leaves[:, 2].view(np.float32)
    assert np.all(np.isfinite(slope)) and np.all(slope >= 0)


def round_f32(v):
    """The float32 nearest to the rational v (ties to even), as a Python float."""
    if v == 0:
        return 0.0
    sign, v = (-1 if v < 0 else 1), abs(v)
    e = v.numerator.bit_length() - v.denominator.bit_length()
    while v >= Fraction(2) ** (e + 1):
        e += 1
    while v < Fraction(2) ** e:
        e -= 1
    e = max(e, -126)                                  # subnormals share the least exponent
    q = v / Fraction(2) ** (e - 23)
    m, r = divmod(q.numerator, q.denominator)
    if 2 * r > q.denominator or (2 * r == q.denominator and m % 2):
        m += 1
    return sign * m * 2.0 ** (e - 23)


def mlp_value(blob, xs):
    """The MLP root of a model blob before its scaling to leaves, evaluated as the kernels
    do: segment j = number of knots below x, then sb[j] * x + sa[j] rounded once to
    float32 (a fused multiply-add), computed exactly here."""
    f = blob[:576].view(np.float32)
    t, sa, sb = f[8:40], f[73:106], f[106:139]       # byte offsets 32, 292 and 424
    j = np.sum(t[None, :] < xs[:, None], axis=1)
    y = [round_f32(Fraction(float(sb[i])) * Fraction(float(x)) + Fraction(float(sa[i])))
         for i, x in zip(j, xs)]
    return np.array(y), t, sb


@pytest.mark.parametrize("leaves", [18, 22])
def test_rmi_mlp_root_is_monotone(gpu, ref_index, leaves):
    # leaf starts are written by one lane each, which needs routing monotone in the key:
    # the trained root never decreases, across every knot and between samples of [0, 1]
    ref, offs, ek, ev, ix = ref_index
    blob = gpu.rmi_train(ix, root="mlp", log2_leaves=leaves).rmi.cpu().numpy()
    assert blob[4:8].view(np.uint32)[0] == 1            # the MLP root was kept
    _, t, sb = mlp_value(blob, np.zeros(1, np.float32))
    assert np.all(sb >= 0)
    steps = np.arange(-4, 5, dtype=np.int32)
    near = (t.view(np.int32)[:, None] + steps[None, :]).ravel().view(np.float32)
    rng = np.random.default_rng(3)
    xs = np.concatenate([near[(near >= 0) & (near <= 1)], rng.random(20_000, np.float32),
                         np.float32([0, 1])])
    y, _, _ = mlp_value(blob, np.unique(xs))
    assert np.all(np.diff(y) >= 0)


def test_rmi_corrupted_model_falls_back(gpu, ref_index):
    ref, offs, ek, ev, ix = ref_index
    q = queries_from(ek)
    qt = torch.from_numpy(q.view(np.int64)).cuda()
    m = gpu.rmi_train(ix, root="mlp", log2_leaves=12)
    words = m.rmi.view(torch.int32)                 # header 576 B, then 16-B leaves
    leaves = words[144:].view(-1, 4)                # khi, base, slope, err_lo|err_hi
    leaves[:, 3] = 0                                # both errors 0
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


def test_rmi_model_beyond_its_bytes_is_ignored(gpu, ref_index):
    # a model whose leaves would lie past the bytes the index declares is not read (the
    # buffers below are allocated large enough that even a read would stay inside them)
    import ctypes
    from paper_2211_08157_amd import api
    ref, offs, ek, ev, ix = ref_index
    q = queries_from(ek)
    qt = torch.from_numpy(q.view(np.int64)).cuda()
    elb, eocc = oracle.lookup(ek, q)
    L = api.lib()
    size12, size13 = L.godiet_rmi_size(12), L.godiet_rmi_size(13)
    blob = torch.zeros(size13 + 64, dtype=torch.uint8, device="cuda")
    off = (-blob.data_ptr()) % 64
    blob = blob[off:off + size13]
    r = L.godiet_rmi_train(ctypes.byref(ix.c()), 1, 12, ctypes.c_void_p(blob.data_ptr()), size13,
                           api._stream())
    assert r == api.OK
    reads = gpu.to_device(*datagen.fixed_reads(ref, 500, 150, 45, sub=0.01)[:2])
    for case in ("truncated", "leaf count"):
        if case == "truncated":
            b = blob[:size12 // 2]                    # half the leaves' bytes declared
        else:
            blob.view(torch.int32)[2] = 13            # header claims 2^13 leaves ...
            b = blob[:size12]                         # ... but declares 2^12 leaves' bytes
        lb, occ = gpu.lookup(ix.with_rmi(b), qt)
        assert np.array_equal(u32(lb).astype(np.uint64), elb)
        assert np.array_equal(u32(occ).astype(np.uint64), eocc)
        a, _, _ = gpu.seed(ix.with_rmi(b), reads, "10", 15, 10)
        a0, _, _ = gpu.seed(ix, reads, "10", 15, 10)
        assert a.shape[0] > 0 and torch.equal(a, a0), case
    # fewer bytes than a header and two leaves: refused on the host
    with pytest.raises(api.GodietError):
        gpu.lookup(ix.with_rmi(blob[:300]), qt)


def test_rmi_stats_account_for_every_query(gpu, ref_index):
    # the diagnostics see every query once; a fitted model brackets every present key, a
    # model with its error bounds zeroed misses some, and each query's window is the one
    # the lookups read (their results stay those of binary search either way)
    ref, offs, ek, ev, ix = ref_index
    q = queries_from(ek)
    qt = torch.from_numpy(q.view(np.int64)).cuda()
    m = gpu.rmi_train(ix, root="mlp", log2_leaves=12)
    st = gpu.rmi_stats(m, qt)
    assert st["queries"] == q.size and st["fallbacks"] + sum(st["window_keys"]) == q.size
    present = torch.from_numpy(ek[::7].view(np.int64)).cuda()
    assert gpu.rmi_stats(m, present)["fallbacks"] == 0
    m.rmi.view(torch.int32)[144:].view(-1, 4)[:, 3] = 0     # err_lo = err_hi = 0
    st0 = gpu.rmi_stats(m, present)
    assert 0 < st0["fallbacks"] < present.numel()
    # every bracketing window is [p, p + 1) with its two brackets: 3 keys (fewer at the ends)
    assert sum(st0["window_keys"][:3]) == present.numel() - st0["fallbacks"]
    lb, occ = gpu.lookup(m, present)
    elb, eocc = oracle.lookup(ek, ek[::7])
    assert np.array_equal(u32(lb).astype(np.uint64), elb)


def test_random_gather_probe(gpu):
    # the probe behind the lookups' random-request roofline: out[i] = src[idx[i]], with an
    # out-of-range index reported in the status word (and 0 written)
    import torch
    src = torch.arange(7, 7 + 100_003, dtype=torch.int64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    for n in (0, 1, 999, 300_001):
        idx = torch.randint(0, src.numel(), (n,), device="cuda", generator=g)
        out, st = gpu.random_gather(src, idx)
        assert torch.equal(out, src[idx]) and int(st.item()) == 0
    idx = torch.tensor([0, 100_003, 5, 1 << 40], dtype=torch.int64, device="cuda")
    out, st = gpu.random_gather(src, idx)
    assert out.cpu().tolist() == [7, 0, 12, 0] and int(st.item()) == gpu.STATUS_RANGE
