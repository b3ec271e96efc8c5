"""The workspace-free sketch entry point, godiet_sketch_static (for callers that cannot
allocate), against godiet_sketch through the C ABI: two calls in a row on one GPU, the
second on a smaller batch with other parameters, every output element equal; and a batch
whose sketch scratch exceeds the library's static array is refused on the host before
anything is enqueued."""
import ctypes

import numpy as np
import pytest

import datagen
from paper_2211_08157_amd import api


def static_sketch(seqs, pattern, k, w, capacity):
    import torch
    L = api.lib()
    keys = torch.empty(max(capacity, 1), dtype=torch.int64, device="cuda")
    vals = torch.empty(max(capacity, 1), dtype=torch.int32, device="cuda")
    mz = torch.empty(seqs.n_seq + 1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    prm = api.Params(pattern.encode(), k, w, 0)
    r = L.godiet_sketch_static(ctypes.byref(seqs.c()), ctypes.byref(prm), None,
                               ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                               ctypes.c_void_p(mz.data_ptr()), capacity,
                               ctypes.c_void_p(st.data_ptr()),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert r == api.OK, r
    torch.cuda.synchronize()
    return keys, vals, mz, int(st.item())


def batch(seed, n_reads, ref_len):
    ref = datagen.random_genome(ref_len, seed)
    reads, offs, _, _ = datagen.fixed_reads(ref, n_reads, 150, seed + 1, sub=0.01)
    codes = np.concatenate([ref, reads])
    offsets = np.concatenate([[0], ref.size + offs]).astype(np.int64)
    return codes, offsets


@pytest.mark.gpu
def test_static_sketch_equals_workspace_sketch(gpu):
    # a chromosome-like sequence plus reads, then a smaller batch: the second call reuses
    # the static array the first one filled
    cases = [(batch(71, 3000, 2_000_000), "10", 21, 11),
             (batch(72, 300, 50_000), "110", 15, 10)]
    for (codes, offsets), pattern, k, w in cases:
        seqs = gpu.to_device(codes, offsets)
        ek, ev, emz = gpu.sketch(seqs, pattern, k, w)
        n = ek.numel()
        assert n > 1000
        gk, gv, gmz, st = static_sketch(seqs, pattern, k, w, n)
        assert st == 0
        assert np.array_equal(gmz.cpu().numpy(), emz.cpu().numpy())
        assert np.array_equal(gk[:n].cpu().numpy(), ek.cpu().numpy())
        assert np.array_equal(gv[:n].cpu().numpy(), ev.cpu().numpy())
        # a short capacity still reports the required count and sets the capacity bit
        gk, gv, gmz, st = static_sketch(seqs, pattern, k, w, n // 2)
        assert st & api.STATUS_CAPACITY and int(gmz[-1].item()) == n


def test_static_sketch_refuses_batches_beyond_its_scratch():
    L = api.lib()
    cap = L.godiet_sketch_static_max_bytes()
    assert cap == 64 << 20
    fake = ctypes.c_void_p(0x1000)        # never dereferenced: the call stops on the host
    prm = api.Params(b"10", 21, 11, 0)
    for n_bases, expect in ((1 << 34, api.E_WORKSPACE), (1 << 49, api.E_INVAL)):
        s = api.Seqs(fake, fake, 1, n_bases, None)
        need = L.godiet_workspace_size(api.OP_SKETCH, ctypes.byref(s), ctypes.byref(prm), 0)
        assert expect == api.E_INVAL or need > cap
        r = L.godiet_sketch_static(ctypes.byref(s), ctypes.byref(prm), None, fake, fake, fake,
                                   16, fake, None)
        assert r == expect
