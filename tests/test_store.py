"""Saved seed indexes load back bit for bit (CPU tensors; the GPU round trip through
seeding is in test_gpu_table.py), and damaged files are refused."""
import os

import numpy as np
import pytest
import torch

from paper_2211_08157_amd import api, store
from paper_2211_08157_amd.store import load_index, save_index


def blobs(keys, rng):
    """A learned-index model (2^4 leaves) and a hash table (2^11 slots) of these keys:
    valid headers, random bodies (loading checks headers and sizes, not bodies)."""
    n = keys.size
    rmi = rng.integers(0, 255, store.RMI_HEADER + store.RMI_LEAF * 16, dtype=np.uint8)
    rmi[:12] = np.array([store.RMI_MAGIC, 1, 4], np.uint32).view(np.uint8)
    rmi[16:24] = np.array([n], np.uint64).view(np.uint8)
    table = rng.integers(0, 255, store.TABLE_HEADER + store.TABLE_SLOT * 2048, dtype=np.uint8)
    table[:8] = np.array([store.TABLE_MAGIC, 11], np.uint32).view(np.uint8)
    fp = store.keys_fingerprint(keys.view(np.uint64))
    table[8:24] = np.array([n, fp], np.uint64).view(np.uint8)
    return rmi, table


def make(vb, with_models):
    rng = np.random.default_rng(vb)
    n = 1000
    keys = np.sort(rng.integers(0, 2**63, n, dtype=np.int64))
    vals = rng.integers(0, 2**31, n, dtype=np.int64 if vb == 64 else np.int32)
    rmi = table = None
    if with_models:
        r, t = blobs(keys, rng)
        rmi, table = torch.from_numpy(r), torch.from_numpy(t)
    return api.DeviceIndex(torch.from_numpy(keys), torch.from_numpy(vals), n, vb, rmi, table)


@pytest.mark.parametrize("vb,with_models", [(32, False), (32, True), (64, True)])
def test_round_trip(tmp_path, vb, with_models):
    ix = make(vb, with_models)
    p = str(tmp_path / "ix.bin")
    save_index(p, ix, "110", 19, 9)
    got, head = load_index(p, device="cpu")
    assert head["pattern"] == "110" and head["k"] == 19 and head["w"] == 9
    assert got.n == ix.n and got.val_bits == vb
    assert torch.equal(got.keys, ix.keys) and torch.equal(got.vals, ix.vals)
    for a, b in ((got.rmi, ix.rmi), (got.table, ix.table)):
        assert (a is None and b is None) or torch.equal(a, b)


def test_damaged_files_are_refused(tmp_path):
    p = str(tmp_path / "ix.bin")
    save_index(p, make(32, True), "10", 21, 11)
    data = open(p, "rb").read()
    open(p, "wb").write(data[:-100])                      # truncated
    with pytest.raises(ValueError):
        load_index(p, device="cpu")
    open(p, "wb").write(b"NOTANIDX" + data[8:])           # wrong magic
    with pytest.raises(ValueError):
        load_index(p, device="cpu")


@pytest.mark.parametrize("what", ["rmi_log2", "rmi_short", "rmi_keys", "table_fp", "table_short",
                                  "table_magic"])
def test_foreign_or_damaged_models_are_refused(tmp_path, what):
    ix = make(32, True)
    rmi, table = ix.rmi.clone(), ix.table.clone()
    if what == "rmi_log2":
        rmi[8:12] = torch.from_numpy(np.array([40], np.uint32).view(np.uint8))
    elif what == "rmi_short":
        rmi = rmi[:store.RMI_HEADER + 100]
    elif what == "rmi_keys":
        rmi[16:24] = torch.from_numpy(np.array([999], np.uint64).view(np.uint8))
    elif what == "table_fp":
        # the same key count, other keys: the fingerprint gives it away
        other = np.sort(np.random.default_rng(9).integers(0, 2**63, ix.n, dtype=np.int64))
        table = torch.from_numpy(blobs(other, np.random.default_rng(9))[1])
    elif what == "table_short":
        table = table[:store.TABLE_HEADER + 16 * 100]
    else:
        table[:4] = 0
    bad = api.DeviceIndex(ix.keys, ix.vals, ix.n, 32, rmi, table)
    p = str(tmp_path / "ix.bin")
    save_index(p, bad, "10", 21, 11)
    with pytest.raises(ValueError):
        load_index(p, device="cpu")
