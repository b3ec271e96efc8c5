"""Saved seed indexes load back bit for bit (CPU tensors; the GPU round trip through
seeding is in test_gpu_table.py), and damaged files are refused."""
import os

import numpy as np
import pytest
import torch

from paper_2211_08157_amd import api
from paper_2211_08157_amd.store import load_index, save_index


def make(vb, with_models):
    rng = np.random.default_rng(vb)
    n = 1000
    keys = np.sort(rng.integers(0, 2**63, n, dtype=np.int64))
    vals = rng.integers(0, 2**31, n, dtype=np.int64 if vb == 64 else np.int32)
    rmi = torch.from_numpy(rng.integers(0, 255, 777, dtype=np.uint8)) if with_models else None
    table = torch.from_numpy(rng.integers(0, 255, 4160, dtype=np.uint8)) if with_models else None
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
