"""Saving and loading a built seed index (the paper builds its index once and reuses it,
Section 2.3; this is the persistence of that index).

File layout: 8-byte magic "GODIETIX", 8-byte little-endian length of a JSON header, the
header (format version, record count, value width, pattern, k, w, and the byte sizes of
the optional learned-index model and hash table), zero padding to a multiple of 64, then
the arrays, each starting on a 64-byte boundary: keys (uint64 x n), vals (uint32 or
uint64 x n), the learned-index model bytes, the hash-table bytes.  Loading reads the JSON
and raw arrays only (nothing is executed from the file), checks every size against the
file length, and checks that the model's and the table's headers belong to the keys and
fit their sizes.
"""
import json
import os

import numpy as np

from .api import DeviceIndex

MAGIC = b"GODIETIX"
VERSION = 1
RMI_MAGIC, RMI_HEADER, RMI_LEAF = 0x524D4932, 576, 16      # learned-index model layout
TABLE_MAGIC, TABLE_HEADER, TABLE_SLOT = 0x48544231, 64, 16   # hash-table layout
M64 = (1 << 64) - 1


def keys_fingerprint(keys):
    """The hash table's fingerprint of a sorted key array (its count and eight keys spread
    over it, mixed), as the library writes it into the table header."""
    n = int(keys.size)
    h = (n * 0x9E3779B97F4A7C15) & M64
    for i in range(8 if n > 0 else 0):
        h ^= int(keys[(n - 1) * i // 7])
        h = ((h ^ (h >> 29)) * 0xBF58476D1CE4E5B9) & M64
    return h ^ (h >> 32)


def check_models(keys, rmi, table):
    """Raise ValueError unless the model and table blobs are headers of this index's kind
    whose leaves / slots fit their byte sizes (a damaged or foreign file is refused)."""
    n = int(keys.size)
    if rmi.size:
        if rmi.size < RMI_HEADER:
            raise ValueError("learned-index model shorter than its header")
        magic, kind, log2 = (int(x) for x in rmi[:12].view(np.uint32))
        nk = int(rmi[16:24].view(np.uint64)[0])
        if (magic != RMI_MAGIC or kind > 1 or not 1 <= log2 <= 24 or nk != n or
                RMI_HEADER + (RMI_LEAF << log2) > rmi.size):
            raise ValueError("learned-index model does not belong to this index")
    if table.size:
        if table.size < TABLE_HEADER:
            raise ValueError("hash table shorter than its header")
        magic, log2 = (int(x) for x in table[:8].view(np.uint32))
        nk, fp = (int(x) for x in table[8:24].view(np.uint64))
        if (magic != TABLE_MAGIC or log2 > 40 or nk != n or fp != keys_fingerprint(keys) or
                TABLE_HEADER + (TABLE_SLOT << log2) > table.size):
            raise ValueError("hash table does not belong to this index")


def _pad(n):
    return (-n) % 64


def save_index(path, index, pattern, k, w):
    """Write index (a DeviceIndex, on any device) with its sketch parameters."""
    keys = index.keys[:index.n].cpu().numpy()
    vals = index.vals[:index.n].cpu().numpy()
    rmi = index.rmi.cpu().numpy() if index.rmi is not None else np.zeros(0, np.uint8)
    table = index.table.cpu().numpy() if index.table is not None else np.zeros(0, np.uint8)
    head = json.dumps(dict(version=VERSION, n=int(index.n), val_bits=int(index.val_bits),
                           pattern=pattern, k=int(k), w=int(w), rmi_bytes=int(rmi.nbytes),
                           table_bytes=int(table.nbytes))).encode()
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        f.write(np.uint64(len(head)).tobytes())
        f.write(head)
        f.write(b"\0" * _pad(16 + len(head)))
        for arr in (keys, vals, rmi, table):
            f.write(np.ascontiguousarray(arr).tobytes())
            f.write(b"\0" * _pad(arr.nbytes))
    os.replace(tmp, path)


def load_index(path, device="cuda"):
    """Read a saved index; returns (DeviceIndex on `device`, header dict)."""
    import torch
    size = os.path.getsize(path)
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError("%s is not a saved seed index" % path)
        hlen = int(np.frombuffer(f.read(8), np.uint64)[0])
        if hlen > 1 << 20 or 16 + hlen > size:
            raise ValueError("corrupt index header in %s" % path)
        head = json.loads(f.read(hlen).decode())
        if head.get("version") != VERSION:
            raise ValueError("unsupported index format version %r" % head.get("version"))
        n, vb = int(head["n"]), int(head["val_bits"])
        if vb not in (32, 64) or n < 0:
            raise ValueError("corrupt index header in %s" % path)
        vdt = np.uint32 if vb == 32 else np.uint64
        sizes = [8 * n, (vb // 8) * n, int(head["rmi_bytes"]), int(head["table_bytes"])]
        pos = 16 + hlen + _pad(16 + hlen)
        if pos + sum(s + _pad(s) for s in sizes) > size:
            raise ValueError("%s is shorter than its header says" % path)
        out = []
        for nbytes, dt in zip(sizes, (np.uint64, vdt, np.uint8, np.uint8)):
            f.seek(pos)
            out.append(np.fromfile(f, dtype=dt, count=nbytes // np.dtype(dt).itemsize))
            pos += nbytes + _pad(nbytes)
    keys, vals, rmi, table = out
    check_models(keys, rmi, table)

    def dev(a, signed):
        return torch.from_numpy(a.view(signed)).to(device)

    ix = DeviceIndex(dev(keys, np.int64), dev(vals, np.int32 if vb == 32 else np.int64), n, vb,
                     dev(rmi, np.uint8) if rmi.size else None,
                     dev(table, np.uint8) if table.size else None)
    return ix, head
