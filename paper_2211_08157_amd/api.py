"""ctypes declarations of libgodiet.so and torch-based argument marshalling."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libgodiet.so")

OK, E_INVAL, E_RANGE, E_WORKSPACE, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_CAPACITY, STATUS_RANGE, STATUS_SHIFT = 1, 2, 4
OP_SPARSIFY, OP_SKETCH, OP_INDEX_BUILD, OP_SEED, OP_RMI_TRAIN, OP_CONTAIN, OP_VOTE = 1, 2, 3, 4, 5, 6, 7
VOTE_RESCUE = 1


class GodietError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().godiet_status_string(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (%d)" % (what, msg, code))
        self.code = code


class Seqs(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n_seq", ctypes.c_uint32), ("n_bases", ctypes.c_uint64),
                ("nmask", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("pattern", ctypes.c_char_p), ("k", ctypes.c_int32), ("w", ctypes.c_int32),
                ("hash", ctypes.c_int32)]


HASHES = {"splitmix64": 0, "wang": 1}


class Index(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("val_bits", ctypes.c_int32), ("rmi", ctypes.c_void_p),
                ("rmi_bytes", ctypes.c_size_t), ("table", ctypes.c_void_p),
                ("table_bytes", ctypes.c_size_t)]


class SeedOpts(ctypes.Structure):
    _fields_ = [("shift_mode", ctypes.c_int32), ("align_t", ctypes.c_uint32),
                ("max_occ", ctypes.c_uint32), ("long_records", ctypes.c_uint32),
                ("lookup_blocks", ctypes.c_uint32), ("long_blocks", ctypes.c_uint32),
                ("index_ready", ctypes.c_void_p)]


TUNING_KEYS = ("long_records", "lookup_blocks", "long_blocks")


def seed_opts(shift_mode=-1, align_t=0, max_occ=0, tuning=None, index_ready=None):
    """godiet_seed_opts from a tuning dict (missing launch parameters: library default)."""
    t = tuning or {}
    bad = set(t) - set(TUNING_KEYS)
    if bad:
        raise ValueError("unknown launch parameters: %s" % ", ".join(sorted(bad)))
    return SeedOpts(shift_mode=int(shift_mode), align_t=int(align_t), max_occ=int(max_occ),
                    index_ready=index_ready, **{k: int(t.get(k, 0)) for k in TUNING_KEYS})


class VoteOpts(ctypes.Structure):
    _fields_ = [("max_dist", ctypes.c_uint32), ("min_votes", ctypes.c_uint32),
                ("max_winners", ctypes.c_uint32), ("sort", ctypes.c_uint32)]


VOTE_SORTS = {"adaptive": 0, "radix": 1, "merge": 2, "heap": 3}


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise ImportError("libgodiet.so not built: run __graft_entry__.build() or "
                              "python paper_2211_08157_amd/build.py")
        L = ctypes.CDLL(lib_path)
        P, S = ctypes.c_void_p, ctypes.POINTER
        u32, u64, i32, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t
        L.godiet_status_string.argtypes = [i32]
        L.godiet_status_string.restype = ctypes.c_char_p
        L.godiet_workspace_size.argtypes = [i32, S(Seqs), S(Params), u64]
        L.godiet_workspace_size.restype = sz
        L.godiet_kept_bound.argtypes = [S(Seqs), ctypes.c_char_p]
        L.godiet_kept_bound.restype = u64
        L.godiet_sketch_bound.argtypes = [S(Seqs), S(Params)]
        L.godiet_sketch_bound.restype = u64
        L.godiet_sparsify_bytes.argtypes = [S(Seqs), ctypes.c_char_p]
        L.godiet_sparsify_bytes.restype = sz
        L.godiet_sparsify.argtypes = [S(Seqs), ctypes.c_char_p, P, P, P, P, P, sz, P, P]
        L.godiet_sparsify.restype = i32
        L.godiet_seed_match.argtypes = [S(Seqs), S(Seqs), S(Params), P, P, P]
        L.godiet_seed_match.restype = i32
        L.godiet_edit_distance.argtypes = [S(Seqs), S(Seqs), P, P, P]
        L.godiet_edit_distance.restype = i32
        L.godiet_accepted_ws_size.argtypes = [u32]
        L.godiet_accepted_ws_size.restype = sz
        L.godiet_accepted_pairs.argtypes = [P, P, u32, i32, u32, P, P, sz, P]
        L.godiet_accepted_pairs.restype = i32
        L.godiet_pack_bytes.argtypes = [u64]
        L.godiet_pack_bytes.restype = sz
        L.godiet_pack_ascii.argtypes = [P, u64, P, P, P]
        L.godiet_pack_ascii.restype = i32
        L.godiet_sketch.argtypes = [S(Seqs), S(Params), P, P, P, P, u64, P, sz, P, P]
        L.godiet_sketch.restype = i32
        L.godiet_sketch_static_max_bytes.argtypes = []
        L.godiet_sketch_static_max_bytes.restype = sz
        L.godiet_sketch_static.argtypes = [S(Seqs), S(Params), P, P, P, P, u64, P, P]
        L.godiet_sketch_static.restype = i32
        L.godiet_index_build.argtypes = [S(Seqs), S(Params), P, P, i32, u64, P, P, sz, P, P]
        L.godiet_index_build.restype = i32
        L.godiet_seed.argtypes = [S(Index), S(Seqs), S(Params), S(SeedOpts), P, u64, P, P, P, sz,
                                  P, P]
        L.godiet_seed.restype = i32
        L.godiet_contain.argtypes = [S(Index), S(Seqs), S(Params), S(SeedOpts), u32, P, P, P, sz,
                                     P, P]
        L.godiet_contain.restype = i32
        L.godiet_vote.argtypes = [P, P, u32, u64, S(VoteOpts), P, P, P, sz, P, P]
        L.godiet_vote.restype = i32
        L.godiet_table_size.argtypes = [u64]
        L.godiet_table_size.restype = sz
        L.godiet_table_build.argtypes = [S(Index), P, sz, P]
        L.godiet_table_build.restype = i32
        L.godiet_rmi_stats.argtypes = [S(Index), P, u64, P, P]
        L.godiet_rmi_stats.restype = i32
        L.godiet_lookup.argtypes = [S(Index), P, u64, P, P, P]
        L.godiet_lookup.restype = i32
        L.godiet_random_gather.argtypes = [P, u64, P, u64, P, P, P]
        L.godiet_random_gather.restype = i32
        L.godiet_rmi_size.argtypes = [u32]
        L.godiet_rmi_size.restype = sz
        L.godiet_rmi_train.argtypes = [S(Index), i32, u32, P, sz, P]
        L.godiet_rmi_train.restype = i32
        L.godiet_trace_enable.argtypes = [ctypes.c_int]
        L.godiet_trace_enable.restype = None
        L.godiet_trace_dump.argtypes = [ctypes.c_char_p, sz]
        L.godiet_trace_dump.restype = sz
        L.godiet_trace_filter.argtypes = [ctypes.c_char_p]
        L.godiet_trace_filter.restype = None
        _lib = L
    return _lib


def trace_enable(on=True):
    lib().godiet_trace_enable(1 if on else 0)


def trace_filter(prefix=None):
    """Trace only kernels whose name starts with prefix (None: all)."""
    lib().godiet_trace_filter(prefix.encode() if prefix else None)


def trace_dump():
    """{kernel name: (launches, total ms)} of the launches traced since the last dump.
    The caller must have synchronised the streams the kernels ran on."""
    L = lib()
    need = L.godiet_trace_dump(None, 0)
    buf = ctypes.create_string_buffer(max(need, 1) + 4096)
    L.godiet_trace_dump(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.rsplit(" ", 2)
        out[name] = (int(n), float(ms))
    return out


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(code, what):
    if code != OK:
        raise GodietError(code, what)


def pack(codes):
    """2-bit pack base codes (A=0, C=1, G=2, T=3): base i -> bits 2*(i%4) of byte i//4.
    The result is padded with zero bytes to a multiple of 16."""
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    if c.size and c.max() > 3:
        raise ValueError("only A, C, G, T (codes 0..3) can be packed; N goes into pack_n")
    n = c.size
    padded = np.zeros((n + 63) // 64 * 64, np.uint8)
    padded[:n] = c
    q = padded.reshape(-1, 4)
    return (q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)).astype(np.uint8)


def pack_n(is_n):
    """N bit mask of a batch: bit i%32 of 32-bit word i//32 set iff base i is N, padded
    with zero bits to 64 bits per 64 bases (as uint8 bytes)."""
    b = np.ascontiguousarray(is_n, dtype=bool)
    padded = np.zeros((b.size + 63) // 64 * 64, bool)
    padded[:b.size] = b
    return np.packbits(padded, bitorder="little")


class DeviceSeqs:
    """A 2-bit packed batch of sequences resident in device memory, with an optional N
    bit mask (uint8 tensor, or None when the batch holds no N)."""

    def __init__(self, bases, offsets, n_seq, n_bases, nmask=None):
        self.bases, self.offsets = bases, offsets
        self.n_seq, self.n_bases = int(n_seq), int(n_bases)
        self.nmask = nmask

    def c(self):
        return Seqs(self.bases.data_ptr(), self.offsets.data_ptr(), self.n_seq, self.n_bases,
                    self.nmask.data_ptr() if self.nmask is not None else None)


def _offsets(offsets, n):
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    if offs.size < 1 or offs[0] != 0 or np.any(np.diff(offs) < 0):
        raise ValueError("offsets must start at 0 and be non-decreasing")
    if offs[-1] > n:
        raise ValueError("offsets exceed the number of bases")
    return offs


def to_device(codes, offsets, device="cuda"):
    """Upload base codes (A=0, C=1, G=2, T=3; 4 = the ambiguous base N) with their
    n_seq + 1 offsets.  An N mask is attached only when some code is 4."""
    torch = _torch()
    c = np.asarray(codes, dtype=np.uint8)
    offs = _offsets(offsets, c.size)
    if c.size and c.max() > 4:
        raise ValueError("base codes must be 0..3, or 4 for N")
    nm = None
    if c.size and c.max() == 4:
        is_n = c == 4
        nm = torch.from_numpy(pack_n(is_n)).to(device)
        c = np.where(is_n, 0, c).astype(np.uint8)
    b = torch.from_numpy(pack(c)).to(device)
    o = torch.from_numpy(offs).to(device)
    return DeviceSeqs(b, o, offs.size - 1, int(offs[-1]), nm)


def to_device_ascii(text, offsets, device="cuda"):
    """Upload sequence text (bytes, str or a uint8 array; the batch's sequences back to
    back) and pack it on the device: A/C/G/T/U in either case are bases, every other
    character is N.  Always attaches an N mask."""
    torch = _torch()
    if isinstance(text, str):
        text = text.encode()
    raw = np.frombuffer(bytes(text), np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    offs = _offsets(offsets, raw.size)
    L = lib()
    nb = L.godiet_pack_bytes(raw.size)
    t = torch.from_numpy(raw.copy()).to(device) if raw.size else None
    bases = _empty(nb, torch.uint8)
    nmask = _empty(max(nb // 2, 4), torch.uint8)
    _check(L.godiet_pack_ascii(_ptr(t), raw.size, _ptr(bases), _ptr(nmask), _stream()),
           "godiet_pack_ascii")
    o = torch.from_numpy(offs).to(device)
    return DeviceSeqs(bases, o, offs.size - 1, int(offs[-1]), nmask)


def _params(pattern, k, w, hash="splitmix64"):
    if hash not in HASHES:
        raise ValueError("hash must be one of %s" % sorted(HASHES))
    return Params(pattern.encode(), int(k), int(w), HASHES[hash])


def workspace_size(op, seqs, pattern, k, w, n_index=0):
    s = seqs.c()
    return lib().godiet_workspace_size(op, ctypes.byref(s), ctypes.byref(_params(pattern, k, w)),
                                       int(n_index))


def kept_bound(seqs, pattern):
    s = seqs.c()
    return lib().godiet_kept_bound(ctypes.byref(s), pattern.encode())


def _empty(n, dtype):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=dtype, device="cuda")


def _status_value(st):
    return int(st.item())


def sparsify(seqs, pattern, shift=None, with_nmask=False):
    """Returns (packed patterned bases as uint8 tensor, patterned offsets int64 tensor),
    and with with_nmask the N mask of the kept bases (uint8 tensor, None when the batch
    has none) as a third element."""
    torch = _torch()
    s = seqs.c()
    L = lib()
    nbytes = L.godiet_sparsify_bytes(ctypes.byref(s), pattern.encode())
    ws = _empty(workspace_size(OP_SPARSIFY, seqs, pattern, 1, 1), torch.uint8)
    out = _empty(nbytes, torch.uint8)
    offs = _empty(seqs.n_seq + 1, torch.int64)
    st = _empty(1, torch.int32)
    sh = None if shift is None else torch.as_tensor(np.asarray(shift, np.uint32).view(np.int32),
                                                     device="cuda")
    pn = _empty(max(nbytes // 2, 4), torch.uint8) if seqs.nmask is not None else None
    _check(L.godiet_sparsify(ctypes.byref(s), pattern.encode(), _ptr(sh), _ptr(out), _ptr(offs),
                             _ptr(pn), _ptr(ws), ws.numel(), _ptr(st), _stream()),
           "godiet_sparsify")
    if _status_value(st) & STATUS_SHIFT:
        raise ValueError("a shift is >= the pattern length")
    return (out, offs, pn) if with_nmask else (out, offs)


def sketch(seqs, pattern, k, w, shift=None, capacity=None, hash="splitmix64"):
    """Minimizers of every sequence.  Returns (keys int64 tensor holding uint64 bits,
    vals int32 tensor holding uint32 pos<<1|strand, mz_offsets int64 tensor)."""
    torch = _torch()
    s = seqs.c()
    L = lib()
    prm = _params(pattern, k, w, hash)
    if capacity is None:
        capacity = max(1024, int(kept_bound(seqs, pattern) * 2.2 / (w + 1)) + 4096)
    sh = None if shift is None else torch.as_tensor(np.asarray(shift, np.uint32).view(np.int32),
                                                     device="cuda")
    ws = _empty(workspace_size(OP_SKETCH, seqs, pattern, k, w), torch.uint8)
    mz = _empty(seqs.n_seq + 1, torch.int64)
    st = _empty(1, torch.int32)
    while True:
        keys = _empty(capacity, torch.int64)
        vals = _empty(capacity, torch.int32)
        _check(L.godiet_sketch(ctypes.byref(s), ctypes.byref(prm), _ptr(sh), _ptr(keys), _ptr(vals),
                               _ptr(mz), capacity, _ptr(ws), ws.numel(), _ptr(st), _stream()),
               "godiet_sketch")
        status = _status_value(st)
        n = int(mz[-1].item())
        if status & STATUS_CAPACITY:
            capacity = n
            continue
        if status & STATUS_SHIFT:
            raise ValueError("a shift is >= the pattern length")
        if status & STATUS_RANGE:
            raise ValueError("a sequence is too long for 31-bit positions")
        return keys[:n], vals[:n], mz


class DeviceIndex:
    """A sorted seed index in device memory (keys as int64 bit patterns of uint64), with an
    optional learned-index model and an optional hash table (uint8 tensors) used for its
    lookups."""

    def __init__(self, keys, vals, n, val_bits, rmi=None, table=None):
        self.keys, self.vals, self.n, self.val_bits = keys, vals, int(n), int(val_bits)
        self.rmi = rmi
        self.table = table

    def c(self):
        return Index(self.keys.data_ptr(), self.vals.data_ptr(), self.n, self.val_bits,
                     self.rmi.data_ptr() if self.rmi is not None else None,
                     self.rmi.numel() if self.rmi is not None else 0,
                     self.table.data_ptr() if self.table is not None else None,
                     self.table.numel() if self.table is not None else 0)

    def with_rmi(self, rmi):
        return DeviceIndex(self.keys, self.vals, self.n, self.val_bits, rmi, self.table)

    def with_table(self, table):
        return DeviceIndex(self.keys, self.vals, self.n, self.val_bits, self.rmi, table)


def table_build(index):
    """Build the hash-table form of index (seeding and containment lookups use it);
    returns a copy of the index that carries it."""
    torch = _torch()
    L = lib()
    nbytes = L.godiet_table_size(index.n)
    if nbytes == 0:
        raise ValueError("index too large for a hash table")
    blob = _empty(nbytes, torch.uint8)
    _check(L.godiet_table_build(ctypes.byref(index.c()), _ptr(blob), nbytes, _stream()),
           "godiet_table_build")
    return index.with_table(blob)


def rmi_train(index, root="mlp", log2_leaves=18):
    """Train a learned index on index.keys; returns a copy of the index that uses it."""
    torch = _torch()
    L = lib()
    nbytes = L.godiet_rmi_size(int(log2_leaves))
    if nbytes == 0:
        raise ValueError("log2_leaves must be in 1..24")
    blob = torch.empty(nbytes + 64, dtype=torch.uint8, device="cuda")
    off = (-blob.data_ptr()) % 64
    blob = blob[off:off + nbytes]
    ix = index.c()
    kind = {"linear": 0, "mlp": 1}[root]
    _check(L.godiet_rmi_train(ctypes.byref(ix), kind, int(log2_leaves), _ptr(blob), nbytes,
                              _stream()), "godiet_rmi_train")
    return index.with_rmi(blob)


def lookup(index, queries):
    """(lb, occ) int32 tensors (uint32 bits) of int64 query tensor `queries` (uint64 bits)."""
    torch = _torch()
    n = queries.numel()
    lb = _empty(n, torch.int32)
    occ = _empty(n, torch.int32)
    ix = index.c()
    _check(lib().godiet_lookup(ctypes.byref(ix), _ptr(queries), n, _ptr(lb), _ptr(occ),
                               _stream()), "godiet_lookup")
    return lb[:n], occ[:n]


def random_gather(src, idx):
    """out[i] = src[idx[i]] through the library's random-gather probe (int64 tensors);
    returns (out, status tensor)."""
    torch = _torch()
    out = _empty(idx.numel(), torch.int64)
    st = _empty(1, torch.int32)
    _check(lib().godiet_random_gather(_ptr(src), src.numel(), _ptr(idx), idx.numel(), _ptr(out),
                                      _ptr(st), _stream()), "godiet_random_gather")
    return out[:idx.numel()], st


RMI_STAT_WORDS = 20


def rmi_stats(index, queries):
    """Learned-index diagnostics over an int64 query tensor: dict(queries, fallbacks,
    window_keys) with window_keys[b] = windows of w keys, 2^(b-1) < w <= 2^b (the last
    entry open-ended)."""
    torch = _torch()
    st = _empty(RMI_STAT_WORDS, torch.int64)
    _check(lib().godiet_rmi_stats(ctypes.byref(index.c()), _ptr(queries), queries.numel(),
                                  _ptr(st), _stream()), "godiet_rmi_stats")
    v = st.cpu().numpy().view(np.uint64)
    return dict(queries=int(v[0]), fallbacks=int(v[1]), window_keys=[int(x) for x in v[2:]])


def index_build(ref, pattern, k, w, val_bits=32, capacity=None, hash="splitmix64"):
    torch = _torch()
    s = ref.c()
    L = lib()
    prm = _params(pattern, k, w, hash)
    if capacity is None:
        capacity = max(1024, int(kept_bound(ref, pattern) * 2.2 / (w + 1)) + 4096)
    st = _empty(1, torch.int32)
    n_out = _empty(1, torch.int64)
    while True:
        ws = _empty(workspace_size(OP_INDEX_BUILD, ref, pattern, k, w, capacity), torch.uint8)
        keys = _empty(capacity, torch.int64)
        vals = _empty(capacity, torch.int32 if val_bits == 32 else torch.int64)
        _check(L.godiet_index_build(ctypes.byref(s), ctypes.byref(prm), _ptr(keys), _ptr(vals),
                                    val_bits, capacity, _ptr(n_out), _ptr(ws), ws.numel(), _ptr(st),
                                    _stream()), "godiet_index_build")
        status = _status_value(st)
        n = int(n_out.item())
        if status & STATUS_CAPACITY:
            capacity = n
            continue
        if status & STATUS_RANGE:
            raise ValueError("a position does not fit the value encoding")
        return DeviceIndex(keys[:n], vals[:n], n, val_bits)


def seed(index, reads, pattern, k, w, shift_mode=-1, align_t=0, max_occ=0, capacity=None,
         tuning=None, hash="splitmix64", index_ready=None):
    """Pattern alignment + compressed seeding.  Returns (anchors int32 tensor (n, 4) of
    read_id, qpos, rpos, strand; read_anchor_off int64 tensor; shift uint8 tensor).
    index_ready: a torch.cuda.Event recorded after the index was built on another stream
    (the read sketches then run before waiting on it)."""
    torch = _torch()
    s = reads.c()
    L = lib()
    prm = _params(pattern, k, w, hash)
    ix = index.c()
    opts = seed_opts(shift_mode, align_t, max_occ, tuning,
                     index_ready.cuda_event if index_ready is not None else None)
    ws = _empty(workspace_size(OP_SEED, reads, pattern, k, w, index.n), torch.uint8)
    off = _empty(reads.n_seq + 1, torch.int64)
    shift = _empty(reads.n_seq, torch.uint8)
    st = _empty(1, torch.int32)
    if capacity is None:
        capacity = max(4096, reads.n_bases // 4)
    while True:
        anchors = _empty(capacity * 4, torch.int32)
        _check(L.godiet_seed(ctypes.byref(ix), ctypes.byref(s), ctypes.byref(prm),
                             ctypes.byref(opts), _ptr(anchors), capacity, _ptr(off), _ptr(shift),
                             _ptr(ws), ws.numel(), _ptr(st), _stream()), "godiet_seed")
        status = _status_value(st)
        n = int(off[-1].item())
        if status & STATUS_CAPACITY:
            capacity = n
            continue
        return anchors[:4 * n].view(n, 4), off, shift[:reads.n_seq]


def contain(index, reads, pattern, k, w, n_genomes, shift_mode=-1, align_t=0, max_occ=0,
            hash="splitmix64"):
    """Per-genome shared distinct minimizer counts against a 64-bit-val (genome id) index.
    Returns (counts, sizes) int32 tensors (uint32 bits)."""
    torch = _torch()
    s = reads.c()
    L = lib()
    prm = _params(pattern, k, w, hash)
    ix = index.c()
    opts = seed_opts(shift_mode, align_t, max_occ)
    ws = _empty(workspace_size(OP_CONTAIN, reads, pattern, k, w, index.n), torch.uint8)
    counts = _empty(n_genomes, torch.int32)
    sizes = _empty(n_genomes, torch.int32)
    st = _empty(1, torch.int32)
    _check(L.godiet_contain(ctypes.byref(ix), ctypes.byref(s), ctypes.byref(prm),
                            ctypes.byref(opts), int(n_genomes), _ptr(counts), _ptr(sizes),
                            _ptr(ws), ws.numel(), _ptr(st), _stream()), "godiet_contain")
    if _status_value(st) & STATUS_RANGE:
        raise ValueError("an index record names a genome id >= n_genomes")
    return counts[:n_genomes], sizes[:n_genomes]


def vote(anchors, read_off, max_dist, min_votes, max_winners, capacity=None, sort="adaptive"):
    """Location voting over seeding anchors (int32 tensor (n, 4), read_off int64 tensor
    [n_reads+1]).  Returns (winners int32 tensor (n_reads, max_winners, 6): the 24-byte
    records loc (two words), read_id, strand, votes, flags; n_win int32 tensor)."""
    torch = _torch()
    n_reads = read_off.numel() - 1
    if capacity is None:
        capacity = anchors.numel() // 4
    L = lib()
    rs = Seqs(None, None, n_reads, 0)           # workspace sizing reads only n_seq
    need = L.godiet_workspace_size(OP_VOTE, ctypes.byref(rs), None, int(capacity))
    if need == 0:
        raise ValueError("sizes out of range for location voting")
    ws = _empty(need, torch.uint8)
    out = _empty(max(n_reads, 1) * max_winners * 6, torch.int32)
    nw = _empty(max(n_reads, 1), torch.int32)
    st = _empty(1, torch.int32)
    if sort not in VOTE_SORTS:
        raise ValueError("sort must be one of %s" % sorted(VOTE_SORTS))
    opts = VoteOpts(int(max_dist), int(min_votes), int(max_winners), VOTE_SORTS[sort])
    _check(L.godiet_vote(_ptr(anchors) if anchors.numel() else None, _ptr(read_off), n_reads,
                         int(capacity), ctypes.byref(opts), _ptr(out), _ptr(nw), _ptr(ws),
                         ws.numel(), _ptr(st), _stream()), "godiet_vote")
    status = _status_value(st)
    if status & STATUS_CAPACITY:
        raise ValueError("more anchors than the capacity given")
    if status & STATUS_RANGE:
        raise ValueError("anchors are not grouped by read as read_off says")
    return out[:n_reads * max_winners * 6].view(n_reads, max_winners, 6), nw[:n_reads]


def winners_rows(winners, n_win):
    """Host rows (read, strand, votes, flags, loc) of every output winner, in order."""
    import numpy as np
    w = winners.cpu().numpy()
    nw = n_win.cpu().numpy()
    rows = []
    if w.size == 0:
        return np.zeros((0, 5), np.int64)
    loc = w[:, :, 0].astype(np.int64) & 0xFFFFFFFF | (w[:, :, 1].astype(np.int64) << 32)
    idx = np.arange(w.shape[1])[None, :] < nw[:, None]
    r, j = np.nonzero(idx)
    return np.stack([w[r, j, 2].astype(np.int64), w[r, j, 3].astype(np.int64),
                     w[r, j, 4].astype(np.int64), w[r, j, 5].astype(np.int64), loc[r, j]], 1)


FIG4_ALGORITHMS = ("all", "minimizers", "spaced", "god")


def seed_match(orig, copy, pattern, k, w, hash="splitmix64"):
    """Seed-matching experiment over pairs (sequence i of orig, sequence i of copy): int32
    tensor (n_pairs, 4, 2) of (matched seeds of the copy, seeds of the copy) for the
    algorithms FIG4_ALGORITHMS."""
    torch = _torch()
    if orig.n_seq != copy.n_seq:
        raise ValueError("both batches need the same number of sequences")
    a, b = orig.c(), copy.c()
    counts = _empty(8 * orig.n_seq, torch.int32)
    st = _empty(1, torch.int32)
    _check(lib().godiet_seed_match(ctypes.byref(a), ctypes.byref(b),
                                   ctypes.byref(_params(pattern, k, w, hash)), _ptr(counts),
                                   _ptr(st), _stream()), "godiet_seed_match")
    if _status_value(st) & STATUS_RANGE:
        raise ValueError("a sequence of a pair is longer than 1,024 bases")
    return counts[:8 * orig.n_seq].view(orig.n_seq, 4, 2)


def edit_distance(orig, copy):
    """Levenshtein distance of every pair: int32 tensor (n_pairs)."""
    torch = _torch()
    if orig.n_seq != copy.n_seq:
        raise ValueError("both batches need the same number of sequences")
    a, b = orig.c(), copy.c()
    dist = _empty(orig.n_seq, torch.int32)
    st = _empty(1, torch.int32)
    _check(lib().godiet_edit_distance(ctypes.byref(a), ctypes.byref(b), _ptr(dist), _ptr(st),
                                      _stream()), "godiet_edit_distance")
    if _status_value(st) & STATUS_RANGE:
        raise ValueError("an original sequence is longer than 1,024 bases")
    return dist[:orig.n_seq]


def accepted_pairs(dist, counts, algorithm, max_e):
    """Accepted pairs per edit-distance threshold 0..max_e for one algorithm (name or
    index): int32 tensor (max_e + 1)."""
    torch = _torch()
    g = FIG4_ALGORITHMS.index(algorithm) if isinstance(algorithm, str) else int(algorithm)
    n = dist.numel()
    L = lib()
    ws = _empty(L.godiet_accepted_ws_size(max_e), torch.uint8)
    acc = _empty(max_e + 1, torch.int32)
    _check(L.godiet_accepted_pairs(_ptr(dist), _ptr(counts), n, g, max_e, _ptr(acc), _ptr(ws),
                                   ws.numel(), _stream()), "godiet_accepted_pairs")
    return acc[:max_e + 1]
