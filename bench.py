"""Benchmark of the sparsified-seeding hot path on one MI355X.

One step = the whole path over one batch: compressed indexing of the reference
(sparsify + sketch + sort into the seed index, then the learned index's training)
followed by pattern alignment and compressed seeding of the read batch (sketch at every
shift, lookups, shift choice, anchor expansion).  Inputs are generated (seeded,
synthetic) and resident in HBM before the timed region; nothing is copied to or from the
host inside it.

Headline workload (uneven-1Gbp): 1 Gbp reference with 5 % repeats and one mixed batch of
2M x 150 bp, 20k HiFi-like and 20k ONT-like reads (800 Mbp), pattern "10", k=21, w=11,
launch parameters from the autotuner.  The same step runs with the learned index (the
headline), with plain binary search and with the hash-table index; outputs must be
identical.  The step is also replayed as one HIP graph, the seeding pass alone is timed
with the index prebuilt, and pattern "110" is reported beside "10".

Prints one JSON line: reads/s of the learned-index step, the dominant kernel's roofline
(timed live with HIP events on the stream the kernels run on), the sketch kernel's
roofline in the same step, the index build's rate, and the CPU oracle timed on the
host's cores.  Beside the headline: 500M lookups in the 1 Gbp key arrays of patterns "10"
and "11"; the 1 Gbp reference sketch; the 100 Mbp Illumina-like step (1M reads) with its
own roofline and oracle baseline; location voting and its per-read sorts; the step on a
workload with ambiguous bases; the seed-matching experiment; the 1,000-genome
containment search.  --sections selects parts (counter runs time a few steps of one).
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
# 256 CUs x 64 lanes x 2.4 GHz: int32 vector lane-operations per second, in GOP/s
ALU_PEAK_GOPS = 256 * 64 * 2.4
# Algorithmic int32 lane-operations of one k-mer in the sketch: forward and reverse-
# complement codes 4, canonical choice and strand 3, the splitmix64 finalizer 17 (two
# 64-bit multiplies of 4 each, three 64-bit xor-shifts of 3 each), window minimum and
# opening with 3 amortised 64-bit compare-selects each (6 x 3 = 18).
OPS_PER_KMER = 4 + 3 + 17 + 18
# Algorithmic bytes of one lookup: the query in, (lower bound, count) out, one 64-byte
# line of the index.
LOOKUP_BYTES = 8 + 8 + 64
# Algorithmic bytes of the index sort per record: one read and one write of the 12-byte
# (key, value) record.
SORT_BYTES = 24
SORT_KERNELS = ("k_top_hist", "k_digit", "k_hist", "k_scatter", "k_bucket_sort", "k_coarse",
                "k_fine_scatter")
# HBM bytes measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a 1 GiB copy) for a
# kernel source on a workload; reported only while that source is unchanged.
MEASURED_TRAFFIC = {
    ("k_lookup<2>", "uneven-1Gbp/10"): dict(
        summary="profiles/k_lookup_uneven-1Gbp_hbm_bytes.md",
        src="paper_2211_08157_amd/csrc/gd_seed.hip", sha256_16="f85d4bd549d06727",
        bytes_per_step=37771.8e6),
    ("k_sketch<11,0>", "uneven-1Gbp/10"): dict(
        summary="profiles/k_sketch_uneven-1Gbp_hbm_bytes.md",
        src="paper_2211_08157_amd/csrc/gd_sketch.hip", sha256_16="dc3215cf367ec9ef",
        bytes_per_step=2921.9e6),
}
METRIC = "reads/sec seeded (bit-exact anchors), learned-index vs binary search; sketch GB/s"
SECTIONS = ("uneven", "lookups", "sketch1g", "illumina", "extras", "containment")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads():
    """Worker threads for the oracle: the cores this process may run on, at most 16 (one
    GPU's share of the host on the GPU machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def host_cores():
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return dict(nproc=os.cpu_count(), affinity=aff)


class Session:
    """One workload's step with preallocated buffers, so that a step only enqueues
    kernels: index build of the reference, then learned-index training (learned_index) or
    hash-table build (hash_table) or nothing (binary_search), then seeding of the batch."""

    def __init__(self, gd, ref, reads, ref_offsets, read_offsets, pattern, k, w,
                 log2_leaves=18, tuning=None):
        import torch
        from paper_2211_08157_amd import api
        self.torch, self.api, self.gd = torch, api, gd
        self.pattern, self.k, self.w = pattern, k, w
        self.ref_offsets = np.asarray(ref_offsets, np.int64)
        self.read_lengths = np.diff(np.asarray(read_offsets, np.int64))
        self.ref, self.reads = ref, reads
        self.prm = api.Params(pattern.encode(), k, w)
        self.cref, self.creads = self.ref.c(), self.reads.c()
        self.tuning = dict(tuning or {})
        dev = "cuda"
        # learn the index size once (same inputs every step)
        ix = gd.index_build(self.ref, pattern, k, w)
        self.n_index = ix.n
        self.capacity = ix.n
        self.ikeys = torch.empty(self.capacity, dtype=torch.int64, device=dev)
        self.ivals = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.n_out = torch.empty(1, dtype=torch.int64, device=dev)
        self.st_i = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_i = torch.empty(api.workspace_size(api.OP_INDEX_BUILD, self.ref, pattern, k, w,
                                                   self.capacity), dtype=torch.uint8, device=dev)
        a, off, _ = gd.seed(ix, self.reads, pattern, k, w, tuning=self.tuning)
        self.n_anchors = int(off[-1].item())
        self.acap = self.n_anchors
        self.anchors = torch.empty(max(self.acap, 1) * 4, dtype=torch.int32, device=dev)
        self.roff = torch.empty(self.reads.n_seq + 1, dtype=torch.int64, device=dev)
        self.shift = torch.empty(self.reads.n_seq, dtype=torch.uint8, device=dev)
        self.st_s = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_s = torch.empty(api.workspace_size(api.OP_SEED, self.reads, pattern, k, w, ix.n),
                                dtype=torch.uint8, device=dev)
        self.log2_leaves = int(log2_leaves)
        nb = api.lib().godiet_rmi_size(self.log2_leaves)
        blob = torch.empty(nb + 64, dtype=torch.uint8, device=dev)
        off = (-blob.data_ptr()) % 64
        self.rmi = blob[off:off + nb]
        self.cix = api.Index(self.ikeys.data_ptr(), self.ivals.data_ptr(), self.n_index, 32, None, 0)
        self.cix_rmi = api.Index(self.ikeys.data_ptr(), self.ivals.data_ptr(), self.n_index, 32,
                                 self.rmi.data_ptr(), self.rmi.numel())
        self.table = torch.empty(api.lib().godiet_table_size(self.n_index), dtype=torch.uint8,
                                 device=dev)
        self.cix_table = api.Index(self.ikeys.data_ptr(), self.ivals.data_ptr(), self.n_index, 32,
                                   None, 0, self.table.data_ptr(), self.table.numel())
        t = self.tuning
        self.opts = api.seed_opts(tuning=t)
        # with overlap, index construction runs on a side stream (default priority) and
        # overlaps the read sketches of seeding; events order the two streams both ways
        self.overlap = False
        self.side = torch.cuda.Stream()
        self.ev_index = torch.cuda.Event()
        self.ev_seed = torch.cuda.Event()
        del ix, a, off
        # per-shift query counts (minimizers of the reads at every shift) for byte accounting
        self.queries_per_shift = []
        for s in range(len(pattern)):
            kq, _, _ = gd.sketch(self.reads, pattern, k, w,
                                 shift=np.full(self.reads.n_seq, s, np.uint32))
            self.queries_per_shift.append(kq.numel())
            del kq
        self.queries = sum(self.queries_per_shift)
        torch.cuda.synchronize()

    def index_step(self, mode, st):
        L = self.api.lib()
        r = L.godiet_index_build(ctypes.byref(self.cref), ctypes.byref(self.prm),
                                 ctypes.c_void_p(self.ikeys.data_ptr()),
                                 ctypes.c_void_p(self.ivals.data_ptr()), 32, self.capacity,
                                 ctypes.c_void_p(self.n_out.data_ptr()),
                                 ctypes.c_void_p(self.ws_i.data_ptr()), self.ws_i.numel(),
                                 ctypes.c_void_p(self.st_i.data_ptr()), st)
        if r != 0:
            raise RuntimeError("godiet_index_build failed: %d" % r)
        if mode == "learned_index":
            r = L.godiet_rmi_train(ctypes.byref(self.cix), 1, self.log2_leaves,
                                   ctypes.c_void_p(self.rmi.data_ptr()), self.rmi.numel(), st)
            if r != 0:
                raise RuntimeError("godiet_rmi_train failed: %d" % r)
        elif mode == "hash_table":
            r = L.godiet_table_build(ctypes.byref(self.cix), ctypes.c_void_p(self.table.data_ptr()),
                                     self.table.numel(), st)
            if r != 0:
                raise RuntimeError("godiet_table_build failed: %d" % r)

    def seed_step(self, mode, st):
        L = self.api.lib()
        cix = {"learned_index": self.cix_rmi, "hash_table": self.cix_table}.get(mode, self.cix)
        r = L.godiet_seed(ctypes.byref(cix), ctypes.byref(self.creads), ctypes.byref(self.prm),
                          ctypes.byref(self.opts), ctypes.c_void_p(self.anchors.data_ptr()),
                          self.acap, ctypes.c_void_p(self.roff.data_ptr()),
                          ctypes.c_void_p(self.shift.data_ptr()),
                          ctypes.c_void_p(self.ws_s.data_ptr()), self.ws_s.numel(),
                          ctypes.c_void_p(self.st_s.data_ptr()), st)
        if r != 0:
            raise RuntimeError("godiet_seed failed: %d" % r)

    def step(self, mode="binary_search", index=True):
        """One step (index=False: the seeding pass alone, on the index built last)."""
        if mode not in STEP_MODES:
            raise ValueError("unknown step mode %r" % (mode,))
        main = self.torch.cuda.current_stream()
        st = ctypes.c_void_p(main.cuda_stream)
        if self.overlap:
            self.side.wait_event(self.ev_seed)      # the last step's seeding has read the index
            st_i = ctypes.c_void_p(self.side.cuda_stream)
        else:
            st_i = st
        if index:
            self.index_step(mode, st_i)
        if self.overlap:
            self.ev_index.record(self.side)
            self.opts.index_ready = self.ev_index.cuda_event
        else:
            self.opts.index_ready = None
        self.seed_step(mode, st)
        if self.overlap:
            self.ev_seed.record(main)

    def check(self):
        self.torch.cuda.synchronize()
        if int(self.st_i.item()) != 0 or int(self.st_s.item()) != 0:
            raise RuntimeError("device status set: index %d seed %d" % (int(self.st_i.item()),
                                                                         int(self.st_s.item())))
        if int(self.n_out.item()) != self.n_index or int(self.roff[-1].item()) != self.n_anchors:
            raise RuntimeError("output sizes changed between steps")

    def digest(self):
        h = hashlib.sha256()
        h.update(self.ikeys.cpu().numpy().tobytes())
        h.update(self.ivals.cpu().numpy().tobytes())
        h.update(self.anchors[:4 * self.n_anchors].cpu().numpy().tobytes())
        h.update(self.roff.cpu().numpy().tobytes())
        h.update(self.shift.cpu().numpy().tobytes())
        return h.hexdigest()[:16]


def traced(gd, torch, fn, reps):
    """{kernel: (launches, ms)} of reps calls of fn (events around every launch)."""
    torch.cuda.synchronize()
    gd.trace_filter(None)
    gd.trace_dump()
    gd.trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    gd.trace_enable(False)
    return gd.trace_dump()


def time_modes(gd, torch, s, modes, steps, warmup, index=True):
    """Per mode: warm-up, a traced pass of `steps` steps for the per-kernel breakdown, then
    the timed region of `steps` steps with events around the dominant kernel's launches
    only.  Every mode must give the same outputs."""
    out = {}
    for mode in modes:
        for _ in range(warmup):
            s.step(mode, index)
        s.check()
        digest = s.digest()
        trace = traced(gd, torch, lambda: s.step(mode, index), steps)
        # the largest kernel that has an algorithmic model (under counter collection, which
        # serialises dispatches, another kernel can be larger)
        cand = [kv for kv in trace.items() if modeled(kv[0])] or list(trace.items())
        dom = max(cand, key=lambda kv: kv[1][1])[0]
        gd.trace_filter(dom)
        gd.trace_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step(mode, index)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gd.trace_enable(False)
        live = gd.trace_dump()
        gd.trace_filter(None)
        s.check()
        if s.digest() != digest:
            raise RuntimeError("outputs changed between steps")
        ms = (t1 - t0) * 1e3 / steps
        out[mode] = dict(ms_per_step=ms, reads_per_s=s.reads.n_seq / (ms * 1e-3), digest=digest,
                         trace=trace, dominant=dom, live=live)
        log("[bench] %s%s: %.3f ms/step, %.3e reads/s" % (
            mode.replace("_", " "), "" if index else " (seeding pass)", ms,
            s.reads.n_seq / (ms * 1e-3)))
    ref = out[modes[0]]["digest"]
    for mode in modes[1:]:
        if out[mode]["digest"] != ref:
            raise RuntimeError("%s outputs differ from %s outputs" % (mode, modes[0]))
    return out


OVERLAP_NOTE = ("index build + learned-index training on a side stream, seeding waits on "
                "their event after its read sketches")


def overlapped_step(torch, s, steps, warmup, digest):
    """ms per learned-index step with index construction on a second stream overlapping
    the read sketches (outputs must equal the one-stream step's)."""
    s.overlap = True
    try:
        for _ in range(warmup):
            s.step("learned_index")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step("learned_index")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        s.check()
        if s.digest() != digest:
            raise RuntimeError("overlapped steps changed the outputs")
    finally:
        s.overlap = False
    return ms


def graph_step(torch, s, mode, steps):
    """The whole step (index build, training, seeding) captured as one HIP graph and
    replayed; returns ms per replay.  Outputs must equal the eager step's."""
    digest = s.digest()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        s.step(mode)
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        s.step(mode)
    # outputs cleared (outside the graph), so a replay that wrote nothing cannot pass
    s.anchors.zero_()
    s.ikeys.zero_()
    g.replay()
    s.check()
    if s.digest() != digest:
        raise RuntimeError("graph replay changed the outputs")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    s.check()
    if s.digest() != digest:
        raise RuntimeError("graph replay changed the outputs")
    ms = e0.elapsed_time(e1) / steps
    del g
    return ms


def per_kernel(trace, steps):
    return {kn: dict(launches=n // steps, ms_per_step=ms / steps)
            for kn, (n, ms) in sorted(trace.items(), key=lambda kv: -kv[1][1])}


def work_units(s):
    """k-mers, patterned bases and original bases one step sketches (reference, then every
    read shift)."""
    k = s.k
    rl = np.diff(s.ref_offsets)
    ref_np = int(kept_counts(rl, s.pattern, 0).sum())
    ref_km = int(np.maximum(kept_counts(rl, s.pattern, 0) - k + 1, 0).sum())
    read_np = read_km = 0
    for a in range(len(s.pattern)):
        kc = kept_counts(s.read_lengths, s.pattern, a)
        read_np += int(kc.sum())
        read_km += int(np.maximum(kc - k + 1, 0).sum())
    return dict(ref_bases=int(rl.sum()), read_bases=int(s.read_lengths.sum()),
                shifts=len(s.pattern), ref_np=ref_np, ref_kmers=ref_km, read_np=read_np,
                read_kmers=read_km)


def measured_traffic(name, workload, launches_per_step):
    """HBM bytes per launch from the committed counter runs, or None if the kernel's source
    changed since they were taken."""
    m = MEASURED_TRAFFIC.get((name, workload))
    if m is None:
        return None
    with open(os.path.join(ROOT, m["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != m["sha256_16"]:
            return None
    return m["bytes_per_step"] / launches_per_step


def modeled(name):
    """Whether roofline() has an algorithmic model for this kernel."""
    return name.startswith(("k_sketch", "k_lookup", "k_bucket_sort", "k_scatter", "k_expand"))


def sketch_bytes(s, units):
    """Algorithmic bytes of the sketches of one step: ceil(L/4) of every sketched batch
    (the reference once, the reads once per shift) + 12 bytes per minimizer record."""
    return ((units["ref_bases"] + 3) // 4 + 12 * s.n_index +
            units["shifts"] * ((units["read_bases"] + 3) // 4) + 12 * s.queries)


def roofline(name, s, units, ms_total, steps, launches, workload):
    """Roofline entry of one kernel from its traced time over `steps` steps."""
    sec = ms_total * 1e-3 / steps
    base = dict(kernel=name, avg_launch_ms=ms_total / launches,
                launches_per_step=launches / steps,
                traffic=measured_traffic(name, workload, launches / steps))
    if name.startswith("k_sketch"):
        kmers = units["ref_kmers"] + units["read_kmers"]
        achieved = kmers * OPS_PER_KMER / sec / 1e9
        by = sketch_bytes(s, units)
        base.update(bound="alu", achieved=achieved, peak=ALU_PEAK_GOPS, unit="GOP/s",
                    frac=achieved / ALU_PEAK_GOPS, ops_per_kmer=OPS_PER_KMER,
                    kmers_per_launch=kmers * steps / launches,
                    algorithmic_bytes_per_launch=by * steps / launches,
                    hbm_view=dict(achieved=by / sec / 1e9, peak=HBM_PEAK_GBPS, unit="GB/s",
                                  frac=by / sec / 1e9 / HBM_PEAK_GBPS,
                                  bytes_rule="ceil(L/4) of every sketched batch (original "
                                             "bases) + 12 B per minimizer record"))
        return base
    if name.startswith("k_lookup"):
        by = s.queries * LOOKUP_BYTES
        base["bytes_rule"] = "8 B query + 8 B (lower bound, count) + one 64-B index line"
    elif name.startswith("k_bucket_sort") or name.startswith("k_scatter"):
        by = SORT_BYTES * s.n_index
        base["bytes_rule"] = "12-B record read + written"
    elif name.startswith("k_expand"):
        by = 16 * s.n_anchors
        base["bytes_rule"] = "16-B anchor written"
    else:
        return None
    achieved = by / sec / 1e9
    base.update(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBPS, unit="GB/s",
                frac=achieved / HBM_PEAK_GBPS, algorithmic_bytes_per_launch=by * steps / launches)
    return base


def index_build_rate(gd, torch, s, reps=5):
    """Index build of the reference alone: device time of one godiet_index_build call
    (sparsify, sketch, sort) and of its sort kernels, with the sort's rate at 24 B per
    record (one read and one write of each 12-byte record)."""
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    tr = traced(gd, torch, lambda: s.index_step("binary_search", st), reps)
    total = sum(v[1] for v in tr.values()) / reps
    sort = sum(v[1] for kn, v in tr.items() if kn.startswith(SORT_KERNELS)) / reps
    s.check()
    return dict(records=s.n_index, call_ms=total, sort_ms=sort,
                sort_GBps=SORT_BYTES * s.n_index / (sort * 1e-3) / 1e9,
                call_GBps=((s.ref.n_bases + 3) // 4 + SORT_BYTES * s.n_index) / (total * 1e-3)
                / 1e9,
                bytes_rule="sort: 24 B per record; call: ceil(L/4) + 24 B per record",
                kernels_ms={kn: v[1] / reps for kn, v in sorted(tr.items(), key=lambda kv: -kv[1][1])})


def sketch_gbps(gd, torch, seqs, pattern, k, w, reps=5):
    """Reference sketch throughput: (ceil(L/4) + 12 bytes per minimizer) / the summed device
    time of the kernels of one godiet_sketch call (kept counts, scan, sparsify, sketch; the
    fill that clears the tile states and the gaps between launches are not counted)."""
    keys, vals, mz = gd.sketch(seqs, pattern, k, w)
    m = keys.numel()
    del keys, vals, mz
    tr = traced(gd, torch, lambda: gd.sketch(seqs, pattern, k, w, capacity=m), reps)
    ms = sum(v[1] for kname, v in tr.items() if not kname.startswith("k_fill")) / reps
    by = (seqs.n_bases + 3) // 4 + 12 * m
    return by / (ms * 1e-3) / 1e9, ms, m, {kn: v[1] / reps for kn, v in tr.items()}


VOTE_PARAMS = (16, 3, 4)     # location voting on the step's anchors: D, V, max winners


def voting(gd, torch, s, steps, cpu=True):
    """Location voting over the learned-index step's anchors: GPU time per pass (K passes
    on the current stream, after one untimed pass) and the oracle on the same anchors."""
    D, V, cap = VOTE_PARAMS
    anchors = s.anchors[:4 * s.n_anchors].view(-1, 4)
    w, nw = gd.vote(anchors, s.roff, D, V, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        w, nw = gd.vote(anchors, s.roff, D, V, cap)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    rows = gd.winners_rows(w, nw)
    out = dict(D=D, V=V, max_winners=cap, ms_per_pass=ms,
               reads_per_s=s.reads.n_seq / (ms * 1e-3), winners=int(rows.shape[0]),
               rescued=int((rows[:, 3] & 1).sum()),
               reads_with_winner=int(((nw.cpu().numpy() > 0)).sum()))
    if cpu:
        import oracle
        a = anchors.cpu().numpy().view(np.uint32)
        off = s.roff.cpu().numpy().view(np.uint64)
        t0 = time.perf_counter()
        oracle.vote(a, off, D, V, cap)
        sec = time.perf_counter() - t0
        out["cpu_oracle"] = dict(reads_per_s=s.reads.n_seq / sec, cores=1,
                                 sample="all reads of the step")
    return out



def location_sorts(gd, torch, s, data, reps=3):
    """Sorting each read's retrieved locations before voting (a synthetic analogue of
    Table 10): the adaptive default, one digit sort of the whole batch, a per-read merge of
    the runs the anchors already form, a per-read heapsort; on the step's Illumina-like
    anchors and on HiFi- and ONT-like reads seeded against the same index.  Every way gives
    the same winners (checked here)."""
    import datagen
    rng = np.random.default_rng(1205)
    ix = gd.index_build(s.ref, s.pattern, s.k, s.w)
    batches = {"illumina": (s.anchors[:4 * s.n_anchors].view(-1, 4), s.roff, 16)}
    for name, lens, err in (("hifi", datagen.hifi_lengths(2000, rng), (0.005, 0.0025, 0.0025)),
                            ("ont", datagen.ont_lengths(2000, rng), (0.04, 0.02, 0.02))):
        codes, offs = datagen.variable_reads(data["ref"], lens, 1206, *err)[:2]
        a, off, _ = gd.seed(ix, gd.to_device(codes, offs), s.pattern, s.k, s.w)
        batches[name] = (a, off, 100)
    out = {}
    sort_kernels = ("k_vote_read_sort", "k_vote_long_sort", "k_digit", "k_hist", "k_scatter",
                    "k_bucket_sort", "k_coarse_starts", "k_scan")
    for name, (a, off, D) in batches.items():
        res = dict(reads=int(off.numel() - 1), locations=int(a.shape[0]), D=D, V=3)
        ref_rows = None
        for sort in ("adaptive", "radix", "merge", "heap"):
            w, nw = gd.vote(a, off, D, 3, 4, sort=sort)
            rows = gd.winners_rows(w, nw)
            if ref_rows is None:
                ref_rows = rows
            elif not np.array_equal(rows, ref_rows):
                raise RuntimeError("location sort %s changed the winners" % sort)
            torch.cuda.synchronize()
            gd.trace_dump()
            gd.trace_enable(True)
            for _ in range(reps):
                gd.vote(a, off, D, 3, 4, sort=sort)
            torch.cuda.synchronize()
            gd.trace_enable(False)
            tr = gd.trace_dump()
            total = sum(v[1] for v in tr.values()) / reps
            srt = sum(v[1] for kn, v in tr.items() if kn.startswith(sort_kernels)) / reps
            res[sort] = dict(sort_ms=srt, vote_ms=total)
        out[name] = res
    return out


FIG4_SETTINGS = [("10", 8, 6), ("100", 8, 6), ("1110110110111", 13, 9), ("10", 21, 11)]



def fig4_experiment(gd, torch, reps=3, cpu=True):
    """Seed-matching experiment on 100,000 pairs of 1,000 bases: device time of the seed
    counts (four algorithms) per setting, of the edit distances and of the accepted-pairs
    curves; the oracle on a sample of pairs for comparison."""
    import datagen
    o, oo, c, co, _ = datagen.workload_fig4()
    n = oo.size - 1
    so, sc = gd.to_device(o, oo), gd.to_device(c, co)
    out = dict(workload="fig4-100k: 100,000 pairs of 1,000 bases, per-pair substitution "
                        "rate uniform in [0, 0.6]", pairs=n)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        gd.trace_dump()
        gd.trace_enable(True)
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        gd.trace_enable(False)
        tr = gd.trace_dump()
        return r, {kn: v[1] / reps for kn, v in tr.items() if not kn.startswith("k_fill")}

    dist, kt = timed(lambda: gd.edit_distance(so, sc))
    ms = sum(kt.values())
    out["edit_distance"] = dict(ms=ms, pairs_per_s=n / (ms * 1e-3),
                                cells_per_s=1000.0 * 1000.0 * n / (ms * 1e-3))
    max_e = int(dist.max().item())
    out["seed_match"] = {}
    for pattern, k, w in FIG4_SETTINGS:
        counts, kt = timed(lambda: gd.seed_match(so, sc, pattern, k, w))
        ms = sum(kt.values())
        flat = counts.reshape(-1)
        _, ka = timed(lambda: [gd.accepted_pairs(dist, flat, g, max_e) for g in range(4)])
        accepted = {alg: gd.accepted_pairs(dist, flat, alg, max_e).cpu().numpy()
                    for alg in gd.FIG4_ALGORITHMS}
        out["seed_match"]["%s/%d/%d" % (pattern, k, w)] = dict(
            ms=ms, pairs_per_s=n / (ms * 1e-3), accepted_curves_ms=sum(ka.values()),
            accepted_fraction_at_ed_138={a: float(v[min(138, max_e)]) / n
                                        for a, v in accepted.items()})
    if cpu:
        import oracle
        m = 500
        t0 = time.perf_counter()
        oracle.seed_match(o[:oo[m]], oo[:m + 1], c[:co[m]], co[:m + 1], "10", 8, 6)
        t1 = time.perf_counter()
        for i in range(m // 5):
            oracle.edit_distance(o[oo[i]:oo[i + 1]], c[co[i]:co[i + 1]])
        t2 = time.perf_counter()
        out["cpu_oracle"] = dict(seed_match_pairs_per_s=m / (t1 - t0),
                                 edit_distance_pairs_per_s=(m // 5) / (t2 - t1), cores=1,
                                 sample="first 500 pairs (seed counts, 10/8/6), first 100 "
                                        "pairs (edit distance)")
    return out



def copy_gbps(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time): the measured HBM
    ceiling next to the published 8 TB/s."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9



def gather_rate(torch, n_keys, n_q, reps=5):
    """Random 8-byte gathers per second into an array of n_keys, by the library's gather
    probe (independent loads, four in flight per lane): the random-request reference for
    the lookups.  The probe's output is checked against torch's indexing."""
    import paper_2211_08157_amd as gd
    keys = torch.arange(n_keys, dtype=torch.int64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(404)
    idx = torch.randint(0, n_keys, (n_q,), device="cuda", generator=g)
    out, st = gd.random_gather(keys, idx)
    if not torch.equal(out, idx) or int(st.item()) != 0:
        raise RuntimeError("random-gather probe returned wrong values")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gd.random_gather(keys, idx)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del keys, idx, out
    return n_q / (ms * 1e-3)



def containment(gd, torch, reps):
    """Containment-style search: the 1,000-genome database (pattern 10, k=21, w=11, values
    carrying the genome id) and 10M x 150 bp reads drawn from 50 of its genomes; one call
    gives every genome's count of distinct minimizers shared with the reads, through binary
    search and through the learned index (identical counts required)."""
    import datagen
    d = datagen.workload_containment()
    ng = d["ref_offsets"].size - 1
    db = gd.to_device(d["ref"], d["ref_offsets"])
    reads = gd.to_device(d["reads"], d["read_offsets"])
    n_reads, db_bases = reads.n_seq, db.n_bases
    del d
    ix = gd.index_build(db, "10", 21, 11, val_bits=64)
    del db
    out = dict(genomes=ng, database_bases=db_bases, index_records=ix.n, reads=n_reads)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ref_counts = None
    for name, index in (("binary_search", ix),
                        ("learned_index", gd.rmi_train(ix, root="mlp", log2_leaves=18))):
        counts, sizes = gd.contain(index, reads, "10", 21, 11, ng)
        e0.record()
        for _ in range(reps):
            counts, sizes = gd.contain(index, reads, "10", 21, 11, ng)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if ref_counts is None:
            ref_counts = counts.clone()
        elif not torch.equal(counts, ref_counts):
            raise RuntimeError("learned-index containment counts differ from binary search")
        out[name] = dict(ms=ms, reads_per_s=n_reads / (ms * 1e-3))
    out["genomes_with_shared_minimizers"] = int((ref_counts != 0).sum().item())
    del ix, reads, ref_counts
    torch.cuda.empty_cache()
    return out



def kept_counts(lengths, pattern, shift):
    """Kept bases of sequences of the given lengths (closed form, for accounting)."""
    p, x = len(pattern), pattern.count("1")
    rot = [pattern[(t - shift) % p] == "1" for t in range(p)]
    first = np.concatenate([[0], np.cumsum(rot)])          # ones among the first r phases
    L = np.asarray(lengths, np.int64)
    return (L // p) * x + first[L % p]



# launch-parameter grid searched on the mixed batch (every candidate's anchors must match):
# 12 candidates
TUNE_GRID = {"long_records": [64, 192], "lookup_blocks": [8192, 32768],
             "long_blocks": [256, 1024, 4096]}
STEP_MODES = ("learned_index", "binary_search", "hash_table")


def leaves_for(n):
    """Learned-index size: about 32 keys per leaf, at least 2^18 leaves."""
    return max(18, int(np.ceil(np.log2(max(n, 1) / 32))))


def uneven_section(gd, torch, d, args):
    """The headline: the mixed batch on the 1 Gbp reference, per pattern: the whole step
    with each lookup form, the step as one graph replay, the seeding pass alone, the index
    build's rate and the rooflines."""
    from paper_2211_08157_amd import autotune
    ref = gd.to_device(d["ref"], d["ref_offsets"])
    reads = gd.to_device(d["reads"], d["read_offsets"])
    res = {}
    for pat in args.patterns:
        head = pat == "10"
        ix = gd.index_build(ref, pat, d["k"], d["w"])
        leaves = leaves_for(ix.n)
        ixl = gd.rmi_train(ix, root="mlp", log2_leaves=leaves)
        tuning, report = autotune.tune(ixl, reads, pat, d["k"], d["w"], grid=TUNE_GRID, reps=1,
                                       use_cache=False)
        del ix, ixl
        torch.cuda.empty_cache()
        s = Session(gd, ref, reads, d["ref_offsets"], d["read_offsets"], pat, d["k"], d["w"],
                    log2_leaves=leaves, tuning=tuning)
        steps = args.steps if head else max(3, args.steps // 4)
        warm = args.warmup if head else 1
        log("[bench] uneven 1 Gbp batch, pattern %s: %d index records, %d anchors, %d lookups"
            % (pat, s.n_index, s.n_anchors, s.queries))
        modes = time_modes(gd, torch, s, STEP_MODES, steps, warm)
        passes = time_modes(gd, torch, s, STEP_MODES, steps, 1, index=False)
        units = work_units(s)
        li = modes["learned_index"]
        r = dict(index_records=s.n_index, anchors=s.n_anchors, lookups_per_step=s.queries,
                 log2_leaves=leaves, tuning=tuning,
                 tuning_report=dict(candidates=len(report), winner=tuning,
                                    winner_ms=min(ms for _, ms in report),
                                    slowest_ms=max(ms for _, ms in report),
                                    note="seeding pass per candidate (index and model built)",
                                    rows=[dict(tuning=t, ms=ms) for t, ms in report]),
                 work_per_step=units, output_sha256_16=li["digest"])
        for m in STEP_MODES:
            r[m] = dict(ms_per_step=modes[m]["ms_per_step"], reads_per_s=modes[m]["reads_per_s"],
                        kernels=per_kernel(modes[m]["trace"], steps))
        r["learned_vs_binary_speedup"] = (modes["binary_search"]["ms_per_step"] /
                                          li["ms_per_step"])
        r["seeding_pass"] = {m: dict(ms=passes[m]["ms_per_step"],
                                     reads_per_s=passes[m]["reads_per_s"])
                             for m in STEP_MODES}
        r["seeding_pass"]["learned_vs_binary_speedup"] = (
            passes["binary_search"]["ms_per_step"] / passes["learned_index"]["ms_per_step"])
        r["seeding_pass"]["note"] = "index, learned index and hash table built beforehand"
        dom = li["dominant"]
        n_l, ms_l = li["live"][dom]
        roof = roofline(dom, s, units, ms_l, steps, n_l, "uneven-1Gbp/" + pat)
        roof["timing"] = "HIP events around this kernel's launches inside the timed region"
        if roof and roof["kernel"].startswith("k_lookup"):
            # the lookups as random requests: one launch's time at the rate of random 8-byte
            # gathers into an array of the index's size, per query of the launch
            g = gather_rate(torch, s.n_index, s.queries_per_shift[0])
            roof["random_gather_per_s"] = g
            roof["requests_per_query"] = (roof["avg_launch_ms"] * 1e-3 * g /
                                          (s.queries / roof["launches_per_step"]))
        r["roofline"] = roof
        sk = [kv for kv in li["trace"].items() if kv[0].startswith("k_sketch")]
        if sk:
            kn, (n, ms) = sk[0]
            r["roofline_sketch"] = roofline(kn, s, units, ms, steps, n, "uneven-1Gbp/" + pat)
            r["roofline_sketch"]["timing"] = "HIP events around every launch (traced pass)"
        if head:
            gms = graph_step(torch, s, "learned_index", steps)
            r["graph_step"] = dict(ms_per_step=gms, reads_per_s=s.reads.n_seq / (gms * 1e-3),
                                   note="the whole learned-index step captured as one HIP "
                                        "graph and replayed")
            log("[bench] graph-replayed step: %.3f ms" % gms)
            oms = overlapped_step(torch, s, steps, warm, li["digest"])
            r["overlapped_step"] = dict(ms_per_step=oms, reads_per_s=s.reads.n_seq / (oms * 1e-3),
                                        note=OVERLAP_NOTE)
            log("[bench] overlapped step: %.3f ms" % oms)
        r["index_build"] = index_build_rate(gd, torch, s)
        log("[bench] index build, pattern %s: %.3f ms per call, sort %.3f ms = %.0f GB/s"
            % (pat, r["index_build"]["call_ms"], r["index_build"]["sort_ms"],
               r["index_build"]["sort_GBps"]))
        res[pat] = r
        del s
        torch.cuda.empty_cache()
    return ref, reads, res


def lookups_1gbp(gd, torch, ref, reads, reps):
    """Learned index against binary search on the 1 Gbp key arrays of patterns '10' (about
    83M keys) and '11' (no base dropped, about 167M keys), k=21, w=11: 500M queries, 80 %
    drawn from the mixed batch's read minimizers under the same pattern and 20 % random
    64-bit keys (seeded device generator), two-stage FP32 models with an MLP root at 2^18
    and at about 32 keys per leaf.  Every model must return the binary-search (lower
    bound, run length) of every query; each model's fallback fraction (queries its window
    does not bracket) and histogram of window widths (keys read, powers of two) are
    reported."""
    out = {}
    for pat in ("10", "11"):
        ix = gd.index_build(ref, pat, 21, 11)
        rk, _, _ = gd.sketch(reads, pat, 21, 11)
        g = torch.Generator(device="cuda")
        g.manual_seed(404)
        n_total = 500_000_000
        n_abs = n_total // 5
        n_pres = n_total - n_abs
        q = torch.empty(n_total, dtype=torch.int64, device="cuda")
        idx = torch.randint(0, rk.numel(), (n_pres,), device="cuda", generator=g)
        q[:n_pres] = rk[idx]
        del idx, rk
        q[n_pres:] = torch.randint(-2**63, 2**63 - 1, (n_abs,), dtype=torch.int64,
                                   device="cuda", generator=g)
        res = dict(queries=n_total, index_records=ix.n)
        ref_lb = ref_occ = None
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        big = leaves_for(ix.n)
        models = [("binary_search", ix, None),
                  ("learned_index", gd.rmi_train(ix, root="mlp", log2_leaves=18), 18),
                  ("learned_index_%d_leaves" % (1 << big),
                   gd.rmi_train(ix, root="mlp", log2_leaves=big), big)]
        for name, index, lv in models:
            lb, occ = gd.lookup(index, q)
            e0.record()
            for _ in range(reps):
                lb, occ = gd.lookup(index, q)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if ref_lb is None:
                ref_lb, ref_occ = lb, occ
            elif not (torch.equal(lb, ref_lb) and torch.equal(occ, ref_occ)):
                raise RuntimeError("learned-index lookups differ from binary search")
            res[name] = dict(ms=ms, lookups_per_s=n_total / (ms * 1e-3))
            if lv is not None:
                st = gd.rmi_stats(index, q)
                res[name].update(log2_leaves=lv, fallback_fraction=st["fallbacks"] / n_total,
                                 window_keys_hist=st["window_keys"])
            del lb, occ
        res["found"] = int((ref_occ != 0).sum().item())
        res["random_keys_found"] = int((ref_occ[n_pres:] != 0).sum().item())
        res["learned_vs_binary_speedup"] = (res["binary_search"]["ms"] /
                                            res["learned_index"]["ms"])
        log("[bench] 500M lookups, %d keys ('%s'): binary search %.1f ms, learned index %.1f "
            "ms (2^18 leaves), %.1f ms (2^%d)" % (ix.n, pat, res["binary_search"]["ms"],
                                                 res["learned_index"]["ms"],
                                                 res["learned_index_%d_leaves" % (1 << big)]["ms"],
                                                 big))
        out[pat] = res
        del q, ref_lb, ref_occ, ix, models
        torch.cuda.empty_cache()
    return out


def cpu_seed_parallel(oracle, ik, iv, codes, offsets, lo, hi, pattern, k, w, threads):
    """oracle.seed over reads [lo, hi) split into read ranges of about equal bases."""
    from concurrent.futures import ThreadPoolExecutor
    offsets = np.asarray(offsets, np.int64)
    n_tasks = 8 * threads
    cum = offsets[lo:hi + 1] - offsets[lo]
    cuts = np.unique(np.searchsorted(cum, np.linspace(0, cum[-1], n_tasks + 1)[1:-1]) + lo)
    bounds = [lo] + [int(c) for c in cuts if lo < c < hi] + [hi]

    def one(i):
        r0, r1 = bounds[i], bounds[i + 1]
        oracle.seed(ik, iv, codes[offsets[r0]:offsets[r1]], offsets[r0:r1 + 1] - offsets[r0],
                    pattern, k, w)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(len(bounds) - 1)))


def cpu_baseline(d, pattern, k, w, read_frac, classes=None):
    """The oracle on the host's cores: the index of the reference built chunk by chunk on
    every thread (chunks with a margin of context, then merged; identical to one call),
    then seeding of the first read_frac of every read class on every thread, each class's
    time scaled to the whole class.  The oracle is C called through ctypes, which releases
    the interpreter lock."""
    import oracle
    threads = host_threads()
    if d["ref_offsets"].size != 2:
        raise ValueError("the chunked oracle index takes one reference sequence")
    t0 = time.perf_counter()
    ik, iv = oracle.index_build_chunked(d["ref"], pattern, k, w, threads)
    t_index = time.perf_counter() - t0
    ro = np.asarray(d["read_offsets"], np.int64)
    n_reads = ro.size - 1
    classes = classes or {"all": (0, n_reads)}
    t_seed, parts = 0.0, []
    for name, (lo, hi) in classes.items():
        m = max(1, int(round((hi - lo) * read_frac)))
        t0 = time.perf_counter()
        cpu_seed_parallel(oracle, ik, iv, d["reads"], ro, lo, lo + m, pattern, k, w, threads)
        dt = time.perf_counter() - t0
        t_seed += dt * (hi - lo) / m
        parts.append("%s: first %d of %d reads in %.2f s" % (name, m, hi - lo, dt))
    total = t_index + t_seed
    return dict(value=n_reads / total, unit="reads/s", cores=threads, kind="oracle",
                host=host_cores(), index_records=int(ik.size),
                sample="index of the whole reference on %d threads (%.1f s, %d chunks with a "
                       "margin of context, merged); seeding on %d threads, %s, scaled to "
                       "each class" % (threads, t_index, 4 * threads, threads, "; ".join(parts)),
                seconds=dict(index=t_index, seeding_scaled=t_seed))


def illumina_section(gd, torch, data, args):
    """The 100 Mbp / 1M-read Illumina-like workload: the step with each lookup form, the
    overlapped step, its rooflines."""
    pattern, k, w = "10", data["k"], data["w"]
    s = Session(gd, gd.to_device(data["ref"], data["ref_offsets"]),
                gd.to_device(data["reads"], data["read_offsets"]), data["ref_offsets"],
                data["read_offsets"], pattern, k, w)
    log("[bench] illumina: index %d records, %d anchors, %d lookups per step"
        % (s.n_index, s.n_anchors, s.queries))
    modes = time_modes(gd, torch, s, STEP_MODES, args.steps, args.warmup)
    ms_ov = overlapped_step(torch, s, args.steps, args.warmup, modes["learned_index"]["digest"])
    units = work_units(s)
    li = modes["learned_index"]
    dom = li["dominant"]
    n_l, ms_l = li["live"][dom]
    roof = roofline(dom, s, units, ms_l, args.steps, n_l, "illumina-100Mbp")
    roof["timing"] = "HIP events around this kernel's launches inside the timed region"
    others = [kv for kv in li["trace"].items() if kv[0] != dom and modeled(kv[0])]
    second = max(others, key=lambda kv: kv[1][1]) if others else None
    roof_next = (roofline(second[0], s, units, second[1][1], args.steps, second[1][0],
                          "illumina-100Mbp") if second else None)
    r = dict(workload="illumina-100Mbp: 100 Mbp reference (5% repeats), 1M x 150 bp reads, "
                      "pattern 10, k=21, w=11",
             index_records=s.n_index, anchors=s.n_anchors, lookups_per_step=s.queries,
             work_per_step=units, output_sha256_16=li["digest"],
             learned_vs_binary_speedup=modes["binary_search"]["ms_per_step"] / li["ms_per_step"],
             overlapped_step=dict(ms_per_step=ms_ov, reads_per_s=s.reads.n_seq / (ms_ov * 1e-3),
                                  note=OVERLAP_NOTE),
             roofline=roof, roofline_second_kernel=roof_next)
    for m in STEP_MODES:
        r[m] = dict(ms_per_step=modes[m]["ms_per_step"], reads_per_s=modes[m]["reads_per_s"],
                    kernels=per_kernel(modes[m]["trace"], args.steps))
    log("[bench] illumina overlapped learned-index step: %.3f ms/step" % ms_ov)
    return s, r


def gapped_step(gd, torch, steps, warmup):
    """The learned-index step on the Illumina-like workload with assembly gaps (about 5 %
    N in the reference) and N calls in the reads, which takes the N-aware path; plus the
    device text packer on the reference's text."""
    import datagen
    d = datagen.workload_gapped()
    g = Session(gd, gd.to_device(d["ref"], d["ref_offsets"]),
                gd.to_device(d["reads"], d["read_offsets"]), d["ref_offsets"], d["read_offsets"],
                "10", d["k"], d["w"])
    for _ in range(warmup):
        g.step("learned_index")
    g.check()
    trace = traced(gd, torch, lambda: g.step("learned_index"), steps)
    kernels = per_kernel(trace, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step("learned_index")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    g.check()
    n_frac_ref = float((d["ref"] == 4).mean())
    n_frac_reads = float((d["reads"] == 4).mean())
    text = datagen.to_text(d["ref"], seed=7)
    n_reads = g.reads.n_seq
    del g
    gd.to_device_ascii(text, [0, len(text)])
    tr = traced(gd, torch, lambda: gd.to_device_ascii(text, [0, len(text)]), 5)
    pk = tr.get("k_pack_ascii", (5, float("nan")))[1] / 5
    n = len(text)
    return dict(workload="illumina-gapped-100Mbp: the Illumina-like workload with 50 gaps of "
                         "20-180 kbp and 20,000 isolated N in the reference, one N call per "
                         "1,000 read bases",
                ms_per_step=ms, reads_per_s=n_reads / (ms * 1e-3),
                n_fraction_reference=n_frac_ref, n_fraction_reads=n_frac_reads,
                pack_ascii_ms=pk, pack_ascii_GBps=(n + n // 4 + n // 8) / (pk * 1e-3) / 1e9,
                pack_ascii_bytes_rule="text in + 2-bit codes + N bits out", kernels=kernels)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-read-frac", type=float, default=0.5,
                    help="share of every read class the CPU oracle seeds (then scaled)")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated parts to run: " + ", ".join(SECTIONS) +
                         " (the headline needs 'uneven')")
    ap.add_argument("--patterns", default="10,110",
                    help="patterns of the uneven section ('10' is the headline and required)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the index is "
              "replicated and reads split by range when it is sharded); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    args.patterns = [x for x in args.patterns.split(",") if x]
    if "10" not in args.patterns or set(args.patterns) - {"10", "110"}:
        print("--patterns: a comma-separated subset of 10,110 that holds 10", file=sys.stderr)
        sys.exit(2)
    sections = set(x for x in args.sections.split(",") if x)
    bad = sections - set(SECTIONS)
    if bad:
        print("unknown sections: %s" % ", ".join(sorted(bad)), file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_2211_08157_amd as gd
    torch.cuda.set_device(0)
    out = {"metric": METRIC, "value": None, "unit": "reads/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic"}

    if sections & {"uneven", "lookups", "sketch1g"}:
        log("[bench] generating the 1 Gbp reference and the mixed batch")
        d = datagen.workload_uneven()
        n_reads = d["read_offsets"].size - 1
        ref = reads = None
        if "uneven" in sections:
            ref, reads, un = uneven_section(gd, torch, d, args)
            h = un["10"]
            li = h["learned_index"]
            out.update(value=li["reads_per_s"], ms_per_step=li["ms_per_step"])
            out["config"] = {
                "workload": "uneven-1Gbp: 1 Gbp reference (5%% repeats); one mixed batch of "
                            "2,000,000 x 150 bp + 20,000 HiFi-like + 20,000 ONT-like reads "
                            "(%d bases); pattern 10, k=21, w=11; step = index build + "
                            "learned-index training + seeding of the whole batch (pattern "
                            "alignment, anchors)" % int(d["reads"].size),
                "lookup": "learned_index (2-stage FP32 RMI, MLP root, 2^%d leaves)"
                          % h["log2_leaves"],
                "launch_parameters": h["tuning"], "global_batch": n_reads,
                "parallelism": "single GPU"}
            out["binary_search"] = h["binary_search"]
            out["learned_vs_binary_speedup"] = h["learned_vs_binary_speedup"]
            out["hash_table"] = h["hash_table"]
            out["graph_step"] = h["graph_step"]
            out["overlapped_step"] = h["overlapped_step"]
            out["seeding_pass"] = h["seeding_pass"]
            out["roofline"] = h["roofline"]
            out["roofline_sketch"] = h.get("roofline_sketch")
            out["index_build"] = h["index_build"]
            out["index_build_GBps"] = h["index_build"]["sort_GBps"]
            out["work_per_step"] = h["work_per_step"]
            out["kernels"] = h["learned_index"]["kernels"]
            out["output_sha256_16"] = h["output_sha256_16"]
            out["tuning_report"] = h["tuning_report"]
            if "110" in un:
                out["pattern_110"] = un["110"]
        if ref is None:
            ref = gd.to_device(d["ref"], d["ref_offsets"])
            reads = gd.to_device(d["reads"], d["read_offsets"])
        if "lookups" in sections:
            out["lookups_500M"] = lookups_1gbp(gd, torch, ref, reads, max(2, args.steps // 4))
        del reads
        if "sketch1g" in sections:
            sk = {}
            for pat in ("10", "110"):
                g, ms, m, kern = sketch_gbps(gd, torch, ref, pat, d["k"], d["w"])
                sk[pat] = dict(GBps=g, ms=ms, minimizers=m, frac_of_hbm_peak=g / HBM_PEAK_GBPS,
                               kernels_ms=kern)
                log("[bench] 1 Gbp sketch, pattern %s: %.3f ms, %.1f GB/s" % (pat, ms, g))
            out["sketch_1Gbp"] = sk
            out["sketch_bytes_rule"] = ("ceil(L/4) + 12 B per minimizer over the summed device "
                                        "time of the call's kernels (fill and gaps excluded)")
        del ref
        torch.cuda.empty_cache()
        if "uneven" in sections and not args.no_cpu_baseline:
            log("[bench] timing the CPU oracle on the mixed batch")
            out["cpu_baseline"] = cpu_baseline(d, "10", d["k"], d["w"], args.cpu_read_frac,
                                               d["classes"])
            log("[bench] CPU oracle: %.3e reads/s on %d threads" % (
                out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"]))
        del d

    if sections & {"illumina", "extras"}:
        log("[bench] generating the 100 Mbp / 1M-read workload")
        data = datagen.workload_illumina()
        s, il = illumina_section(gd, torch, data, args)
        if "illumina" in sections:
            gbps, sk_ms, sk_m, sk_kernels = sketch_gbps(gd, torch, s.ref, "10", data["k"],
                                                        data["w"])
            il.update(sketch_GBps=gbps, sketch_ms=sk_ms, sketch_kernels_ms=sk_kernels)
            il["random_gather_per_s"] = gather_rate(torch, s.n_index, s.queries)
            rn = il["roofline_second_kernel"]
            if rn and rn["kernel"].startswith("k_lookup"):
                il["lookup_requests_per_query"] = (rn["avg_launch_ms"] * 1e-3 *
                                                   il["random_gather_per_s"] /
                                                   (s.queries / rn["launches_per_step"]))
            log("[bench] illumina reference sketch %.3f ms, %.1f GB/s" % (sk_ms, gbps))
        if "extras" in sections:
            il["location_voting"] = voting(gd, torch, s, args.steps,
                                           cpu=not args.no_cpu_baseline)
            log("[bench] location voting: %.3f ms per pass" % il["location_voting"]["ms_per_pass"])
            il["location_sorts"] = location_sorts(gd, torch, s, data)
        del s
        torch.cuda.empty_cache()
        if "illumina" in sections and not args.no_cpu_baseline:
            log("[bench] timing the CPU oracle on the Illumina-like batch")
            il["cpu_baseline"] = cpu_baseline(data, "10", data["k"], data["w"], 1.0)
        out["illumina_100Mbp"] = il
        del data
        if "extras" in sections:
            out["n_aware_step"] = gapped_step(gd, torch, args.steps, args.warmup)
            log("[bench] gapped workload: %.3f ms/step" % out["n_aware_step"]["ms_per_step"])
            out["seed_matching_experiment"] = fig4_experiment(gd, torch,
                                                              cpu=not args.no_cpu_baseline)
            torch.cuda.empty_cache()
    if "containment" in sections:
        log("[bench] generating the 1,000-genome containment database and 10M reads")
        c = containment(gd, torch, max(2, args.steps // 4))
        out["containment_1000_genomes"] = c
        log("[bench] containment: binary search %.2f ms, learned index %.2f ms"
            % (c["binary_search"]["ms"], c["learned_index"]["ms"]))
    out["measured_copy_GBps"] = copy_gbps(torch)
    if out.get("sketch_1Gbp"):
        out["sketch_frac_of_measured_copy"] = {p: v["GBps"] / out["measured_copy_GBps"]
                                               for p, v in out["sketch_1Gbp"].items()}
    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 1 << 30
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
