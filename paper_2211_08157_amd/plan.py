"""Preallocated seeding plans and their HIP-graph capture.

A SeedPlan binds one read batch, one index and one parameter set to buffers allocated
once (workspace, anchors, offsets, shifts, status word).  run() then only enqueues the
library's kernels on the current stream -- no allocation, no host synchronisation, no
memset -- so a whole seeding pass over a mixed batch of short, HiFi-like and ONT-like
reads can be captured into one HIP graph and replayed with a single launch.
"""
import ctypes

from . import api


class SeedPlan:
    def __init__(self, index, reads, pattern, k, w, shift_mode=-1, align_t=0, max_occ=0,
                 tuning=None, capacity=None):
        import torch
        self.torch = torch
        self.index, self.reads = index, reads
        self.pattern, self.k, self.w = pattern, int(k), int(w)
        t = tuning or {}
        self.tuning = dict(t)
        self.opts = api.seed_opts(shift_mode, align_t, max_occ, t)
        self.prm = api.Params(pattern.encode(), self.k, self.w)
        self.cix = index.c()
        self.creads = reads.c()
        dev = "cuda"
        ws_bytes = api.workspace_size(api.OP_SEED, reads, pattern, k, w, index.n)
        self.ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.read_off = torch.empty(reads.n_seq + 1, dtype=torch.int64, device=dev)
        self.shift = torch.empty(max(reads.n_seq, 1), dtype=torch.uint8, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        if capacity is None:
            # size the anchor buffer with one eager pass (outside any capture)
            self.capacity = 0
            self.anchors = torch.empty(4, dtype=torch.int32, device=dev)
            self.run()
            torch.cuda.synchronize()
            capacity = int(self.read_off[-1].item())
        self.capacity = int(capacity)
        self.anchors = torch.empty(max(self.capacity, 1) * 4, dtype=torch.int32, device=dev)
        self.graph = None

    def run(self):
        """Enqueue one seeding pass on the current stream."""
        st = ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)
        r = api.lib().godiet_seed(ctypes.byref(self.cix), ctypes.byref(self.creads),
                                  ctypes.byref(self.prm), ctypes.byref(self.opts),
                                  ctypes.c_void_p(self.anchors.data_ptr()), self.capacity,
                                  ctypes.c_void_p(self.read_off.data_ptr()),
                                  ctypes.c_void_p(self.shift.data_ptr()),
                                  ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                  ctypes.c_void_p(self.status.data_ptr()), st)
        if r != api.OK:
            raise api.GodietError(r, "godiet_seed")

    def capture(self):
        """Capture run() into a HIP graph (one launch per replay)."""
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()                      # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def check(self):
        """Synchronise and raise if the device status word reports a problem."""
        self.torch.cuda.synchronize()
        st = int(self.status.item())
        if st & api.STATUS_CAPACITY:
            raise RuntimeError("anchor capacity exceeded (need %d)" % int(self.read_off[-1].item()))
        if st:
            raise RuntimeError("device status %d" % st)

    def outputs(self):
        n = int(self.read_off[-1].item())
        return (self.anchors[:4 * n].view(n, 4), self.read_off,
                self.shift[:self.reads.n_seq])
