"""MI355X (gfx950) sparsified seeding (Genome-on-Diet, arXiv 2211.08157).

Thin Python binding of libgodiet.so (C ABI in include/godiet.h).  This module only
marshals arguments: it packs base codes into the 2-bit layout, allocates device buffers
and workspaces with PyTorch, and passes raw pointers and the current HIP stream to the
library.  Every step of sparsification, sketching, index construction and seeding runs
in the library's HIP kernels; nothing here computes a minimizer, a sort or a lookup.

If the shared library is missing the import of the binding raises; there is no CPU
fallback.
"""
from .store import save_index, load_index
from .api import (GodietError, DeviceSeqs, DeviceIndex, pack, pack_n, to_device,
                  to_device_ascii, sparsify, sketch, index_build, seed, rmi_train, rmi_stats,
                  lookup, random_gather, contain, lib, lib_path, workspace_size, kept_bound,
                  trace_enable, trace_dump, trace_filter, vote, winners_rows, table_build,
                  seed_match, edit_distance, accepted_pairs, FIG4_ALGORITHMS, STATUS_CAPACITY,
                  STATUS_RANGE, STATUS_SHIFT)

__all__ = ["GodietError", "DeviceSeqs", "DeviceIndex", "pack", "pack_n", "to_device",
           "to_device_ascii", "sparsify", "sketch", "index_build", "seed", "rmi_train",
           "rmi_stats", "lookup", "random_gather", "contain", "lib", "lib_path",
           "workspace_size", "kept_bound", "trace_enable", "trace_dump", "trace_filter", "vote",
           "winners_rows", "table_build", "save_index", "load_index", "seed_match",
           "edit_distance", "accepted_pairs", "FIG4_ALGORITHMS", "STATUS_CAPACITY",
           "STATUS_RANGE", "STATUS_SHIFT"]
