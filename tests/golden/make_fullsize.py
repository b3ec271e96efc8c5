"""Record the oracle's results on the full-size workloads as digests.

Writes tests/golden/fullsize_oracle.json, which the full-size GPU tests compare against.
Every value in it comes from the oracle (oracle/) on inputs from datagen; nothing here
calls the GPU library.  Run from the repository root:

    python tests/golden/make_fullsize.py [--out FILE] [illumina] [gapped] [fig4] [uneven]
        [lookups | lookups10 | lookups11] [containment]

(no argument: all; "lookups" records both key arrays).  It needs about 20 GB of memory and takes tens of minutes on 8 cores.
Seeding and lookups are split over threads by read and query ranges (each read's anchors
and each query's result are independent of the others); index builds and containment
counts run as one oracle call each.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import datagen  # noqa: E402
import fullsize  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "fullsize_oracle.json")
K, W = 21, 11
# patterns of the 1 Gbp key arrays queried 500M times: '10' (about 83M keys) and '11'
# (about 167M keys, the unsparsified array)
LOOKUP_PATTERNS = ("10", "11")


def log(msg, t0=[time.perf_counter()]):
    print("[%7.1f s] %s" % (time.perf_counter() - t0[0], msg), flush=True)


def parallel_seed(ik, iv, codes, offsets, pattern, chunk=20_000):
    """oracle.seed over consecutive read ranges on threads (every read's anchors depend
    only on that read and the index), stitched back into one batch's output."""
    offsets = np.asarray(offsets, np.int64)
    n_reads = offsets.size - 1
    starts = list(range(0, n_reads, chunk))

    def one(r0):
        r1 = min(r0 + chunk, n_reads)
        o = offsets[r0:r1 + 1] - offsets[r0]
        return oracle.seed(ik, iv, codes[offsets[r0]:offsets[r1]], o, pattern, K, W)

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        res = list(ex.map(one, starts))
    total = sum(r[0].shape[0] for r in res)
    anchors = np.empty((total, 4), np.uint32)
    read_off = np.zeros(n_reads + 1, np.uint64)
    shift = np.empty(n_reads, np.uint32)
    pos = 0
    for r0, (a, off, sh) in zip(starts, res):
        m = a.shape[0]
        anchors[pos:pos + m] = a
        anchors[pos:pos + m, 0] += np.uint32(r0)
        read_off[r0:r0 + off.size] = off + np.uint64(pos)
        shift[r0:r0 + sh.size] = sh
        pos += m
    return anchors, read_off, shift


# location-voting parameters per workload: (D, V, max_winners)
VOTE = {"illumina-100Mbp": (16, 3, 4), "illumina-gapped-100Mbp": (16, 3, 4),
        "uneven-1Gbp": (100, 3, 4)}


def vote_rows(out, nw):
    r, j = np.nonzero(np.arange(out.shape[1])[None, :] < nw[:, None])
    return np.concatenate([r[:, None].astype(np.int64), out[r, j]], axis=1)


def seed_entry(d, pattern):
    ik, iv = oracle.index_build(d["ref"], d["ref_offsets"], pattern, K, W)
    log("%s %s: index %d records" % (d["name"], pattern, ik.size))
    ent = dict(index=fullsize.index_digest(ik, iv))
    a, off, sh = parallel_seed(ik, iv, d["reads"], d["read_offsets"], pattern)
    log("%s %s: %d anchors" % (d["name"], pattern, a.shape[0]))
    ent["anchors"] = fullsize.anchors_digest(a, off, sh)
    D, V, cap = VOTE[d["name"]]
    out, nw = oracle.vote(a, off, D, V, cap)
    ent["votes"] = dict(fullsize.votes_digest(nw, vote_rows(out, nw)), D=D, V=V, cap=cap)
    log("%s %s: %d winners" % (d["name"], pattern, ent["votes"]["n"]))
    return ent, ik


def parallel_lookup(ik, q, chunk=10_000_000):
    lb = np.empty(q.size, np.uint32)
    occ = np.empty(q.size, np.uint32)

    def one(lo):
        hi = min(lo + chunk, q.size)
        l, o = oracle.lookup(ik, q[lo:hi])
        lb[lo:hi] = l
        occ[lo:hi] = o

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        list(ex.map(one, range(0, q.size, chunk)))
    return lb, occ


# seed-matching experiment (Fig. 4): (pattern, k, w) settings recorded at full size
FIG4 = [("10", 8, 6), ("100", 8, 6), ("1110110110111", 13, 9), ("10", 21, 11)]


def fig4_entry():
    """Oracle results on the 100,000-pair experiment: edit distances, per-pair seed counts
    of every setting, and the accepted-pairs curves (thresholds 0..max distance)."""
    o, oo, c, co, _ = datagen.workload_fig4()
    n = oo.size - 1
    log("fig4 workload generated")
    dist = np.zeros(n, np.uint32)

    def ed(lo):
        for i in range(lo, min(lo + 2000, n)):
            dist[i] = oracle.edit_distance(o[oo[i]:oo[i + 1]], c[co[i]:co[i + 1]])

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        list(ex.map(ed, range(0, n, 2000)))
    log("fig4: edit distances done (max %d)" % dist.max())
    max_e = int(dist.max())
    ent = dict(dist=fullsize.pairs_digest(dist), max_e=max_e, settings={})
    for pattern, k, w in FIG4:
        counts = np.zeros((n, 4, 2), np.uint32)

        def sm(lo):
            hi = min(lo + 5000, n)
            counts[lo:hi] = oracle.seed_match(o[oo[lo]:oo[hi]], oo[lo:hi + 1] - oo[lo],
                                              c[co[lo]:co[hi]], co[lo:hi + 1] - co[lo],
                                              pattern, k, w)

        with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
            list(ex.map(sm, range(0, n, 5000)))
        acc = {alg: oracle.accepted(dist, counts[:, g, 0], counts[:, g, 1], max_e).tolist()
               for g, alg in enumerate(oracle.FIG4_ALGORITHMS)}
        ent["settings"]["%s/%d/%d" % (pattern, k, w)] = dict(
            counts=fullsize.pairs_digest(counts.reshape(n, 8)), accepted=acc)
        log("fig4 %s k%d w%d done" % (pattern, k, w))
    return ent


def main(which):
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    oracle.lib()
    if "illumina" in which:
        d = datagen.workload_illumina()
        log("illumina workload generated")
        ent, _ = seed_entry(d, "10")
        table["illumina-100Mbp/10"] = ent
        del d
    if "gapped" in which:
        d = datagen.workload_gapped()
        log("gapped workload generated")
        ent, _ = seed_entry(d, "10")
        table["illumina-gapped-100Mbp/10"] = ent
        del d
    if "fig4" in which:
        table["fig4-100k"] = fig4_entry()
    if "uneven" in which or any(x.startswith("lookups") for x in which):
        d = datagen.workload_uneven()
        log("uneven workload generated")
        for pattern in (["10", "110"] if "uneven" in which else []):
            ent, ik = seed_entry(d, pattern)
            table["uneven-1Gbp/" + pattern] = ent
            del ik
        for pattern in LOOKUP_PATTERNS:
            if "lookups" not in which and "lookups" + pattern not in which:
                continue
            # the key array of the 1 Gbp reference under the pattern ('11': no base
            # dropped), queried with the mixed batch's minimizers under the same pattern
            ik, iv = oracle.index_build(d["ref"], d["ref_offsets"], pattern, K, W)
            del iv
            rk, _, _ = oracle.sketch(d["reads"], d["read_offsets"], pattern, K, W)
            log("lookups %s: %d index keys, %d read minimizers" % (pattern, ik.size, rk.size))
            q = fullsize.lookup_queries(rk)
            del rk
            lb, occ = parallel_lookup(ik, q)
            log("lookups %s: %d queries done" % (pattern, q.size))
            table["lookups-1Gbp/" + pattern] = dict(index_keys=int(ik.size),
                                                    lookups=fullsize.lookup_digest(lb, occ))
            del q, lb, occ, ik
        del d
    if "containment" in which:
        d = datagen.workload_containment()
        log("containment workload generated")
        ng = d["ref_offsets"].size - 1
        ik, iv = oracle.index_build(d["ref"], d["ref_offsets"], "10", K, W, val_bits=64)
        log("containment: index %d records" % ik.size)
        counts, sizes = oracle.contain(ik, iv, d["reads"], d["read_offsets"], "10", K, W, ng)
        log("containment: counts done")
        table["containment-1000/10"] = dict(index=fullsize.index_digest(ik, iv),
                                            counts=counts.tolist(), sizes=sizes.tolist())
        del d, ik, iv
    with open(OUT, "w") as f:
        json.dump(table, f, indent=0, sort_keys=True)
        f.write("\n")
    log("wrote " + OUT)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args[:1] == ["--out"]:
        OUT = args[1]
        args = args[2:]
    main(set(args or ["illumina", "gapped", "fig4", "uneven", "lookups", "containment"]))
