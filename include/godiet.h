/*
 * godiet.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path of
 * Genome-on-Diet's sparsified genomics (Alser, Eudine, Mutlu, arXiv 2211.08157):
 * sparsify sequences with a repeating keep/skip pattern, sketch the patterned sequences
 * into canonical (w,k)-minimizers, build the sorted minimizer index of a reference, and
 * seed reads against it (pattern alignment + compressed seeding) to emit anchors.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers unless marked [host].  Every buffer is owned by the
 *    caller; the library never allocates, frees, copies to the host or synchronises
 *    inside a call.  All work is enqueued on the caller's stream, so a call may be
 *    captured into a HIP graph.
 *  - Scratch memory is the caller's `ws` of at least godiet_workspace_size() bytes for
 *    the same operation and sizes.
 *  - Argument errors (bad pattern, k or w out of range, NULL pointers, workspace too
 *    small, sizes that cannot fit the value encoding) are detected on the host before
 *    anything is enqueued and returned synchronously; nothing is written then.
 *  - Data-dependent problems (an output larger than the caller's capacity, a position
 *    that does not fit 31 bits, a per-sequence shift >= p) are reported through the
 *    device status word `status` (bits GODIET_ST_*), which each call clears first.  The
 *    call still writes the REQUIRED count, so the caller can synchronise, read the status,
 *    resize and call again.  Outputs other than the counts are unspecified then.
 *  - A failed kernel launch returns GODIET_E_HIP.
 *  - Calls that share a workspace must not overlap; otherwise the library keeps no
 *    state and calls on different streams with different workspaces are independent.
 *
 * Sequence layout (the paper's 2-bit encoding of A, C, G, T; Section 3.6.1)
 * -----------------------------------------------------------------------
 *  A batch of n_seq sequences is one 2-bit packed byte array: base i of the batch is
 *  bits [2*(i%4), 2*(i%4)+1] of byte i/4, with A=0, C=1, G=2, T=3.  offsets[n_seq+1]
 *  (uint64, non-decreasing, offsets[0] = 0, offsets[n_seq] = n_bases) delimit the
 *  sequences; they need not be multiples of 4.  The byte array must hold at least
 *  ceil(n_bases / 4) bytes.
 *  Ambiguous bases (N) ride beside the codes in an optional bit mask nmask: bit (i%32)
 *  of 32-bit word i/32 is set iff base i is N (its 2-bit code is then ignored), at
 *  least ceil(n_bases / 32) words.  With nmask NULL the batch holds no N.
 *  godiet_pack_ascii builds both arrays from text.
 *
 * The method (Section 3; Sections 3.1-3.3)
 * -----------------------------------------
 *  pattern P = p characters '0'/'1' (1 <= p <= 256, weight x >= 1 ones).  With shift a,
 *  base j of a sequence is kept iff P[(j - a) mod p] == '1' (the cyclic form of the
 *  paper's {Q[i+a] * P[i mod p]}).  The reference uses a = 0.
 *  k-mer code: 2k bits, first base most significant; canonical code = min(forward,
 *  reverse complement), strand = 1 iff the reverse complement is smaller; a k-mer equal
 *  to its own reverse complement is never a minimizer.  hash = splitmix64 finalizer of
 *  the canonical code.  A k-mer of the patterned sequence is a minimizer iff its hash
 *  equals the minimum over some full window of w consecutive k-mers (all ties kept).
 *  Locations are coordinates in the ORIGINAL sequence of the k-mer's first kept base.
 *  An N among the KEPT bases ends the current run of patterned bases and the next run
 *  starts right after it (Section 3.6.1): no k-mer contains an N and no window spans
 *  one, so every run is sketched as if it were a sequence of its own (its locations
 *  stay those of the original sequence).  An N at a dropped position is dropped with
 *  it and changes nothing.
 */
#ifndef GODIET_H
#define GODIET_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t godiet_status;
#define GODIET_OK            0
#define GODIET_E_INVAL      (-1)  /* bad argument */
#define GODIET_E_RANGE      (-2)  /* sizes do not fit the value encoding */
#define GODIET_E_WORKSPACE  (-3)  /* ws NULL or smaller than godiet_workspace_size() */
#define GODIET_E_HIP        (-4)  /* a HIP launch failed */
#define GODIET_E_UNSUPPORTED (-5) /* valid request the library does not handle */

/* bits of the device status word */
#define GODIET_ST_CAPACITY 1u  /* output larger than capacity; required count written */
#define GODIET_ST_RANGE    2u  /* a position needs more than 31 bits */
#define GODIET_ST_SHIFT    4u  /* a per-sequence shift is >= p */

/* operations for godiet_workspace_size */
#define GODIET_OP_SPARSIFY    1
#define GODIET_OP_SKETCH      2
#define GODIET_OP_INDEX_BUILD 3
#define GODIET_OP_SEED        4
#define GODIET_OP_RMI_TRAIN   5
#define GODIET_OP_CONTAIN     6
#define GODIET_OP_VOTE        7

typedef struct {
    const uint8_t *bases;     /* 2-bit packed bases (layout above) */
    const uint64_t *offsets;  /* n_seq + 1 base offsets */
    uint32_t n_seq;           /* [host] */
    uint64_t n_bases;         /* [host] must equal offsets[n_seq] */
    const uint32_t *nmask;    /* N bit mask (layout above), or NULL: no N in the batch */
} godiet_seqs;

typedef struct {
    const char *pattern;      /* [host] NUL-terminated '0'/'1' string, 1..256 chars, >= one '1' */
    int32_t k;                /* 1..32 */
    int32_t w;                /* 1..256 */
    int32_t hash;             /* k-mer hash: 0 = splitmix64 finalizer (default); 1 = Thomas
                                 Wang's 64-bit integer hash with every step masked to 2k bits
                                 (the paper's hash, Section 3.6.1, in minimap2's form).  An
                                 index and the reads seeded against it must use the same. */
} godiet_sketch_params;

/* A sorted seed index as produced by godiet_index_build.  val_bits 32: vals is uint32
 * global position << 1 | strand; val_bits 64: vals is uint64 sequence id << 32 |
 * position << 1 | strand.  rmi: NULL for binary-search lookups, else a learned index
 * trained on exactly these keys by godiet_rmi_train (rmi_bytes its size, at least
 * godiet_rmi_size(1), else calls return GODIET_E_INVAL).  The lookup kernels read the
 * model only after checking that its header names this key count and that its leaves lie
 * inside rmi_bytes; any other model is ignored (binary search), and a model's content
 * never changes a result (every window is checked against the keys).  table/table_bytes:
 * see godiet_table_build. */
typedef struct {
    const uint64_t *keys;
    const void *vals;
    uint64_t n;               /* [host] number of records (< 2^32) */
    int32_t val_bits;
    const void *rmi;
    size_t rmi_bytes;         /* [host] */
    const void *table;        /* NULL, or the hash-table form built by godiet_table_build on
                                 exactly these keys; used by seeding and containment lookups */
    size_t table_bytes;       /* [host] */
} godiet_index;

typedef struct {
    int32_t shift_mode;       /* -1: pattern alignment (Section 3.2); 0..p-1: fixed shift */
    uint32_t align_t;         /* 0: no limit; else at most t minimizers scored per shift */
    uint32_t max_occ;         /* 0: off; else minimizers with >= max_occ index hits are
                                 skipped in alignment scores and in seeding */
    /* launch tuning, 0 = library default; these never change any result */
    uint32_t long_records;    /* reads with more minimizer records (summed over the sketched
                                 shifts) than this get a wave each instead of a thread */
    uint32_t lookup_blocks;   /* workgroups of each lookup launch */
    uint32_t long_blocks;     /* workgroups of the long-read alignment/expansion launches */
    /* NULL, or an event the caller records after building the index on another stream:
       the call enqueues the read sketches of every shift first (they need no index),
       then makes `stream` wait on this event before the first index lookup, so index
       construction and read sketching overlap.  The caller keeps the index alive and
       unmodified until this call's work has finished. */
    hipEvent_t index_ready;
} godiet_seed_opts;

typedef struct {
    uint32_t read_id, qpos, rpos, strand;   /* 16 bytes */
} godiet_anchor;

/* Location voting parameters (Section 3.4): D, V and the cap on the winning list. */
typedef struct {
    uint32_t max_dist;        /* D: votes of L0 are the locations in [L0, L0 + D] */
    uint32_t min_votes;       /* V: a location wins with >= V votes */
    uint32_t max_winners;     /* 1..16: winners kept per read */
    uint32_t sort;            /* how each read's adjusted locations are sorted before the
                                 sweep (Section 3.6.2); every choice gives the same winners:
                                 0 adaptive (default): a register sorting network for
                                   reads with at most 16 locations, one workgroup per longer
                                   read;
                                 1 one digit (radix-style) sort of the whole batch;
                                 2 per read, a natural merge sort merging the ascending runs
                                   that the anchors already form (the index keeps every
                                   minimizer's locations sorted);
                                 3 per read, heapsort */
} godiet_vote_opts;

/* One winning (or rescue) mapping location, 24 bytes.  loc is the adjusted location:
 * rpos - qpos for strand 0 (may be negative), rpos + qpos for strand 1. */
typedef struct {
    int64_t loc;
    uint32_t read_id, strand, votes;
    uint32_t flags;           /* GODIET_VOTE_RESCUE: below V, the read's best candidate */
} godiet_winner;
#define GODIET_VOTE_RESCUE 1u

/* Human-readable text of a status code. */
const char *godiet_status_string(godiet_status s);

/* [host] Bytes of scratch an operation needs for these sizes.  `seqs` is the batch the
 * operation sketches (reference for INDEX_BUILD, reads for SEED/CONTAIN); only its host
 * fields are read.  n_index is the index size for SEED/CONTAIN/RMI_TRAIN, the output
 * capacity for SKETCH/INDEX_BUILD.  Returns 0 on invalid arguments. */
size_t godiet_workspace_size(int32_t op, const godiet_seqs *seqs,
                             const godiet_sketch_params *prm, uint64_t n_index);

/* [host] Upper bound on the number of kept bases of the batch under any shift
 * (floor(n_bases / p) * x + n_seq * x, capped at n_bases).  Returns UINT64_MAX on a bad
 * pattern. */
uint64_t godiet_kept_bound(const godiet_seqs *seqs, const char *pattern);

/* [host] Upper bound on the number of minimizer records a sketch of the batch can emit
 * (Section 3.1 step 3: every minimizer is a k-mer of a patterned sequence): the sum over
 * sequences s of max(0, K_s - k + 1), where K_s is the largest kept count of sequence s
 * under any shift (so the bound holds for the reference at shift 0 and for reads at every
 * shift of pattern alignment).  Unlike every other call, this one reads seqs->offsets on
 * the HOST: pass a godiet_seqs whose offsets array (n_seq + 1 entries) is host memory;
 * bases and nmask are not read (ambiguous bases only remove k-mers).  Returns UINT64_MAX
 * on invalid arguments (bad pattern or k, NULL offsets, decreasing offsets). */
uint64_t godiet_sketch_bound(const godiet_seqs *seqs, const godiet_sketch_params *prm);

/* [host] Bytes godiet_sparsify writes to out_bases (a multiple of 4, including zero
 * padding), or 0 on a bad pattern. */
size_t godiet_sparsify_bytes(const godiet_seqs *seqs, const char *pattern);

/* Sparsification (Section 3.1 steps 1-2; Section 3, definition of PR and PQ):
 * keep base j of sequence s iff P[(j - a_s) mod p] == '1', a_s = shift[s] (shift NULL:
 * all 0).  out_bases receives the kept bases of all sequences back to back in the same
 * 2-bit layout, zero-padded to godiet_sparsify_bytes(); out_offsets[n_seq+1] their
 * boundaries.  out_nmask (may be NULL; ignored when in->nmask is NULL) receives the N
 * mask of the kept bases in the layout above, godiet_sparsify_bytes() / 2 bytes. */
godiet_status godiet_sparsify(const godiet_seqs *in, const char *pattern, const uint32_t *shift,
                              uint8_t *out_bases, uint64_t *out_offsets, uint32_t *out_nmask,
                              void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream);

/* [host] Bytes godiet_pack_ascii writes to bases (16 per 64 characters, rounded up);
 * the N mask takes half as many. */
size_t godiet_pack_bytes(uint64_t n_chars);

/* Text to the batch layout (Section 3.6.1: 2-bit codes, with N kept aside): character i
 * of `text` (n_chars bytes, device) becomes base i; A/a = 0, C/c = 1, G/g = 2, T/t and
 * U/u = 3; every other byte is the ambiguous base N (code 0 with its nmask bit set).
 * Writes godiet_pack_bytes(n_chars) bytes to bases and half of that to nmask, padding
 * with zero codes and clear bits.  Offsets are the caller's: the text of the batch's
 * sequences back to back, without separators. */
godiet_status godiet_pack_ascii(const char *text, uint64_t n_chars, uint8_t *bases,
                                uint32_t *nmask, hipStream_t stream);

/* Minimizer sketch (Section 3.1 step 3, canonical (w,k)-minimizers of both strands;
 * Section 3.6.1):
 * the minimizers of every sequence, sparsified with its shift (NULL: 0), as records
 * keys[i] = hash, vals[i] = position << 1 | strand (position in that sequence's own
 * original coordinates), in ascending sequence then position order.
 * mz_offsets[n_seq+1] delimit each sequence's records.  At most `capacity` records are
 * written; mz_offsets[n_seq] is the required count either way. */
godiet_status godiet_sketch(const godiet_seqs *in, const godiet_sketch_params *prm,
                            const uint32_t *shift, uint64_t *keys, uint32_t *vals,
                            uint64_t *mz_offsets, uint64_t capacity,
                            void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream);

/* [host] Scratch bytes godiet_sketch_static can use (64 MiB): the largest
 * godiet_workspace_size(GODIET_OP_SKETCH, ...) it accepts. */
size_t godiet_sketch_static_max_bytes(void);

/* godiet_sketch without a workspace, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments and results as godiet_sketch minus ws / ws_bytes.  Its scratch is a
 * library-owned device array of godiet_sketch_static_max_bytes() bytes, one per GPU,
 * located on the first call on each device and kept until the process ends; the call
 * allocates and frees nothing.  A batch whose sketch workspace would exceed that size
 * returns GODIET_E_WORKSPACE before anything is enqueued (use godiet_sketch then).  Every
 * call on one GPU shares that GPU's array, so calls that overlap on one GPU (concurrent
 * streams, or host threads) race and give undefined results; serialise them. */
godiet_status godiet_sketch_static(const godiet_seqs *in, const godiet_sketch_params *prm,
                                   const uint32_t *shift, uint64_t *keys, uint32_t *vals,
                                   uint64_t *mz_offsets, uint64_t capacity, uint32_t *status,
                                   hipStream_t stream);

/* Compressed indexing (Section 3.1): minimizers of the sparsified reference (shift 0),
 * appended and sorted ascending by (hash, val) into keys[] / vals[].  val_bits 32: vals is
 * uint32 (global position in the batch) << 1 | strand, needs n_bases < 2^31; val_bits
 * 64: vals is uint64 sequence id << 32 | position << 1 | strand.  *n_out (device)
 * receives the number of records; at most `capacity` are written. */
godiet_status godiet_index_build(const godiet_seqs *ref, const godiet_sketch_params *prm,
                                 uint64_t *keys, void *vals, int32_t val_bits,
                                 uint64_t capacity, uint64_t *n_out,
                                 void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream);

/* Pattern alignment (Section 3.2) and compressed seeding (Section 3.3) of a read batch
 * against a 32-bit-val index.  For each read r: with shift_mode -1, every shift s in
 * [0, p) is sketched; the first n* = min_s |M_s| minimizers of each shift (n* capped at
 * align_t when align_t > 0) are scored by their summed index occurrences (skipping those
 * with >= max_occ when max_occ > 0); a_r = the smallest shift of maximal score (0 when
 * every score is 0 or p == 1).  Then, for every minimizer of shift a_r in ascending read
 * position (skipping >= max_occ when set) and every index entry e with the same hash in
 * index order, one anchor {r, qpos, vals[e] >> 1, (qval ^ vals[e]) & 1} is written.
 * Anchors are therefore sorted by (read_id, qpos, rpos).  read_anchor_off[n_reads+1]
 * delimits each read's anchors (its last entry is the required count); shift_out
 * (nullable) receives a_r.  At most `capacity` anchors are written. */
godiet_status godiet_seed(const godiet_index *index, const godiet_seqs *reads,
                          const godiet_sketch_params *prm, const godiet_seed_opts *opts,
                          godiet_anchor *anchors, uint64_t capacity, uint64_t *read_anchor_off,
                          uint8_t *shift_out, void *ws, size_t ws_bytes, uint32_t *status,
                          hipStream_t stream);

/* Containment-style search (Section 2.3, the k-mer-set intersection behind containment
 * search; the paper then thresholds these counts): index is a multi-genome index built
 * with val_bits 64 (genome id = val >> 32).  H_sample = distinct hashes of every read's
 * minimizers at its aligned shift (alignment exactly as in godiet_seed, opts included);
 * for genome g, H_g = distinct hashes among its index records.  counts[g] =
 * |H_sample intersect H_g| and genome_sizes[g] = |H_g| for g < n_genomes (device arrays,
 * overwritten).  Records whose genome id is >= n_genomes are skipped and raise
 * GODIET_ST_RANGE.  ws: godiet_workspace_size(GODIET_OP_CONTAIN, reads, prm, index->n). */
godiet_status godiet_contain(const godiet_index *index, const godiet_seqs *reads,
                             const godiet_sketch_params *prm, const godiet_seed_opts *opts,
                             uint32_t n_genomes, uint32_t *counts, uint32_t *genome_sizes,
                             void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream);

/* Location voting (Section 3.4 steps 1-4, the short-read form, with the rescue location
 * of Section 3.6.3) over the anchors of godiet_seed: for each read r, its anchors
 * [read_anchor_off[r], read_anchor_off[r+1]) (all with read_id r) get the adjusted
 * location rpos - qpos (strand 0) or rpos + qpos (strand 1) and are sorted by (strand,
 * location).  The first entry is the temporary location L0; its votes are the entries of
 * its strand in [L0, L0 + D]; it wins with >= V votes; the first entry beyond L0 + D
 * becomes the next L0.  out[r * max_winners + i], i < n_win[r], receives the winners by
 * votes descending, then strand and location ascending, at most max_winners of them;
 * with no winner it receives the candidate with the most votes (the first such),
 * flagged GODIET_VOTE_RESCUE; a read without anchors gets n_win[r] = 0.
 * anchor_capacity [host] bounds read_anchor_off[n_reads] (GODIET_ST_CAPACITY if
 * exceeded); anchors not grouped by read raise GODIET_ST_RANGE.  Needs n_reads < 2^31
 * and positions < 2^31.  ws: godiet_workspace_size(GODIET_OP_VOTE, reads, NULL,
 * anchor_capacity), where only reads->n_seq (= n_reads) is read.  Device arrays:
 * anchors, read_anchor_off, out (n_reads * max_winners), n_win (n_reads). */
godiet_status godiet_vote(const godiet_anchor *anchors, const uint64_t *read_anchor_off,
                          uint32_t n_reads, uint64_t anchor_capacity,
                          const godiet_vote_opts *opts, godiet_winner *out, uint32_t *n_win,
                          void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream);

/* Exact-match lookups in a sorted index (Section 3.3: each read minimizer is matched
 * exactly against the seed index): for every query q[i], lb[i] = first index e with
 * keys[e] >= q[i] and occ[i] = number of e with keys[e] == q[i].  Uses index->rmi when it
 * is non-NULL, plain binary search otherwise; the results are identical either way.
 * q, lb, occ: device arrays of n_q entries.  Needs index->n < 2^32. */
godiet_status godiet_lookup(const godiet_index *index, const uint64_t *q, uint64_t n_q,
                            uint32_t *lb, uint32_t *occ, hipStream_t stream);

/* Hash-table form of the seed index (Section 3.1: every distinct minimizer hash maps to
 * its sorted location list; here the list is the run [start, start + count) of the sorted
 * keys/vals).  Open addressing with linear probing: a 64-byte header, then 2^b slots of
 * 16 bytes {uint64 key, uint32 start, uint32 count}, 2^b the smallest power of two >=
 * 2 * index->n (load factor <= 1/2), home slot = the key's low b bits, count 0 = empty.
 * godiet_table_size(n) is the byte size (0 if n >= 2^32); godiet_table_build writes the
 * whole buffer (16-byte aligned, table_bytes >= that size) from index->keys.  godiet_seed
 * and godiet_contain then look read minimizers up in it when index->table is set, with
 * results identical to binary search; godiet_lookup ignores it (a table has no lower
 * bound for an absent key).  table_bytes below godiet_table_size(index->n) returns
 * GODIET_E_INVAL.  The header records the key count and a fingerprint of the keys (their
 * count and eight keys spread over them); the lookup kernels use the table only when
 * both match index->keys and its slots lie inside table_bytes, and take a slot's run only
 * when it lies inside the keys; otherwise they search the sorted keys. */
size_t godiet_table_size(uint64_t n_index);
godiet_status godiet_table_build(const godiet_index *index, void *table, size_t table_bytes,
                                 hipStream_t stream);

/* Learned index (not part of the paper; its counterpart there is the hash table of
 * Section 3.1): a two-stage recursive model index over index->keys.  The root (root_kind
 * 0: linear, 1: 1->32->1 ReLU network with knots at key quantiles) routes the FP32 image
 * of a key to one of 2^log2_leaves linear leaves, each predicting the key's rank from its
 * integer offset to the leaf's first key and storing its largest under/over-prediction.
 * Training makes the network's FP32 evaluation non-decreasing in the key (its segments
 * are made to agree in order at every knot), so routing is monotone; should that fail,
 * the model is built with the linear root instead and its header's root kind says 0.
 * A lookup searches only the predicted window after checking that it brackets the
 * answer, and falls back to binary search otherwise, so results equal binary search.
 * rmi: device buffer of godiet_rmi_size(log2_leaves) bytes, 64-byte aligned, written
 * entirely by this call (no workspace needed); log2_leaves in 1..24. */
size_t godiet_rmi_size(uint32_t log2_leaves);
godiet_status godiet_rmi_train(const godiet_index *index, int32_t root_kind, uint32_t log2_leaves,
                               void *rmi, size_t rmi_bytes, hipStream_t stream);

/* Learned-index diagnostics (a measurement aid; lookups never need it): for each of the
 * n_q queries q (device uint64), whether the model's key window brackets it or the lookup
 * falls back to binary search, and how many keys the window spans with its two brackets.
 * stats (device, GODIET_RMI_STAT_WORDS uint64 words, overwritten): [0] queries, [1]
 * fallbacks (the model unusable for this index, or a window that does not bracket the
 * query), [2 + b] windows of w keys with 2^(b-1) < w <= 2^b for b = 0..16, and [19]
 * windows of more than 2^16 keys.  index->rmi must be set. */
#define GODIET_RMI_STAT_WORDS 20
godiet_status godiet_rmi_stats(const godiet_index *index, const uint64_t *q, uint64_t n_q,
                               uint64_t *stats, hipStream_t stream);

/* Random-gather probe, a measurement aid outside the method: the rate at which the GPU
 * serves independent random 8-byte loads sets the roofline of the lookups (each lookup is
 * a short chain of such loads).  out[i] = src[idx[i]] for i < n_idx (device arrays; every
 * idx[i] < n_src is checked in the kernel and an out-of-range index writes 0 and sets
 * GODIET_ST_RANGE in the device status word, which the call clears first).  Each lane
 * keeps four independent loads in flight. */
godiet_status godiet_random_gather(const uint64_t *src, uint64_t n_src, const uint64_t *idx,
                                   uint64_t n_idx, uint64_t *out, uint32_t *status,
                                   hipStream_t stream);

/* Kernel tracing, a profiling aid outside the method.  While enabled, every kernel launch
 * of the library is bracketed by HIP events recorded on the launch's stream.  After the
 * caller has synchronised, godiet_trace_dump writes one line "kernel launches total_ms"
 * per kernel into buf (truncated to len bytes, NUL-terminated) and forgets the records;
 * with buf NULL or len 0 it only measures.  Returns the bytes the full text needs
 * including the NUL. */
void godiet_trace_enable(int on);
size_t godiet_trace_dump(char *buf, size_t len);
/* Restricts tracing to kernels whose name (as reported by godiet_trace_dump) begins with
 * prefix; NULL or "" traces every kernel again.  The string is copied. */
void godiet_trace_filter(const char *prefix);

/* ---- Seed-matching experiment (Section 2.1.1, Fig. 4; Section 2.1.2) ----------------
 * Pairs: sequence i of `orig` and sequence i of `copy` (a copy with substitutions), each
 * at most 1,024 bases, no N mask.  Four seeding algorithms, in this order:
 *   0 all seeds: every k-mer;  1 minimizers: (w,k)-minimizers (pattern '1');
 *   2 spaced seeds: at every start i the bases i + j with M[j] == '1', M = the pattern
 *     repeated to span k (a pattern of length k as it is);
 *   3 Genome-on-Diet: (w,k)-minimizers of the patterned sequence (shift 0).
 * A seed is identified by the canonical code of its bases (a string and its reverse
 * complement are one seed); minimizer seeds by their hash (prm->hash), a bijection of
 * that code.  The matching rate of a pair is (seeds of the copy, with multiplicity,
 * present among the original's seeds) / (seeds of the copy). */
#define GODIET_FIG4_ALGORITHMS 4

/* counts[8i + 2g] = matched seeds of the copy, counts[8i + 2g + 1] = seeds of the copy,
 * for pair i and algorithm g.  n_seq of both batches must be equal.  A pair longer than
 * 1,024 bases gets zeros and sets GODIET_ST_RANGE. */
godiet_status godiet_seed_match(const godiet_seqs *orig, const godiet_seqs *copy,
                                const godiet_sketch_params *prm, uint32_t *counts,
                                uint32_t *status, hipStream_t stream);

/* Levenshtein distance (unit-cost substitution, insertion, deletion) of every pair into
 * dist[i]; the original may have at most 1,024 bases (else 0 and GODIET_ST_RANGE). */
godiet_status godiet_edit_distance(const godiet_seqs *orig, const godiet_seqs *copy,
                                   uint32_t *dist, uint32_t *status, hipStream_t stream);

/* [host] Workspace bytes of godiet_accepted_pairs for thresholds 0..max_e. */
size_t godiet_accepted_ws_size(uint32_t max_e);

/* Accepted sequence pairs (Section 2.1.2) for algorithm g: for every edit-distance
 * threshold E in [0, max_e], the rate threshold is the smallest matching rate among the
 * pairs with dist <= E, and accepted[E] is the number of pairs whose rate reaches it (0
 * when no pair has dist <= E).  dist and counts as written by the two calls above;
 * rates are compared exactly (totals stay below 2^16). */
godiet_status godiet_accepted_pairs(const uint32_t *dist, const uint32_t *counts, uint32_t n_pairs,
                                    int32_t g, uint32_t max_e, uint32_t *accepted, void *ws,
                                    size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GODIET_H */
