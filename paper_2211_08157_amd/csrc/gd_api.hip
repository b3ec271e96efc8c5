// C ABI entry points: host-side validation, workspace layout and kernel sequencing.
#include <string.h>

#include <atomic>
#include <mutex>

#include "../../include/godiet.h"
#include "gd_internal.h"

using namespace gd;

namespace {

bool parse_pattern(const char *s, Pattern *P)
{
    if (!s) return false;
    const size_t n = strnlen(s, kMaxPattern + 1);
    if (n < 1 || n > kMaxPattern) return false;
    memset(P, 0, sizeof(*P));
    P->p = (uint32_t)n;
    for (size_t i = 0; i < n; i++) {
        if (s[i] == '1') {
            if (i < 64) P->mask |= 1ull << i;
            else P->hi[(i - 64) >> 6] |= 1ull << ((i - 64) & 63);
            P->ones[P->x++] = (uint8_t)i;
        } else if (s[i] != '0') {
            return false;
        }
    }
    return P->x >= 1;
}

bool valid_seqs(const godiet_seqs *q)
{
    if (!q || !q->offsets) return false;
    if (q->n_bases > 0 && !q->bases) return false;
    return q->n_bases < (1ull << 48);
}

bool valid_params(const godiet_sketch_params *prm, Pattern *P)
{
    if (!prm || !parse_pattern(prm->pattern, P)) return false;
    return prm->k >= 1 && prm->k <= 32 && prm->w >= 1 && prm->w <= 256 &&
           (prm->hash == 0 || prm->hash == 1);
}

uint64_t kept_bound(const godiet_seqs *q, const Pattern &P)
{
    const uint64_t b = (q->n_bases / P.p) * P.x + (uint64_t)q->n_seq * P.x;
    return b < q->n_bases ? b : q->n_bases;
}

// An index's learned-index model must hold at least its header and smallest leaf table,
// its hash table the size built for its key count (the kernels check the rest).
bool models_fit(const godiet_index *ix)
{
    if (ix->rmi && ix->rmi_bytes < rmi_bytes(1)) return false;
    if (ix->table && ix->table_bytes < table_bytes(ix->n)) return false;
    return true;
}

Batch batch_of(const godiet_seqs *q)
{
    return Batch{q->bases, q->offsets, q->n_seq, q->n_bases, q->nmask};
}

#define GD_TRY(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return GODIET_E_HIP; \
    } while (0)

// ---- workspace plans: the same code measures (ws == nullptr) and carves ----

struct SketchWs {
    uint64_t *kept, *scan, *pofs;
    uint32_t *psw;
    uint32_t *pnw;        // N bits of the patterned stream (null without an N mask)
    uint64_t *tiles;      // tile states + the tile ticket counter
    uint32_t *lohi;       // sequence ranges of the sparsify workgroups
    uint32_t *lohi_sk;    // sequence ranges of the sketch tiles
};

void plan_sketch_ws(Bump &b, const godiet_seqs *q, uint64_t npb, int w, SketchWs *o)
{
    const uint32_t n_seq = q->n_seq;
    o->kept = b.take<uint64_t>((size_t)n_seq + 1);
    o->scan = b.take<uint64_t>(scan_scratch((size_t)n_seq + 1));
    o->pofs = b.take<uint64_t>((size_t)n_seq + 1);
    o->psw = b.take<uint32_t>(psw_words(npb));
    o->pnw = q->nmask ? b.take<uint32_t>(pnw_words(npb)) : nullptr;
    o->tiles = b.take<uint64_t>(sketch_tiles_bound(npb, w) + 1);
    o->lohi = b.take<uint32_t>(sparsify_lohi(psw_words(npb)));
    o->lohi_sk = b.take<uint32_t>(2 * sketch_tiles_bound(npb, w));
}

// kept counts -> pofs -> sequence ranges (sparsify and sketch of window w) -> patterned
// stream, for a per-sequence or uniform shift
hipError_t sparsify_to_stream(const godiet_seqs *in, const Pattern &P, const uint32_t *shift,
                              uint32_t uniform, const SketchWs &W, uint64_t npb, int w,
                              uint32_t *status, hipStream_t s)
{
    const Batch bt = batch_of(in);
    hipError_t e = launch_kept(bt, P, shift, uniform, W.kept, status, s);
    if (e != hipSuccess) return e;
    e = exclusive_scan_u64(W.kept, W.pofs, in->n_seq, W.scan, s);
    if (e != hipSuccess) return e;
    if (in->n_seq > 0) {
        e = launch_window_ranges(W.pofs, in->n_seq, psw_words(npb), npb, w, W.lohi, W.lohi_sk, s);
        if (e != hipSuccess) return e;
    }
    return launch_sparsify(bt, P, shift, uniform, W.pofs, W.psw, W.pnw, psw_words(npb), W.lohi,
                           in->n_seq > 0, s);
}

struct IndexWs {
    SketchWs sk;
    SortWs so;
    SortPlan sp;
};

void plan_index_ws(Bump &b, const godiet_seqs *ref, const Pattern &P, int w, uint64_t capacity,
                   int val_bytes, IndexWs *o)
{
    const uint64_t npb = kept_bound(ref, P);
    plan_sketch_ws(b, ref, npb, w, &o->sk);
    uint64_t expected = npb * 2 / (uint64_t)(w + 1) + 1;
    if (expected > capacity) expected = capacity;
    o->sp = sort_plan(expected, capacity, val_bytes);
    o->so.hist = b.take<uint32_t>(o->sp.digits ? o->sp.nchunks * o->sp.nfine : o->sp.nfine);
    o->so.tot = o->sp.digits ? b.take<uint32_t>(o->sp.nfine) : nullptr;
    o->so.top = o->sp.digits ? b.take<uint32_t>(sort_top_bins()) : nullptr;
    o->so.cdf = o->sp.digits ? b.take<uint64_t>(sort_top_bins() + 1) : nullptr;
    o->so.fofs = b.take<uint64_t>(o->sp.nfine + 1);
    o->so.rank = o->sp.digits ? nullptr : b.take<uint32_t>(capacity);
    o->so.scan_tmp = b.take<uint64_t>(scan_scratch(o->sp.nfine > sort_top_bins() ? o->sp.nfine
                                                                                 : sort_top_bins()));
    o->so.trec = b.take<ulonglong2>(capacity);
    o->so.tmp = o->sp.two_level ? b.take<ulonglong2>(capacity) : nullptr;
    o->so.cmat = o->sp.two_level ? b.take<uint32_t>(o->sp.nchunks * 256) : nullptr;
    o->so.cstart = b.take<uint32_t>(o->sp.ncoarse + 1);
    o->so.overflow = b.take<uint32_t>(o->sp.ncoarse);
    o->so.blist = b.take<uint32_t>(o->sp.ncoarse);
    o->so.overflow_n = b.take<uint32_t>(2);
}

struct VoteWs {
    uint64_t *keys;
    uint32_t *vals;
    uint32_t *long_ids, *long_n;
    SortWs so;
    SortPlan sp;
};

void plan_vote_ws(Bump &b, uint32_t n_reads, uint64_t capacity, VoteWs *o)
{
    o->keys = b.take<uint64_t>(capacity);
    o->vals = b.take<uint32_t>(capacity);
    o->long_ids = b.take<uint32_t>(n_reads);
    o->long_n = b.take<uint32_t>(1);
    o->sp = sort_plan(capacity, capacity > 0 ? capacity : 1, 4);
    o->so.hist = b.take<uint32_t>(o->sp.digits ? o->sp.nchunks * o->sp.nfine : o->sp.nfine);
    o->so.tot = o->sp.digits ? b.take<uint32_t>(o->sp.nfine) : nullptr;
    o->so.top = o->sp.digits ? b.take<uint32_t>(sort_top_bins()) : nullptr;
    o->so.cdf = o->sp.digits ? b.take<uint64_t>(sort_top_bins() + 1) : nullptr;
    o->so.fofs = b.take<uint64_t>(o->sp.nfine + 1);
    o->so.rank = o->sp.digits ? nullptr : b.take<uint32_t>(capacity);
    o->so.scan_tmp = b.take<uint64_t>(scan_scratch(o->sp.nfine > sort_top_bins() ? o->sp.nfine
                                                                                 : sort_top_bins()));
    o->so.trec = b.take<ulonglong2>(capacity);
    o->so.tmp = o->sp.two_level ? b.take<ulonglong2>(capacity) : nullptr;
    o->so.cmat = o->sp.two_level ? b.take<uint32_t>(o->sp.nchunks * 256) : nullptr;
    o->so.cstart = b.take<uint32_t>(o->sp.ncoarse + 1);
    o->so.overflow = b.take<uint32_t>(o->sp.ncoarse);
    o->so.blist = b.take<uint32_t>(o->sp.ncoarse);
    o->so.overflow_n = b.take<uint32_t>(2);
}

struct SeedWs {
    SketchWs sk;
    uint64_t *mzofs;      // n_shift * (n_reads + 1)
    uint64_t *qkeys;      // n_shift * stride
    uint32_t *qvals, *lb, *occ;
    uint32_t *slot, *cnt;
    uint32_t *long_ids, *long_n;
    uint64_t *scan;
    size_t stride;
};

void plan_seed_ws(Bump &b, const godiet_seqs *reads, const Pattern &P, int w, uint32_t n_shift,
                  SeedWs *o)
{
    const uint64_t npb = kept_bound(reads, P);
    plan_sketch_ws(b, reads, npb, w, &o->sk);
    o->stride = (size_t)npb + 1;
    const size_t nr = (size_t)reads->n_seq;
    o->mzofs = b.take<uint64_t>((nr + 1) * n_shift);
    o->qkeys = b.take<uint64_t>(o->stride * n_shift);
    o->qvals = b.take<uint32_t>(o->stride * n_shift);
    o->lb = b.take<uint32_t>(o->stride * n_shift);
    o->occ = b.take<uint32_t>(o->stride * n_shift);
    o->slot = b.take<uint32_t>(nr + 1);
    o->cnt = b.take<uint32_t>(nr + 1);
    o->long_ids = b.take<uint32_t>(nr + 1);     // long reads from the front, huge from the back
    o->long_n = b.take<uint32_t>(2);            // counts of both lists
    o->scan = b.take<uint64_t>(scan_scratch(nr + 1));
}

// Pattern alignment front end shared by seeding and containment: every shift (or the
// fixed one) is sparsified, sketched and looked up, then each read's shift is chosen.
// With mark non-null the workspace also carries an index-sized byte array for it.
godiet_status seed_front(const godiet_index *index, const godiet_seqs *reads, const Pattern &P,
                         const godiet_sketch_params *prm, const godiet_seed_opts *opts, void *ws,
                         size_t ws_bytes, uint8_t *shift_out, uint32_t *status, hipStream_t stream,
                         SeedWs *Wp, AlignArgs *Ap, uint8_t **mark)
{
    if (index->n > 0 && (!index->keys || !index->vals)) return GODIET_E_INVAL;
    if (index->n >= (1ull << 32)) return GODIET_E_RANGE;
    if (!models_fit(index)) return GODIET_E_INVAL;
    if (opts->shift_mode < -1 || opts->shift_mode >= (int32_t)P.p) return GODIET_E_INVAL;
    const uint64_t npb = kept_bound(reads, P);
    const uint32_t n_shift = opts->shift_mode >= 0 ? 1u : P.p;
    Bump b(ws);
    SeedWs &W = *Wp;
    plan_seed_ws(b, reads, P, prm->w, n_shift, &W);
    if (mark) *mark = b.take<uint8_t>((index->n + 3) / 4 * 4);
    if (!ws || ws_bytes < b.off) return GODIET_E_WORKSPACE;
    const size_t nr = reads->n_seq;
    GD_TRY(fill_u32(status, 0, 1, stream));
    // every shift's sketch first (they need no index), then the lookups, so that an index
    // built on another stream can overlap the sketches
    for (uint32_t si = 0; si < n_shift; si++) {
        const uint32_t a = opts->shift_mode >= 0 ? (uint32_t)opts->shift_mode : si;
        GD_TRY(sparsify_to_stream(reads, P, nullptr, a, W.sk, npb, prm->w, status, stream));
        uint64_t *mz = W.mzofs + si * (nr + 1);
        uint64_t *qk = W.qkeys + si * W.stride;
        uint32_t *qv = W.qvals + si * W.stride;
        SketchOut o{qk, qv, VAL_LOCAL32, mz, (uint64_t)W.stride, nullptr};
        GD_TRY(launch_sketch(batch_of(reads), P, nullptr, a, W.sk.pofs, W.sk.psw, W.sk.pnw, npb,
                             prm->k, prm->w, prm->hash, o, W.sk.tiles, W.sk.lohi_sk,
                             reads->n_seq > 0, status, stream));
    }
    if (opts->index_ready) GD_TRY(hipStreamWaitEvent(stream, opts->index_ready, 0));
    for (uint32_t si = 0; si < n_shift; si++) {
        const uint64_t *mz = W.mzofs + si * (nr + 1);
        GD_TRY(launch_lookup(index->keys, index->n, W.qkeys + si * W.stride, mz + nr, W.stride,
                             W.lb + si * W.stride, W.occ + si * W.stride, index->rmi,
                             index->rmi_bytes, index->table, index->table_bytes,
                             opts->lookup_blocks, stream));
    }
    AlignArgs &A = *Ap;
    A.mzofs = W.mzofs;
    A.occ = W.occ;
    A.lb = W.lb;
    A.qval = W.qvals;
    A.stride = W.stride;
    A.n_reads = reads->n_seq;
    A.n_shift = n_shift;
    A.fixed_shift = opts->shift_mode;
    A.align_t = opts->align_t;
    A.max_occ = opts->max_occ;
    A.long_records = opts->long_records ? opts->long_records : 192u;
    A.long_blocks = opts->long_blocks ? opts->long_blocks : 4096u;
    GD_TRY(launch_align(A, shift_out, W.slot, W.cnt, W.long_ids, W.long_n, stream));
    return GODIET_OK;
}

}  // namespace

extern "C" {

const char *godiet_status_string(godiet_status s)
{
    switch (s) {
    case GODIET_OK: return "ok";
    case GODIET_E_INVAL: return "invalid argument";
    case GODIET_E_RANGE: return "sizes do not fit the value encoding";
    case GODIET_E_WORKSPACE: return "workspace missing or too small";
    case GODIET_E_HIP: return "HIP launch failed";
    case GODIET_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

uint64_t godiet_kept_bound(const godiet_seqs *seqs, const char *pattern)
{
    Pattern P;
    if (!seqs || !parse_pattern(pattern, &P)) return UINT64_MAX;
    return kept_bound(seqs, P);
}

uint64_t godiet_sketch_bound(const godiet_seqs *seqs, const godiet_sketch_params *prm)
{
    Pattern P;
    if (!seqs || !seqs->offsets || !prm || !parse_pattern(prm->pattern, &P) || prm->k < 1 ||
        prm->k > 32)
        return UINT64_MAX;
    // most[r]: the largest number of ones among r consecutive characters of the cyclic
    // pattern, i.e. the largest kept count of the first r bases of a period over all shifts
    uint32_t most[kMaxPattern + 1];
    for (uint32_t r = 0; r <= P.p; r++) {
        uint32_t best = 0;
        for (uint32_t a = 0; a < P.p; a++) {
            uint32_t c = 0;
            for (uint32_t t = 0; t < r; t++) c += pattern_bit(P, (a + t) % P.p) ? 1u : 0u;
            best = c > best ? c : best;
        }
        most[r] = best;
    }
    uint64_t total = 0;
    for (uint32_t s = 0; s < seqs->n_seq; s++) {
        if (seqs->offsets[s + 1] < seqs->offsets[s]) return UINT64_MAX;
        const uint64_t L = seqs->offsets[s + 1] - seqs->offsets[s];
        const uint64_t K = (L / P.p) * P.x + most[L % P.p];
        if (K >= (uint64_t)prm->k) total += K - (uint64_t)prm->k + 1;
    }
    return total;
}

size_t godiet_sparsify_bytes(const godiet_seqs *seqs, const char *pattern)
{
    Pattern P;
    if (!seqs || !parse_pattern(pattern, &P)) return 0;
    return psw_words(kept_bound(seqs, P)) * 4;
}

size_t godiet_workspace_size(int32_t op, const godiet_seqs *seqs, const godiet_sketch_params *prm,
                             uint64_t n_index)
{
    Pattern P;
    if (!seqs) return 0;
    Bump b(nullptr);
    switch (op) {
    case GODIET_OP_SPARSIFY: {
        if (!prm || !parse_pattern(prm->pattern, &P)) return 0;
        b.take<uint64_t>((size_t)seqs->n_seq + 1);
        b.take<uint64_t>(scan_scratch((size_t)seqs->n_seq + 1));
        b.take<uint32_t>(sparsify_lohi(psw_words(kept_bound(seqs, P))));
        return b.off;
    }
    case GODIET_OP_SKETCH: {
        if (!valid_params(prm, &P)) return 0;
        SketchWs o;
        plan_sketch_ws(b, seqs, kept_bound(seqs, P), prm->w, &o);
        return b.off;
    }
    case GODIET_OP_INDEX_BUILD: {
        // enough for either value width (the sort's partition depends on it)
        if (!valid_params(prm, &P)) return 0;
        IndexWs o;
        Bump b4(nullptr);
        plan_index_ws(b, seqs, P, prm->w, n_index, 8, &o);
        plan_index_ws(b4, seqs, P, prm->w, n_index, 4, &o);
        return b.off > b4.off ? b.off : b4.off;
    }
    case GODIET_OP_SEED:
    case GODIET_OP_CONTAIN: {
        if (!valid_params(prm, &P)) return 0;
        SeedWs o;
        plan_seed_ws(b, seqs, P, prm->w, P.p, &o);
        if (op == GODIET_OP_CONTAIN) b.take<uint8_t>((n_index + 3) / 4 * 4);
        return b.off;
    }
    case GODIET_OP_VOTE: {
        if (n_index >= (1ull << 32) || seqs->n_seq >= (1u << 31)) return 0;
        VoteWs o;
        plan_vote_ws(b, seqs->n_seq, n_index, &o);
        return b.off;
    }
    default: return 0;
    }
}

godiet_status godiet_sparsify(const godiet_seqs *in, const char *pattern, const uint32_t *shift,
                              uint8_t *out_bases, uint64_t *out_offsets, uint32_t *out_nmask,
                              void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream)
{
    Pattern P;
    if (!valid_seqs(in) || !parse_pattern(pattern, &P) || !out_bases || !out_offsets || !status)
        return GODIET_E_INVAL;
    if (((uintptr_t)out_bases & 3) != 0 || ((uintptr_t)out_nmask & 3) != 0) return GODIET_E_INVAL;
    Bump b(ws);
    uint64_t *kept = b.take<uint64_t>((size_t)in->n_seq + 1);
    uint64_t *scan = b.take<uint64_t>(scan_scratch((size_t)in->n_seq + 1));
    const uint64_t npb = kept_bound(in, P);
    uint32_t *lohi = b.take<uint32_t>(sparsify_lohi(psw_words(npb)));
    if (!ws || ws_bytes < b.off) return GODIET_E_WORKSPACE;
    const Batch bt = batch_of(in);
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(launch_kept(bt, P, shift, 0, kept, status, stream));
    GD_TRY(exclusive_scan_u64(kept, out_offsets, in->n_seq, scan, stream));
    GD_TRY(launch_sparsify(bt, P, shift, 0, out_offsets, (uint32_t *)out_bases, out_nmask,
                           psw_words(npb), lohi, false, stream));
    return GODIET_OK;
}

godiet_status godiet_seed_match(const godiet_seqs *orig, const godiet_seqs *copy,
                                const godiet_sketch_params *prm, uint32_t *counts,
                                uint32_t *status, hipStream_t stream)
{
    Pattern P;
    if (!valid_seqs(orig) || !valid_seqs(copy) || !valid_params(prm, &P) || !status)
        return GODIET_E_INVAL;
    if (orig->n_seq != copy->n_seq || (orig->n_seq > 0 && !counts)) return GODIET_E_INVAL;
    if (orig->nmask || copy->nmask) return GODIET_E_UNSUPPORTED;
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(launch_seed_match(orig, copy, P, prm->k, prm->w, prm->hash, counts, status, stream));
    return GODIET_OK;
}

godiet_status godiet_edit_distance(const godiet_seqs *orig, const godiet_seqs *copy,
                                   uint32_t *dist, uint32_t *status, hipStream_t stream)
{
    if (!valid_seqs(orig) || !valid_seqs(copy) || !status) return GODIET_E_INVAL;
    if (orig->n_seq != copy->n_seq || (orig->n_seq > 0 && !dist)) return GODIET_E_INVAL;
    if (orig->nmask || copy->nmask) return GODIET_E_UNSUPPORTED;
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(launch_edit_distance(orig, copy, dist, status, stream));
    return GODIET_OK;
}

size_t godiet_accepted_ws_size(uint32_t max_e) { return ((size_t)max_e + 1) * 8 + 256; }

godiet_status godiet_accepted_pairs(const uint32_t *dist, const uint32_t *counts, uint32_t n_pairs,
                                    int32_t g, uint32_t max_e, uint32_t *accepted, void *ws,
                                    size_t ws_bytes, hipStream_t stream)
{
    if (g < 0 || g >= GODIET_FIG4_ALGORITHMS || !accepted || max_e >= (1u << 24))
        return GODIET_E_INVAL;
    if (n_pairs > 0 && (!dist || !counts)) return GODIET_E_INVAL;
    if (!ws || ws_bytes < godiet_accepted_ws_size(max_e) || ((uintptr_t)ws & 7) != 0)
        return GODIET_E_WORKSPACE;
    GD_TRY(launch_accepted(dist, counts, n_pairs, g, max_e, (uint64_t *)ws, accepted, stream));
    return GODIET_OK;
}

size_t godiet_pack_bytes(uint64_t n_chars) { return (size_t)((n_chars + 63) / 64) * 16; }

godiet_status godiet_pack_ascii(const char *text, uint64_t n_chars, uint8_t *bases,
                                uint32_t *nmask, hipStream_t stream)
{
    if (n_chars > 0 && (!text || !bases || !nmask)) return GODIET_E_INVAL;
    if (((uintptr_t)bases & 3) != 0 || ((uintptr_t)nmask & 3) != 0) return GODIET_E_INVAL;
    if (n_chars >= (1ull << 48)) return GODIET_E_RANGE;
    GD_TRY(launch_pack_ascii(text, n_chars, (uint32_t *)bases, (uint16_t *)nmask, stream));
    return GODIET_OK;
}

godiet_status godiet_sketch(const godiet_seqs *in, const godiet_sketch_params *prm,
                            const uint32_t *shift, uint64_t *keys, uint32_t *vals,
                            uint64_t *mz_offsets, uint64_t capacity, void *ws, size_t ws_bytes,
                            uint32_t *status, hipStream_t stream)
{
    Pattern P;
    if (!valid_seqs(in) || !valid_params(prm, &P) || !mz_offsets || !status) return GODIET_E_INVAL;
    if (capacity > 0 && (!keys || !vals)) return GODIET_E_INVAL;
    const uint64_t npb = kept_bound(in, P);
    Bump b(ws);
    SketchWs W;
    plan_sketch_ws(b, in, npb, prm->w, &W);
    if (!ws || ws_bytes < b.off) return GODIET_E_WORKSPACE;
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(sparsify_to_stream(in, P, shift, 0, W, npb, prm->w, status, stream));
    SketchOut o{keys, vals, VAL_LOCAL32, mz_offsets, capacity, nullptr};
    GD_TRY(launch_sketch(batch_of(in), P, shift, 0, W.pofs, W.psw, W.pnw, npb, prm->k, prm->w,
                         prm->hash, o, W.tiles, W.lohi_sk, in->n_seq > 0, status, stream));
    return GODIET_OK;
}

}  // extern "C"

namespace {

// Scratch of godiet_sketch_static: one copy per GPU, held until the process ends.  Host
// code never uses the array's name as an address: each device's copy is found once with
// hipGetSymbolAddress (with that device current) and that pointer is passed on.
constexpr size_t kStaticScratch = (size_t)64 << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratch];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// This device's copy of `scratch` (null if the runtime cannot provide it).
void *device_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return nullptr;
        g_scratch[dev].store(q, std::memory_order_release);
        p = q;
    }
    return p;
}

}  // namespace

extern "C" {

size_t godiet_sketch_static_max_bytes(void) { return kStaticScratch; }

godiet_status godiet_sketch_static(const godiet_seqs *in, const godiet_sketch_params *prm,
                                   const uint32_t *shift, uint64_t *keys, uint32_t *vals,
                                   uint64_t *mz_offsets, uint64_t capacity, uint32_t *status,
                                   hipStream_t stream)
{
    Pattern P;
    if (!valid_seqs(in) || !valid_params(prm, &P) || !mz_offsets || !status) return GODIET_E_INVAL;
    if (capacity > 0 && (!keys || !vals)) return GODIET_E_INVAL;
    // the same workspace plan as godiet_sketch, measured before any HIP call
    const uint64_t npb = kept_bound(in, P);
    Bump m(nullptr);
    SketchWs W;
    plan_sketch_ws(m, in, npb, prm->w, &W);
    if (m.off > kStaticScratch) return GODIET_E_WORKSPACE;
    void *ws = device_scratch();
    if (!ws) return GODIET_E_HIP;
    Bump b(ws);
    plan_sketch_ws(b, in, npb, prm->w, &W);
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(sparsify_to_stream(in, P, shift, 0, W, npb, prm->w, status, stream));
    SketchOut o{keys, vals, VAL_LOCAL32, mz_offsets, capacity, nullptr};
    GD_TRY(launch_sketch(batch_of(in), P, shift, 0, W.pofs, W.psw, W.pnw, npb, prm->k, prm->w,
                         prm->hash, o, W.tiles, W.lohi_sk, in->n_seq > 0, status, stream));
    return GODIET_OK;
}

godiet_status godiet_index_build(const godiet_seqs *ref, const godiet_sketch_params *prm,
                                 uint64_t *keys, void *vals, int32_t val_bits, uint64_t capacity,
                                 uint64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status,
                                 hipStream_t stream)
{
    Pattern P;
    if (!valid_seqs(ref) || !valid_params(prm, &P) || !n_out || !status) return GODIET_E_INVAL;
    if (val_bits != 32 && val_bits != 64) return GODIET_E_INVAL;
    if (capacity > 0 && (!keys || !vals)) return GODIET_E_INVAL;
    if (capacity >= (1ull << 32)) return GODIET_E_RANGE;
    if (val_bits == 32 && ref->n_bases >= (1ull << 31)) return GODIET_E_RANGE;
    const uint64_t npb = kept_bound(ref, P);
    const int vb = val_bits / 8;
    Bump b(ws);
    IndexWs W;
    plan_index_ws(b, ref, P, prm->w, capacity, vb, &W);
    if (!ws || ws_bytes < b.off) return GODIET_E_WORKSPACE;
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(sparsify_to_stream(ref, P, nullptr, 0, W.sk, npb, prm->w, status, stream));
    SketchOut o{keys, vals, val_bits == 32 ? VAL_GLOBAL32 : VAL_SEQ64, nullptr, capacity, n_out};
    GD_TRY(launch_sketch(batch_of(ref), P, nullptr, 0, W.sk.pofs, W.sk.psw, W.sk.pnw, npb, prm->k,
                         prm->w, prm->hash, o, W.sk.tiles, W.sk.lohi_sk, ref->n_seq > 0, status,
                         stream));
    if (capacity > 0) GD_TRY(launch_sort(W.sp, W.so, keys, vals, vb, n_out, capacity, stream));
    return GODIET_OK;
}

godiet_status godiet_seed(const godiet_index *index, const godiet_seqs *reads,
                          const godiet_sketch_params *prm, const godiet_seed_opts *opts,
                          godiet_anchor *anchors, uint64_t capacity, uint64_t *read_anchor_off,
                          uint8_t *shift_out, void *ws, size_t ws_bytes, uint32_t *status,
                          hipStream_t stream)
{
    Pattern P;
    if (!index || !valid_seqs(reads) || !valid_params(prm, &P) || !opts || !read_anchor_off ||
        !status)
        return GODIET_E_INVAL;
    if (index->val_bits != 32) return GODIET_E_UNSUPPORTED;
    if (capacity > 0 && !anchors) return GODIET_E_INVAL;
    SeedWs W;
    AlignArgs A;
    godiet_status st = seed_front(index, reads, P, prm, opts, ws, ws_bytes, shift_out, status,
                                  stream, &W, &A, nullptr);
    if (st != GODIET_OK) return st;
    GD_TRY(exclusive_scan_u32(W.cnt, read_anchor_off, reads->n_seq, W.scan, stream));
    GD_TRY(launch_expand(A, W.slot, read_anchor_off, index->vals, (uint32_t *)anchors, capacity,
                         status, W.long_ids, W.long_n, stream));
    return GODIET_OK;
}

godiet_status godiet_contain(const godiet_index *index, const godiet_seqs *reads,
                             const godiet_sketch_params *prm, const godiet_seed_opts *opts,
                             uint32_t n_genomes, uint32_t *counts, uint32_t *genome_sizes,
                             void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream)
{
    Pattern P;
    if (!index || !valid_seqs(reads) || !valid_params(prm, &P) || !opts || !status)
        return GODIET_E_INVAL;
    if (index->val_bits != 64) return GODIET_E_UNSUPPORTED;
    if (n_genomes > 0 && (!counts || !genome_sizes)) return GODIET_E_INVAL;
    SeedWs W;
    AlignArgs A;
    uint8_t *mark = nullptr;
    godiet_status st = seed_front(index, reads, P, prm, opts, ws, ws_bytes, nullptr, status,
                                  stream, &W, &A, &mark);
    if (st != GODIET_OK) return st;
    GD_TRY(launch_contain(A, W.slot, index->keys, (const uint64_t *)index->vals, index->n, mark,
                          n_genomes, counts, genome_sizes, status, stream));
    return GODIET_OK;
}

godiet_status godiet_vote(const godiet_anchor *anchors, const uint64_t *read_anchor_off,
                          uint32_t n_reads, uint64_t anchor_capacity,
                          const godiet_vote_opts *opts, godiet_winner *out, uint32_t *n_win,
                          void *ws, size_t ws_bytes, uint32_t *status, hipStream_t stream)
{
    if (!opts || !status || opts->max_winners < 1 || opts->max_winners > 16 || opts->sort > 3)
        return GODIET_E_INVAL;
    if (n_reads > 0 && (!read_anchor_off || !out || !n_win)) return GODIET_E_INVAL;
    if (anchor_capacity > 0 && !anchors) return GODIET_E_INVAL;
    if (n_reads >= (1u << 31) || anchor_capacity >= (1ull << 32)) return GODIET_E_RANGE;
    Bump b(ws);
    VoteWs W;
    plan_vote_ws(b, n_reads, anchor_capacity, &W);
    if (!ws || ws_bytes < b.off) return GODIET_E_WORKSPACE;
    VoteArgs A;
    A.max_dist = opts->max_dist;
    A.min_votes = opts->min_votes;
    A.max_win = opts->max_winners;
    A.sort = (int)opts->sort;
    int rb = 0;                                   // bits of the largest read id
    while (rb < 31 && ((uint64_t)(n_reads > 0 ? n_reads - 1 : 0) >> rb) != 0) rb++;
    A.lz = 64 - 33 - rb;
    GD_TRY(fill_u32(status, 0, 1, stream));
    GD_TRY(launch_vote(A, (const uint4 *)anchors, read_anchor_off, n_reads, anchor_capacity,
                       W.sp, W.so, W.keys, W.vals, W.long_ids, W.long_n, out, n_win, status,
                       stream));
    return GODIET_OK;
}

size_t godiet_table_size(uint64_t n_index)
{
    if (n_index >= (1ull << 32)) return 0;
    return table_bytes(n_index);
}

godiet_status godiet_table_build(const godiet_index *index, void *table, size_t table_bytes_,
                                 hipStream_t stream)
{
    if (!index || !table) return GODIET_E_INVAL;
    if (index->n > 0 && !index->keys) return GODIET_E_INVAL;
    if (index->n >= (1ull << 32)) return GODIET_E_RANGE;
    if (table_bytes_ < table_bytes(index->n)) return GODIET_E_WORKSPACE;
    if (((uintptr_t)table & 15) != 0) return GODIET_E_INVAL;
    GD_TRY(launch_table_build(index->keys, index->n, table, stream));
    return GODIET_OK;
}

size_t godiet_rmi_size(uint32_t log2_leaves)
{
    if (log2_leaves < 1 || log2_leaves > 24) return 0;
    return rmi_bytes(log2_leaves);
}

godiet_status godiet_rmi_train(const godiet_index *index, int32_t root_kind, uint32_t log2_leaves,
                               void *rmi, size_t rmi_bytes_, hipStream_t stream)
{
    if (!index || !rmi || (root_kind != 0 && root_kind != 1)) return GODIET_E_INVAL;
    if (index->n > 0 && !index->keys) return GODIET_E_INVAL;
    if (index->n >= (1ull << 32)) return GODIET_E_RANGE;
    const size_t need = godiet_rmi_size(log2_leaves);
    if (need == 0) return GODIET_E_INVAL;
    if (rmi_bytes_ < need) return GODIET_E_WORKSPACE;
    if (((uintptr_t)rmi & 63) != 0) return GODIET_E_INVAL;
    GD_TRY(launch_rmi_train(index->keys, index->n, root_kind, log2_leaves, rmi, stream));
    return GODIET_OK;
}

godiet_status godiet_rmi_stats(const godiet_index *index, const uint64_t *q, uint64_t n_q,
                               uint64_t *stats, hipStream_t stream)
{
    if (!index || !index->rmi || !stats || (n_q > 0 && !q)) return GODIET_E_INVAL;
    if (index->n > 0 && !index->keys) return GODIET_E_INVAL;
    if (index->n >= (1ull << 32)) return GODIET_E_RANGE;
    if (!models_fit(index)) return GODIET_E_INVAL;
    GD_TRY(launch_rmi_stats(index->keys, index->n, index->rmi, index->rmi_bytes, q, n_q, stats,
                            stream));
    return GODIET_OK;
}

godiet_status godiet_random_gather(const uint64_t *src, uint64_t n_src, const uint64_t *idx,
                                   uint64_t n_idx, uint64_t *out, uint32_t *status,
                                   hipStream_t stream)
{
    if (!status || (n_idx > 0 && (!src || !idx || !out))) return GODIET_E_INVAL;
    GD_TRY(launch_random_gather(src, n_src, idx, n_idx, out, status, stream));
    return GODIET_OK;
}

godiet_status godiet_lookup(const godiet_index *index, const uint64_t *q, uint64_t n_q,
                            uint32_t *lb, uint32_t *occ, hipStream_t stream)
{
    if (!index || (n_q > 0 && (!q || !lb || !occ))) return GODIET_E_INVAL;
    if (index->n > 0 && !index->keys) return GODIET_E_INVAL;
    if (index->n >= (1ull << 32)) return GODIET_E_RANGE;
    if (!models_fit(index)) return GODIET_E_INVAL;
    if (n_q == 0) return GODIET_OK;
    GD_TRY(launch_lookup(index->keys, index->n, q, nullptr, n_q, lb, occ, index->rmi,
                         index->rmi_bytes, nullptr, 0, 0,
                         stream));
    return GODIET_OK;
}

}  // extern "C"
