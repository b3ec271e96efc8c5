/*
 * godiet_oracle.c -- plain, slow CPU oracle of the sparsified-seeding hot path of
 * Genome-on-Diet (Alser, Eudine, Mutlu: "Genome-on-Diet: Taming Large-Scale Genomic
 * Analyses via Sparsified Genomics", arXiv 2211.08157).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no source, header, table or
 * helper with the GPU library; the two meet only in the seeded synthetic inputs.
 *
 * Every routine follows the definition in the paper as directly as possible, with no
 * blocking, fusion or reordering: sequences are handled one at a time, k-mer codes are
 * recomputed from their k bases, window minima are recomputed from their w members.
 *
 * Inputs are bases as one code per byte (A=0, C=1, G=2, T=3, and 4 for the ambiguous
 * base N) plus n_seq+1 offsets.
 * Positions stored in minimizer records are coordinates of the ORIGINAL (unpatterned)
 * sequence (Section 3.1, step 3).
 *
 * Readings of points the paper leaves open (each one is listed with its reason in the
 * design notes of the repository):
 *   - pattern phase for reads: base j is kept iff P[(j - a) mod p] == 1 (cyclic form of
 *     the set {Q[i+a] * P[i mod p]} of Section 3);
 *   - hash: splitmix64 finalizer of the canonical 2k-bit code (the workloads fix it), or
 *     Thomas Wang's hash masked to 2k bits (the paper's, Section 3.6.1) after
 *     gdo_set_hash(1);
 *   - window ties: every k-mer attaining a window minimum is a minimizer;
 *   - only full windows of w k-mers count; palindromic k-mers (fwd == rc) are never
 *     minimizers and never lower a window minimum;
 *   - pattern alignment scores the first n* = min_s |M_s| minimizers of every shift
 *     (capped by t when t > 0), skips occurrences >= max_occ when max_occ > 0, and picks
 *     the smallest shift of maximal score (0 when p == 1);
 *   - location voting: the adjusted location of an anchor is its diagonal rpos - qpos
 *     on the forward strand and its anti-diagonal rpos + qpos on the reverse strand;
 *     locations vote only within their strand; every anchor is one vote; winners are
 *     ordered by votes (descending), then strand and location (ascending).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GDO_OK 0
#define GDO_EINVAL (-1)
#define GDO_ECAP (-2)
#define GDO_ENOMEM (-3)

#define GDO_MAX_PATTERN 256

typedef struct {
    int p;                    /* pattern length */
    int x;                    /* weight = number of ones */
    unsigned char bit[GDO_MAX_PATTERN];
} gdo_pattern;

static int parse_pattern(const char *s, gdo_pattern *P)
{
    if (!s) return GDO_EINVAL;
    size_t n = strlen(s);
    if (n < 1 || n > GDO_MAX_PATTERN) return GDO_EINVAL;
    P->p = (int)n;
    P->x = 0;
    for (size_t i = 0; i < n; i++) {
        if (s[i] == '1') { P->bit[i] = 1; P->x++; }
        else if (s[i] == '0') P->bit[i] = 0;
        else return GDO_EINVAL;
    }
    return P->x >= 1 ? GDO_OK : GDO_EINVAL;
}

/* Section 3 and Section 3.1 steps (1)-(2): the user pattern is repeated along the
 * sequence; with the pattern shifted right by a, base j is kept iff P[(j - a) mod p]. */
static int is_kept(const gdo_pattern *P, uint64_t j, uint32_t a)
{
    uint64_t p = (uint64_t)P->p;
    uint64_t t = (j % p + p - (a % p)) % p;
    return P->bit[t];
}

/* splitmix64 finalizer (Steele, Lea, Flood 2014: the output function of SplitMix64). */
uint64_t gdo_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Thomas Wang's 64-bit integer hash (his integer-hash note; the k-mer hash of Section
 * 3.6.1), with every step reduced to the 2k-bit code space as minimap2 applies it to k-mer
 * codes.  Steps: key = ~key + key*2^21; key ^= key >> 24; key *= 265; key ^= key >> 14;
 * key *= 21; key ^= key >> 28; key *= 2^31 + 1, each result taken mod 2^(2k). */
uint64_t gdo_wang64(uint64_t key, int k)
{
    const uint64_t mask = k >= 32 ? ~0ULL : ((1ULL << (2 * k)) - 1);
    key = (~key + (key << 21)) & mask;
    key = key ^ (key >> 24);
    key = (key * 265u) & mask;
    key = key ^ (key >> 14);
    key = (key * 21u) & mask;
    key = key ^ (key >> 28);
    key = (key * ((1ULL << 31) + 1)) & mask;
    return key;
}

/* Which k-mer hash the sketches use: 0 splitmix64 finalizer, 1 Wang's hash (set before
 * the calls; a test-infrastructure switch, not thread-safe). */
static int g_hash = 0;

int gdo_set_hash(int kind)
{
    if (kind != 0 && kind != 1) return GDO_EINVAL;
    g_hash = kind;
    return GDO_OK;
}

/* Number of kept bases of a sequence of length L under shift a, counted by definition. */
uint64_t gdo_kept_count(uint64_t L, const char *pattern, uint32_t a)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK) return UINT64_MAX;
    uint64_t n = 0;
    for (uint64_t j = 0; j < L; j++) n += is_kept(&P, j, a);
    return n;
}

/* Sparsify every sequence of a batch (Section 3.1 (1)-(2)).  out_codes receives the kept
 * bases of all sequences back to back, out_offsets[n_seq+1] their boundaries and, when
 * non-NULL, out_orig the original in-sequence coordinate of every kept base.
 * shifts may be NULL (all zero).  Returns the total number of kept bases. */
int64_t gdo_sparsify(const uint8_t *codes, const uint64_t *offsets, uint32_t n_seq,
                     const char *pattern, const uint32_t *shifts,
                     uint8_t *out_codes, uint64_t *out_offsets, uint64_t *out_orig)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK) return GDO_EINVAL;
    uint64_t n = 0;
    out_offsets[0] = 0;
    for (uint32_t s = 0; s < n_seq; s++) {
        uint32_t a = shifts ? shifts[s] : 0;
        if (a >= (uint32_t)P.p) return GDO_EINVAL;
        for (uint64_t j = offsets[s]; j < offsets[s + 1]; j++) {
            if (is_kept(&P, j - offsets[s], a)) {
                out_codes[n] = codes[j];
                if (out_orig) out_orig[n] = j - offsets[s];
                n++;
            }
        }
        out_offsets[s + 1] = n;
    }
    return (int64_t)n;
}

/* Steps 2-3 of the sketch on one run of patterned bases PS[0..n) with no ambiguous base:
 *   2. for every k-mer: forward code (first base most significant), reverse-complement
 *      code, canonical = smaller, strand = rc < fwd, hash = mix64(canonical) (or Wang's);
 *   3. a k-mer is a minimizer iff its hash equals the minimum of some full window of w
 *      consecutive k-mers containing it.
 * Records (key = hash, val = orig << 1 | strand) are appended in ascending k-mer order.
 * Returns the number of records, GDO_ECAP if more than cap would be written. */
static int64_t sketch_run(const uint8_t *PS, const uint64_t *orig, uint64_t n, int k, int w,
                          uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    int64_t out = 0;
    if (n < (uint64_t)k || n - (uint64_t)k + 1 < (uint64_t)w) return 0;
    uint64_t nk = n - (uint64_t)k + 1;
    uint64_t *h = (uint64_t *)malloc(nk * sizeof(uint64_t));
    uint8_t *ok = (uint8_t *)malloc(nk);
    uint8_t *strand = (uint8_t *)malloc(nk);
    uint64_t nwin = nk - (uint64_t)w + 1;
    uint64_t *wmin = (uint64_t *)malloc(nwin * sizeof(uint64_t));
    uint8_t *wany = (uint8_t *)malloc(nwin);
    if (!h || !ok || !strand || !wmin || !wany) {
        free(h); free(ok); free(strand); free(wmin); free(wany);
        return GDO_ENOMEM;
    }
    for (uint64_t i = 0; i < nk; i++) {
        uint64_t fwd = 0, rc = 0;
        for (int t = 0; t < k; t++) fwd = fwd * 4 + PS[i + t];
        for (int t = 0; t < k; t++) rc = rc * 4 + (uint64_t)(3 - PS[i + (uint64_t)k - 1 - t]);
        if (fwd == rc) { ok[i] = 0; h[i] = 0; strand[i] = 0; continue; }
        ok[i] = 1;
        strand[i] = rc < fwd ? 1 : 0;
        h[i] = g_hash ? gdo_wang64(rc < fwd ? rc : fwd, k) : gdo_mix64(rc < fwd ? rc : fwd);
    }
    for (uint64_t s = 0; s < nwin; s++) {
        wany[s] = 0;
        wmin[s] = 0;
        for (uint64_t t = s; t < s + (uint64_t)w; t++) {
            if (!ok[t]) continue;
            if (!wany[s] || h[t] < wmin[s]) wmin[s] = h[t];
            wany[s] = 1;
        }
    }
    for (uint64_t i = 0; i < nk; i++) {
        if (!ok[i]) continue;
        uint64_t s_lo = i + 1 >= (uint64_t)w ? i + 1 - (uint64_t)w : 0;
        uint64_t s_hi = i < nwin - 1 ? i : nwin - 1;
        int sel = 0;
        for (uint64_t s = s_lo; s <= s_hi; s++)
            if (wany[s] && h[i] == wmin[s]) { sel = 1; break; }
        if (!sel) continue;
        if ((uint64_t)out >= cap) { out = GDO_ECAP; break; }
        keys[out] = h[i];
        vals[out] = (orig[i] << 1) | strand[i];
        out++;
    }
    free(h); free(ok); free(strand); free(wmin); free(wany);
    return out;
}

/* Minimizers of one sequence (Section 3.1 step (3) and its minimizer definition):
 *   1. sparsify with shift a, remembering the original coordinate of each kept base;
 *   1b. an ambiguous base (code 4, N) among the kept bases ends the current run of
 *      patterned bases and the next run starts right after it (Section 3.6.1): every run
 *      is sketched on its own, so no k-mer and no window contains an N or spans one.
 *      An N at a dropped position is dropped with it and splits nothing;
 *   2-3. each run as in sketch_run.
 * Records are in ascending k-mer order.  Returns the number of records, or GDO_ECAP if
 * more than cap would be written. */
static int64_t sketch_one(const uint8_t *S, uint64_t L, const gdo_pattern *P, uint32_t a,
                          int k, int w, uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    uint8_t *PS = (uint8_t *)malloc(L ? L : 1);
    uint64_t *orig = (uint64_t *)malloc((L ? L : 1) * sizeof(uint64_t));
    if (!PS || !orig) { free(PS); free(orig); return GDO_ENOMEM; }
    uint64_t n = 0;
    for (uint64_t j = 0; j < L; j++)
        if (is_kept(P, j, a)) { PS[n] = S[j]; orig[n] = j; n++; }

    int64_t out = 0;
    uint64_t r0 = 0;                        /* start of the current run */
    for (uint64_t i = 0; i <= n; i++) {
        if (i < n && PS[i] != 4) continue;
        int64_t r = sketch_run(PS + r0, orig + r0, i - r0, k, w, keys + out, vals + out,
                               cap - (uint64_t)out);
        if (r < 0) { out = r; break; }
        out += r;
        r0 = i + 1;
    }
    free(PS);
    free(orig);
    return out;
}

/* Minimizers of every sequence of a batch.  vals hold orig << 1 | strand in the
 * sequence's own coordinates; mz_offsets[n_seq+1] delimit each sequence's records.
 * Returns the total, GDO_ECAP when cap is too small, GDO_EINVAL on bad arguments. */
int64_t gdo_sketch(const uint8_t *codes, const uint64_t *offsets, uint32_t n_seq,
                   const char *pattern, const uint32_t *shifts, int k, int w,
                   uint64_t *keys, uint64_t *vals, uint64_t *mz_offsets, uint64_t cap)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK || k < 1 || k > 32 || w < 1) return GDO_EINVAL;
    uint64_t n = 0;
    mz_offsets[0] = 0;
    for (uint32_t s = 0; s < n_seq; s++) {
        uint32_t a = shifts ? shifts[s] : 0;
        if (a >= (uint32_t)P.p) return GDO_EINVAL;
        int64_t r = sketch_one(codes + offsets[s], offsets[s + 1] - offsets[s], &P, a, k, w,
                               keys + n, vals + n, cap - n);
        if (r < 0) return r;
        n += (uint64_t)r;
        mz_offsets[s + 1] = n;
    }
    return (int64_t)n;
}

typedef struct { uint64_t key, val; } gdo_rec;

static int rec_cmp(const void *pa, const void *pb)
{
    const gdo_rec *a = (const gdo_rec *)pa, *b = (const gdo_rec *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->val != b->val) return a->val < b->val ? -1 : 1;
    return 0;
}

/* Seed index (Section 3.1 step (3)): all minimizer records of the reference, appended to
 * one array and sorted by (hash, location).  val_bits == 32: val = global position in the
 * concatenated batch << 1 | strand; val_bits == 64: val = sequence id << 32 |
 * position << 1 | strand.  Returns the number of records. */
int64_t gdo_index_build(const uint8_t *codes, const uint64_t *offsets, uint32_t n_seq,
                        const char *pattern, int k, int w, int val_bits,
                        uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    if (val_bits != 32 && val_bits != 64) return GDO_EINVAL;
    uint64_t *mz = (uint64_t *)malloc(((uint64_t)n_seq + 1) * sizeof(uint64_t));
    if (!mz) return GDO_ENOMEM;
    int64_t n = gdo_sketch(codes, offsets, n_seq, pattern, NULL, k, w, keys, vals, mz, cap);
    if (n < 0) { free(mz); return n; }
    gdo_rec *r = (gdo_rec *)malloc(((uint64_t)n + 1) * sizeof(gdo_rec));
    if (!r) { free(mz); return GDO_ENOMEM; }
    for (uint32_t s = 0; s < n_seq; s++) {
        for (uint64_t i = mz[s]; i < mz[s + 1]; i++) {
            uint64_t pos = vals[i] >> 1, strand = vals[i] & 1;
            r[i].key = keys[i];
            if (val_bits == 32) r[i].val = ((offsets[s] + pos) << 1) | strand;
            else r[i].val = ((uint64_t)s << 32) | (pos << 1) | strand;
        }
    }
    qsort(r, (size_t)n, sizeof(gdo_rec), rec_cmp);
    for (int64_t i = 0; i < n; i++) { keys[i] = r[i].key; vals[i] = r[i].val; }
    free(r);
    free(mz);
    return n;
}

/* Exact-match lookup: lb = first i with keys[i] >= q, ub = first i with keys[i] > q. */
static uint64_t lower_bound(const uint64_t *keys, uint64_t n, uint64_t q)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < q) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static uint64_t upper_bound(const uint64_t *keys, uint64_t n, uint64_t q)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] <= q) lo = mid + 1; else hi = mid;
    }
    return lo;
}

void gdo_lookup(const uint64_t *keys, uint64_t n, const uint64_t *q, uint64_t m,
                uint64_t *lb, uint64_t *occ)
{
    for (uint64_t i = 0; i < m; i++) {
        uint64_t l = lower_bound(keys, n, q[i]);
        lb[i] = l;
        occ[i] = upper_bound(keys, n, q[i]) - l;
    }
}

/* Pattern alignment (Section 3.2) for one read: returns the alignment index a. */
static int64_t align_read(const uint8_t *S, uint64_t L, const gdo_pattern *P, int k, int w,
                          const uint64_t *ikeys, uint64_t in, uint32_t t, uint32_t max_occ)
{
    if (P->p == 1) return 0;
    uint64_t **mk = (uint64_t **)calloc((size_t)P->p, sizeof(uint64_t *));
    uint64_t **mv = (uint64_t **)calloc((size_t)P->p, sizeof(uint64_t *));
    int64_t *cnt = (int64_t *)calloc((size_t)P->p, sizeof(int64_t));
    if (!mk || !mv || !cnt) { free(mk); free(mv); free(cnt); return GDO_ENOMEM; }
    int64_t status = 0;
    uint64_t cap = L + 1;
    for (int s = 0; s < P->p && status == 0; s++) {
        mk[s] = (uint64_t *)malloc(cap * sizeof(uint64_t));
        mv[s] = (uint64_t *)malloc(cap * sizeof(uint64_t));
        if (!mk[s] || !mv[s]) { status = GDO_ENOMEM; break; }
        cnt[s] = sketch_one(S, L, P, (uint32_t)s, k, w, mk[s], mv[s], cap);
        if (cnt[s] < 0) status = cnt[s];
    }
    int64_t best = 0;
    if (status == 0) {
        uint64_t nstar = (uint64_t)cnt[0];
        for (int s = 1; s < P->p; s++) if ((uint64_t)cnt[s] < nstar) nstar = (uint64_t)cnt[s];
        if (t > 0 && (uint64_t)t < nstar) nstar = t;
        uint64_t best_score = 0;
        for (int s = 0; s < P->p; s++) {
            uint64_t score = 0;
            for (uint64_t j = 0; j < nstar; j++) {
                uint64_t occ = upper_bound(ikeys, in, mk[s][j]) - lower_bound(ikeys, in, mk[s][j]);
                if (max_occ == 0 || occ < max_occ) score += occ;
            }
            if (score > best_score) { best_score = score; best = s; }
        }
    }
    for (int s = 0; s < P->p; s++) { free(mk[s]); free(mv[s]); }
    free(mk); free(mv); free(cnt);
    return status ? status : best;
}

/* Pattern alignment + compressed seeding (Sections 3.2, 3.3) over a batch of reads.
 * Index: sorted keys[in], vals[in] with val = global reference position << 1 | strand.
 * shift_mode < 0 runs pattern alignment; shift_mode >= 0 forces that shift.
 * For every read r (in order), every minimizer of the read at its shift a (ascending
 * k-mer order), unless max_occ > 0 and its occurrence count >= max_occ, and every index
 * entry e with the same hash (ascending), one anchor
 *     (read_id = r, qpos = read position, rpos = vals[e] >> 1, strand = (qval ^ vals[e]) & 1)
 * is written as four uint32.  read_off[n_reads+1] delimits each read's anchors and
 * shift_out[n_reads] receives a.  Returns the number of anchors or GDO_ECAP. */
int64_t gdo_seed(const uint64_t *ikeys, const uint64_t *ivals, uint64_t in,
                 const uint8_t *codes, const uint64_t *offsets, uint32_t n_reads,
                 const char *pattern, int k, int w, int shift_mode, uint32_t t, uint32_t max_occ,
                 uint32_t *anchors, uint64_t cap, uint64_t *read_off, uint32_t *shift_out)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK || k < 1 || k > 32 || w < 1) return GDO_EINVAL;
    if (shift_mode >= P.p) return GDO_EINVAL;
    uint64_t n = 0;
    read_off[0] = 0;
    int64_t status = 0;
    for (uint32_t r = 0; r < n_reads && status == 0; r++) {
        const uint8_t *S = codes + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        int64_t a = shift_mode >= 0 ? shift_mode
                                    : align_read(S, L, &P, k, w, ikeys, in, t, max_occ);
        if (a < 0) { status = a; break; }
        if (shift_out) shift_out[r] = (uint32_t)a;
        uint64_t *mk = (uint64_t *)malloc((L + 1) * sizeof(uint64_t));
        uint64_t *mv = (uint64_t *)malloc((L + 1) * sizeof(uint64_t));
        if (!mk || !mv) { free(mk); free(mv); status = GDO_ENOMEM; break; }
        int64_t m = sketch_one(S, L, &P, (uint32_t)a, k, w, mk, mv, L + 1);
        if (m < 0) status = m;
        for (int64_t j = 0; j < m && status == 0; j++) {
            uint64_t lb = lower_bound(ikeys, in, mk[j]);
            uint64_t ub = upper_bound(ikeys, in, mk[j]);
            if (max_occ > 0 && ub - lb >= max_occ) continue;
            for (uint64_t e = lb; e < ub; e++) {
                if (n >= cap) { status = GDO_ECAP; break; }
                anchors[4 * n + 0] = r;
                anchors[4 * n + 1] = (uint32_t)(mv[j] >> 1);
                anchors[4 * n + 2] = (uint32_t)(ivals[e] >> 1);
                anchors[4 * n + 3] = (uint32_t)((mv[j] ^ ivals[e]) & 1);
                n++;
            }
        }
        free(mk);
        free(mv);
        read_off[r + 1] = n;
    }
    return status ? status : (int64_t)n;
}

static int u64_cmp(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Containment-style counts (the k-mer-set intersection of Section 2.3): H_sample is the
 * set of hashes of all reads' minimizers at their aligned shift; for genome g, H_g is the
 * set of hashes among index records whose val >> 32 == g (val_bits 64);
 * counts[g] = |H_sample intersect H_g| and sizes[g] = |H_g|. */
int64_t gdo_contain(const uint64_t *ikeys, const uint64_t *ivals, uint64_t in,
                    const uint8_t *codes, const uint64_t *offsets, uint32_t n_reads,
                    const char *pattern, int k, int w, int shift_mode, uint32_t t,
                    uint32_t max_occ, uint32_t n_genomes, uint32_t *counts, uint32_t *sizes)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK || k < 1 || k > 32 || w < 1) return GDO_EINVAL;
    if (shift_mode >= P.p) return GDO_EINVAL;
    uint64_t cap = offsets[n_reads] + 1;
    uint64_t *sample = (uint64_t *)malloc(cap * sizeof(uint64_t));
    uint64_t *tmpv = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!sample || !tmpv) { free(sample); free(tmpv); return GDO_ENOMEM; }
    uint64_t ns = 0;
    for (uint32_t r = 0; r < n_reads; r++) {
        const uint8_t *S = codes + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        int64_t a = shift_mode >= 0 ? shift_mode
                                    : align_read(S, L, &P, k, w, ikeys, in, t, max_occ);
        if (a < 0) { free(sample); free(tmpv); return a; }
        int64_t m = sketch_one(S, L, &P, (uint32_t)a, k, w, sample + ns, tmpv, cap - ns);
        if (m < 0) { free(sample); free(tmpv); return m; }
        ns += (uint64_t)m;
    }
    free(tmpv);
    qsort(sample, (size_t)ns, sizeof(uint64_t), u64_cmp);
    uint64_t nu = 0;
    for (uint64_t i = 0; i < ns; i++)
        if (nu == 0 || sample[nu - 1] != sample[i]) sample[nu++] = sample[i];

    for (uint32_t g = 0; g < n_genomes; g++) { counts[g] = 0; sizes[g] = 0; }
    /* pairs (genome, hash), sorted, then distinct pairs counted */
    gdo_rec *gh = (gdo_rec *)malloc((in + 1) * sizeof(gdo_rec));
    if (!gh) { free(sample); return GDO_ENOMEM; }
    for (uint64_t i = 0; i < in; i++) { gh[i].key = ivals[i] >> 32; gh[i].val = ikeys[i]; }
    qsort(gh, (size_t)in, sizeof(gdo_rec), rec_cmp);
    for (uint64_t i = 0; i < in; i++) {
        if (i > 0 && gh[i].key == gh[i - 1].key && gh[i].val == gh[i - 1].val) continue;
        uint64_t g = gh[i].key;
        if (g >= n_genomes) { free(gh); free(sample); return GDO_EINVAL; }
        sizes[g]++;
        if (bsearch(&gh[i].val, sample, (size_t)nu, sizeof(uint64_t), u64_cmp)) counts[g]++;
    }
    free(gh);
    free(sample);
    return (int64_t)nu;
}

/* Location voting for short reads (Section 3.4 steps 1-4, Illumina form) with the rescue
 * location of Section 3.6.3.  For read r, its anchors [read_off[r], read_off[r+1]) of
 * rows (read_id, qpos, rpos, strand):
 *   1. adjusted location: strand 0: rpos - qpos; strand 1: rpos + qpos;
 *   2. the (strand, location) pairs are sorted into one list;
 *   3. the first entry is the temporary mapping location L0; its votes are the entries of
 *      the same strand with location <= L0 + D;
 *   4. if votes >= V, (strand, L0, votes) is a winner; the first entry beyond L0 + D (or
 *      of the other strand) becomes the next temporary location, until the list ends.
 * Winners are ordered by votes descending (ties: strand, then location ascending) and the
 * first max_win are kept.  The rescue location is the candidate with the most votes (the
 * first such in list order); when there is no winner it is the output, flagged 1.
 * Output per read in out[r*max_win + i], i < n_win[r], rows (strand, votes, flags, loc)
 * as four int64 values.  Returns the total number of rows written. */
typedef struct { int64_t loc; uint32_t strand; uint32_t votes; } gdo_cand;

static int loc_cmp(const void *pa, const void *pb)
{
    const gdo_cand *a = (const gdo_cand *)pa, *b = (const gdo_cand *)pb;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    return a->loc < b->loc ? -1 : (a->loc > b->loc ? 1 : 0);
}

static int win_cmp(const void *pa, const void *pb)
{
    const gdo_cand *a = (const gdo_cand *)pa, *b = (const gdo_cand *)pb;
    if (a->votes != b->votes) return a->votes > b->votes ? -1 : 1;
    return loc_cmp(pa, pb);
}

int64_t gdo_vote(const uint32_t *anchors, const uint64_t *read_off, uint32_t n_reads,
                 uint32_t D, uint32_t V, uint32_t max_win, int64_t *out, uint32_t *n_win)
{
    if (max_win == 0) return GDO_EINVAL;
    int64_t total = 0;
    for (uint32_t r = 0; r < n_reads; r++) {
        const uint64_t b = read_off[r], m = read_off[r + 1] - b;
        n_win[r] = 0;
        if (m == 0) continue;
        gdo_cand *list = (gdo_cand *)malloc(m * sizeof(gdo_cand));
        gdo_cand *win = (gdo_cand *)malloc(m * sizeof(gdo_cand));
        if (!list || !win) { free(list); free(win); return GDO_ENOMEM; }
        for (uint64_t i = 0; i < m; i++) {
            const uint32_t *a = anchors + 4 * (b + i);
            list[i].strand = a[3];
            list[i].loc = a[3] ? (int64_t)a[2] + (int64_t)a[1] : (int64_t)a[2] - (int64_t)a[1];
            list[i].votes = 0;
        }
        qsort(list, (size_t)m, sizeof(gdo_cand), loc_cmp);
        uint64_t nw = 0, i = 0;
        gdo_cand rescue = list[0];
        rescue.votes = 0;
        while (i < m) {
            gdo_cand c = list[i];
            uint64_t j = i;
            while (j < m && list[j].strand == c.strand && list[j].loc <= c.loc + (int64_t)D) j++;
            c.votes = (uint32_t)(j - i);
            if (c.votes >= V) win[nw++] = c;
            if (c.votes > rescue.votes) rescue = c;
            i = j;
        }
        if (nw > 0) {
            qsort(win, (size_t)nw, sizeof(gdo_cand), win_cmp);
            if (nw > max_win) nw = max_win;
            for (uint64_t t = 0; t < nw; t++) {
                int64_t *o = out + 4 * ((uint64_t)r * max_win + t);
                o[0] = win[t].strand; o[1] = win[t].votes; o[2] = 0; o[3] = win[t].loc;
            }
            n_win[r] = (uint32_t)nw;
        } else {
            int64_t *o = out + 4 * ((uint64_t)r * max_win);
            o[0] = rescue.strand; o[1] = rescue.votes; o[2] = 1; o[3] = rescue.loc;
            n_win[r] = 1;
        }
        total += n_win[r];
        free(list);
        free(win);
    }
    return total;
}

/* ---------------------------------------------------------------------------------
 * Seed-matching experiment (Section 2.1.1, Fig. 4): a sequence and a copy with random
 * substitutions; four seeding algorithms; seed matching rates and edit distance.
 *
 * Readings (the program itself is not in the paper):
 *   - a seed is identified by the canonical code of its base string (the string and its
 *     reverse complement are one seed); minimizer and Genome-on-Diet seeds by their hash,
 *     which is a bijection of that code;
 *   - all seeds: every k-mer; minimizers: the sketch with pattern '1'; Genome-on-Diet:
 *     the sketch of the patterned sequence (shift 0); spaced seeds: at every start i the
 *     bases i + j with M[j] == 1, M = the pattern repeated to span k (a pattern of
 *     length k is used as it is);
 *   - matching rate = (seeds of the copy, with multiplicity, found among the original's
 *     seeds) / (seeds of the copy); a copy without seeds has rate 0.
 * ------------------------------------------------------------------------------- */

static uint64_t canon_code(const uint8_t *s, int n)
{
    uint64_t f = 0, r = 0;
    for (int t = 0; t < n; t++) f = f * 4 + s[t];
    for (int t = 0; t < n; t++) r = r * 4 + (uint64_t)(3 - s[n - 1 - t]);
    return f < r ? f : r;
}

static int u64_cmp_plain(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Seeds of one sequence under algorithm alg (0 all, 1 minimizers, 2 spaced, 3
 * Genome-on-Diet), appended to out[]; returns their number or a negative error. */
static int64_t fig4_seeds(const uint8_t *S, uint64_t L, int alg, const gdo_pattern *P, int k,
                          int w, uint64_t *out)
{
    if (alg == 0 || alg == 2) {
        if (L < (uint64_t)k) return 0;
        uint8_t buf[32];
        for (uint64_t i = 0; i + (uint64_t)k <= L; i++) {
            int n = 0;
            for (int j = 0; j < k; j++)
                if (alg == 0 || P->bit[j % P->p]) buf[n++] = S[i + (uint64_t)j];
            out[i] = canon_code(buf, n);
        }
        return (int64_t)(L - (uint64_t)k + 1);
    }
    gdo_pattern one;
    one.p = 1; one.x = 1; one.bit[0] = 1;
    uint64_t *vals = (uint64_t *)malloc((L + 1) * sizeof(uint64_t));
    if (!vals) return GDO_ENOMEM;
    int64_t n = sketch_one(S, L, alg == 1 ? &one : P, 0, k, w, out, vals, L + 1);
    free(vals);
    return n;
}

/* For every pair i (sequence i of a = the original, of b = the mutated copy) and every
 * algorithm g: out[8i + 2g] = matched seeds of the copy, out[8i + 2g + 1] = seeds of the
 * copy.  Codes must be 0..3. */
int gdo_seed_match(const uint8_t *ca, const uint64_t *oa, const uint8_t *cb, const uint64_t *ob,
                   uint32_t n_pairs, const char *pattern, int k, int w, uint32_t *out)
{
    gdo_pattern P;
    if (parse_pattern(pattern, &P) != GDO_OK || k < 1 || k > 32 || w < 1) return GDO_EINVAL;
    for (uint32_t i = 0; i < n_pairs; i++) {
        const uint64_t la = oa[i + 1] - oa[i], lb = ob[i + 1] - ob[i];
        for (uint64_t j = 0; j < la; j++) if (ca[oa[i] + j] > 3) return GDO_EINVAL;
        for (uint64_t j = 0; j < lb; j++) if (cb[ob[i] + j] > 3) return GDO_EINVAL;
        uint64_t *sa = (uint64_t *)malloc((la + 1) * sizeof(uint64_t));
        uint64_t *sb = (uint64_t *)malloc((lb + 1) * sizeof(uint64_t));
        if (!sa || !sb) { free(sa); free(sb); return GDO_ENOMEM; }
        for (int g = 0; g < 4; g++) {
            int64_t na = fig4_seeds(ca + oa[i], la, g, &P, k, w, sa);
            int64_t nb = fig4_seeds(cb + ob[i], lb, g, &P, k, w, sb);
            if (na < 0 || nb < 0) { free(sa); free(sb); return GDO_ENOMEM; }
            qsort(sa, (size_t)na, sizeof(uint64_t), u64_cmp_plain);
            uint32_t hit = 0;
            for (int64_t t = 0; t < nb; t++)
                if (na > 0 && bsearch(&sb[t], sa, (size_t)na, sizeof(uint64_t), u64_cmp_plain))
                    hit++;
            out[8 * (uint64_t)i + 2 * g] = hit;
            out[8 * (uint64_t)i + 2 * g + 1] = (uint32_t)nb;
        }
        free(sa);
        free(sb);
    }
    return GDO_OK;
}

/* Levenshtein distance (unit-cost substitutions, insertions and deletions) by its
 * recurrence D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a_i != b_j]),
 * row by row. */
uint64_t gdo_edit_distance(const uint8_t *a, uint64_t la, const uint8_t *b, uint64_t lb)
{
    uint64_t *prev = (uint64_t *)malloc((lb + 1) * sizeof(uint64_t));
    uint64_t *cur = (uint64_t *)malloc((lb + 1) * sizeof(uint64_t));
    if (!prev || !cur) { free(prev); free(cur); return UINT64_MAX; }
    for (uint64_t j = 0; j <= lb; j++) prev[j] = j;
    for (uint64_t i = 1; i <= la; i++) {
        cur[0] = i;
        for (uint64_t j = 1; j <= lb; j++) {
            uint64_t d = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0);
            if (prev[j] + 1 < d) d = prev[j] + 1;
            if (cur[j - 1] + 1 < d) d = cur[j - 1] + 1;
            cur[j] = d;
        }
        uint64_t *t = prev; prev = cur; cur = t;
    }
    uint64_t r = prev[lb];
    free(prev);
    free(cur);
    return r;
}

/* Accepted sequence pairs (Section 2.1.2): for every edit-distance threshold E in
 * [0, max_e], the seed-matching-rate threshold is the smallest rate among pairs with
 * distance <= E, and accepted[E] counts the pairs whose rate reaches it (0 when no pair
 * is that close).  Rates matched/total are compared as exact fractions (total 0 counts
 * as rate 0). */
void gdo_accepted(const uint32_t *dist, const uint32_t *matched, const uint32_t *total,
                  uint32_t n, uint32_t max_e, uint32_t *accepted)
{
    for (uint32_t E = 0; E <= max_e; E++) {
        int have = 0;
        uint64_t tm = 0, tt = 1;                     /* threshold fraction tm / tt */
        for (uint32_t i = 0; i < n; i++) {
            if (dist[i] > E) continue;
            uint64_t m = total[i] ? matched[i] : 0, t = total[i] ? total[i] : 1;
            if (!have || m * tt < tm * t) { tm = m; tt = t; have = 1; }
        }
        uint32_t c = 0;
        if (have)
            for (uint32_t i = 0; i < n; i++) {
                uint64_t m = total[i] ? matched[i] : 0, t = total[i] ? total[i] : 1;
                if (m * tt >= tm * t) c++;
            }
        accepted[E] = c;
    }
}
