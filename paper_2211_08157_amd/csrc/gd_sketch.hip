// Sparsification and minimizer sketching on gfx950.
//
// Layout: a batch of sequences is first sparsified into one "patterned stream" (2-bit
// packed, 16 bases per uint32 word, sequences back to back, boundaries pofs[]).  The
// sketch kernel then tiles the patterned positions of the whole batch: a workgroup of
// kSkBlock = 512 threads, 16 positions each, owns T consecutive positions (k-mer starts)
// plus a halo of H positions on each side, so that every window touching an owned position lies in its LDS.  A
// position whose k-mer would cross the end of its sequence gets an "empty" hash, and a
// window is valid only when its w k-mers lie in one sequence, so tiles may span any
// number of sequences (reads) or cover part of one (a chromosome).
//
// Minimizer selection uses the identity: position i is a minimizer iff its hash equals
// max over the valid windows containing i of the window minimum (every window minimum
// is <= h_i, and equality holds exactly for the windows where i attains the minimum).
// For w = 2..17 both sliding reductions run in registers (prefix and suffix scans of each
// thread's 16 values plus two neighbour exchanges through LDS); other w use doubling in
// LDS.  The output is compacted in position order with a single-pass decoupled look-back
// across tiles.
#include "gd_internal.h"

namespace gd {

TileGeom tile_geom(int w)
{
    TileGeom g;
    g.H = ((w - 1 + 15) / 16) * 16;
    if (g.H == 0) g.H = 16;
    g.T = kSkBlock * 16 - 2 * g.H;
    return g;
}

size_t sketch_tiles_bound(uint64_t np_bound, int w)
{
    const TileGeom g = tile_geom(w);
    return (size_t)(np_bound / (uint64_t)g.T) + 2;
}

namespace {

__device__ __forceinline__ uint32_t seq_shift(const uint32_t *shift, uint32_t uniform, uint32_t s)
{
    return shift ? shift[s] : uniform;
}

// Sequence boundaries of one workgroup's range of patterned positions, cached in LDS.
// A batch of reads puts tens of sequences into every tile; looking each position's
// sequence up with a binary search over millions of global offsets would dominate.
constexpr int kSeqCache = 512;

struct SeqCache {
    const uint64_t *pofs;   // global boundaries, n_seq + 1 entries
    uint32_t n_seq;
    const uint64_t *sh;     // LDS copy of pofs[lo .. lo + n]
    const uint64_t *offs;   // original offsets (global) and, if osh, their LDS copy
    const uint64_t *osh;
    uint32_t lo, n;         // n == 0: no cache (nothing was loaded into sh / osh)
    __device__ __forceinline__ uint64_t at(uint32_t s) const
    {
        const uint32_t d = s - lo;
        return (n > 0 && d <= n) ? sh[d] : pofs[s];
    }
    __device__ __forceinline__ uint64_t orig(uint32_t s) const
    {
        const uint32_t d = s - lo;
        return (osh && n > 0 && d <= n) ? osh[d] : offs[s];
    }
    // last s with pofs[s] <= j (j < pofs[n_seq])
    __device__ __forceinline__ uint32_t find(uint64_t j) const
    {
        if (n > 0 && j >= sh[0] && j < sh[n]) {
            // the guess that is exact for sequences of equal length (a batch of reads),
            // then bisection on the side it leaves
            const float f = (float)(j - sh[0]) * ((float)n / (float)(sh[n] - sh[0]));
            uint32_t g = f < (float)n ? (uint32_t)f : n - 1;
            uint32_t a, b;                  // sh[a] <= j < sh[b]
            if (sh[g] <= j) {
                if (j < sh[g + 1]) return lo + g;
                a = g + 1;
                b = n;
            } else {
                a = 0;
                b = g;
            }
            while (b - a > 1) {
                const uint32_t m = (a + b) >> 1;
                if (sh[m] <= j) a = m; else b = m;
            }
            return lo + a;
        }
        return last_le(pofs, n_seq, j);
    }
};

// Last s in [0, n] with a[s] <= v, as last_le, for a[0] <= v < np = a[n]: the search
// starts where v would fall if the positions were spread evenly over the sequences (as
// they nearly are in a read batch) and gallops outwards to a bracket, so a batch of
// similar reads needs a few loads instead of log2(n) dependent ones.
__device__ __forceinline__ uint32_t last_le_guess(const uint64_t *a, uint32_t n, uint64_t v,
                                                  uint64_t np)
{
    const double f = (double)v / (double)np * (double)n;
    uint32_t g = f < (double)n ? (uint32_t)f : n - 1;
    if (g >= n) g = n - 1;
    uint32_t lo, hi;                 // a[lo] <= v, and a[hi] > v or hi == n + 1
    if (a[g] <= v) {
        lo = g;
        uint64_t step = 1;
        while (true) {
            const uint64_t nx = (uint64_t)lo + step;
            if (nx > n) { hi = n + 1; break; }
            if (a[nx] > v) { hi = (uint32_t)nx; break; }
            lo = (uint32_t)nx;
            step <<= 1;
        }
    } else {
        hi = g;
        uint64_t step = 1;
        while (true) {
            if (hi < step) { lo = 0; break; }          // a[0] <= v
            const uint32_t nx = (uint32_t)(hi - step);
            if (a[nx] <= v) { lo = nx; break; }
            hi = nx;
            step <<= 1;
        }
    }
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Sequences holding the first and last position of window i of the patterned stream,
// for all windows at once (one thread each), so that no workgroup starts with a serial
// search over the batch's offsets.  Window i covers [max(i*stride - before, 0),
// i*stride - before + span] clamped to the stream; lohi[2i] and lohi[2i+1] are the first and
// last sequence (both n_seq when the window lies past the stream's end).
__device__ __forceinline__ void window_range(const uint64_t *pofs, uint32_t n_seq, uint64_t np,
                                             uint64_t i, uint64_t stride, uint64_t before,
                                             uint64_t span, uint32_t *lohi)
{
    const int64_t a0 = (int64_t)(i * stride) - (int64_t)before;
    const uint64_t a = a0 > 0 ? (uint64_t)a0 : 0;
    const int64_t b0 = a0 + (int64_t)span;
    uint64_t b = b0 > 0 ? (uint64_t)b0 : 0;
    uint32_t lo = n_seq, hi = n_seq;
    if (a < np) {
        if (b >= np) b = np - 1;
        lo = last_le_guess(pofs, n_seq, a, np);
        hi = last_le_guess(pofs, n_seq, b, np);
    }
    lohi[2 * i] = lo;
    lohi[2 * i + 1] = hi;
}

__global__ __launch_bounds__(kBlock) void k_window_seqs(const uint64_t *pofs, uint32_t n_seq,
                                                        uint64_t stride, uint64_t before,
                                                        uint64_t span, uint64_t count,
                                                        uint32_t *lohi)
{
    const uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    if (i >= count) return;
    window_range(pofs, n_seq, pofs[n_seq], i, stride, before, span, lohi);
}

// The ranges of the sparsify workgroups (kSpSpan positions each) and of the sketch tiles
// of the same stream in one launch.
__global__ __launch_bounds__(kBlock) void k_window_seqs2(const uint64_t *pofs, uint32_t n_seq,
                                                         uint64_t count_sp, uint32_t *lohi_sp,
                                                         uint64_t T, uint64_t H,
                                                         uint64_t count_sk, uint32_t *lohi_sk)
{
    const uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    const uint64_t np = pofs[n_seq];
    if (i < count_sp)
        window_range(pofs, n_seq, np, i, kSpSpan, 0, kSpSpan - 1, lohi_sp);
    if (i < count_sk) window_range(pofs, n_seq, np, i, T, H, T + 2 * H + 48, lohi_sk);
}

// Fill the cache with the boundaries of sequences lo..hi from k_window_seqs (all threads
// of the workgroup call this).
// With offs/osh set, the sequences' original offsets are cached as well (loaded together
// with the boundaries, so no later load waits on the sequence search).
__device__ __forceinline__ SeqCache seq_cache(const uint64_t *pofs, uint32_t n_seq,
                                              const uint32_t *lohi, uint64_t win, uint64_t *sh,
                                              const uint64_t *offs = nullptr,
                                              uint64_t *osh = nullptr)
{
    SeqCache c;
    c.pofs = pofs;
    c.n_seq = n_seq;
    c.sh = sh;
    c.offs = offs;
    c.osh = osh;
    const uint32_t lo = lohi[2 * win], hi = lohi[2 * win + 1];
    c.lo = lo;
    c.n = lo < n_seq ? hi - lo + 1 : 0;      // sequences lo..hi, boundaries lo..hi+1
    if (c.n + 1 > (uint32_t)kSeqCache) c.n = 0;
    for (uint32_t i = threadIdx.x; c.n > 0 && i <= c.n; i += blockDim.x) {
        sh[i] = pofs[c.lo + i];
        if (osh) osh[i] = offs[c.lo + i];
    }
    __syncthreads();
    return c;
}

// ---------------------------------------------------------------- kept counts

__global__ __launch_bounds__(kBlock) void k_kept(const uint64_t *offsets, uint32_t n_seq,
                                                 Pattern P, const uint32_t *shift,
                                                 uint32_t uniform, uint64_t *kept,
                                                 uint32_t *status)
{
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_seq) return;
    uint32_t a = seq_shift(shift, uniform, s);
    if (a >= P.p) { set_status(status, 4u); a = 0; }
    kept[s] = kept_count(P, offsets[s + 1] - offsets[s], a);
}

// ---------------------------------------------------------------- sparsify

// (li / x, li % x) without an integer divide: a double estimate, corrected.
__device__ __forceinline__ void div_x(uint64_t li, uint32_t x, double inv_x, uint64_t *q,
                                      uint32_t *r)
{
    int64_t qq = (int64_t)((double)li * inv_x);
    int64_t rr = (int64_t)li - qq * (int64_t)x;
    while (rr < 0) { qq--; rr += x; }
    while (rr >= (int64_t)x) { qq++; rr -= x; }
    *q = (uint64_t)qq;
    *r = (uint32_t)rr;
}


__device__ __forceinline__ uint32_t base_at(const uint8_t *bases, uint64_t g)
{
    return (bases[g >> 2] >> ((g & 3) * 2)) & 3u;
}

// Bases 2i (i = 0..15) of a 64-bit run of 32 bases: the kept half under a period-2
// pattern, compacted into one 16-base word.
__device__ __forceinline__ uint32_t unzip_even(uint64_t y)
{
    y &= 0x3333333333333333ull;
    y = (y | (y >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    y = (y | (y >> 4)) & 0x00FF00FF00FF00FFull;
    y = (y | (y >> 8)) & 0x0000FFFF0000FFFFull;
    y = (y | (y >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)y;
}

// Offset within the period of the only kept phase of a one-one pattern under shift a
// (kept_phase(P, a, 0) for x == 1, read without a per-lane table index).
__device__ __forceinline__ uint32_t phase1(const Pattern &P, uint32_t a)
{
    const uint32_t v = P.ones[0] + a;
    return v >= P.p ? v - P.p : v;
}

// Input bases o, o + 2, .., o + 30 (every other base of the 32 from o) as one word, from
// the three input words from o >> 4: one funnel shift and a bit unzip.
__device__ __forceinline__ uint32_t unzip_run(uint32_t W0, uint32_t W1, uint32_t W2, uint64_t o)
{
    const int sh = 2 * (int)(o & 15);
    const uint32_t lo = __builtin_amdgcn_alignbit(W1, W0, sh);
    const uint32_t hi = __builtin_amdgcn_alignbit(W2, W1, sh);
    return unzip_even(((uint64_t)hi << 32) | lo);
}

// The 16 kept bases [16q, 16q+16) of the batch as one word (q below the stream's words).
// nbytes = ceil(n_bases / 4), the readable size of `bases`.  Three paths:
//  * period 2 with one kept base, word inside one sequence: the 16 kept bases are every
//    other base of a run of 32, one funnel shift and a bit unzip;
//  * compact patterns (16 kept bases always within 49 original bases): per sequence
//    segment of the word, one 64-base window of the input in registers, the kept phases
//    walked as the set bits of the rotated pattern (no tables, no divisions per base);
//  * otherwise one 2-bit load per base.
__device__ uint32_t sparsify_word(const SeqCache &C, const uint8_t *bases, const Pattern &P,
                                  const uint32_t *shift, uint32_t uniform, uint64_t np,
                                  size_t q, uint64_t nbytes, int compact, double inv_x)
{
    const uint64_t j0 = (uint64_t)q * 16;
    uint32_t word = 0;
    if (j0 < np) {
        uint32_t s = C.find(j0);
        uint64_t beg = C.at(s), end = C.at(s + 1);
        while (j0 >= end) { s++; beg = end; end = C.at(s + 1); }
        uint32_t a = seq_shift(shift, uniform, s);
        if (a >= P.p) a = 0;
        if (P.p == 2 && P.x == 1) {
            // 16 kept bases from original position o: every other base of a run of 32
            const uint32_t *wd = (const uint32_t *)bases;
            auto run16 = [&](uint64_t o) -> uint32_t {
                const uint64_t g = o >> 4;
                return unzip_run(wd[g], wd[g + 1], wd[g + 2], o);
            };
            const uint64_t o0 = C.orig(s) + (j0 - beg) * 2 + phase1(P, a);   // x == 1
            if (j0 + 16 <= end && ((o0 >> 4) + 3) * 4 <= nbytes) {
                return run16(o0);
            }
            // a word that ends inside the next non-empty sequence (most read boundaries):
            // the first n1 bases from this sequence, the rest from the start of the next;
            // both runs are read at once
            if (j0 + 16 > end && j0 + 16 <= np) {
                uint32_t s2 = s + 1;
                while (C.at(s2 + 1) == C.at(s2)) s2++;        // skip empty sequences
                const uint64_t end2 = C.at(s2 + 1);
                uint32_t a2 = seq_shift(shift, uniform, s2);
                if (a2 >= P.p) a2 = 0;
                const uint64_t o2 = C.orig(s2) + phase1(P, a2);
                if (j0 + 16 <= end2 && ((o0 >> 4) + 3) * 4 <= nbytes &&
                    ((o2 >> 4) + 3) * 4 <= nbytes) {
                    const int n1 = (int)(end - j0);           // 1..15
                    const uint32_t w1 = run16(o0), w2 = run16(o2);
                    return (w1 & ((1u << (2 * n1)) - 1u)) | (w2 << (2 * n1));
                }
            }
        }
        int u = 0;
        while (u < 16) {
            const uint64_t j = j0 + (uint64_t)u;
            if (j >= np) break;
            if (j >= end) {
                while (j >= end) { s++; beg = end; end = C.at(s + 1); }
                a = seq_shift(shift, uniform, s);
                if (a >= P.p) a = 0;
            }
            const int seg = (int)min((uint64_t)(16 - u), end - j);   // bases of sequence s
            const uint64_t li = j - beg;
            uint64_t per;
            uint32_t r;
            div_x(li, P.x, inv_x, &per, &r);
            if (P.p > 64) {
                // long pattern: the kept phases by rank, (ones[(r + front) mod x] + a) mod p
                uint64_t pb = C.orig(s) + per * P.p;
                uint32_t idx = r + kept_front(P, a);
                if (idx >= P.x) idx -= P.x;
                for (int i = 0; i < seg; i++) {
                    uint32_t v = P.ones[idx] + a;
                    if (v >= P.p) v -= P.p;
                    word |= base_at(bases, pb + v) << (2 * (u + i));
                    if (++r == P.x) { r = 0; pb += P.p; }
                    if (++idx == P.x) idx = 0;
                }
                u += seg;
                continue;
            }
            const uint64_t rot = rotated_mask(P, a);
            uint64_t m = rot;                      // kept phases of the period not yet used
            for (uint32_t t = 0; t < r; t++) m &= m - 1;
            const uint64_t ob = C.orig(s) + per * P.p;                // period start
            const uint64_t g = (ob + (uint64_t)__builtin_ctzll(m)) >> 4;
            if (compact && (g + 4) * 4 <= nbytes) {
                const uint32_t *wd = (const uint32_t *)bases;
                const uint64_t lo64 = ((uint64_t)wd[g + 1] << 32) | wd[g];
                const uint64_t hi64 = ((uint64_t)wd[g + 3] << 32) | wd[g + 2];
                int64_t rel = (int64_t)(ob - 16 * g);                  // period start in window
                for (int i = 0; i < seg; i++) {
                    const int off = (int)(rel + __builtin_ctzll(m));   // < 64
                    const uint64_t src = off < 32 ? lo64 : hi64;
                    const uint32_t b2 = (uint32_t)(src >> (2 * (off & 31))) & 3u;
                    word |= b2 << (2 * (u + i));
                    m &= m - 1;
                    if (m == 0) { m = rot; rel += P.p; }
                }
            } else {
                uint64_t pb = ob;
                for (int i = 0; i < seg; i++) {
                    word |= base_at(bases, pb + (uint64_t)__builtin_ctzll(m)) << (2 * (u + i));
                    m &= m - 1;
                    if (m == 0) { m = rot; pb += P.p; }
                }
            }
            u += seg;
        }
    }
    return word;
}


// kSpWords output words per thread, kBlock apart (so that each round of stores is
// coalesced), in one workgroup per kSpSpan patterned positions: the workgroup's sequence
// range is loaded once for all of them.  Under a period-2 pattern the words that lie
// inside one sequence (all but a few per read) first compute their input offsets, then
// issue every input load at once, so one memory round trip serves all of a thread's
// words; the others take sparsify_word.
__global__ __launch_bounds__(kBlock) void k_sparsify(const uint8_t *bases, const uint64_t *offsets,
                                                     uint32_t n_seq, Pattern P,
                                                     const uint32_t *shift, uint32_t uniform,
                                                     const uint64_t *pofs, uint32_t *psw,
                                                     size_t words, uint64_t nbytes, int compact,
                                                     double inv_x, const uint32_t *lohi)
{
    __shared__ uint64_t sh_pofs[kSeqCache];
    __shared__ uint64_t sh_offs[kSeqCache];
    const SeqCache C = seq_cache(pofs, n_seq, lohi, blockIdx.x, sh_pofs, offsets, sh_offs);
    const size_t q0 = blockIdx.x * (size_t)kBlock * kSpWords + threadIdx.x;
    const uint64_t np = pofs[n_seq];
    if (P.p == 2 && P.x == 1) {
        uint64_t o[kSpWords];
        bool fast[kSpWords];
#pragma unroll
        for (int u = 0; u < kSpWords; u++) {
            const size_t q = q0 + (size_t)u * kBlock;
            const uint64_t j0 = (uint64_t)q * 16;
            fast[u] = false;
            o[u] = 0;
            if (q < words && j0 < np) {
                uint32_t s = C.find(j0);
                uint64_t beg = C.at(s), end = C.at(s + 1);
                while (j0 >= end) { s++; beg = end; end = C.at(s + 1); }
                uint32_t a = seq_shift(shift, uniform, s);
                if (a >= P.p) a = 0;
                const uint64_t oo = C.orig(s) + (j0 - beg) * 2 + phase1(P, a);   // x == 1
                fast[u] = j0 + 16 <= end && ((oo >> 4) + 3) * 4 <= nbytes;
                o[u] = fast[u] ? oo : 0;
            }
        }
        // every load in flight before the first use; a word off the fast path reads the
        // input's first three words, which exist whenever some word is fast
        uint32_t W[kSpWords][3];
        const uint32_t *wd = (const uint32_t *)bases;
        if (nbytes >= 12) {
#pragma unroll
            for (int u = 0; u < kSpWords; u++)
#pragma unroll
                for (int k = 0; k < 3; k++) W[u][k] = wd[(o[u] >> 4) + k];
        }
#pragma unroll
        for (int u = 0; u < kSpWords; u++) {
            const size_t q = q0 + (size_t)u * kBlock;
            if (q >= words) break;
            psw[q] = fast[u] ? unzip_run(W[u][0], W[u][1], W[u][2], o[u])
                             : sparsify_word(C, bases, P, shift, uniform, np, q, nbytes, compact,
                                             inv_x);
        }
        return;
    }
    for (int u = 0; u < kSpWords; u++) {
        const size_t q = q0 + (size_t)u * kBlock;
        if (q >= words) break;
        psw[q] = sparsify_word(C, bases, P, shift, uniform, np, q, nbytes, compact, inv_x);
    }
}

// N bits of the kept bases: the 16 bits of output word q (the words of k_sparsify, with the
// same workgroups and sequence ranges).  Each base is located as in the per-base path of
// sparsify_word; N runs are rare, so nothing faster is needed.
__device__ uint16_t sparsify_nword(const SeqCache &C, const uint32_t *nmask, const Pattern &P,
                                   const uint32_t *shift, uint32_t uniform, uint64_t np,
                                   size_t q, double inv_x, uint64_t nwords)
{
    const uint64_t j0 = (uint64_t)q * 16;
    uint32_t bits = 0;
    if (j0 < np) {
        uint32_t s = C.find(j0);
        uint64_t beg = C.at(s), end = C.at(s + 1);
        while (j0 >= end) { s++; beg = end; end = C.at(s + 1); }
        if (P.p == 2 && P.x == 1) {
            // period 2: the bits of every other base of a run of 31, one funnel shift and
            // a bit unzip (the next mask word is read only when the run reaches into it);
            // a word that ends inside the next sequence takes its tail from a second run
            auto run16 = [&](uint64_t o) -> uint32_t {
                const uint64_t g = o >> 5;
                const uint32_t sh = (uint32_t)(o & 31);
                const uint32_t lo = nmask[g], hi = sh >= 2 ? nmask[g + 1] : 0u;
                uint32_t x = __builtin_amdgcn_alignbit(hi, lo, sh) & 0x55555555u;
                x = (x | (x >> 1)) & 0x33333333u;
                x = (x | (x >> 2)) & 0x0F0F0F0Fu;
                x = (x | (x >> 4)) & 0x00FF00FFu;
                return (x | (x >> 8)) & 0x0000FFFFu;
            };
            uint32_t a = seq_shift(shift, uniform, s);
            if (a >= P.p) a = 0;
            const uint64_t o0 = C.orig(s) + (j0 - beg) * 2 + phase1(P, a);
            if (j0 + 16 <= end) {
                return (uint16_t)run16(o0);
            }
            if (j0 + 16 <= np) {
                uint32_t s2 = s + 1;
                while (C.at(s2 + 1) == C.at(s2)) s2++;        // skip empty sequences
                uint32_t a2 = seq_shift(shift, uniform, s2);
                if (a2 >= P.p) a2 = 0;
                const uint64_t o2 = C.orig(s2) + phase1(P, a2);
                // both runs' reads stay inside the mask (ceil(n_bases / 32) words)
                if (j0 + 16 <= C.at(s2 + 1) && ((o0 + 30) >> 5) < nwords &&
                    ((o2 + 30) >> 5) < nwords) {
                    const int n1 = (int)(end - j0);           // 1..15
                    return (uint16_t)((run16(o0) & ((1u << n1) - 1u)) | (run16(o2) << n1));
                }
            }
        }
        int u = 0;
        while (u < 16) {
            const uint64_t j = j0 + (uint64_t)u;
            if (j >= np) break;
            while (j >= end) { s++; beg = end; end = C.at(s + 1); }
            uint32_t a = seq_shift(shift, uniform, s);
            if (a >= P.p) a = 0;
            const int seg = (int)min((uint64_t)(16 - u), end - j);
            uint64_t per;
            uint32_t r;
            div_x(j - beg, P.x, inv_x, &per, &r);
            if (P.p > 64) {
                uint64_t pb = C.orig(s) + per * P.p;
                uint32_t idx = r + kept_front(P, a);
                if (idx >= P.x) idx -= P.x;
                for (int i = 0; i < seg; i++) {
                    uint32_t v = P.ones[idx] + a;
                    if (v >= P.p) v -= P.p;
                    const uint64_t g = pb + v;
                    bits |= ((nmask[g >> 5] >> (g & 31)) & 1u) << (u + i);
                    if (++r == P.x) { r = 0; pb += P.p; }
                    if (++idx == P.x) idx = 0;
                }
                u += seg;
                continue;
            }
            const uint64_t rot = rotated_mask(P, a);
            uint64_t m = rot;
            for (uint32_t t = 0; t < r; t++) m &= m - 1;
            uint64_t pb = C.orig(s) + per * P.p;
            for (int i = 0; i < seg; i++) {
                const uint64_t g = pb + (uint64_t)__builtin_ctzll(m);
                bits |= ((nmask[g >> 5] >> (g & 31)) & 1u) << (u + i);
                m &= m - 1;
                if (m == 0) { m = rot; pb += P.p; }
            }
            u += seg;
        }
    }
    return (uint16_t)bits;
}


__global__ __launch_bounds__(kBlock) void k_sparsify_n(const uint32_t *nmask,
                                                       const uint64_t *offsets, uint32_t n_seq,
                                                       Pattern P, const uint32_t *shift,
                                                       uint32_t uniform, const uint64_t *pofs,
                                                       uint16_t *pnw, size_t words, double inv_x,
                                                       const uint32_t *lohi, uint64_t nwords)
{
    __shared__ uint64_t sh_pofs[kSeqCache];
    __shared__ uint64_t sh_offs[kSeqCache];
    const SeqCache C = seq_cache(pofs, n_seq, lohi, blockIdx.x, sh_pofs, offsets, sh_offs);
    const size_t q0 = blockIdx.x * (size_t)kBlock * kSpWords + threadIdx.x;
    const uint64_t np = pofs[n_seq];
    for (int u = 0; u < kSpWords; u++) {
        const size_t q = q0 + (size_t)u * kBlock;
        if (q >= words) break;
        pnw[q] = sparsify_nword(C, nmask, P, shift, uniform, np, q, inv_x, nwords);
    }
}

// Code of one character (4 = N).
__device__ __forceinline__ uint32_t base_code(uint32_t ch)
{
    const uint32_t c = ch | 0x20u;                                  // lower case
    return c == 'a' ? 0u : c == 'c' ? 1u : c == 'g' ? 2u : (c == 't' || c == 'u') ? 3u : 4u;
}

// Text to codes: one thread per 16 characters (one 16-byte load when the text is
// 16-byte aligned and the group is whole), one 2-bit word and 16 N bits.
__global__ __launch_bounds__(kBlock) void k_pack_ascii(const uint8_t *text, uint64_t n,
                                                       uint32_t *bases, uint16_t *nmask,
                                                       size_t words, int aligned)
{
    const size_t q = blockIdx.x * (size_t)kBlock + threadIdx.x;
    if (q >= words) return;
    uint32_t code = 0, nb = 0;
    const uint64_t i0 = (uint64_t)q * 16;
    if (aligned && i0 + 16 <= n) {
        const uint4 v = *(const uint4 *)(text + i0);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const uint32_t b = base_code((wd[u >> 2] >> (8 * (u & 3))) & 0xFFu);
            code |= (b & 3u) << (2 * u);
            nb |= (b >> 2) << u;
        }
    } else {
        for (int u = 0; u < 16; u++) {
            if (i0 + u < n) {
                const uint32_t b = base_code(text[i0 + u]);
                code |= (b & 3u) << (2 * u);
                nb |= (b >> 2) << u;
            }
        }
    }
    bases[q] = code;
    nmask[q] = (uint16_t)nb;
}

// ---------------------------------------------------------------- sketch

constexpr int kE = kSkBlock * 16;   // LDS positions per tile (T + 2H)
constexpr uint64_t kFlagA = 1ull << 62, kFlagP = 2ull << 62, kValMask = (1ull << 62) - 1;
constexpr int kMaxRegW = 17;        // largest w handled by the register path

struct SketchArgs {
    const uint32_t *psw;
    const uint32_t *pnw;            // N bits of the patterned stream, or null
    const uint64_t *pofs;
    const uint64_t *offsets;
    const uint32_t *shift;
    uint32_t uniform;
    uint32_t n_seq;
    Pattern P;
    double inv_x;                   // 1 / x, for the period division
    int k, w, H, T;
    uint64_t kmask;
    uint64_t *keys;
    void *vals;
    int val_mode;
    uint64_t *mz_offsets;
    uint64_t capacity;
    uint64_t *n_out;
    uint64_t *tile_state;
    const uint32_t *lohi;           // per-tile sequence range (k_window_seqs)
    uint32_t *tile_counter;
    uint32_t *status;
};

// A 16-base word with base 0 in the low bits turned into one with base 0 in the top
// bits (bit reversal, then the two bits of every base swapped back).
__device__ __forceinline__ uint32_t msb_first(uint32_t w)
{
    w = __builtin_bitreverse32(w);
    return ((w >> 1) & 0x55555555u) | ((w & 0x55555555u) << 1);
}

// 64 bits of the patterned stream starting at base u of the chunk, base u in the low bits
// (the reverse-complement code is its complement), from LSB-first words w0..w2.
__device__ __forceinline__ uint64_t kmer_lsb(uint32_t w0, uint32_t w1, uint32_t w2, int u)
{
    const uint32_t lo = u == 0 ? w0 : __builtin_amdgcn_alignbit(w1, w0, 2 * u);
    const uint32_t hi = u == 0 ? w1 : __builtin_amdgcn_alignbit(w2, w1, 2 * u);
    return ((uint64_t)hi << 32) | lo;
}

// 64 bits of the patterned stream starting at base u, base u in the top bits (shifted
// right by 64 - 2k it is the forward code), from MSB-first words m0..m2.
__device__ __forceinline__ uint64_t kmer_msb(uint32_t m0, uint32_t m1, uint32_t m2, int u)
{
    const uint32_t hi = u == 0 ? m0 : __builtin_amdgcn_alignbit(m0, m1, 32 - 2 * u);
    const uint32_t lo = u == 0 ? m1 : __builtin_amdgcn_alignbit(m1, m2, 32 - 2 * u);
    return ((uint64_t)hi << 32) | lo;
}

// First N of the patterned stream in [a, b), else b (b - a is at most a few hundred).
__device__ __forceinline__ uint64_t first_n(const uint32_t *pnw, uint64_t a, uint64_t b)
{
    while (a < b) {
        uint32_t wd = pnw[a >> 5] >> (a & 31);
        uint64_t avail = 32 - (a & 31);
        if (b - a < avail) {
            avail = b - a;
            wd &= (1u << avail) - 1u;
        }
        if (wd) return a + (uint64_t)(__ffs(wd) - 1);
        a += avail;
    }
    return b;
}

// Whether [a, b) holds an N: up to four mask words loaded at once when the range spans
// at most 96 positions (the loads issue together with the chunk's stream words), the
// scanning loop otherwise.
__device__ __forceinline__ bool any_n(const uint32_t *pnw, uint64_t a, uint64_t b)
{
    if (b <= a) return false;
    if (b - a > 96) return first_n(pnw, a, b) != b;
    const uint64_t wa = a >> 5, wb = (b - 1) >> 5;       // wb - wa <= 3
    uint32_t m[4];
#pragma unroll
    for (int i = 0; i < 4; i++) m[i] = wa + i <= wb ? pnw[wa + i] : 0u;
    m[0] &= ~0u << (a & 31);
    const uint32_t top = (uint32_t)((b - 1) & 31);
    const uint32_t keep = top == 31 ? ~0u : ((2u << top) - 1u);
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (wa + i == wb) m[i] &= keep;
    return (m[0] | m[1] | m[2] | m[3]) != 0;
}

// One past the last N of the patterned stream in [a, b), else a.
__device__ __forceinline__ uint64_t after_last_n(const uint32_t *pnw, uint64_t a, uint64_t b)
{
    while (b > a) {
        const uint64_t top = b - 1;               // highest position of this step
        uint32_t wd = pnw[top >> 5] << (31 - (top & 31));     // bit 31 = position top
        uint64_t avail = (top & 31) + 1;
        if (b - a < avail) {
            avail = b - a;
            wd &= ~((1u << (32 - avail)) - 1u);
        }
        if (wd) return top - (uint64_t)__clz(wd) + 1;
        b -= avail;
    }
    return a;
}

// Bits u in [0, 16) with u <= x.
__device__ __forceinline__ uint32_t mask_le(int64_t x)
{
    return x < 0 ? 0u : (x >= 15 ? 0xFFFFu : (2u << x) - 1u);
}


// Minimizer selection for the 16 positions of this thread, w = W known at compile time,
// on values of type T: the full 64-bit hashes, or their high 32-bit words (see
// sketch_tile for how the result is kept exact).  Window minima of the windows starting
// in the chunk come from the chunk's suffix minima and the next chunk's prefix minima
// (windows reaching into it) or from a split at a position common to all windows inside
// the chunk; the opening (max over the windows containing a position) is built the same
// way from the previous chunk's suffix maxima.  ex is an LDS array of kE values of type T
// used for the two neighbour exchanges.  Returns the owned positions equal to their
// opening (and allowed by selm); *eq_all receives the same bits for any thread.
template <int W, typename T>
__device__ __forceinline__ uint32_t select_reg(const T (&v)[16], uint32_t selm, uint32_t winm,
                                               T *ex, bool owner, uint32_t *eq_all = nullptr)
{
    constexpr T kTop = ~T(0);
    const int t = threadIdx.x;
    T P[16], S[16], mw[16];
    P[0] = v[0];
#pragma unroll
    for (int u = 1; u < 16; u++) P[u] = min(P[u - 1], v[u]);
#pragma unroll
    for (int u = 0; u < W - 1; u++) ex[u * kSkBlock + t] = P[u];
    __syncthreads();
    T Pn[W > 1 ? W - 1 : 1];
#pragma unroll
    for (int u = 0; u < W - 1; u++) Pn[u] = t + 1 < kSkBlock ? ex[u * kSkBlock + t + 1] : kTop;
    __syncthreads();
    S[15] = v[15];
#pragma unroll
    for (int u = 14; u >= 0; u--) S[u] = min(S[u + 1], v[u]);
    // windows reaching into the next chunk
#pragma unroll
    for (int s = (17 - W > 0 ? 17 - W : 0); s < 16; s++) mw[s] = W == 1 ? v[s] : min(S[s], Pn[s + W - 1 - 16]);
    // windows inside the chunk (none when W == 17)
    if constexpr (W >= 9 && W <= 16) {
        constexpr int m = 16 - W;               // contained in every inner window
        T SA[m + 1], PB[16];
        SA[m] = v[m];
#pragma unroll
        for (int s = m - 1; s >= 0; s--) SA[s] = min(SA[s + 1], v[s]);
        PB[m + 1] = v[m + 1];
#pragma unroll
        for (int e = m + 2; e < 16; e++) PB[e] = min(PB[e - 1], v[e]);
#pragma unroll
        for (int s = 0; s <= m; s++) mw[s] = min(SA[s], PB[s + W - 1]);
    } else if constexpr (W <= 8) {
#pragma unroll
        for (int s = 0; s <= 16 - W; s++) {
            T x = v[s];
#pragma unroll
            for (int d = 1; d < W; d++) x = min(x, v[s + d]);
            mw[s] = x;
        }
    }
    if (__ballot(winm != 0xFFFFu) != 0) {       // skipped by waves whose windows are all valid
#pragma unroll
        for (int s = 0; s < 16; s++) mw[s] = ((winm >> s) & 1u) ? mw[s] : T(0);
    }

    // opening
    T SM[16], PM[16], op[16];
    SM[15] = mw[15];
#pragma unroll
    for (int u = 14; u >= 0; u--) SM[u] = max(SM[u + 1], mw[u]);
#pragma unroll
    for (int u = 17 - W; u < 16; u++) ex[u * kSkBlock + t] = SM[u];
    __syncthreads();
    T Sp[W > 1 ? W - 1 : 1];
#pragma unroll
    for (int j = 0; j < W - 1; j++) Sp[j] = t > 0 ? ex[(17 - W + j) * kSkBlock + t - 1] : T(0);
    PM[0] = mw[0];
#pragma unroll
    for (int u = 1; u < 16; u++) PM[u] = max(PM[u - 1], mw[u]);
#pragma unroll
    for (int u = 0; u < (W - 1 < 16 ? W - 1 : 16); u++) op[u] = max(PM[u], Sp[u]);
    if constexpr (W >= 9 && W <= 16) {
        constexpr int m = W - 1;                // contained in every inner range
        T SA[m + 1], PB[16];
        SA[m] = mw[m];
#pragma unroll
        for (int s = m - 1; s >= 0; s--) SA[s] = max(SA[s + 1], mw[s]);
        if constexpr (m < 16) op[m] = SA[0];
        if constexpr (m + 1 < 16) {
            PB[m + 1] = mw[m + 1];
#pragma unroll
            for (int e = m + 2; e < 16; e++) PB[e] = max(PB[e - 1], mw[e]);
#pragma unroll
            for (int u = m + 1; u < 16; u++) op[u] = max(SA[u - W + 1], PB[u]);
        }
    } else if constexpr (W <= 8) {
#pragma unroll
        for (int u = (W - 1 > 0 ? W - 1 : 0); u < 16; u++) {
            T x = mw[u];
#pragma unroll
            for (int d = 1; d < W; d++) x = max(x, mw[u - d]);
            op[u] = x;
        }
    }
    uint32_t eq = 0;
#pragma unroll
    for (int u = 0; u < 16; u++) eq |= (v[u] == op[u] ? 1u : 0u) << u;
    eq &= selm;
    if (eq_all) *eq_all = eq;
    return owner ? eq : 0u;
}

// Any w: window minima and the opening by doubling in LDS (ex holds kE words).
__device__ uint32_t select_lds(const uint64_t (&v)[16], uint32_t selm, uint32_t winm, uint64_t *ex,
                               int w, bool owner)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 16; u++) ex[16 * t + u] = v[u];
    __syncthreads();
    int q2 = 1;                       // largest power of two <= w
    while (q2 * 2 <= w) q2 *= 2;
    const int r2 = w - q2;
    for (int d = 1; d < q2; d *= 2) {
        uint64_t x[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int i = 16 * t + u;
            x[u] = min(ex[i], i + d < kE ? ex[i + d] : kMax64);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) ex[16 * t + u] = x[u];
        __syncthreads();
    }
    {
        uint64_t x[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int i = 16 * t + u;
            x[u] = ((winm >> u) & 1u) ? min(ex[i], i + r2 < kE ? ex[i + r2] : kMax64) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) ex[16 * t + u] = x[u];
        __syncthreads();
    }
    for (int d = 1; d < q2; d *= 2) {
        uint64_t x[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int i = 16 * t + u;
            x[u] = max(ex[i], i - d >= 0 ? ex[i - d] : 0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) ex[16 * t + u] = x[u];
        __syncthreads();
    }
    uint32_t sel = 0;
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int i = 16 * t + u;
        const uint64_t opened = max(ex[i], i - r2 >= 0 ? ex[i - r2] : 0);
        if (owner && ((selm >> u) & 1u) && v[u] == opened) sel |= 1u << u;
    }
    return sel;
}

// N bits of the patterned stream read from the mask in memory.
struct MemN {
    const uint32_t *pnw;
    __device__ __forceinline__ bool at(uint64_t c) const { return (pnw[c >> 5] >> (c & 31)) & 1u; }
    __device__ __forceinline__ uint64_t first(uint64_t a, uint64_t b) const
    {
        return first_n(pnw, a, b);
    }
    __device__ __forceinline__ uint64_t after_last(uint64_t a, uint64_t b) const
    {
        return after_last_n(pnw, a, b);
    }
};

// N bits of positions [jc - 64, jc + 64) held in two registers (Y below jc, X from jc):
// the run loop then waits on no load.  Valid for the queries it makes when L <= 48.
struct RegN {
    uint64_t X, Y;
    uint64_t jc;
    __device__ __forceinline__ bool at(uint64_t c) const { return (X >> (c - jc)) & 1u; }
    // first N in [a, b), a >= jc, b <= jc + 64
    __device__ __forceinline__ uint64_t first(uint64_t a, uint64_t b) const
    {
        if (b <= a) return b;
        uint64_t m = X >> (a - jc);
        if (b - a < 64) m &= (1ull << (b - a)) - 1;
        return m ? a + (uint64_t)__builtin_ctzll(m) : b;
    }
    // one past the last N in [a, b), b == jc, jc - a <= 64
    __device__ __forceinline__ uint64_t after_last(uint64_t a, uint64_t b) const
    {
        if (b <= a) return a;
        const uint64_t m = Y >> (64 - (b - a));          // bit i: position a + i
        return m ? a + 64 - (uint64_t)__builtin_clzll(m) : a;
    }
};

// Masks of a chunk near an N (kv: the k-mer fits, wv: a window starts, okm: the position
// lies in a run long enough for one window): with ambiguous bases the runs between Ns
// within a sequence play the part of sequences.  A run's start before jc - L or its end
// beyond jc + 16 + L changes no mask, so the searches stop there.
template <typename NB>
__device__ __forceinline__ void run_masks(const NB &nb, const SeqCache &C, int64_t jc,
                                          uint32_t seq, uint64_t seq_beg, uint64_t seq_end,
                                          uint64_t np, int k, uint64_t L, uint32_t &kv,
                                          uint32_t &wv, uint32_t &okm)
{
    uint64_t c = (uint64_t)jc;
    uint32_t s = seq;
    uint64_t sb = seq_beg, se = seq_end;
    const uint64_t far = (uint64_t)jc + 16 + L;
    while (c < (uint64_t)jc + 16 && c < np) {
        if (c >= se) {
            s++;
            sb = se;
            se = C.at(s + 1);
            continue;
        }
        if (nb.at(c)) {                                  // an N: in no run
            c++;
            continue;
        }
        uint64_t b = c;
        if (c == (uint64_t)jc && c > sb) {
            const uint64_t lo = (uint64_t)jc - sb > L ? (uint64_t)jc - L : sb;
            b = nb.after_last(lo, c);
        }
        const uint64_t e = nb.first(c, se < far ? se : far);
        const int lo = (int)(c - (uint64_t)jc);
        const int hi = e - (uint64_t)jc >= 16 ? 16 : (int)(e - (uint64_t)jc);
        const uint32_t span = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
        kv |= span & mask_le((int64_t)e - (int64_t)k - jc);
        wv |= span & mask_le((int64_t)e - (int64_t)L - jc);
        if (e - b >= L) okm |= span;
        c = e;
    }
}

// One tile: the T positions [tile*T, tile*T + T) of the batch's patterned stream.
template <int W, int HK>
__device__ __forceinline__ void sketch_tile(const SketchArgs &A, uint64_t tile, uint64_t np,
                                            uint64_t n_tiles, uint64_t *ex, uint64_t *sh_scan,
                                            uint64_t *sh_misc, const SeqCache &C,
                                            const uint8_t *ones, uint32_t w0, uint32_t w1,
                                            uint32_t w2)
{
    const int t = threadIdx.x;
    const int H = A.H, T = A.T, w = W > 0 ? W : A.w, k = A.k;

    const int64_t j0 = (int64_t)(tile * (uint64_t)T);
    const int64_t jc = j0 - H + 16 * t;                  // first position of this chunk

    // ---- stage 1: canonical k-mer hashes and flags of the 16 positions of the chunk.
    // hv = hash (kMax64 where there is no k-mer or it is a palindrome); bit u of selm:
    // position u may be selected, of winm: a valid window starts there, of smask: strand.
    uint64_t hv[16];
    uint32_t selm = 0, winm = 0, smask = 0;   // bit u: may be selected / window starts / strand
#pragma unroll
    for (int u = 0; u < 16; u++) hv[u] = kMax64;
    uint32_t seq0 = 0;
    uint64_t beg0 = 0, end0 = 0;
    if (jc >= 0 && (uint64_t)jc < np) {
        uint32_t seq = C.find((uint64_t)jc);
        uint64_t seq_beg = C.at(seq), seq_end = C.at(seq + 1);
        while ((uint64_t)jc >= seq_end) { seq++; seq_beg = seq_end; seq_end = C.at(seq + 1); }
        seq0 = seq; beg0 = seq_beg; end0 = seq_end;
        // an N within k + w - 1 positions of the chunk needs the run-aware masks below
        const uint64_t L = (uint64_t)(k + w - 1);
        bool n_near = false;
        if (A.pnw) {
            const uint64_t lo = (uint64_t)jc > L ? (uint64_t)jc - L : 0;
            const uint64_t hi = (uint64_t)jc + 16 + L < np ? (uint64_t)jc + 16 + L : np;
            n_near = any_n(A.pnw, lo, hi);
        }
        const uint32_t mw0 = msb_first(w0), mw1 = msb_first(w1), mw2 = msb_first(w2);
        const int fsh = 64 - 2 * k;
        // every position of the chunk has its k-mer and a valid window in one sequence
        // (and, with ambiguous bases, no N among the bases those windows cover)
        bool interior = (uint64_t)jc + 16 + (uint64_t)(k + w - 2) <= seq_end &&
                        seq_end - seq_beg >= L;
        if (interior && n_near)
            interior = first_n(A.pnw, (uint64_t)jc, (uint64_t)jc + 15 + L) == (uint64_t)jc + 15 + L;
        // One path per wave: the masked path below is exact for interior chunks too, and a
        // wave whose lanes split between the two would execute both.
        interior = __ballot(!interior) == 0;
        if (interior && (k & 1)) {
            // odd k: a k-mer never equals its reverse complement
            selm = winm = 0xFFFFu;
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const uint64_t X = kmer_lsb(w0, w1, w2, u);
                const uint64_t F = kmer_msb(mw0, mw1, mw2, u);
                const uint64_t rc = (~X) & A.kmask;
                const uint64_t fwd = F >> fsh;
                const bool strand = rc < fwd;
                hv[u] = kmer_hash<HK>(strand ? rc : fwd, A.kmask);
                smask |= (strand ? 1u : 0u) << u;
            }
        } else if (interior) {
            winm = 0xFFFFu;
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const uint64_t X = kmer_lsb(w0, w1, w2, u);
                const uint64_t F = kmer_msb(mw0, mw1, mw2, u);
                const uint64_t rc = (~X) & A.kmask;
                const uint64_t fwd = F >> fsh;
                const bool strand = rc < fwd;
                const uint64_t h = kmer_hash<HK>(strand ? rc : fwd, A.kmask);
                const bool pal = fwd == rc;
                hv[u] = pal ? kMax64 : h;
                selm |= (pal ? 0u : 1u) << u;
                smask |= (strand ? 1u : 0u) << u;
            }
        } else {
            // The chunk meets a sequence end (reads put one into most chunks): bit masks of
            // the positions whose k-mer (kv) and window (wv) fit in their sequence and of
            // those in sequences long enough for one full window (okm), one run of the
            // loop per sequence overlapping the chunk; then all 16 positions are hashed
            // as in the interior and masked, without per-position branches.
            uint32_t kv = 0, wv = 0, okm = 0;
            // the N-aware masks are exact without an N too: one branch per wave
            n_near = __ballot(n_near) != 0;
            if (n_near && L <= 48) {
                // N bits of [jc - 64, jc + 64) from five words loaded at once
                const int64_t q0 = jc >> 5;
                const uint32_t sh = (uint32_t)(jc & 31);
                uint32_t nw[5];
#pragma unroll
                for (int i = 0; i < 5; i++) nw[i] = q0 - 2 + i >= 0 ? A.pnw[q0 - 2 + i] : 0u;
                RegN nb;
                nb.jc = (uint64_t)jc;
                nb.Y = ((uint64_t)__builtin_amdgcn_alignbit(nw[2], nw[1], sh) << 32) |
                       __builtin_amdgcn_alignbit(nw[1], nw[0], sh);
                nb.X = ((uint64_t)__builtin_amdgcn_alignbit(nw[4], nw[3], sh) << 32) |
                       __builtin_amdgcn_alignbit(nw[3], nw[2], sh);
                run_masks(nb, C, jc, seq, seq_beg, seq_end, np, k, L, kv, wv, okm);
            } else if (n_near) {
                MemN nb{A.pnw};
                run_masks(nb, C, jc, seq, seq_beg, seq_end, np, k, L, kv, wv, okm);
            } else {
                uint64_t b = seq_beg, e = seq_end;
                uint32_t s = seq;
                int lo = 0;
                while (true) {
                    const int hi = e - (uint64_t)jc >= 16 ? 16 : (int)(e - (uint64_t)jc);
                    const uint32_t span = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                    kv |= span & mask_le((int64_t)e - (int64_t)k - jc);
                    wv |= span & mask_le((int64_t)e - (int64_t)(k + w - 1) - jc);
                    if (e - b >= (uint64_t)(k + w - 1)) okm |= span;
                    if (hi >= 16 || e >= np) break;
                    s++;
                    b = e;
                    e = C.at(s + 1);
                    lo = hi;
                }
            }
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const uint64_t X = kmer_lsb(w0, w1, w2, u);
                const uint64_t F = kmer_msb(mw0, mw1, mw2, u);
                const uint64_t rc = (~X) & A.kmask;
                const uint64_t fwd = F >> fsh;
                const bool strand = rc < fwd;
                const uint64_t h = kmer_hash<HK>(strand ? rc : fwd, A.kmask);
                const bool use = ((kv >> u) & 1u) && !((k & 1) == 0 && fwd == rc);
                hv[u] = use ? h : kMax64;
                selm |= (use ? 1u : 0u) << u;
                smask |= (strand ? 1u : 0u) << u;
            }
            selm &= okm;
            winm = wv;
        }
    }

    // ---- stage 2: minimizer selection (window minima, then the opening).
    // For w = 3..17 the reductions first run on the hashes' high 32-bit words (one 32-bit
    // min or max per step instead of a 64-bit compare and two selects).  A k-mer equal to
    // the minimum of a window also has the smallest high word of that window, so every
    // minimizer is selected, and a k-mer is selected wrongly only if, in some window, two
    // positions share the smallest high word with different hashes.  Then two positions
    // that are consecutive among the selected ones lie in that window with equal high
    // words and different hashes (no selected position can lie between two positions of
    // a window that attain its smallest high word).  Such a pair is either two consecutive
    // owned records of this tile or the tile's first owned record and the last position of
    // the chunk before the owned range that the same rule selects there (with fewer
    // windows in view it selects a subset, which still holds the pair).  The tile checks
    // every such pair on its compacted records; if one matches, or the records do not fit
    // the exchange array, it selects again on the full hashes.
    const bool owner = 16 * t >= H && 16 * t < H + T;
    const int vbytes = A.val_mode == VAL_SEQ64 ? 8 : 4;
    uint32_t sel = 0;
    uint64_t total = 0, excl = 0;
    bool staged = false;
    // exclusive record offset of this thread, the tile's count, whether it is staged
    auto count = [&]() {
        uint32_t tot32;
        excl = block_excl_scan<uint32_t, kSkBlock>((uint32_t)__popc(sel), (uint32_t *)sh_scan,
                                                   &tot32);
        total = tot32;
        staged = total * (uint64_t)(8 + vbytes) <= (uint64_t)kE * 8;     // workgroup-uniform
    };
    // the selected hashes, compacted in position order into the exchange array
    auto compact = [&]() {
        uint32_t loc = (uint32_t)excl;
#pragma unroll
        for (int u = 0; u < 16; u++)
            if ((sel >> u) & 1u) ex[loc++] = hv[u];
    };
    bool full = true;
    if constexpr (W >= 3) {
        uint32_t hi[16];
#pragma unroll
        for (int u = 0; u < 16; u++) hi[u] = (uint32_t)(hv[u] >> 32);
        uint32_t eq_all;
        sel = select_reg<W, uint32_t>(hi, selm, winm, (uint32_t *)ex, owner, &eq_all);
        if (t == H / 16 - 1) {                     // the chunk before the owned range
            uint64_t last = 0;
#pragma unroll
            for (int u = 0; u < 16; u++)
                if ((eq_all >> u) & 1u) last = hv[u];
            sh_misc[1] = last;
            sh_misc[2] = eq_all != 0;
        }
        count();                                   // its barriers publish sh_misc
        bool bad = !staged;
        if (staged) {
            compact();
            __syncthreads();
            for (uint32_t i = t; i < (uint32_t)total; i += kSkBlock) {
                const uint64_t cur = ex[i];
                const uint64_t prev = i > 0 ? ex[i - 1] : sh_misc[1];
                const bool has = i > 0 || sh_misc[2] != 0;
                if (has && (cur >> 32) == (prev >> 32) && cur != prev) bad = true;
            }
        }
        full = __syncthreads_or(bad) != 0;
    }
    if (full) {
        if constexpr (W > 0) sel = select_reg<W, uint64_t>(hv, selm, winm, ex, owner);
        else sel = select_lds(hv, selm, winm, ex, w, owner);
        count();
        if (staged) compact();
    }

    // The records of this thread's selected positions: their values (and, when the tile
    // is not staged, their keys) go out in position order.  A staged tile writes values to
    // the exchange array only, so it needs no tile base and runs before the look-back
    // finishes.
    uint32_t *sv32 = (uint32_t *)(ex + total);          // staged values, after the keys
    uint64_t *sv64 = ex + total;
    auto records = [&](uint64_t tile_base) {
        // The original coordinate of patterned position li of a sequence is
        // (li / x) * p + phase(li % x); the division is done once per chunk (or per
        // sequence start) and then advanced by small offsets with a reciprocal multiply.
        uint32_t seq = seq0;
        uint64_t seq_beg = beg0, seq_end = end0;
        uint32_t a = seq_shift(A.shift, A.uniform, seq);
        if (a >= A.P.p) a = 0;
        uint32_t front = kept_front(A.P, a);
        // original offset of the sequence (global positions only), reloaded per sequence
        uint64_t obase = A.val_mode == VAL_GLOBAL32 ? A.offsets[seq] : 0;
        uint64_t per0;
        uint32_t r0;
        div_x((uint64_t)jc - seq_beg, A.P.x, A.inv_x, &per0, &r0);
        uint64_t jb = (uint64_t)jc;                // position whose rank is (per0, r0)
        const uint32_t magic = (65536u + A.P.x - 1) / A.P.x;
        uint64_t idx = excl;                       // record index within the tile
        uint32_t bits = sel;
        while (bits) {
            const int u = __ffs(bits) - 1;
            bits &= bits - 1;
            const uint64_t j = (uint64_t)jc + u;
            if (j >= seq_end) {
                while (j >= seq_end) { seq++; seq_beg = seq_end; seq_end = C.at(seq + 1); }
                a = seq_shift(A.shift, A.uniform, seq);
                if (a >= A.P.p) a = 0;
                front = kept_front(A.P, a);
                if (A.val_mode == VAL_GLOBAL32) obase = A.offsets[seq];
                per0 = 0;
                r0 = 0;
                jb = seq_beg;
            }
            const uint32_t rr = r0 + (uint32_t)(j - jb);          // < x + 16
            const uint32_t q = (rr * magic) >> 16;
            // offset in the period of kept phase r under shift a (ones[] in LDS)
            uint32_t oi = rr - q * A.P.x + front;
            if (oi >= A.P.x) oi -= A.P.x;
            uint32_t ph = ones[oi] + a;
            if (ph >= A.P.p) ph -= A.P.p;
            const uint64_t local = (per0 + q) * A.P.p + ph;
            const uint32_t strand = (smask >> u) & 1u;
            if (A.val_mode == VAL_SEQ64) {
                if (local >= (1ull << 31)) set_status(A.status, 2u);
                const uint64_t v = ((uint64_t)seq << 32) | (local << 1) | strand;
                if (staged) {
                    sv64[idx] = v;
                } else if (tile_base + idx < A.capacity) {
                    A.keys[tile_base + idx] = ex[u * kSkBlock + t];
                    ((uint64_t *)A.vals)[tile_base + idx] = v;
                }
            } else {
                const uint64_t pos = obase + local;
                if (pos >= (1ull << 31)) set_status(A.status, 2u);
                const uint32_t v = (uint32_t)((pos << 1) | strand);
                if (staged) {
                    sv32[idx] = v;
                } else if (tile_base + idx < A.capacity) {
                    A.keys[tile_base + idx] = ex[u * kSkBlock + t];
                    ((uint32_t *)A.vals)[tile_base + idx] = v;
                }
            }
            idx++;
        }
    };

    // ---- stage 3: position-ordered compaction across tiles (decoupled look-back)
    // Wave 0 publishes this tile's aggregate, then looks back over 64 predecessors per
    // step: it adds every aggregate up to the nearest tile that already carries its
    // inclusive prefix, and waits only while one of the tiles in between has not
    // published yet.  The flag and the value share one 64-bit word, so relaxed atomics
    // suffice (no other data of a predecessor is read).
    if (t < kWave) {
        uint64_t before = 0;
        if (t == 0)
            __hip_atomic_store(&A.tile_state[tile], (tile == 0 ? kFlagP : kFlagA) | total,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t end = (int64_t)tile - 1;          // newest predecessor not yet added
        while (end >= 0) {
            const int64_t idx = end - t;
            const uint64_t st = idx >= 0 ? __hip_atomic_load(&A.tile_state[idx], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                                         : kFlagP;
            const uint64_t f = st & ~kValMask;
            const uint64_t pmask = __ballot(f == kFlagP);
            const uint64_t zmask = __ballot(f == 0);
            const int first_p = pmask ? __ffsll((unsigned long long)pmask) - 1 : kWave;
            const int first_z = zmask ? __ffsll((unsigned long long)zmask) - 1 : kWave;
            if (first_z < first_p) {              // a nearer predecessor is not ready yet
                __builtin_amdgcn_s_sleep(2);
                continue;
            }
            uint64_t v = t <= first_p ? (st & kValMask) : 0;
            v = wave_sum<uint64_t>(v);
            before += v;
            if (first_p < kWave) break;
            end -= kWave;
        }
        if (t == 0) {
            if (tile != 0)
                __hip_atomic_store(&A.tile_state[tile], kFlagP | (before + total),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh_misc[0] = before;
            if (tile == n_tiles - 1) {
                if (A.n_out) *A.n_out = before + total;
                if (before + total > A.capacity) set_status(A.status, 1u);
            }
        }
    }
    // waves 1-3 fill in their staged values while wave 0 looks back
    if (staged && owner && (uint64_t)jc <= np && sel != 0) records(0);
    // Records leave the tile in position order.  When they fit in the exchange array
    // (12 or 16 bytes each, which every tile does unless w is tiny or the sequence is of
    // low complexity), the keys were compacted there straight from registers, the values
    // go after them, and the workgroup then writes the tile's contiguous record range
    // with coalesced stores; otherwise the hashes go to LDS by position and each thread
    // writes its own records.  Every read of the exchange array by the selection
    // finished before the scan's barriers.
    if (!staged) {
#pragma unroll
        for (int u = 0; u < 16; u++) ex[u * kSkBlock + t] = hv[u];
    }
    __syncthreads();
    const uint64_t tile_base = sh_misc[0];
    const uint64_t base = tile_base + excl;

    if (owner && (uint64_t)jc <= np) {
        // per-sequence record offsets of the sequences that start inside this chunk
        if (A.mz_offsets) {
            uint32_t s = (uint64_t)jc < np ? seq0 : first_ge(A.pofs, A.n_seq, (uint64_t)jc);
            while (s > 0 && C.at(s - 1) >= (uint64_t)jc) s--;       // empty sequences
            while (s <= A.n_seq && C.at(s) < (uint64_t)jc) s++;
            while (s <= A.n_seq && C.at(s) < (uint64_t)jc + 16) {
                const uint32_t below = (uint32_t)(C.at(s) - (uint64_t)jc);
                A.mz_offsets[s] = base + __popc(sel & ((1u << below) - 1u));
                s++;
            }
        }
        if (!staged && sel != 0) records(tile_base);
    }
    if (staged) {
        __syncthreads();
        const uint64_t n = tile_base + total <= A.capacity
                               ? total
                               : (tile_base < A.capacity ? A.capacity - tile_base : 0);
        if (A.val_mode == VAL_SEQ64) {
            for (uint64_t i = t; i < n; i += kSkBlock) {
                A.keys[tile_base + i] = ex[i];
                ((uint64_t *)A.vals)[tile_base + i] = sv64[i];
            }
        } else {
            for (uint64_t i = t; i < n; i += kSkBlock) {
                A.keys[tile_base + i] = ex[i];
                ((uint32_t *)A.vals)[tile_base + i] = sv32[i];
            }
        }
    }
}

template <int W, int HK>
__global__ __launch_bounds__(kSkBlock) void k_sketch(SketchArgs A)
{
    __shared__ uint64_t ex[kE];       // neighbour exchange / sliding-reduction work array
    __shared__ uint64_t sh_scan[kSkBlock / kWave];
    __shared__ uint64_t sh_misc[3];   // tile base; key and flag of the record before the tile
    __shared__ uint32_t sh_tile;
    __shared__ uint64_t sh_pofs[kSeqCache];
    __shared__ uint8_t sh_ones[kMaxPattern];   // the pattern's kept offsets, read per record

    const uint64_t np = A.pofs[A.n_seq];
    const uint64_t n_tiles = np / (uint64_t)A.T + 1;    // the last tile covers position np
    // tiles are numbered in the order workgroups start, so every predecessor a tile looks
    // back on is already running
    if (threadIdx.x == 0) sh_tile = atomicAdd(A.tile_counter, 1u);
    for (uint32_t i = threadIdx.x; i < A.P.x; i += kSkBlock) sh_ones[i] = A.P.ones[i];
    __syncthreads();
    const uint64_t tile = sh_tile;
    if (tile >= n_tiles) return;
    // the chunk's three stream words (the 16 positions and the 32 after them), loaded
    // before the sequence cache so that the two loads' latencies overlap (unconditionally,
    // from word 0 for chunks outside the stream, whose words are never used: a load under
    // a branch is waited for at the branch's end)
    const int64_t jc = (int64_t)(tile * (uint64_t)A.T) - A.H + 16 * (int64_t)threadIdx.x;
    const size_t wi = jc >= 0 && (uint64_t)jc < np ? (size_t)jc / 16 : 0;
    const uint32_t w0 = A.psw[wi], w1 = A.psw[wi + 1], w2 = A.psw[wi + 2];
    const SeqCache C = seq_cache(A.pofs, A.n_seq, A.lohi, tile, sh_pofs);
    sketch_tile<W, HK>(A, tile, np, n_tiles, ex, sh_scan, sh_misc, C, sh_ones, w0, w1, w2);
}

}  // namespace

hipError_t launch_kept(const Batch &b, const Pattern &P, const uint32_t *shift,
                       uint32_t uniform_shift, uint64_t *kept, uint32_t *status, hipStream_t s)
{
    if (b.n_seq == 0) return hipSuccess;
    const unsigned blocks = (b.n_seq + kBlock - 1) / kBlock;
    GD_LAUNCH(k_kept, dim3(blocks), dim3(kBlock), 0, s, b.offsets, b.n_seq, P, shift,
                       uniform_shift, kept, status);
    return hipGetLastError();
}

hipError_t launch_window_ranges(const uint64_t *pofs, uint32_t n_seq, size_t words,
                                uint64_t np_bound, int w, uint32_t *lohi_sp, uint32_t *lohi_sk,
                                hipStream_t s)
{
    const size_t blocks = sparsify_blocks(words);
    const TileGeom g = tile_geom(w);
    const size_t tiles = sketch_tiles_bound(np_bound, w);
    const size_t count = blocks > tiles ? blocks : tiles;
    GD_LAUNCH(k_window_seqs2, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
              pofs, n_seq, (uint64_t)blocks, lohi_sp, (uint64_t)g.T, (uint64_t)g.H,
              (uint64_t)tiles, lohi_sk);
    return hipGetLastError();
}

hipError_t launch_sparsify(const Batch &b, const Pattern &P, const uint32_t *shift,
                           uint32_t uniform_shift, const uint64_t *pofs, uint32_t *psw,
                           uint32_t *pnw, size_t words, uint32_t *lohi, bool ranges_ready,
                           hipStream_t s)
{
    const size_t blocks = sparsify_blocks(words);
    if (blocks == 0) return hipSuccess;
    if (!ranges_ready)
        GD_LAUNCH(k_window_seqs, dim3((unsigned)((blocks + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                  s, pofs, b.n_seq, kSpSpan, (uint64_t)0, kSpSpan - 1, (uint64_t)blocks, lohi);
    // 16 consecutive kept bases lie in at most ceil(15/x) + 1 periods; with that span
    // <= 48 bases every base of a word's segment is inside a 64-base window that starts
    // at most 15 bases before the segment's first kept base
    const int compact = (int)(((15 + P.x - 1) / P.x + 1) * P.p <= 48);
    GD_LAUNCH(k_sparsify, dim3((unsigned)blocks), dim3(kBlock), 0, s, b.bases, b.offsets,
              b.n_seq, P, shift, uniform_shift, pofs, psw, words, (b.n_bases + 3) / 4, compact,
              1.0 / (double)P.x, (const uint32_t *)lohi);
    if (b.nmask && pnw)
        GD_LAUNCH(k_sparsify_n, dim3((unsigned)blocks), dim3(kBlock), 0, s, b.nmask, b.offsets,
                  b.n_seq, P, shift, uniform_shift, pofs, (uint16_t *)pnw, words,
                  1.0 / (double)P.x, (const uint32_t *)lohi, (b.n_bases + 31) / 32);
    return hipGetLastError();
}

hipError_t launch_pack_ascii(const char *text, uint64_t n, uint32_t *bases, uint16_t *nmask,
                             hipStream_t s)
{
    const size_t words = (size_t)((n + 63) / 64) * 4;
    const size_t blocks = (words + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    GD_LAUNCH(k_pack_ascii, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const uint8_t *)text, n,
              bases, nmask, words, (int)(((uintptr_t)text & 15) == 0));
    return hipGetLastError();
}

hipError_t launch_sketch(const Batch &b, const Pattern &P, const uint32_t *shift,
                         uint32_t uniform_shift, const uint64_t *pofs, const uint32_t *psw,
                         const uint32_t *pnw, uint64_t np_bound, int k, int w, int hash,
                         const SketchOut &o, uint64_t *tile_state, uint32_t *lohi,
                         bool ranges_ready, uint32_t *status, hipStream_t s)
{
    const TileGeom g = tile_geom(w);
    const size_t tiles = sketch_tiles_bound(np_bound, w);
    // tile states and, in the word after them, the tile ticket counter: one fill
    hipError_t e = fill_u64(tile_state, 0, tiles + 1, s);
    if (e != hipSuccess) return e;
    uint32_t *tile_counter = (uint32_t *)(tile_state + tiles);
    // tile t covers [t*T - H, t*T + T + H + 48] (the last 48 for the record loop's lookups)
    if (!ranges_ready)
        GD_LAUNCH(k_window_seqs, dim3((unsigned)((tiles + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                  s, pofs, b.n_seq, (uint64_t)g.T, (uint64_t)g.H, (uint64_t)(g.T + 2 * g.H + 48),
                  (uint64_t)tiles, lohi);
    SketchArgs A;
    A.psw = psw;
    A.pnw = pnw;
    A.pofs = pofs;
    A.offsets = b.offsets;
    A.shift = shift;
    A.uniform = uniform_shift;
    A.n_seq = b.n_seq;
    A.P = P;
    A.k = k;
    A.w = w;
    A.H = g.H;
    A.T = g.T;
    A.kmask = k == 32 ? kMax64 : ((1ull << (2 * k)) - 1);
    A.keys = o.keys;
    A.vals = o.vals;
    A.val_mode = o.val_mode;
    A.mz_offsets = o.mz_offsets;
    A.capacity = o.capacity;
    A.n_out = o.n_out;
    A.tile_state = tile_state;
    A.lohi = lohi;
    A.tile_counter = tile_counter;
    A.status = status;
    A.inv_x = 1.0 / (double)P.x;
    const size_t grid = tiles;
    if (hash == 0 && k == 32) {
        // splitmix64 of full 64-bit codes: the general selection path (k = 32 is rare)
        GD_LAUNCH((k_sketch<0, 2>), dim3((unsigned)grid), dim3(kSkBlock), 0, s, A);
        return hipGetLastError();
    }
    switch (w) {
#define GD_W(n)                                                                             \
    case n:                                                                                 \
        if (hash == 1) GD_LAUNCH((k_sketch<n, 1>), dim3((unsigned)grid), dim3(kSkBlock), 0, s, A); \
        else GD_LAUNCH((k_sketch<n, 0>), dim3((unsigned)grid), dim3(kSkBlock), 0, s, A);          \
        break;
        GD_W(2) GD_W(3) GD_W(4) GD_W(5) GD_W(6) GD_W(7) GD_W(8) GD_W(9) GD_W(10) GD_W(11)
        GD_W(12) GD_W(13) GD_W(14) GD_W(15) GD_W(16) GD_W(17)
#undef GD_W
    default:
        if (hash == 1) GD_LAUNCH((k_sketch<0, 1>), dim3((unsigned)grid), dim3(kSkBlock), 0, s, A);
        else GD_LAUNCH((k_sketch<0, 0>), dim3((unsigned)grid), dim3(kSkBlock), 0, s, A);
        break;
    }
    return hipGetLastError();
}

}  // namespace gd
