// Seed-matching experiment of Section 2.1.1 (Fig. 4) on gfx950: pairs of a sequence and
// a copy with substitutions, seeded four ways, their edit distance, and the number of
// accepted pairs per edit-distance threshold (Section 2.1.2).
//
//  * k_seed_match: one workgroup per pair.  Both sequences (at most 1,024 bases each)
//    are unpacked into LDS; for each algorithm the original's seeds are built in LDS and
//    inserted into an LDS hash set (2,048 slots, linear probing, 64-bit compare-and-swap),
//    then the copy's seeds are built and each one probes the set.  Minimizer selection
//    marks, for every full window, the positions that attain its minimum (all ties), as
//    the sketch does.
//  * k_edit_distance: one thread per pair, the bit-vector form of the edit-distance
//    recurrence (Myers 1999, in Hyyrö's 2003 formulation for Levenshtein distance) over
//    16 words of 64 rows, with the per-letter match masks in LDS.
//  * accepted pairs: a matching rate m/t becomes the integer floor(m * 2^32 / t), which
//    orders rates exactly while totals stay below 2^16; per-distance minima by atomic
//    min, a prefix minimum over distances, then every pair adds one to the first
//    distance threshold it passes (counted in LDS per workgroup, then added to the global
//    counts) and a prefix sum gives the counts.
#include "gd_internal.h"

namespace gd {

namespace {

constexpr int kFig4MaxLen = 1024;     // bases per sequence of a pair
constexpr int kSetSlots = 2048;       // LDS hash-set slots (load <= 1/2)
static_assert(4 * kBlock >= kFig4MaxLen, "4 k-mers per thread cover a sequence");
constexpr uint64_t kEmpty = ~0ull;    // an empty slot; the key ~0 itself is kept aside
constexpr int kEdBlock = 64;          // threads per workgroup of k_edit_distance
constexpr int kEdWords = kFig4MaxLen / 64;

__device__ __forceinline__ uint32_t base_of(const uint8_t *bases, uint64_t g)
{
    return (bases[g >> 2] >> ((g & 3) * 2)) & 3u;
}

struct MatchArgs {
    const uint8_t *ba, *bb;
    const uint64_t *oa, *ob;
    uint32_t n_pairs;
    Pattern P;
    int k, w;
    uint64_t kmask;
    uint32_t spaced;      // bit j: offset j of a k-span takes part in a spaced seed
    uint32_t *counts;
    uint32_t *status;
};

struct MatchLds {
    uint8_t sa[kFig4MaxLen], sb[kFig4MaxLen], ps[kFig4MaxLen];
    uint8_t use[kFig4MaxLen], sel[kFig4MaxLen];
    unsigned long long set[kSetSlots];
    uint64_t kb[kFig4MaxLen], hv[kFig4MaxLen];
    uint32_t n;
    uint32_t has_max;       // the original has a seed equal to kEmpty
    uint32_t red[kBlock / kWave];
};

// Canonical code of the bases s[i + j] for the offsets j < k whose bit is set in sel.
__device__ __forceinline__ uint64_t canon_at(const uint8_t *s, int i, int k, uint32_t sel)
{
    uint64_t f = 0, r = 0;
    int n = 0;
    for (int j = 0; j < k; j++) {
        if (!((sel >> j) & 1u)) continue;
        const uint64_t b = s[i + j];
        f = (f << 2) | b;
        r |= (3ull - b) << (2 * n);
        n++;
    }
    return f < r ? f : r;
}

// Forward and reverse-complement codes of the k-mer at i: built from its k bases when
// `fresh`, otherwise rolled on from the k-mer at i - 1.
__device__ __forceinline__ void roll_kmer(const uint8_t *s, int i, int k, uint64_t kmask,
                                          bool fresh, uint64_t &f, uint64_t &r)
{
    if (fresh) {
        f = 0;
        r = 0;
        for (int j = 0; j < k; j++) {
            const uint64_t b = s[i + j];
            f = (f << 2) | b;
            r |= (3ull - b) << (2 * j);
        }
        return;
    }
    const uint64_t b = s[i + k - 1];
    f = ((f << 2) | b) & kmask;
    r = (r >> 2) | ((3ull - b) << (2 * (k - 1)));
}

// Seeds of sequence s (length L) under algorithm g into out[]; returns their number
// (the same in every thread).  All threads of the workgroup call it.
template <int HK>
__device__ uint32_t fig4_seeds(const MatchArgs &A, MatchLds &M, const uint8_t *s, int L, int g,
                               uint64_t *out)
{
    const int t = threadIdx.x, k = A.k, w = A.w;
    if (g == 2) {
        const int n = L >= k ? L - k + 1 : 0;
        for (int i = t; i < n; i += kBlock) out[i] = canon_at(s, i, k, A.spaced);
        __syncthreads();
        return (uint32_t)n;
    }
    if (g == 0) {
        const int n = L >= k ? L - k + 1 : 0;
        // positions [4t, 4t + 4) of the (at most 1,024) k-mers: one k-mer built, 3 rolled
        uint64_t f = 0, r = 0;
        for (int i = 4 * t; i < 4 * t + 4 && i < n; i++) {
            roll_kmer(s, i, k, A.kmask, i == 4 * t, f, r);
            out[i] = f < r ? f : r;
        }
        __syncthreads();
        return (uint32_t)n;
    }
    // minimizers of s itself (g == 1) or of its patterned sequence (g == 3, shift 0)
    const uint8_t *src = s;
    int n = L;
    if (g == 3) {
        n = (int)kept_count(A.P, (uint64_t)L, 0);
        for (int li = t; li < n; li += kBlock) M.ps[li] = s[orig_of(A.P, (uint64_t)li, 0)];
        src = M.ps;
        __syncthreads();
    }
    const int nk = n >= k ? n - k + 1 : 0;
    if (nk < w) return 0;
    uint64_t f = 0, r = 0;
    for (int i = 4 * t; i < 4 * t + 4 && i < nk; i++) {
        roll_kmer(src, i, k, A.kmask, i == 4 * t, f, r);
        const bool pal = f == r;
        M.hv[i] = pal ? kMax64 : kmer_hash<HK>(f < r ? f : r, A.kmask);
        M.use[i] = pal ? 0 : 1;
        M.sel[i] = 0;
    }
    if (t == 0) M.n = 0;
    __syncthreads();
    for (int s0 = t; s0 + w <= nk; s0 += kBlock) {
        bool any = false;
        uint64_t m = 0;
        for (int j = s0; j < s0 + w; j++)
            if (M.use[j] && (!any || M.hv[j] < m)) { m = M.hv[j]; any = true; }
        if (!any) continue;
        for (int j = s0; j < s0 + w; j++)
            if (M.use[j] && M.hv[j] == m) M.sel[j] = 1;      // every writer stores 1
    }
    __syncthreads();
    for (int i = t; i < nk; i += kBlock)
        if (M.sel[i]) out[atomicAdd(&M.n, 1u)] = M.hv[i];   // order is irrelevant
    __syncthreads();
    return M.n;
}

__device__ __forceinline__ uint32_t set_slot(uint64_t key)
{
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53);        // 11 bits
}

// Inserts keys[0, n) into the LDS hash set (cleared by the caller).
__device__ void set_insert(MatchLds &M, const uint64_t *keys, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        const uint64_t key = keys[i];
        if (key == kEmpty) {
            M.has_max = 1;
            continue;
        }
        uint32_t slot = set_slot(key);
        while (true) {
            const unsigned long long old = atomicCAS(&M.set[slot], (unsigned long long)kEmpty,
                                                     (unsigned long long)key);
            if (old == kEmpty || old == key) break;     // claimed, or already present
            slot = (slot + 1) & (kSetSlots - 1);
        }
    }
}

__device__ __forceinline__ bool set_has(const MatchLds &M, uint64_t key)
{
    if (key == kEmpty) return M.has_max != 0;
    uint32_t slot = set_slot(key);
    while (true) {
        const uint64_t v = M.set[slot];
        if (v == key) return true;
        if (v == kEmpty) return false;
        slot = (slot + 1) & (kSetSlots - 1);
    }
}

template <int HK>
__global__ __launch_bounds__(kBlock) void k_seed_match(MatchArgs A)
{
    __shared__ MatchLds M;
    const int t = threadIdx.x;
    for (uint32_t p = blockIdx.x; p < A.n_pairs; p += gridDim.x) {
        const uint64_t a0 = A.oa[p], b0 = A.ob[p];
        const uint64_t la = A.oa[p + 1] - a0, lb = A.ob[p + 1] - b0;
        if (la > (uint64_t)kFig4MaxLen || lb > (uint64_t)kFig4MaxLen) {
            if (t == 0) set_status(A.status, GODIET_ST_RANGE);
            if (t < 8) A.counts[8 * (uint64_t)p + t] = 0;
            continue;
        }
        for (int i = t; i < (int)la; i += kBlock) M.sa[i] = (uint8_t)base_of(A.ba, a0 + i);
        for (int i = t; i < (int)lb; i += kBlock) M.sb[i] = (uint8_t)base_of(A.bb, b0 + i);
        __syncthreads();
        for (int g = 0; g < 4; g++) {
            for (int i = t; i < kSetSlots; i += kBlock) M.set[i] = kEmpty;
            if (t == 0) M.has_max = 0;
            const uint32_t na = fig4_seeds<HK>(A, M, M.sa, (int)la, g, M.kb);   // syncs
            set_insert(M, M.kb, na);
            __syncthreads();
            const uint32_t nb = fig4_seeds<HK>(A, M, M.sb, (int)lb, g, M.kb);
            uint32_t hit = 0;
            for (uint32_t i = t; i < nb; i += kBlock) hit += set_has(M, M.kb[i]) ? 1u : 0u;
            hit = wave_sum<uint32_t>(hit);
            if ((t & (kWave - 1)) == 0) M.red[t / kWave] = hit;
            __syncthreads();
            if (t == 0) {
                uint32_t sum = 0;
                for (int i = 0; i < kBlock / kWave; i++) sum += M.red[i];
                A.counts[8 * (uint64_t)p + 2 * g] = sum;
                A.counts[8 * (uint64_t)p + 2 * g + 1] = nb;
            }
            __syncthreads();
        }
    }
}

// Levenshtein distance of pair p: the rows are the original's bases (at most 1,024, as
// 16 words of 64), the columns the copy's.  Pv / Mv hold the vertical +1 / -1 deltas of
// the current column; each column adds the match mask through a carry chain over the
// words and shifts the horizontal deltas up by one row, with a +1 entering at row 0
// (the first row of the table is 0, 1, 2, ...).  The distance is m plus the running sum
// of the horizontal deltas of the last row.
__global__ __launch_bounds__(kEdBlock) void k_edit_distance(const uint8_t *ba, const uint64_t *oa,
                                                            const uint8_t *bb, const uint64_t *ob,
                                                            uint32_t n_pairs, uint32_t *dist,
                                                            uint32_t *status)
{
    __shared__ uint64_t peq[4 * kEdWords * kEdBlock];    // [letter][word][thread]
    const int t = threadIdx.x;
    const uint32_t p = blockIdx.x * kEdBlock + t;
    if (p >= n_pairs) return;
    const uint64_t a0 = oa[p], b0 = ob[p];
    const uint64_t m = oa[p + 1] - a0, n = ob[p + 1] - b0;
    if (m > (uint64_t)kFig4MaxLen || n >= (1ull << 31)) {
        set_status(status, GODIET_ST_RANGE);
        dist[p] = 0;
        return;
    }
    if (m == 0) {
        dist[p] = (uint32_t)n;
        return;
    }
    const int W = (int)((m + 63) / 64);
#pragma unroll
    for (int wd = 0; wd < kEdWords; wd++) {
        uint64_t e[4] = {0, 0, 0, 0};
        if (wd < W) {
            for (int b = 0; b < 64; b++) {
                const uint64_t i = 64 * (uint64_t)wd + b;
                if (i >= m) break;
                const uint32_t c = base_of(ba, a0 + i);
                e[0] |= (c == 0 ? 1ull : 0ull) << b;
                e[1] |= (c == 1 ? 1ull : 0ull) << b;
                e[2] |= (c == 2 ? 1ull : 0ull) << b;
                e[3] |= (c == 3 ? 1ull : 0ull) << b;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; c++) peq[(c * kEdWords + wd) * kEdBlock + t] = e[c];
    }
    uint64_t Pv[kEdWords], Mv[kEdWords];
#pragma unroll
    for (int wd = 0; wd < kEdWords; wd++) {
        Pv[wd] = ~0ull;
        Mv[wd] = 0;
    }
    const int top = (int)((m - 1) & 63);          // last row's bit in word W - 1
    int64_t score = (int64_t)m;
    uint32_t byte = 0;
    for (uint64_t j = 0; j < n; j++) {
        const uint64_t g = b0 + j;
        if (j == 0 || (g & 3) == 0) byte = bb[g >> 2];
        const uint32_t c = (byte >> ((g & 3) * 2)) & 3u;
        uint64_t carry = 0, ph_in = 1, mh_in = 0;
#pragma unroll
        for (int wd = 0; wd < kEdWords; wd++) {
            if (wd < W) {
                const uint64_t eq = peq[(c * kEdWords + wd) * kEdBlock + t];
                const uint64_t pv = Pv[wd], mv = Mv[wd];
                const uint64_t xv = eq | mv;
                const uint64_t ep = eq & pv;
                const uint64_t s1 = ep + pv;
                const uint64_t s2 = s1 + carry;
                carry = (s1 < ep || s2 < s1) ? 1ull : 0ull;
                const uint64_t xh = (s2 ^ pv) | eq;
                const uint64_t ph = mv | ~(xh | pv);
                const uint64_t mh = pv & xh;
                if (wd == W - 1) score += (int64_t)((ph >> top) & 1ull) - (int64_t)((mh >> top) & 1ull);
                const uint64_t phs = (ph << 1) | ph_in;
                const uint64_t mhs = (mh << 1) | mh_in;
                ph_in = ph >> 63;
                mh_in = mh >> 63;
                Pv[wd] = mhs | ~(xv | phs);
                Mv[wd] = phs & xv;
            }
        }
    }
    dist[p] = (uint32_t)score;
}

// Rate m / t as an integer with the same order (exact for totals below 2^16).
__device__ __forceinline__ uint64_t rate_key(uint32_t m, uint32_t t)
{
    return t ? (((uint64_t)m << 32) / t) : 0;
}

__global__ __launch_bounds__(kBlock) void k_acc_min(const uint32_t *dist, const uint32_t *counts,
                                                    uint32_t n, int g, uint32_t max_e,
                                                    unsigned long long *minkey)
{
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint32_t d = dist[i];
        if (d > max_e) continue;
        atomicMin(&minkey[d], (unsigned long long)rate_key(counts[8 * (uint64_t)i + 2 * g],
                                                           counts[8 * (uint64_t)i + 2 * g + 1]));
    }
}

// In-place inclusive prefix (min for thresholds, sum for counts) over e[0, n) by one
// workgroup, in chunks of kBlock with a running carry.
template <typename T, bool kMin>
__global__ __launch_bounds__(kBlock) void k_acc_prefix(T *e, uint32_t n)
{
    __shared__ T sh[kBlock];
    __shared__ T carry;
    const int t = threadIdx.x;
    if (t == 0) carry = kMin ? (T)~(T)0 : (T)0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += kBlock) {
        const uint32_t i = base + t;
        T v = i < n ? e[i] : (kMin ? (T)~(T)0 : (T)0);
        sh[t] = v;
        __syncthreads();
        for (int d = 1; d < kBlock; d <<= 1) {
            const T o = t >= d ? sh[t - d] : (kMin ? (T)~(T)0 : (T)0);
            __syncthreads();
            v = kMin ? (o < v ? o : v) : v + o;
            sh[t] = v;
            __syncthreads();
        }
        const T c = carry;
        v = kMin ? (c < v ? c : v) : v + c;
        if (i < n) e[i] = v;
        __syncthreads();
        if (t == kBlock - 1) carry = v;
        __syncthreads();
    }
}

constexpr uint32_t kAccLds = 8192;

// Every pair adds one at the first threshold its rate reaches (thresholds do not rise).
__global__ __launch_bounds__(kBlock) void k_acc_count(const uint32_t *counts, uint32_t n, int g,
                                                      uint32_t max_e,
                                                      const unsigned long long *thr,
                                                      uint32_t *acc)
{
    __shared__ uint32_t hist[kAccLds];          // per-workgroup counts when they fit
    if (max_e < kAccLds) {
        for (uint32_t e = threadIdx.x; e <= max_e; e += kBlock) hist[e] = 0;
        __syncthreads();
    }
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint64_t key = rate_key(counts[8 * (uint64_t)i + 2 * g],
                                      counts[8 * (uint64_t)i + 2 * g + 1]);
        uint32_t lo = 0, hi = max_e + 1;                 // first E with thr[E] <= key
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (thr[mid] <= key) hi = mid; else lo = mid + 1;
        }
        if (lo <= max_e) {
            if (max_e < kAccLds) atomicAdd(&hist[lo], 1u);
            else atomicAdd(&acc[lo], 1u);
        }
    }
    if (max_e < kAccLds) {
        __syncthreads();
        for (uint32_t e = threadIdx.x; e <= max_e; e += kBlock)
            if (hist[e]) atomicAdd(&acc[e], hist[e]);
    }
}

}  // namespace

hipError_t launch_seed_match(const godiet_seqs *a, const godiet_seqs *b, const Pattern &P, int k,
                             int w, int hash, uint32_t *counts, uint32_t *status, hipStream_t s)
{
    if (a->n_seq == 0) return hipSuccess;
    MatchArgs A;
    A.ba = a->bases;
    A.bb = b->bases;
    A.oa = a->offsets;
    A.ob = b->offsets;
    A.n_pairs = a->n_seq;
    A.P = P;
    A.k = k;
    A.w = w;
    A.kmask = k == 32 ? kMax64 : ((1ull << (2 * k)) - 1);
    A.spaced = 0;
    for (int j = 0; j < k; j++)
        if (pattern_bit(P, (uint32_t)j % P.p)) A.spaced |= 1u << j;
    A.counts = counts;
    A.status = status;
    const unsigned grid = a->n_seq < 65536u ? a->n_seq : 65536u;
    if (hash == 1) GD_LAUNCH(k_seed_match<1>, dim3(grid), dim3(kBlock), 0, s, A);
    else if (k == 32) GD_LAUNCH(k_seed_match<2>, dim3(grid), dim3(kBlock), 0, s, A);
    else GD_LAUNCH(k_seed_match<0>, dim3(grid), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_edit_distance(const godiet_seqs *a, const godiet_seqs *b, uint32_t *dist,
                                uint32_t *status, hipStream_t s)
{
    if (a->n_seq == 0) return hipSuccess;
    const unsigned grid = (a->n_seq + kEdBlock - 1) / kEdBlock;
    GD_LAUNCH(k_edit_distance, dim3(grid), dim3(kEdBlock), 0, s, a->bases, a->offsets, b->bases,
              b->offsets, a->n_seq, dist, status);
    return hipGetLastError();
}

hipError_t launch_accepted(const uint32_t *dist, const uint32_t *counts, uint32_t n, int g,
                           uint32_t max_e, uint64_t *minkey, uint32_t *acc, hipStream_t s)
{
    hipError_t e = fill_u64(minkey, kMax64, (size_t)max_e + 1, s);
    if (e != hipSuccess) return e;
    e = fill_u32(acc, 0, (size_t)max_e + 1, s);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    unsigned grid = (n + kBlock - 1) / kBlock;
    if (grid > 4096) grid = 4096;
    unsigned long long *mk = (unsigned long long *)minkey;
    GD_LAUNCH(k_acc_min, dim3(grid), dim3(kBlock), 0, s, dist, counts, n, g, max_e, mk);
    GD_LAUNCH((k_acc_prefix<unsigned long long, true>), dim3(1), dim3(kBlock), 0, s, mk,
              max_e + 1);
    GD_LAUNCH(k_acc_count, dim3(grid), dim3(kBlock), 0, s, counts, n, g, max_e,
              (const unsigned long long *)mk, acc);
    GD_LAUNCH((k_acc_prefix<uint32_t, false>), dim3(1), dim3(kBlock), 0, s, acc, max_e + 1);
    return hipGetLastError();
}

}  // namespace gd
