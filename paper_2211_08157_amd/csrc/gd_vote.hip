// Location voting (Section 3.4 steps 1-4, Illumina form) with the rescue location of
// Section 3.6.3, over the anchors of a seeding pass.
//
// Layout of the work: every anchor becomes one 64-bit key
//     (read_id << 33 | strand << 32 | d) << lz,
//     d = rpos - qpos + 2^31 (forward strand, the diagonal) or rpos + qpos (reverse strand,
//     the anti-diagonal), lz = the unused high bits for this batch's read count (so the
//     read id sits at the top, where the sort partitions),
// with its anchor index as the value.  One sort of the whole batch (the index sort)
// orders every read's adjusted locations by strand and location, and since the read id
// is the top of the key each read keeps its own range [read_off[r], read_off[r+1]).
// Alternatively each read's range is sorted on its own by one thread, by a natural merge
// sort over the runs the anchors already form, or by heapsort (Section 3.6.2 compares
// such choices); the default sorts reads with at most 16 locations in registers (a
// bitonic network) and gives every longer read a workgroup (LDS bitonic chunks, then
// merge-path merges).  The sweep
// reads only the keys, so every choice gives the same winners.
// The sweep then walks each read's run: the first key is the temporary location L0, its
// votes are the keys up to L0 + D of the same read and strand, and the first key beyond
// becomes the next L0.  Reads with few anchors are swept by one thread each; reads with
// many (long reads) by one wave each, which finds the end of every cluster with a ballot
// over 64 keys at a time.  The best max_win candidates by votes (then strand, location)
// are kept in registers; when none reaches V the candidate with the most votes is the
// rescue output.
#include "gd_internal.h"

namespace gd {

namespace {

constexpr int kMaxWin = 16;            // largest max_win
constexpr uint32_t kSeqSweep = 256;    // reads with more anchors are swept by a wave

__global__ __launch_bounds__(kBlock) void k_vote_keys(const uint4 *anchors, const uint64_t *n_ptr,
                                                      uint64_t capacity, int lz, uint64_t *keys,
                                                      uint32_t *vals)
{
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint4 a = anchors[i];                       // read_id, qpos, rpos, strand
        const uint32_t st = a.w & 1u;
        const uint32_t d = st ? a.z + a.y : a.z - a.y + 0x80000000u;
        keys[i] = (((uint64_t)a.x << 33) | ((uint64_t)st << 32) | d) << lz;
        vals[i] = (uint32_t)i;
    }
}

// Per-read sorts of the keys (one thread per read), the alternatives to the batch sort.
// Keys of read r occupy [read_off[r], read_off[r + 1]) in anchor order.

// Heapsort of a[0, n) ascending (sift-down heap, then repeated extraction).
__device__ void heap_sort(uint64_t *a, uint64_t n)
{
    if (n < 2) return;
    auto sift = [&](uint64_t root, uint64_t end) {
        const uint64_t v = a[root];
        while (true) {
            uint64_t c = 2 * root + 1;
            if (c >= end) break;
            if (c + 1 < end && a[c + 1] > a[c]) c++;
            if (a[c] <= v) break;
            a[root] = a[c];
            root = c;
        }
        a[root] = v;
    };
    for (uint64_t i = n / 2; i-- > 0;) sift(i, n);
    for (uint64_t end = n - 1; end > 0; end--) {
        const uint64_t t = a[0];
        a[0] = a[end];
        a[end] = t;
        sift(0, end);
    }
}

// Natural merge sort of a[0, n) with scratch t[0, n): every pass merges adjacent
// ascending runs pairwise; a read's anchors come as per-minimizer runs sorted by
// reference position, so few passes are needed.  The result ends in a.
__device__ void natural_merge_sort(uint64_t *a, uint64_t *t, uint64_t n)
{
    uint64_t *src = a, *dst = t;
    while (true) {
        uint64_t i = 0, runs = 0;
        while (i < n) {
            uint64_t m = i + 1;                           // end of the first run
            while (m < n && src[m - 1] <= src[m]) m++;
            uint64_t e = m;                               // end of the second run
            if (e < n) {
                e++;
                while (e < n && src[e - 1] <= src[e]) e++;
            }
            uint64_t x = i, y = m, o = i;
            while (x < m && y < e) dst[o++] = src[y] < src[x] ? src[y++] : src[x++];
            while (x < m) dst[o++] = src[x++];
            while (y < e) dst[o++] = src[y++];
            runs++;
            i = e;
        }
        uint64_t *sw = src;
        src = dst;
        dst = sw;
        if (runs <= 1) break;
    }
    if (src != a)
        for (uint64_t i = 0; i < n; i++) a[i] = src[i];
}

// kind 2: natural merge sort, 3: heapsort, 0 (adaptive): reads with at most kRegSort keys
// sorted in registers by a fixed bitonic network, longer reads listed for
// k_vote_long_sort (one workgroup each).  Serial sorts in global memory wait on one load
// after another, so beyond a few keys a read is better served by a whole workgroup.
constexpr int kRegSort = 16;

__device__ __forceinline__ void reg_sort16(uint64_t *a, uint32_t n)
{
    uint64_t v[kRegSort];
#pragma unroll
    for (int i = 0; i < kRegSort; i++) v[i] = (uint32_t)i < n ? a[i] : kMax64;
#pragma unroll
    for (int k = 2; k <= kRegSort; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < kRegSort; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const bool asc = (i & k) == 0;
                    const uint64_t x = v[i], y = v[l];
                    const bool sw = (x > y) == asc;
                    v[i] = sw ? y : x;
                    v[l] = sw ? x : y;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kRegSort; i++)
        if ((uint32_t)i < n) a[i] = v[i];
}

__global__ __launch_bounds__(kBlock) void k_vote_read_sort(uint64_t *keys, uint64_t *scratch,
                                                           const uint64_t *read_off,
                                                           uint32_t n_reads, uint64_t capacity,
                                                           int kind, uint32_t *long_ids,
                                                           uint32_t *long_n)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_reads || read_off[n_reads] > capacity) return;
    const uint64_t b = read_off[r], e = read_off[r + 1];
    if (kind == 2) {
        natural_merge_sort(keys + b, scratch + b, e - b);
    } else if (kind == 3) {
        heap_sort(keys + b, e - b);
    } else if (e - b > (uint64_t)kRegSort) {
        long_ids[atomicAdd(long_n, 1u)] = r;
    } else if (e - b > 1) {
        reg_sort16(keys + b, (uint32_t)(e - b));
    }
}

constexpr uint32_t kSortChunk = 4096;        // keys sorted at once in LDS (32 KB)

// Ascending bitonic sort of the LDS array a[0, n2) (n2 a power of two <= kSortChunk).
__device__ void lds_bitonic(uint64_t *a, uint32_t n2)
{
    for (uint32_t size = 2; size <= n2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t c = threadIdx.x; c < n2 / 2; c += kBlock) {
                const uint32_t lo = (c / stride) * stride * 2 + (c % stride);
                const uint32_t hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if ((x > y) == asc) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Elements of A among the first d outputs of merge(A, B), A first on ties (merge path).
__device__ __forceinline__ uint64_t co_rank(uint64_t d, const uint64_t *A, uint64_t na,
                                            const uint64_t *B, uint64_t nb)
{
    uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t i = (lo + hi) >> 1;
        if (A[i] <= B[d - i - 1]) lo = i + 1; else hi = i;
    }
    return lo;
}

// One workgroup per listed (long) read: sorted chunks of kSortChunk keys in LDS, then
// pairwise merges of sorted runs in global memory, every thread merging its own share of
// the output found by a merge-path split.  The result ends in keys.
__global__ __launch_bounds__(kBlock) void k_vote_long_sort(uint64_t *keys, uint64_t *scratch,
                                                           const uint64_t *read_off,
                                                           uint32_t n_reads, uint64_t capacity,
                                                           const uint32_t *long_ids,
                                                           const uint32_t *long_n)
{
    __shared__ uint64_t sh[kSortChunk];
    if (read_off[n_reads] > capacity) return;
    const uint32_t nl = *long_n;
    for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
        const uint32_t r = long_ids[li];
        const uint64_t b = read_off[r], n = read_off[r + 1] - b;
        uint64_t *a = keys + b, *t = scratch + b;
        for (uint64_t c0 = 0; c0 < n; c0 += kSortChunk) {
            const uint32_t m = (uint32_t)(n - c0 < kSortChunk ? n - c0 : kSortChunk);
            uint32_t n2 = 1;
            while (n2 < m) n2 <<= 1;
            for (uint32_t i = threadIdx.x; i < n2; i += kBlock) sh[i] = i < m ? a[c0 + i] : kMax64;
            __syncthreads();
            lds_bitonic(sh, n2);
            for (uint32_t i = threadIdx.x; i < m; i += kBlock) a[c0 + i] = sh[i];
            __syncthreads();
        }
        uint64_t *src = a, *dst = t;
        for (uint64_t width = kSortChunk; width < n; width *= 2) {
            for (uint64_t p0 = 0; p0 < n; p0 += 2 * width) {
                const uint64_t na = n - p0 < width ? n - p0 : width;
                const uint64_t nb = n - p0 - na < width ? n - p0 - na : width;
                const uint64_t *A = src + p0, *B = src + p0 + na;
                const uint64_t len = na + nb;
                const uint64_t d0 = len * threadIdx.x / kBlock;
                const uint64_t d1 = len * (threadIdx.x + 1) / kBlock;
                uint64_t i = co_rank(d0, A, na, B, nb), j = d0 - i;
                for (uint64_t d = d0; d < d1; d++) {
                    const bool take_a = j >= nb || (i < na && A[i] <= B[j]);
                    dst[p0 + d] = take_a ? A[i++] : B[j++];
                }
            }
            __syncthreads();                          // the pass is complete
            uint64_t *sw = src;
            src = dst;
            dst = sw;
        }
        if (src != a) {
            for (uint64_t i = threadIdx.x; i < n; i += kBlock) a[i] = src[i];
        }
        __syncthreads();
    }
}

// Candidates kept in registers: the best nw (<= cap) by votes, then key; and the rescue.
struct Winners {
    uint32_t v[kMaxWin];
    uint64_t k[kMaxWin];
    uint32_t nw;
    uint32_t rv;
    uint64_t rk;

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int t = 0; t < kMaxWin; t++) { v[t] = 0; k[t] = 0; }
        nw = 0;
        rv = 0;
        rk = 0;
    }
    // candidates arrive in ascending key order, so an equal vote count ranks later
    __device__ __forceinline__ void add(uint32_t votes, uint64_t key, uint32_t V, uint32_t cap)
    {
        if (votes > rv) { rv = votes; rk = key; }
        if (votes < V) return;
        // insert after the entries with at least as many votes; everything below moves
        // down one slot (a displaced entry precedes the equal ones it lands on)
        uint32_t cv = votes;
        uint64_t ck = key;
        bool moving = false;
#pragma unroll
        for (int t = 0; t < kMaxWin; t++) {
            if ((uint32_t)t < cap && (moving || cv > v[t])) {
                const uint32_t tv = v[t];
                const uint64_t tk = k[t];
                v[t] = cv;
                k[t] = ck;
                cv = tv;
                ck = tk;
                moving = true;
            }
        }
        if (nw < cap) nw++;
    }
};

__device__ __forceinline__ godiet_winner make_rec(uint32_t r, uint64_t key, uint32_t votes,
                                                    uint32_t flags)
{
    godiet_winner o;
    const uint32_t st = (uint32_t)(key >> 32) & 1u;
    const uint32_t d = (uint32_t)key;
    o.loc = st ? (int64_t)d : (int64_t)d - (int64_t)0x80000000u;
    o.read_id = r;
    o.strand = st;
    o.votes = votes;
    o.flags = flags;
    return o;
}

__device__ __forceinline__ void write_winners(const Winners &W, uint32_t r, uint32_t cap,
                                              godiet_winner *out, uint32_t *n_win, bool any)
{
    godiet_winner *o = out + (size_t)r * cap;
    if (!any) {
        n_win[r] = 0;
    } else if (W.nw == 0) {
        o[0] = make_rec(r, W.rk, W.rv, GODIET_VOTE_RESCUE);
        n_win[r] = 1;
    } else {
#pragma unroll
        for (int t = 0; t < kMaxWin; t++)
            if ((uint32_t)t < W.nw) o[t] = make_rec(r, W.k[t], W.v[t], 0);
        n_win[r] = W.nw;
    }
}

// Largest key of cluster that starts at k0: L0 + D within the same read and strand.
__device__ __forceinline__ uint64_t cluster_limit(uint64_t k0, uint32_t D)
{
    const uint64_t group_end = k0 | 0xffffffffull;
    return (group_end - k0 >= (uint64_t)D) ? k0 + D : group_end;
}

// One thread per read (reads with at most kSeqSweep anchors); longer reads are listed.
__global__ __launch_bounds__(kBlock) void k_vote_sweep(const uint64_t *keys,
                                                       const uint64_t *read_off, uint32_t n_reads,
                                                       uint64_t capacity, VoteArgs A,
                                                       godiet_winner *out, uint32_t *n_win,
                                                       uint32_t *long_ids, uint32_t *long_n,
                                                       uint32_t *status)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_reads) return;
    if (read_off[n_reads] > capacity) {
        if (r == 0) set_status(status, 1u);
        return;
    }
    const uint64_t b = read_off[r], e = read_off[r + 1];
    if (e - b > kSeqSweep) {
        long_ids[atomicAdd(long_n, 1u)] = r;
        return;
    }
    Winners W;
    W.init();
    uint64_t i = b;
    while (i < e) {
        const uint64_t k0 = keys[i] >> A.lz;
        if ((k0 >> 33) != r) set_status(status, 2u);      // anchors not grouped by read
        const uint64_t lim = cluster_limit(k0, A.max_dist);
        uint64_t j = i + 1;
        while (j < e && (keys[j] >> A.lz) <= lim) j++;
        W.add((uint32_t)(j - i), k0, A.min_votes, A.max_win);
        i = j;
    }
    write_winners(W, r, A.max_win, out, n_win, e > b);
}

// One wave per listed read: the end of each cluster is the first key beyond its limit,
// found by a ballot over 64 keys at a time.  Every lane holds the same candidates.
__global__ __launch_bounds__(kBlock) void k_vote_sweep_long(const uint64_t *keys,
                                                            const uint64_t *read_off,
                                                            uint32_t n_reads, uint64_t capacity,
                                                            VoteArgs A, godiet_winner *out,
                                                            uint32_t *n_win,
                                                            const uint32_t *long_ids,
                                                            const uint32_t *long_n,
                                                            uint32_t *status)
{
    if (read_off[n_reads] > capacity) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nl = *long_n;
    for (uint32_t li = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; li < nl;
         li += gridDim.x * (kBlock / kWave)) {
        const uint32_t r = long_ids[li];
        const uint64_t b = read_off[r], e = read_off[r + 1];
        Winners W;
        W.init();
        uint64_t i = b;
        while (i < e) {
            const uint64_t k0 = keys[i] >> A.lz;
            if (lane == 0 && (k0 >> 33) != r) set_status(status, 2u);
            const uint64_t lim = cluster_limit(k0, A.max_dist);
            uint64_t j = i + 1;
            while (true) {
                const uint64_t idx = j + (uint64_t)lane;
                const bool stop = idx >= e || (keys[idx] >> A.lz) > lim;
                const uint64_t beyond = __ballot(stop);
                if (beyond) {
                    j += (uint64_t)(__ffsll((unsigned long long)beyond) - 1);
                    break;
                }
                j += kWave;
            }
            if (j > e) j = e;
            W.add((uint32_t)(j - i), k0, A.min_votes, A.max_win);
            i = j;
        }
        if (lane == 0) write_winners(W, r, A.max_win, out, n_win, e > b);
    }
}

}  // namespace

hipError_t launch_vote(const VoteArgs &A, const uint4 *anchors, const uint64_t *read_off,
                       uint32_t n_reads, uint64_t capacity, const SortPlan &sp,
                       const SortWs &sw, uint64_t *keys, uint32_t *vals, uint32_t *long_ids,
                       uint32_t *long_n, godiet_winner *out, uint32_t *n_win,
                       uint32_t *status, hipStream_t s)
{
    if (n_reads == 0) return hipSuccess;
    const uint64_t *n_ptr = read_off + n_reads;
    hipError_t e = fill_u32(long_n, 0, 1, s);
    if (e != hipSuccess) return e;
    if (capacity > 0) {
        uint64_t blocks = (capacity + kBlock - 1) / kBlock;
        if (blocks > 8192) blocks = 8192;
        GD_LAUNCH(k_vote_keys, dim3((unsigned)blocks), dim3(kBlock), 0, s, anchors, n_ptr,
                  capacity, A.lz, keys, vals);
        if (A.sort == 1) {
            e = launch_sort(sp, sw, keys, vals, 4, n_ptr, capacity, s);
            if (e != hipSuccess) return e;
        } else {
            GD_LAUNCH(k_vote_read_sort, dim3((n_reads + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                      keys, (uint64_t *)sw.trec, read_off, n_reads, capacity, A.sort, long_ids,
                      long_n);
            if (A.sort == 0) {
                GD_LAUNCH(k_vote_long_sort, dim3(1024), dim3(kBlock), 0, s, keys,
                          (uint64_t *)sw.trec, read_off, n_reads, capacity,
                          (const uint32_t *)long_ids, (const uint32_t *)long_n);
            }
            e = fill_u32(long_n, 0, 1, s);                // the sweep lists its own reads
            if (e != hipSuccess) return e;
        }
    }
    GD_LAUNCH(k_vote_sweep, dim3((n_reads + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
              (const uint64_t *)keys, read_off, n_reads, capacity, A, out, n_win, long_ids,
              long_n, status);
    GD_LAUNCH(k_vote_sweep_long, dim3(1024), dim3(kBlock), 0, s, (const uint64_t *)keys,
              read_off, n_reads, capacity, A, out, n_win, (const uint32_t *)long_ids,
              (const uint32_t *)long_n, status);
    return hipGetLastError();
}

}  // namespace gd
