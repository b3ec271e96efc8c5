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
        e = launch_sort(sp, sw, keys, vals, 4, n_ptr, capacity, s);
        if (e != hipSuccess) return e;
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
