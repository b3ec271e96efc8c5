// Sort of the reference minimizer records by (hash, val) for the seed index.
//
// Minimizer hashes are window minima, so they are NOT uniform: small values are several
// times denser than large ones, and fixed top-bit buckets overflow at the dense end.
// The partition is therefore data driven:
//   1. a fine histogram over the top Bf bits (about 2 records per fine bin on average,
//      a few times more at the dense low end); the value each record's atomic returns
//      is its rank inside its bin;
//   2. its exclusive scan gives the start of every fine bin;
//   3. a scatter moves each record to bin start + rank as one 16-byte (key, value)
//      record (no atomics: the ranks are already known);
//   4. coarse bucket c is the run of fine bins whose start lies in [c*T, (c+1)*T), so
//      every coarse bucket holds about T records whatever the key distribution (its
//      first fine bin comes from one pass over the fine bins); one workgroup loads it
//      into LDS and writes every record to its segment's start plus its rank inside its
//      run of one fine bin (runs are already in key order relative to each other), or
//      sorts the whole bucket by an LDS bitonic sort when a run is long (many equal
//      hashes).  The work per bucket depends on its
//      records only, not on the number of (possibly empty) fine bins it spans.
// A coarse bucket larger than the LDS capacity (only possible when one fine bin holds
// thousands of records) is listed and sorted by a fallback kernel in global memory.
// (hash, val) pairs are unique, so the result does not depend on the order in which the
// scatter's atomics land.
//
// Indexes of up to ~200M records with 32-bit values (~100M with 64-bit values) take a
// cheaper partition ("digits" mode) whose digits are balanced by the data: a histogram of
// the top 12 bits of a sample of the keys, scanned, maps a key to its approximate rank
// (the cumulative count of its 12-bit slice plus its share of the slice, by the next 32
// key bits, which is monotone in the key), and the digit is that rank scaled to
// D <= 2^15 digits, so every digit holds about N / D records whatever the skew of the
// hashes.  Digits are counted per chunk of records in LDS.  Below 2^24 records they are
// turned into per-chunk digit offsets by one thread per digit and scattered with LDS
// atomics; from 2^24 records the records move in two coalesced passes (256 coarse digits,
// then the fine digits inside each), staged in LDS so that every group of a step is
// written as one run.  No record touches a global atomic or a random global read.  Coarse
// buckets of whole digits (about 2,048 records, at most that plus one digit) are sorted
// in LDS: binned by their key's offset from the bucket's smallest key, scaled to about
// two bins per record, and placed by rank inside their bin (k_digit_bucket_sort, in three
// launches by bucket size, the largest with up to 128 KB of LDS and over a device-built
// list of its buckets).
#include "gd_internal.h"

namespace gd {

namespace {

// records a workgroup sorts in LDS (a power of two, so bitonic padding fits)
template <typename V> struct Cap { static constexpr int value = sizeof(V) == 4 ? 4096 : 2048; };
// the digits mode's full-capacity buckets: 96 KB (32-bit values) or 64 KB (64-bit) of
// records plus the sub-bins
template <typename V> struct DCap { static constexpr int value = sizeof(V) == 4 ? 8192 : 4096; };
constexpr int kSmall = 48;          // longest fine-bin run placed by ranking

template <typename V>
__device__ __forceinline__ bool rec_less(uint64_t ka, V va, uint64_t kb, V vb)
{
    return ka < kb || (ka == kb && va < vb);
}

__global__ __launch_bounds__(kBlock) void k_hist(const uint64_t *keys, const uint64_t *n_ptr,
                                                 uint64_t capacity, int Bf, uint32_t *hist,
                                                 uint32_t *rank)
{
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock)
        rank[i] = atomicAdd(&hist[keys[i] >> (64 - Bf)], 1u);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t *keys, const V *vals,
                                                    const uint64_t *n_ptr, uint64_t capacity,
                                                    int Bf, const uint64_t *fofs,
                                                    const uint32_t *rank, ulonglong2 *trec)
{
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t key = keys[i];
        trec[fofs[key >> (64 - Bf)] + rank[i]] = make_ulonglong2(key, (uint64_t)vals[i]);
    }
}

// ---- digits mode
constexpr int kDigitBits = 15;      // at most 2^15 digits (128 KB of LDS counters)
constexpr int kBigBlock = 1024;
constexpr int kTopBits = 12;        // slices of the key range whose counts balance the digits
constexpr int kTop = 1 << kTopBits;

// Histogram of the top kTopBits bits of every stride-th key (per workgroup in LDS, then
// added globally).  The digit map only needs the key distribution's shape: any counts give
// a monotone map (so a correct sort), a sample of the keys a balanced one.
__global__ __launch_bounds__(kBigBlock) void k_top_hist(const uint64_t *keys, const uint64_t *n_ptr,
                                                        uint64_t capacity, uint32_t *hist)
{
    __shared__ uint32_t h[kTop];
    for (uint32_t d = threadIdx.x; d < (uint32_t)kTop; d += kBigBlock) h[d] = 0;
    __syncthreads();
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    // every stride-th key, stride (a power of two up to 64) keeping at least 256 sampled
    // keys per slice on average: a strided sample touches only every (stride / 8)-th line
    uint32_t stride = 1;
    while (stride < 64 && n / (2ull * stride) >= (uint64_t)kTop * 256) stride <<= 1;
    for (uint64_t i = (blockIdx.x * (uint64_t)kBigBlock + threadIdx.x) * stride; i < n;
         i += (uint64_t)gridDim.x * kBigBlock * stride)
        atomicAdd(&h[keys[i] >> (64 - kTopBits)], 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < (uint32_t)kTop; d += kBigBlock)
        if (h[d]) atomicAdd(&hist[d], h[d]);
}

// Key -> digit, monotone in the key.  Of the kTop + 1 cumulative slice counts the first
// kTop are in LDS and the total N in a register; a key's approximate rank is its slice's
// start plus the slice's count times the key's position inside the slice (its next 32
// bits), and the digit is rank * D / N.
struct DigitMap {
    const uint32_t *C;                   // the first kTop CDF entries (in LDS)
    uint32_t total;                      // the last one, N
    uint64_t mul;                        // D * 2^32 / N
    __device__ __forceinline__ void init(const uint64_t *cdf, uint32_t *lds, uint32_t D)
    {
        for (uint32_t j = threadIdx.x; j < (uint32_t)kTop; j += blockDim.x) lds[j] = (uint32_t)cdf[j];
        total = (uint32_t)cdf[kTop];
        __syncthreads();
        C = lds;
        mul = total ? ((uint64_t)D << 32) / total : 0;
    }
    __device__ __forceinline__ uint32_t operator()(uint64_t x) const
    {
        const uint32_t j = (uint32_t)(x >> (64 - kTopBits));
        const uint32_t lo = C[j], cnt = (j + 1 < (uint32_t)kTop ? C[j + 1] : total) - lo;
        const uint32_t f = (uint32_t)(x >> (64 - kTopBits - 32));
        const uint32_t rank = lo + (uint32_t)(((uint64_t)cnt * f) >> 32);   // < N
        return (uint32_t)(((uint64_t)rank * mul) >> 32);                    // < D
    }
};

__global__ __launch_bounds__(kBigBlock) void k_digit_count(const uint64_t *keys,
                                                           const uint64_t *n_ptr,
                                                           uint64_t capacity, uint32_t D,
                                                           uint32_t chunk, const uint64_t *cdf,
                                                           uint32_t *mat, uint32_t *cmat,
                                                           int sub_bits)
{
    extern __shared__ uint32_t dyn[];           // D counters, then kTop slice CDF entries
    uint32_t *cnt = dyn, *cl = dyn + D;
    for (uint32_t d = threadIdx.x; d < D; d += kBigBlock) cnt[d] = 0;
    DigitMap dm;
    dm.init(cdf, cl, D);
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    constexpr int U = 4;
    for (uint64_t i0 = c0 + threadIdx.x; i0 < c1; i0 += (uint64_t)kBigBlock * U) {
        uint64_t key[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            if (i0 + (uint64_t)u * kBigBlock < c1) key[u] = keys[i0 + (uint64_t)u * kBigBlock];
#pragma unroll
        for (int u = 0; u < U; u++)
            if (i0 + (uint64_t)u * kBigBlock < c1) atomicAdd(&cnt[dm(key[u])], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < D; d += kBigBlock) mat[(size_t)blockIdx.x * D + d] = cnt[d];
    if (cmat) {                                  // two-level: the chunk's coarse-digit counts
        const uint32_t G = D >> sub_bits;
        for (uint32_t g = threadIdx.x; g < G; g += kBigBlock) {
            uint32_t sum = 0;
            for (uint32_t j = 0; j < (1u << sub_bits); j++) sum += cnt[(g << sub_bits) + j];
            cmat[(size_t)blockIdx.x * G + g] = sum;
        }
    }
}

// One thread per digit: its total over all chunks.
__global__ __launch_bounds__(kBlock) void k_digit_totals(const uint32_t *mat, uint32_t nchunks,
                                                         uint32_t D, uint32_t *tot)
{
    const uint32_t d = blockIdx.x * kBlock + threadIdx.x;
    if (d >= D) return;
    uint32_t sum = 0;
#pragma unroll 8
    for (uint32_t b = 0; b < nchunks; b++) sum += mat[(size_t)b * D + d];
    tot[d] = sum;
}

// One thread per digit: per-chunk counts -> each chunk's first output slot of the digit.
__global__ __launch_bounds__(kBlock) void k_digit_offsets(uint32_t *mat, uint32_t nchunks,
                                                          uint32_t D, const uint64_t *start)
{
    const uint32_t d = blockIdx.x * kBlock + threadIdx.x;
    if (d >= D) return;
    uint32_t run = (uint32_t)start[d];
#pragma unroll 8
    for (uint32_t b = 0; b < nchunks; b++) {
        const uint32_t v = mat[(size_t)b * D + d];
        mat[(size_t)b * D + d] = run;
        run += v;
    }
}

template <typename V>
__global__ __launch_bounds__(kBigBlock) void k_digit_scatter(const uint64_t *keys, const V *vals,
                                                             const uint64_t *n_ptr,
                                                             uint64_t capacity, uint32_t D,
                                                             uint32_t chunk, const uint64_t *cdf,
                                                             const uint32_t *mat, ulonglong2 *trec)
{
    extern __shared__ uint32_t dyn[];           // D offsets, then kTop slice CDF entries
    uint32_t *off = dyn, *cl = dyn + D;
    for (uint32_t d = threadIdx.x; d < D; d += kBigBlock) off[d] = mat[(size_t)blockIdx.x * D + d];
    DigitMap dm;
    dm.init(cdf, cl, D);
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    // four records per thread and step: their loads, LDS atomics and stores overlap
    constexpr int U = 4;
    for (uint64_t i0 = c0 + threadIdx.x; i0 < c1; i0 += (uint64_t)kBigBlock * U) {
        uint64_t key[U];
        V val[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t i = i0 + (uint64_t)u * kBigBlock;
            if (i < c1) {
                key[u] = keys[i];
                val[u] = vals[i];
            }
        }
        uint32_t pos[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            if (i0 + (uint64_t)u * kBigBlock < c1) pos[u] = atomicAdd(&off[dm(key[u])], 1u);
#pragma unroll
        for (int u = 0; u < U; u++)
            if (i0 + (uint64_t)u * kBigBlock < c1)
                trec[pos[u]] = make_ulonglong2(key[u], (uint64_t)val[u]);
    }
}

// cstart[c] = first fine bin whose start is >= c*T (so coarse bucket c is the fine bins
// [cstart[c], cstart[c+1])).  One thread per fine bin writes the c values it is first for:
// c in (fofs[f-1] / T, fofs[f] / T].  Entries past N / T keep the fill value nfine.
__global__ __launch_bounds__(kBlock) void k_coarse_starts(const uint64_t *fofs, uint32_t nfine,
                                                          uint32_t target, uint32_t *cstart,
                                                          uint64_t ncoarse)
{
    const uint64_t f = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    if (f > nfine) return;
    const uint64_t hi = fofs[f];
    const uint64_t c_lo = f == 0 ? 0 : fofs[f - 1] / target + 1;
    const uint64_t c_hi = hi / target;        // c*T <= hi
    for (uint64_t c = c_lo; c <= c_hi && c < ncoarse; c++)
        if (f == 0 || c * target > fofs[f - 1]) cstart[c] = (uint32_t)f;
}

// In-LDS bitonic sort of n records, padded with maximal records to the next power of two
// (the arrays must hold that many).
template <typename V>
__device__ void lds_bitonic(uint64_t *K, V *Vv, int n)
{
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int i = n + threadIdx.x; i < P2; i += kBlock) { K[i] = kMax64; Vv[i] = (V)~(V)0; }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P2 / 2; i += kBlock) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t ka = K[lo], kb = K[hi];
                const V va = Vv[lo], vb = Vv[hi];
                const bool gt = rec_less(kb, vb, ka, va);
                if (gt == up) { K[lo] = kb; K[hi] = ka; Vv[lo] = vb; Vv[hi] = va; }
            }
            __syncthreads();
        }
    }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_bucket_sort(const ulonglong2 *trec,
                                                        const uint64_t *fofs, const uint32_t *cstart,
                                                        int Bf, uint64_t *okeys, V *ovals,
                                                        uint32_t *overflow, uint32_t *overflow_n)
{
    constexpr int kCap = Cap<V>::value;
    __shared__ uint64_t K[kCap];
    __shared__ V Vv[kCap];

    const uint32_t f0 = cstart[blockIdx.x], f1 = cstart[blockIdx.x + 1];
    const uint64_t base = fofs[f0];
    const uint64_t n64 = fofs[f1] - base;
    if (n64 == 0) return;
    if (n64 > (uint64_t)kCap) {
        if (threadIdx.x == 0) overflow[atomicAdd(overflow_n, 1u)] = blockIdx.x;
        return;
    }
    const int n = (int)n64;
    const int t = threadIdx.x;
    constexpr int kPer = kCap / kBlock;
    {
        ulonglong2 r[kPer];                 // all loads in flight before the LDS stores
#pragma unroll
        for (int m = 0; m < kPer; m++) {
            const int i = t + m * kBlock;
            if (i < n) r[m] = trec[base + i];
        }
#pragma unroll
        for (int m = 0; m < kPer; m++) {
            const int i = t + m * kBlock;
            if (i < n) { K[i] = r[m].x; Vv[i] = (V)r[m].y; }
        }
    }
    __syncthreads();
    // The records are grouped by fine bin (a run of one bin is a segment).  Each record's
    // final place is its segment's start plus the number of records of the segment that
    // are smaller than it, so every thread places its own records independently.
    const int sh = 64 - Bf;
    int big = 0;
    int pos[kPer];
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * kBlock;
        pos[m] = i;
        if (i >= n) continue;
        const uint64_t k = K[i];
        const V v = Vv[i];
        const uint64_t b = k >> sh;
        int lo = i, hi = i + 1;
        while (lo > 0 && (K[lo - 1] >> sh) == b && i - lo < kSmall) lo--;
        while (hi < n && (K[hi] >> sh) == b && hi - i < kSmall) hi++;
        if ((lo > 0 && (K[lo - 1] >> sh) == b) || (hi < n && (K[hi] >> sh) == b) ||
            hi - lo > kSmall) {
            big = 1;                        // a long segment: the whole bucket is sorted below
            continue;
        }
        int rank = 0;
        for (int j = lo; j < hi; j++) rank += rec_less<V>(K[j], Vv[j], k, v) ? 1 : 0;
        pos[m] = lo + rank;
    }
    if (__syncthreads_or(big)) {
        lds_bitonic<V>(K, Vv, n);
        for (int i = t; i < n; i += kBlock) { okeys[base + i] = K[i]; ovals[base + i] = Vv[i]; }
        return;
    }
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * kBlock;
        if (i < n) { okeys[base + pos[m]] = K[i]; ovals[base + pos[m]] = Vv[i]; }
    }
}

// In-LDS bitonic sort as lds_bitonic, for a workgroup of NT threads.
template <typename V, int NT>
__device__ void lds_bitonic_nt(uint64_t *K, V *Vv, int n)
{
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int i = n + threadIdx.x; i < P2; i += NT) { K[i] = kMax64; Vv[i] = (V)~(V)0; }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P2 / 2; i += NT) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t ka = K[lo], kb = K[hi];
                const V va = Vv[lo], vb = Vv[hi];
                const bool gt = rec_less(kb, vb, ka, va);
                if (gt == up) { K[lo] = kb; K[hi] = ka; Vv[lo] = vb; Vv[hi] = va; }
            }
            __syncthreads();
        }
    }
}

// Exclusive sum over the NT threads of a workgroup (sh: NT / kWave entries).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *sh)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; i++)
        if (i < wv) before += sh[i];
    __syncthreads();
    return before + inc - v;
}

// ---- two-level scatter (large indexes): records go first to one of kCoarse coarse
// digits (a digit's top kCoarseBits bits), then within each coarse digit to its fine
// digits.  Both passes stage a tile of kTile records in LDS, grouped by (coarse or fine)
// digit, and write every group as one run of consecutive 16-byte records, so each
// workgroup store instruction covers whole lines; a chunk's next tile continues the same
// runs.  (A one-pass scatter to 2^15 digits lands runs of a few records each, whose
// partial lines double the bytes written.)
constexpr int kCoarseBits = 8;
constexpr int kCoarse = 1 << kCoarseBits;
constexpr int kPerThread = 8;               // records per thread and step (158 KB of LDS)
constexpr int kTile = kPerThread * kBigBlock;

// One workgroup per coarse digit: per-chunk coarse counts -> each chunk's first slot of
// it (each thread scans a run of consecutive chunks).
__global__ __launch_bounds__(kCoarse) void k_coarse_offsets(uint32_t *cmat, uint32_t nchunks,
                                                            int sub_bits, const uint64_t *start)
{
    __shared__ uint32_t sh_scan[kCoarse / kWave];
    const uint32_t g = blockIdx.x, t = threadIdx.x;
    const uint32_t per = (nchunks + kCoarse - 1) / kCoarse;
    const uint32_t b0 = t * per < nchunks ? t * per : nchunks;
    const uint32_t b1 = b0 + per < nchunks ? b0 + per : nchunks;
    uint32_t sum = 0;
    for (uint32_t b = b0; b < b1; b++) sum += cmat[(size_t)b * kCoarse + g];
    uint32_t run = (uint32_t)start[(size_t)g << sub_bits] + block_excl_sum<kCoarse>(sum, sh_scan);
    for (uint32_t b = b0; b < b1; b++) {
        const uint32_t v = cmat[(size_t)b * kCoarse + g];
        cmat[(size_t)b * kCoarse + g] = run;
        run += v;
    }
}

// Stage up to kTile records (held kPerThread per thread in r, with group id gid[] and rank
// in its group rk[]) grouped by group id in LDS, then write each group's run at run[group].
// G groups (<= 256); cnt holds the tile's group counts on entry.
template <int G>
__device__ __forceinline__ void stage_and_write(const ulonglong2 (&r)[kPerThread],
                                                const uint32_t (&gid)[kPerThread],
                                                const uint32_t (&rk)[kPerThread], int m,
                                                uint32_t *cnt, uint32_t *lofs, uint32_t *run,
                                                ulonglong2 *stage, uint8_t *sg, uint32_t *sh_scan,
                                                ulonglong2 *out)
{
    const int t = threadIdx.x;
    const uint32_t ex = block_excl_sum<kBigBlock>(t < G ? cnt[t] : 0u, sh_scan);
    if (t < G) lofs[t] = ex;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerThread; u++) {
        const int i = t + u * kBigBlock;
        if (i < m) {
            const uint32_t p = lofs[gid[u]] + rk[u];
            stage[p] = r[u];
            sg[p] = (uint8_t)gid[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPerThread; u++) {
        const int j = t + u * kBigBlock;
        if (j < m) {
            const uint32_t g = sg[j];
            out[run[g] + ((uint32_t)j - lofs[g])] = stage[j];
        }
    }
    __syncthreads();
    if (t < G) {
        run[t] += cnt[t];
        cnt[t] = 0;
    }
    __syncthreads();
}

// Pass 1: one workgroup per chunk; coarse digit = digit >> sub_bits.
template <typename V>
__global__ __launch_bounds__(kBigBlock) void k_coarse_scatter(const uint64_t *keys, const V *vals,
                                                              const uint64_t *n_ptr,
                                                              uint64_t capacity, uint32_t D,
                                                              int sub_bits, uint32_t chunk,
                                                              const uint64_t *cdf,
                                                              const uint32_t *coff,
                                                              ulonglong2 *tmp)
{
    __shared__ uint32_t cl[kTop];
    __shared__ ulonglong2 stage[kTile];
    __shared__ uint8_t sg[kTile];
    __shared__ uint32_t cnt[kCoarse], lofs[kCoarse], run[kCoarse];
    __shared__ uint32_t sh_scan[kBigBlock / kWave];
    const int t = threadIdx.x;
    if (t < kCoarse) {
        cnt[t] = 0;
        run[t] = coff[(size_t)blockIdx.x * kCoarse + t];
    }
    DigitMap dm;
    dm.init(cdf, cl, D);                        // (its barrier also orders the lines above)
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    for (uint64_t t0 = c0; t0 < c1; t0 += kTile) {
        const int m = (int)(c1 - t0 < (uint64_t)kTile ? c1 - t0 : (uint64_t)kTile);
        ulonglong2 r[kPerThread];
        uint32_t gid[kPerThread], rk[kPerThread];
#pragma unroll
        for (int u = 0; u < kPerThread; u++) {
            const int i = t + u * kBigBlock;
            if (i < m) {
                const uint64_t key = keys[t0 + i];
                r[u] = make_ulonglong2(key, (uint64_t)vals[t0 + i]);
                gid[u] = dm(key) >> sub_bits;
            }
        }
#pragma unroll
        for (int u = 0; u < kPerThread; u++)
            if (t + u * kBigBlock < m) rk[u] = atomicAdd(&cnt[gid[u]], 1u);
        __syncthreads();
        stage_and_write<kCoarse>(r, gid, rk, m, cnt, lofs, run, stage, sg, sh_scan, tmp);
    }
}

// Pass 2: one workgroup per coarse digit g, over its range of the pass-1 output; fine
// digit (g << sub_bits) + j goes to its final range at fofs.
__global__ __launch_bounds__(kBigBlock) void k_fine_scatter(const ulonglong2 *tmp, uint32_t D,
                                                            int sub_bits, const uint64_t *cdf,
                                                            const uint64_t *fofs,
                                                            ulonglong2 *trec)
{
    constexpr int kMaxSub = 1 << (kDigitBits - kCoarseBits);
    __shared__ uint32_t cl[kTop];
    __shared__ ulonglong2 stage[kTile];
    __shared__ uint8_t sg[kTile];
    __shared__ uint32_t cnt[kMaxSub], lofs[kMaxSub], run[kMaxSub];
    __shared__ uint32_t sh_scan[kBigBlock / kWave];
    const int t = threadIdx.x;
    const uint32_t g = blockIdx.x, S = 1u << sub_bits;
    if (t < kMaxSub) cnt[t] = 0;
    if (t < (int)S) run[t] = (uint32_t)fofs[((size_t)g << sub_bits) + t];
    DigitMap dm;
    dm.init(cdf, cl, D);
    const uint64_t b0 = fofs[(size_t)g << sub_bits], b1 = fofs[(size_t)(g + 1) << sub_bits];
    for (uint64_t t0 = b0; t0 < b1; t0 += kTile) {
        const int m = (int)(b1 - t0 < (uint64_t)kTile ? b1 - t0 : (uint64_t)kTile);
        ulonglong2 r[kPerThread];
        uint32_t gid[kPerThread], rk[kPerThread];
#pragma unroll
        for (int u = 0; u < kPerThread; u++) {
            const int i = t + u * kBigBlock;
            if (i < m) {
                r[u] = tmp[t0 + i];
                gid[u] = dm(r[u].x) & (S - 1);   // pass 1 put the record in digit group g
            }
        }
#pragma unroll
        for (int u = 0; u < kPerThread; u++)
            if (t + u * kBigBlock < m) rk[u] = atomicAdd(&cnt[gid[u]], 1u);
        __syncthreads();
        stage_and_write<kMaxSub>(r, gid, rk, m, cnt, lofs, run, stage, sg, sh_scan, trec);
    }
}

// Digits mode: a coarse bucket is a run of whole digits holding more than kLo and at most
// kCap records (three launches cover the sizes, with workgroups whose LDS and thread
// count fit them).  Its records are binned in LDS by their key's offset from the
// bucket's smallest key, scaled to NS <= kBins bins (about two per record, or fewer when
// kBins caps them so that more workgroups share a CU; monotone in the key),
// the bins are scanned and filled from registers, and every record is then placed by its
// rank inside its bin, as in k_bucket_sort.  A bucket holding a long bin (many equal
// hashes) is bitonic-sorted.  A bucket larger than kCap is appended to the spill list if
// one is given (the next size's list, or the fallback's).  Launched either over every
// bucket (one workgroup each, those of other sizes exit at once) or, with a list, over the
// listed buckets only (a small grid of workgroups taking entries in turn).
template <typename V, int kCap, int kLo, int NT, int kBins>
__device__ __forceinline__ void digit_bucket_one(uint32_t c, const ulonglong2 *trec,
                                                 const uint64_t *fofs, const uint32_t *cstart,
                                                 uint64_t *okeys, V *ovals, uint32_t *spill,
                                                 uint32_t *spill_n, uint64_t *K, V *Vv,
                                                 uint32_t *sub, uint32_t *sh_scan,
                                                 uint64_t *sh_mm)
{
    constexpr int kSub = kBins;                 // bins
    constexpr int kPer = kCap / NT;
    const uint32_t d0 = cstart[c], d1 = cstart[c + 1];
    const uint64_t base = fofs[d0];
    const uint64_t n64 = fofs[d1] - base;
    if (n64 <= (uint64_t)kLo) return;                       // a smaller launch's bucket
    if (n64 > (uint64_t)kCap) {
        if (spill && threadIdx.x == 0) spill[atomicAdd(spill_n, 1u)] = c;
        return;
    }
    const int n = (int)n64;
    const int t = threadIdx.x;

    ulonglong2 r[kPer];
    uint64_t mn = kMax64, mx = 0;
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * NT;
        if (i < n) {
            r[m] = trec[base + i];
            const uint64_t kx = r[m].x;       // (plain compares: no mixed-type min / max)
            mn = kx < mn ? kx : mn;
            mx = kx > mx ? kx : mx;
        }
    }
    // the bucket's smallest and largest key
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const uint64_t a = __shfl_xor(mn, d, kWave), b = __shfl_xor(mx, d, kWave);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if ((t & (kWave - 1)) == 0) {
        sh_mm[t / kWave] = mn;
        sh_mm[NT / kWave + t / kWave] = mx;
    }
    uint32_t NS = 2;
    while (NS < 2 * (uint32_t)n && NS < (uint32_t)kSub) NS <<= 1;
    for (uint32_t b = t; b <= NS; b += NT) sub[b] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT / kWave; i++) {
        const uint64_t a = sh_mm[i], b = sh_mm[i + NT / kWave];
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    const float scale = (float)NS / ((float)(mx - mn) + 1.0f);
    auto bin_of = [&](uint64_t x) -> uint32_t {
        const uint32_t b = (uint32_t)((float)(x - mn) * scale);
        return b < NS ? b : NS - 1;
    };
    uint32_t slot[kPer];
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * NT;
        if (i < n) slot[m] = atomicAdd(&sub[bin_of(r[m].x)], 1u);
    }
    __syncthreads();
    // exclusive scan of sub[0, NS): each thread takes a run of consecutive entries
    const uint32_t per = (NS + NT - 1) / NT;
    const uint32_t b0 = t * per < NS ? t * per : NS, b1 = b0 + per < NS ? b0 + per : NS;
    uint32_t run = 0;
    for (uint32_t b = b0; b < b1; b++) run += sub[b];
    uint32_t acc = block_excl_sum<NT>(run, sh_scan);
    for (uint32_t b = b0; b < b1; b++) {
        const uint32_t c = sub[b];
        sub[b] = acc;
        acc += c;
    }
    if (t == 0) sub[NS] = (uint32_t)n;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * NT;
        if (i < n) {
            const uint32_t at = sub[bin_of(r[m].x)] + slot[m];
            K[at] = r[m].x;
            Vv[at] = (V)r[m].y;
        }
    }
    __syncthreads();
    int pos[kPer];
    int big = 0;
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * NT;
        pos[m] = i;
        if (i >= n) continue;
        const uint64_t k = K[i];
        const V v = Vv[i];
        const uint32_t b = bin_of(k);
        const int lo = (int)sub[b], hi = (int)sub[b + 1];
        if (hi - lo > kSmall) {
            big = 1;
            continue;
        }
        int rank = 0;
        for (int j = lo; j < hi; j++) rank += rec_less<V>(K[j], Vv[j], k, v) ? 1 : 0;
        pos[m] = lo + rank;
    }
    if (__syncthreads_or(big)) {
        lds_bitonic_nt<V, NT>(K, Vv, n);
        for (int i = t; i < n; i += NT) { okeys[base + i] = K[i]; ovals[base + i] = Vv[i]; }
        return;
    }
#pragma unroll
    for (int m = 0; m < kPer; m++) {
        const int i = t + m * NT;
        if (i < n) { okeys[base + pos[m]] = K[i]; ovals[base + pos[m]] = Vv[i]; }
    }
}

// kList: the listed buckets (list, list_n) with any grid; otherwise bucket blockIdx.x.
// (Two instantiations rather than one kernel with both paths, which would hold the
// registers of both.)
template <typename V, int kCap, int kLo, int NT, int kBins = kCap, bool kList = false>
__global__ __launch_bounds__(NT) void k_digit_bucket_sort(const ulonglong2 *trec,
                                                          const uint64_t *fofs,
                                                          const uint32_t *cstart,
                                                          uint64_t *okeys, V *ovals,
                                                          const uint32_t *list,
                                                          const uint32_t *list_n,
                                                          uint32_t *spill, uint32_t *spill_n)
{
    __shared__ uint64_t K[kCap];
    __shared__ V Vv[kCap];
    __shared__ uint32_t sub[kBins + 1];
    __shared__ uint32_t sh_scan[NT / kWave];
    __shared__ uint64_t sh_mm[2 * (NT / kWave)];
    if constexpr (!kList) {
        digit_bucket_one<V, kCap, kLo, NT, kBins>(blockIdx.x, trec, fofs, cstart, okeys, ovals,
                                                  spill, spill_n, K, Vv, sub, sh_scan, sh_mm);
        return;
    }
    const uint32_t nl = *list_n;
    for (uint32_t i = blockIdx.x; i < nl; i += gridDim.x) {     // workgroup-uniform
        digit_bucket_one<V, kCap, kLo, NT, kBins>(list[i], trec, fofs, cstart, okeys, ovals,
                                                  spill, spill_n, K, Vv, sub, sh_scan, sh_mm);
        __syncthreads();                                        // LDS reused by the next one
    }
}

// Fallback for coarse buckets larger than the LDS capacity: sort runs of kCap records in
// LDS into the output, then merge pairs of runs by ranking (an element's output index is
// its index in its own run plus the number of smaller elements in the other run),
// ping-ponging between the output and the bucket's own part of the scatter buffer (16
// bytes per record, reused as separate key and value arrays once its records are read).
template <typename V>
__device__ uint64_t rank_in(const uint64_t *K, const V *Vv, uint64_t lo, uint64_t n, uint64_t kx,
                            V vx)
{
    uint64_t l = 0, len = n;                 // count of elements < (kx, vx) in [lo, lo+n)
    while (len > 0) {
        const uint64_t half = len / 2;
        if (rec_less(K[lo + l + half], Vv[lo + l + half], kx, vx)) { l += half + 1; len -= half + 1; }
        else len = half;
    }
    return l;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_bucket_sort_big(ulonglong2 *trec, const uint64_t *fofs,
                                                            const uint32_t *cstart,
                                                            const uint32_t *overflow,
                                                            const uint32_t *overflow_n,
                                                            uint64_t *okeys, V *ovals)
{
    constexpr int kCap = Cap<V>::value;
    __shared__ uint64_t K[kCap];
    __shared__ V Vv[kCap];
    const uint32_t nov = *overflow_n;
    for (uint32_t oi = blockIdx.x; oi < nov; oi += gridDim.x) {
        const uint32_t c = overflow[oi];
        const uint64_t base = fofs[cstart[c]];
        const uint64_t n = fofs[cstart[c + 1]] - base;
        for (uint64_t r0 = 0; r0 < n; r0 += kCap) {
            const int m = (int)min((uint64_t)kCap, n - r0);
            for (int i = threadIdx.x; i < m; i += kBlock) {
                const ulonglong2 r = trec[base + r0 + i];
                K[i] = r.x;
                Vv[i] = (V)r.y;
            }
            __syncthreads();
            lds_bitonic<V>(K, Vv, m);
            for (int i = threadIdx.x; i < m; i += kBlock) {
                okeys[base + r0 + i] = K[i];
                ovals[base + r0 + i] = Vv[i];
            }
            __syncthreads();
        }
        uint64_t *sk = okeys + base, *dk = (uint64_t *)(trec + base);
        V *sv = ovals + base, *dv = (V *)(dk + n);
        bool in_out = true;
        for (uint64_t width = kCap; width < n; width *= 2) {
            for (uint64_t lo = 0; lo < n; lo += 2 * width) {
                const uint64_t mid = min(lo + width, n), hi = min(lo + 2 * width, n);
                for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
                    const uint64_t kx = sk[i];
                    const V vx = sv[i];
                    uint64_t pos;
                    if (i < mid) pos = lo + (i - lo) + rank_in(sk, sv, mid, hi - mid, kx, vx);
                    else pos = lo + (i - mid) + rank_in(sk, sv, lo, mid - lo, kx, vx);
                    dk[pos] = kx;
                    dv[pos] = vx;
                }
            }
            __syncthreads();
            uint64_t *tk = sk; sk = dk; dk = tk;
            V *tv = sv; sv = dv; dv = tv;
            in_out = !in_out;
        }
        if (!in_out) {
            for (uint64_t i = threadIdx.x; i < n; i += kBlock) { okeys[base + i] = sk[i]; ovals[base + i] = sv[i]; }
        }
        __syncthreads();
    }
}

// Raise the dynamic-LDS limit of the digit kernels to the CU's 160 KB (once per process).
template <typename V>
hipError_t allow_digit_lds()
{
    static hipError_t once = [] {
        const int bytes = 160 * 1024;
        hipError_t e = hipFuncSetAttribute((const void *)k_digit_count,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_digit_scatter<V>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        return e;
    }();
    return once;
}

template <typename V>
hipError_t sort_impl(const SortPlan &sp, const SortWs &w, uint64_t *keys, V *vals,
                     const uint64_t *n_ptr, uint64_t capacity, hipStream_t s)
{
    hipError_t e;
    if ((e = fill_u32(w.overflow_n, 0, 2, s)) != hipSuccess) return e;
    if (sp.digits) {
        const uint32_t D = (uint32_t)sp.nfine, nc = (uint32_t)sp.nchunks;
        const uint32_t ch = (uint32_t)sp.chunk;
        const unsigned dg = (D + kBlock - 1) / kBlock;
        if ((e = fill_u32(w.top, 0, kTop, s)) != hipSuccess) return e;
        GD_LAUNCH(k_top_hist, dim3(256), dim3(kBigBlock), 0, s, keys, n_ptr, capacity, w.top);
        if ((e = exclusive_scan_u32(w.top, w.cdf, kTop, w.scan_tmp, s)) != hipSuccess) return e;
        // LDS sized to the digits: 80 KB at 2^14 digits, two workgroups per CU
        const size_t lds = ((size_t)D + kTop) * sizeof(uint32_t);
        if ((e = allow_digit_lds<V>()) != hipSuccess) return e;
        const int sb = sp.two_level ? sp.Bf - kCoarseBits : 0;
        GD_LAUNCH(k_digit_count, dim3(nc), dim3(kBigBlock), lds, s, keys, n_ptr, capacity, D, ch,
                  (const uint64_t *)w.cdf, w.hist, sp.two_level ? w.cmat : nullptr, sb);
        GD_LAUNCH(k_digit_totals, dim3(dg), dim3(kBlock), 0, s, (const uint32_t *)w.hist, nc, D,
                  w.tot);
        if ((e = exclusive_scan_u32(w.tot, w.fofs, D, w.scan_tmp, s)) != hipSuccess) return e;
        if (sp.two_level) {
            GD_LAUNCH(k_coarse_offsets, dim3(kCoarse), dim3(kCoarse), 0, s, w.cmat, nc, sb,
                      (const uint64_t *)w.fofs);
            GD_LAUNCH(k_coarse_scatter<V>, dim3(nc), dim3(kBigBlock), 0, s, keys, vals, n_ptr,
                      capacity, D, sb, ch, (const uint64_t *)w.cdf, (const uint32_t *)w.cmat,
                      w.tmp);
            GD_LAUNCH(k_fine_scatter, dim3(kCoarse), dim3(kBigBlock), 0, s,
                      (const ulonglong2 *)w.tmp, D, sb, (const uint64_t *)w.cdf,
                      (const uint64_t *)w.fofs, w.trec);
        } else {
            GD_LAUNCH(k_digit_offsets, dim3(dg), dim3(kBlock), 0, s, w.hist, nc, D,
                      (const uint64_t *)w.fofs);
            GD_LAUNCH(k_digit_scatter<V>, dim3(nc), dim3(kBigBlock), lds, s, keys, vals, n_ptr,
                      capacity, D, ch, (const uint64_t *)w.cdf, (const uint32_t *)w.hist,
                      w.trec);
        }
    } else {
        if ((e = fill_u32(w.hist, 0, sp.nfine, s)) != hipSuccess) return e;
        const unsigned grid = 4096;
        GD_LAUNCH(k_hist, dim3(grid), dim3(kBlock), 0, s, keys, n_ptr, capacity, sp.Bf, w.hist,
                  w.rank);
        if ((e = exclusive_scan_u32(w.hist, w.fofs, sp.nfine, w.scan_tmp, s)) != hipSuccess)
            return e;
        GD_LAUNCH(k_scatter<V>, dim3(grid), dim3(kBlock), 0, s, keys, vals, n_ptr, capacity,
                  sp.Bf, (const uint64_t *)w.fofs, (const uint32_t *)w.rank, w.trec);
    }
    if ((e = fill_u32(w.cstart, (uint32_t)sp.nfine, sp.ncoarse + 1, s)) != hipSuccess) return e;
    GD_LAUNCH(k_coarse_starts, dim3((unsigned)((sp.nfine + kBlock) / kBlock)), dim3(kBlock), 0, s,
              (const uint64_t *)w.fofs, (uint32_t)sp.nfine, (uint32_t)sp.target, w.cstart,
              (uint64_t)sp.ncoarse + 1);
    if (sp.digits) {
        // buckets by size: up to a quarter, a half and the whole of the largest capacity
        // (the half-size launch with a quarter as many bins: 53 KB of LDS, three
        // workgroups per CU, for the ~2.5K-record buckets of the two-level sort)
        constexpr int C = DCap<V>::value;
        const dim3 g((unsigned)sp.ncoarse);
        const ulonglong2 *tr = w.trec;
        const uint64_t *fo = w.fofs;
        const uint32_t *cs = w.cstart;
        // the half-size launch lists the larger buckets for the largest launch, which takes
        // them with a small grid (one workgroup per CU) instead of a workgroup per bucket
        uint32_t *blist_n = w.overflow_n + 1;
        GD_LAUNCH((k_digit_bucket_sort<V, C / 4, 0, kBlock>), g, dim3(kBlock), 0, s, tr, fo, cs,
                  keys, vals, nullptr, nullptr, nullptr, nullptr);
        GD_LAUNCH((k_digit_bucket_sort<V, C / 2, C / 4, 2 * kBlock, C / 8>), g, dim3(2 * kBlock),
                  0, s, tr, fo, cs, keys, vals, nullptr, nullptr, w.blist, blist_n);
        const unsigned gbig = sp.ncoarse < 256 ? (unsigned)sp.ncoarse : 256u;
        GD_LAUNCH((k_digit_bucket_sort<V, C, C / 2, kBigBlock, C, true>), dim3(gbig),
                  dim3(kBigBlock), 0, s, tr, fo, cs, keys, vals, (const uint32_t *)w.blist,
                  (const uint32_t *)blist_n, w.overflow, w.overflow_n);
    }
    else
        GD_LAUNCH(k_bucket_sort<V>, dim3((unsigned)sp.ncoarse), dim3(kBlock), 0, s,
                  (const ulonglong2 *)w.trec, (const uint64_t *)w.fofs,
                  (const uint32_t *)w.cstart, sp.Bf, keys, vals, w.overflow, w.overflow_n);
    GD_LAUNCH(k_bucket_sort_big<V>, dim3(64), dim3(kBlock), 0, s, w.trec,
              (const uint64_t *)w.fofs, (const uint32_t *)w.cstart,
              (const uint32_t *)w.overflow, (const uint32_t *)w.overflow_n, keys, vals);
    return hipGetLastError();
}

}  // namespace

SortPlan sort_plan(uint64_t expected_records, uint64_t capacity, int val_bytes)
{
    SortPlan sp;
    const uint64_t dcap = val_bytes == 4 ? DCap<uint32_t>::value : DCap<uint64_t>::value;
    // digits mode while balanced digits (at most 2^15 of them, about 512 records each when
    // there are fewer) stay within three quarters of the largest bucket capacity
    if (capacity > 0 && capacity <= ((dcap * 3 / 4) << kDigitBits)) {
        // about 512 records per digit for small indexes; large ones keep 2^14 digits while
        // a digit holds at most ~6K records: twice the records of one digit per chunk
        // (longer runs of scattered records, half the LDS of 2^15 counters), buckets still
        // within the largest bucket launch
        int Bd = 4;
        while (Bd < kDigitBits && (capacity >> Bd) > 512) Bd++;
        // from 2^24 records: 2^15 digits through the two-level scatter (buckets of ~2.5K
        // records at 100M, two bucket-sort workgroups per CU); below, one scatter pass
        sp.two_level = capacity >= ((uint64_t)1 << 24);
        if (!sp.two_level && Bd == kDigitBits && (capacity >> (kDigitBits - 1)) <= 6144)
            Bd = kDigitBits - 1;
        sp.digits = true;
        sp.Bf = Bd;
        sp.nfine = (size_t)1 << Bd;
        // chunks of at least 32K records (a multiple of the 4,096 a workgroup step takes),
        // as few as fill 256 CUs at once (two workgroups per CU up to 2^14 digits, one
        // above): the longer a chunk, the longer its run of records in each digit's range
        // (short scattered runs cost partial-line writes)
        const uint64_t slots = Bd <= 14 && !sp.two_level ? 512 : 256;
        uint64_t chunk = (capacity + slots - 1) / slots;
        chunk = (chunk + 4095) / 4096 * 4096;
        if (chunk < 32768) chunk = 32768;
        sp.chunk = (size_t)chunk;
        sp.nchunks = (size_t)((capacity + chunk - 1) / chunk);
        sp.target = (capacity >> Bd) > 512 ? 2048 : 512;
        sp.ncoarse = (size_t)(capacity / sp.target) + 2;
        return sp;
    }
    int Bf = 4;
    while (Bf < 26 && (expected_records >> Bf) > 2) Bf++;
    sp.digits = false;
    sp.two_level = false;
    sp.nchunks = 0;
    sp.chunk = 0;
    sp.Bf = Bf;
    sp.nfine = (size_t)1 << Bf;
    sp.target = val_bytes == 4 ? 2048 : 1024;
    sp.ncoarse = (size_t)(capacity / sp.target) + 2;
    return sp;
}

size_t sort_top_bins() { return kTop; }

hipError_t launch_sort(const SortPlan &sp, const SortWs &w, uint64_t *keys, void *vals,
                       int val_bytes, const uint64_t *n_ptr, uint64_t capacity, hipStream_t s)
{
    if (val_bytes == 4) return sort_impl<uint32_t>(sp, w, keys, (uint32_t *)vals, n_ptr, capacity, s);
    return sort_impl<uint64_t>(sp, w, keys, (uint64_t *)vals, n_ptr, capacity, s);
}

}  // namespace gd
