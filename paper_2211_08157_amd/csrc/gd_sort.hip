// Sort of the reference minimizer records by (hash, val) for the seed index.
//
// Most-significant-digit bucketing: the top B bits of the 64-bit hash pick one of 2^B
// buckets (hashes are uniform, so B is chosen for ~512 records per bucket).  A histogram
// and a scan give bucket offsets, a scatter moves every record into its bucket, and one
// workgroup per bucket finishes the bucket in LDS: a counting sort on the next 8 hash
// bits followed by an insertion sort of each (tiny) sub-bucket, or an LDS bitonic sort
// when a sub-bucket is large (many equal hashes).  Buckets larger than the LDS capacity
// are listed and sorted by a fallback kernel in global memory (LDS-sorted runs merged by
// ranking).  (hash, val) pairs are unique, so the result does not depend on the order in
// which the scatter's atomics land.
#include "gd_internal.h"

namespace gd {

namespace {

// records a workgroup sorts in LDS (a power of two, so bitonic padding fits)
template <typename V> struct Cap { static constexpr int value = sizeof(V) == 4 ? 2048 : 1024; };
constexpr int kSmall = 24;          // sub-bucket size handled by insertion sort

template <typename V>
__device__ __forceinline__ bool rec_less(uint64_t ka, V va, uint64_t kb, V vb)
{
    return ka < kb || (ka == kb && va < vb);
}

__global__ __launch_bounds__(kBlock) void k_hist(const uint64_t *keys, const uint64_t *n_ptr,
                                                 uint64_t capacity, int B, uint32_t *hist)
{
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock)
        atomicAdd(&hist[keys[i] >> (64 - B)], 1u);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t *keys, const V *vals,
                                                    const uint64_t *n_ptr, uint64_t capacity,
                                                    int B, const uint64_t *bofs,
                                                    uint32_t *cursor, uint64_t *tkeys, V *tvals)
{
    uint64_t n = *n_ptr;
    if (n > capacity) n = capacity;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t key = keys[i];
        const uint64_t b = key >> (64 - B);
        const uint64_t pos = bofs[b] + atomicAdd(&cursor[b], 1u);
        tkeys[pos] = key;
        tvals[pos] = vals[i];
    }
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
__global__ __launch_bounds__(kBlock) void k_bucket_sort(const uint64_t *tkeys, const V *tvals,
                                                        const uint64_t *bofs, int B,
                                                        uint64_t *okeys, V *ovals,
                                                        uint32_t *overflow, uint32_t *overflow_n)
{
    constexpr int kCap = Cap<V>::value;
    __shared__ uint64_t K0[kCap], K1[kCap];
    __shared__ V V0[kCap], V1[kCap];
    __shared__ uint32_t cnt[256], start[257], fill[256];
    __shared__ uint32_t sh_max;

    const uint32_t b = blockIdx.x;
    const uint64_t base = bofs[b];
    const uint64_t n64 = bofs[b + 1] - base;
    if (n64 == 0) return;
    if (n64 > (uint64_t)kCap) {
        if (threadIdx.x == 0) overflow[atomicAdd(overflow_n, 1u)] = b;
        return;
    }
    const int n = (int)n64;
    const int t = threadIdx.x;
    for (int i = t; i < n; i += kBlock) { K0[i] = tkeys[base + i]; V0[i] = tvals[base + i]; }
    cnt[t] = 0;
    fill[t] = 0;
    if (t == 0) sh_max = 0;
    __syncthreads();
    const int sh = 56 - B;           // next 8 bits below the bucket bits
    for (int i = t; i < n; i += kBlock) atomicAdd(&cnt[(K0[i] >> sh) & 255u], 1u);
    __syncthreads();
    if (t < kWave) {                 // one wave scans the 256 counts
        uint32_t c[4], s4 = 0, mx = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) { c[j] = cnt[4 * t + j]; s4 += c[j]; mx = c[j] > mx ? c[j] : mx; }
        const uint32_t inc = wave_incl_scan<uint32_t>(s4);
        uint32_t run = inc - s4;
#pragma unroll
        for (int j = 0; j < 4; j++) { start[4 * t + j] = run; run += c[j]; }
        if (t == kWave - 1) start[256] = inc;
        atomicMax(&sh_max, mx);
    }
    __syncthreads();
    for (int i = t; i < n; i += kBlock) {
        const uint32_t d = (K0[i] >> sh) & 255u;
        const uint32_t slot = start[d] + atomicAdd(&fill[d], 1u);
        K1[slot] = K0[i];
        V1[slot] = V0[i];
    }
    __syncthreads();
    if (sh_max <= (uint32_t)kSmall) {
        const int lo = start[t], hi = start[t + 1];
        for (int i = lo + 1; i < hi; i++) {
            const uint64_t kx = K1[i];
            const V vx = V1[i];
            int j = i - 1;
            while (j >= lo && rec_less(kx, vx, K1[j], V1[j])) {
                K1[j + 1] = K1[j];
                V1[j + 1] = V1[j];
                j--;
            }
            K1[j + 1] = kx;
            V1[j + 1] = vx;
        }
        __syncthreads();
    } else {
        lds_bitonic<V>(K1, V1, n);
    }
    for (int i = t; i < n; i += kBlock) { okeys[base + i] = K1[i]; ovals[base + i] = V1[i]; }
}

// Fallback for buckets larger than the LDS capacity: sort runs of kCap in LDS (in place in the
// scatter buffer), then merge pairs of runs by ranking (an element's output index is its
// index in its own run plus the number of smaller elements in the other run), ping-
// ponging between the scatter buffer and the output.
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
__global__ __launch_bounds__(kBlock) void k_bucket_sort_big(uint64_t *tkeys, V *tvals,
                                                            const uint64_t *bofs,
                                                            const uint32_t *overflow,
                                                            const uint32_t *overflow_n,
                                                            uint64_t *okeys, V *ovals)
{
    constexpr int kCap = Cap<V>::value;
    __shared__ uint64_t K[kCap];
    __shared__ V Vv[kCap];
    const uint32_t nov = *overflow_n;
    for (uint32_t oi = blockIdx.x; oi < nov; oi += gridDim.x) {
        const uint32_t b = overflow[oi];
        const uint64_t base = bofs[b];
        const uint64_t n = bofs[b + 1] - base;
        for (uint64_t r0 = 0; r0 < n; r0 += kCap) {
            const int m = (int)min((uint64_t)kCap, n - r0);
            for (int i = threadIdx.x; i < m; i += kBlock) {
                K[i] = tkeys[base + r0 + i];
                Vv[i] = tvals[base + r0 + i];
            }
            __syncthreads();
            lds_bitonic<V>(K, Vv, m);
            for (int i = threadIdx.x; i < m; i += kBlock) {
                tkeys[base + r0 + i] = K[i];
                tvals[base + r0 + i] = Vv[i];
            }
            __syncthreads();
        }
        uint64_t *sk = tkeys + base, *dk = okeys + base;
        V *sv = tvals + base, *dv = ovals + base;
        bool in_out = false;
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

template <typename V>
hipError_t sort_impl(const SortPlan &sp, const SortWs &w, uint64_t *keys, V *vals,
                     const uint64_t *n_ptr, uint64_t capacity, hipStream_t s)
{
    hipError_t e;
    if ((e = fill_u32(w.hist, 0, sp.nbuckets, s)) != hipSuccess) return e;
    if ((e = fill_u32(w.cursor, 0, sp.nbuckets, s)) != hipSuccess) return e;
    if ((e = fill_u32(w.overflow_n, 0, 1, s)) != hipSuccess) return e;
    const unsigned grid = 4096;
    GD_LAUNCH(k_hist, dim3(grid), dim3(kBlock), 0, s, keys, n_ptr, capacity, sp.B, w.hist);
    if ((e = exclusive_scan_u32(w.hist, w.bofs, sp.nbuckets, w.scan_tmp, s)) != hipSuccess) return e;
    GD_LAUNCH(k_scatter<V>, dim3(grid), dim3(kBlock), 0, s, keys, vals, n_ptr, capacity,
                       sp.B, w.bofs, w.cursor, w.tkeys, (V *)w.tvals);
    GD_LAUNCH(k_bucket_sort<V>, dim3((unsigned)sp.nbuckets), dim3(kBlock), 0, s, w.tkeys,
                       (const V *)w.tvals, w.bofs, sp.B, keys, vals, w.overflow, w.overflow_n);
    GD_LAUNCH(k_bucket_sort_big<V>, dim3(64), dim3(kBlock), 0, s, w.tkeys, (V *)w.tvals,
                       w.bofs, w.overflow, w.overflow_n, keys, vals);
    return hipGetLastError();
}

}  // namespace

SortPlan sort_plan(uint64_t expected_records)
{
    SortPlan sp;
    int B = 1;
    while (B < 22 && (expected_records >> B) > 512) B++;
    sp.B = B;
    sp.nbuckets = (size_t)1 << B;
    return sp;
}

hipError_t launch_sort(const SortPlan &sp, const SortWs &w, uint64_t *keys, void *vals,
                       int val_bytes, const uint64_t *n_ptr, uint64_t capacity, hipStream_t s)
{
    if (val_bytes == 4) return sort_impl<uint32_t>(sp, w, keys, (uint32_t *)vals, n_ptr, capacity, s);
    return sort_impl<uint64_t>(sp, w, keys, (uint64_t *)vals, n_ptr, capacity, s);
}

}  // namespace gd
