// Device-side building blocks shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr uint64_t kMax64 = ~0ull;

constexpr uint32_t kMaxPattern = 256;

// A keep/skip pattern (Section 3: P[0..p-1], weight x; 1 <= p <= 256).  Passed by value
// to kernels.  Patterns of up to 64 characters (all the paper uses) live in `mask` and
// take the bit-mask paths; longer ones also use `hi` and the rank-walking paths.
struct Pattern {
    uint64_t mask;                // bit t set iff P[t] == '1', t < 64
    uint64_t hi[3];               // bit t - 64 - 64i of hi[i] for P[64..256)
    uint32_t p, x;
    uint8_t ones[kMaxPattern];    // positions of the ones in ascending order
};

__host__ __device__ __forceinline__ uint32_t popc64(uint64_t v)
{
#ifdef __HIP_DEVICE_COMPILE__
    return (uint32_t)__popcll(v);
#else
    return (uint32_t)__builtin_popcountll(v);
#endif
}

__host__ __device__ __forceinline__ bool pattern_bit(const Pattern &P, uint32_t t)
{
    return t < 64 ? (P.mask >> t) & 1ull : (P.hi[(t - 64) >> 6] >> ((t - 64) & 63)) & 1ull;
}

// Ones of P among its first n characters (n <= p).
__host__ __device__ __forceinline__ uint32_t ones_below(const Pattern &P, uint32_t n)
{
    if (n < 64) return popc64(P.mask & ((1ull << n) - 1));
    uint32_t c = popc64(P.mask);
    for (uint32_t i = 0; i < 3; i++) {
        const uint32_t lo = 64 + 64 * i;
        if (n <= lo) break;
        const uint32_t take = n - lo >= 64 ? 64 : n - lo;
        c += popc64(take == 64 ? P.hi[i] : (P.hi[i] & ((1ull << take) - 1)));
    }
    return c;
}

// splitmix64 output function (the k-mer hash; Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Thomas Wang's 64-bit integer hash restricted to the 2k-bit code space (each step masked
// to 2k bits, as minimap2 applies it to k-mer codes): the paper's k-mer hash (Section
// 3.6.1).  Every step is invertible on the masked space, so it permutes the codes.
__device__ __forceinline__ uint64_t wang64(uint64_t key, uint64_t mask)
{
    key = (~key + (key << 21)) & mask;
    key = key ^ (key >> 24);
    key = ((key + (key << 3)) + (key << 8)) & mask;
    key = key ^ (key >> 14);
    key = ((key + (key << 2)) + (key << 4)) & mask;
    key = key ^ (key >> 28);
    key = (key + (key << 31)) & mask;
    return key;
}

// mix64 of a code below 2^62 (k <= 31): z >> 30 then fits 32 bits, so the first
// xor-shift leaves the high word alone and is one funnel shift and one xor.
__device__ __forceinline__ uint64_t mix64_short(uint64_t z)
{
    const uint32_t lo = (uint32_t)z, hi = (uint32_t)(z >> 32);
    z = ((uint64_t)hi << 32) | (lo ^ __builtin_amdgcn_alignbit(hi, lo, 30));
    z *= 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// k-mer hash of a canonical code: kHash 0 = splitmix64 finalizer of a code of k <= 31
// bases, 1 = Thomas Wang's hash, 2 = splitmix64 finalizer of any code (k = 32).
template <int kHash>
__device__ __forceinline__ uint64_t kmer_hash(uint64_t code, uint64_t mask)
{
    if constexpr (kHash == 1) return wang64(code, mask);
    else if constexpr (kHash == 2) return mix64(code);
    else return mix64_short(code);
}

// Pattern rotated right by a: bit t set iff P[(t - a) mod p] == '1' (p <= 64 only).
__host__ __device__ __forceinline__ uint64_t rotated_mask(const Pattern &P, uint32_t a)
{
    const uint64_t full = P.p == 64 ? kMax64 : ((1ull << P.p) - 1);
    if (a == 0) return P.mask;
    return ((P.mask << a) | (P.mask >> (P.p - a))) & full;
}

// Kept bases of a length-L sequence under shift a: floor(L/p)*x + ones of the rotated
// pattern among the first L mod p phases.
__device__ __forceinline__ uint64_t kept_count(const Pattern &P, uint64_t L, uint32_t a)
{
    const uint64_t q = L / P.p;
    const uint32_t rem = (uint32_t)(L - q * P.p);
    if (P.p > 64) {
        // phases t < rem map to pattern positions (t - a) mod p: [p - a, p - a + min(rem,
        // a)) before the wrap, [0, rem - a) after it
        if (a == 0) return q * P.x + ones_below(P, rem);
        const uint32_t head = rem < a ? rem : a;
        uint64_t c = ones_below(P, P.p - a + head) - ones_below(P, P.p - a);
        if (rem > a) c += ones_below(P, rem - a);
        return q * P.x + c;
    }
    const uint64_t m = rotated_mask(P, a);
    const uint64_t low = rem == 64 ? m : (m & ((1ull << rem) - 1));
    return q * P.x + (uint64_t)__popcll(low);
}

// Ones of P with u < p - a (those that do not wrap under shift a); x when a == 0.
__device__ __forceinline__ uint32_t kept_front(const Pattern &P, uint32_t a)
{
    if (a == 0) return P.x;
    if (P.p > 64) return ones_below(P, P.p - a);
    return (uint32_t)__popcll(P.mask & ((1ull << (P.p - a)) - 1));
}

// Offset within a period of the r-th kept phase under shift a (0 <= r < x).  The ones
// u_i of P move to (u_i + a) mod p; those with u_i >= p - a wrap to the front.
__device__ __forceinline__ uint32_t kept_phase(const Pattern &P, uint32_t a, uint32_t r)
{
    const uint32_t front = kept_front(P, a);
    uint32_t idx = r + front;
    if (idx >= P.x) idx -= P.x;
    uint32_t v = P.ones[idx] + a;
    if (v >= P.p) v -= P.p;
    return v;
}

// Original coordinate of the li-th kept base of a sequence under shift a.
__device__ __forceinline__ uint64_t orig_of(const Pattern &P, uint64_t li, uint32_t a)
{
    const uint64_t q = li / P.x;
    const uint32_t r = (uint32_t)(li - q * P.x);
    return q * P.p + kept_phase(P, a, r);
}

// Last s in [0, n] with a[s] <= v (a non-decreasing, a[0] <= v).
__device__ __forceinline__ uint32_t last_le(const uint64_t *a, uint32_t n, uint64_t v)
{
    uint32_t lo = 0, hi = n;              // invariant: a[lo] <= v, answer in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (a[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// First s in [0, n] with a[s] >= v, n + 1 if none.
__device__ __forceinline__ uint32_t first_ge(const uint64_t *a, uint32_t n, uint64_t v)
{
    uint32_t lo = 0, hi = n + 1;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Wave64 inclusive prefix sum.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Workgroup exclusive prefix sum over kBlock threads; returns the exclusive value and
// writes the workgroup total to *total.  `sh` must hold kBlock / kWave elements.
template <typename T, int NT = kBlock>
__device__ __forceinline__ T block_excl_scan(T v, T *sh, T *total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; i++) {
        const T s = sh[i];
        if (i < wv) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ void set_status(uint32_t *status, uint32_t bits)
{
    if (status) atomicOr(status, bits);
}

}  // namespace gd
