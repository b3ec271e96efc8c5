// Fill kernels (used instead of memset so calls stay safe to capture in a HIP graph) and a
// device-wide exclusive scan (one launch for small inputs, two up to 4M, three beyond).
#include "gd_internal.h"

namespace gd {

namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, T v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

template <typename T>
hipError_t fill(T *p, T v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    GD_LAUNCH(k_fill<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

constexpr int kItems = 16;                      // items per thread
constexpr size_t kTile = (size_t)kBlock * kItems;

// Phase 1: per-block sums.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const Tin *in, size_t n, uint64_t *bsum)
{
    __shared__ uint64_t sh[kBlock / kWave];
    const size_t base = blockIdx.x * kTile;
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const size_t idx = base + (size_t)i * kBlock + threadIdx.x;
        if (idx < n) acc += (uint64_t)in[idx];
    }
    uint64_t tot;
    block_excl_scan<uint64_t>(acc, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Phase 2: exclusive scan of the block sums by one workgroup (any number of blocks).
__global__ __launch_bounds__(kBlock) void k_scan_top(uint64_t *bsum, size_t nb)
{
    __shared__ uint64_t sh[kBlock / kWave];
    uint64_t carry = 0;
    for (size_t b0 = 0; b0 < nb; b0 += kBlock) {
        const size_t i = b0 + threadIdx.x;
        const uint64_t v = i < nb ? bsum[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan<uint64_t>(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

// Phase 3: per-block exclusive scan plus the block offset; out[n] = total.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const Tin *in, uint64_t *out, size_t n,
                                                       const uint64_t *bsum, size_t nb)
{
    __shared__ uint64_t sh[kBlock / kWave];
    const size_t base = blockIdx.x * kTile + (size_t)threadIdx.x * kItems;   // contiguous
    uint64_t v[kItems];
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const size_t idx = base + i;
        v[i] = idx < n ? (uint64_t)in[idx] : 0;
        acc += v[i];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<uint64_t>(acc, sh, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const size_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = bsum[nb];
}

// Phases 2 and 3 in one launch for up to kFusedBlocks blocks: each block adds up the sums of
// the blocks before it (a few hundred values) instead of waiting for a separate top scan.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_scan_apply_fused(const Tin *in, uint64_t *out,
                                                             size_t n, const uint64_t *bsum,
                                                             size_t nb)
{
    __shared__ uint64_t sh[kBlock / kWave];
    uint64_t off = 0;
    for (size_t b0 = 0; b0 < blockIdx.x; b0 += kBlock) {        // uniform in the block
        const size_t i = b0 + threadIdx.x;
        uint64_t part;
        block_excl_scan<uint64_t>(i < blockIdx.x ? bsum[i] : 0, sh, &part);
        off += part;
    }
    const size_t base = blockIdx.x * kTile + (size_t)threadIdx.x * kItems;   // contiguous
    uint64_t v[kItems];
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const size_t idx = base + i;
        v[i] = idx < n ? (uint64_t)in[idx] : 0;
        acc += v[i];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<uint64_t>(acc, sh, &tot) + off;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const size_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = off + tot;
}

// Small inputs: one workgroup walks the tiles in order with a running carry (one launch
// instead of three).
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_scan_single(const Tin *in, uint64_t *out, size_t n)
{
    __shared__ uint64_t sh[kBlock / kWave];
    uint64_t carry = 0;
    for (size_t base0 = 0; base0 < n; base0 += kTile) {
        const size_t base = base0 + (size_t)threadIdx.x * kItems;
        uint64_t v[kItems];
        uint64_t acc = 0;
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const size_t idx = base + i;
            v[i] = idx < n ? (uint64_t)in[idx] : 0;
            acc += v[i];
        }
        uint64_t tot;
        uint64_t run = block_excl_scan<uint64_t>(acc, sh, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const size_t idx = base + i;
            if (idx < n) out[idx] = run;
            run += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

constexpr size_t kSingleScan = 16 * kTile;      // 65,536 inputs
constexpr size_t kFusedBlocks = 1024;           // up to 4M inputs: two launches

template <typename Tin>
hipError_t scan(const Tin *in, uint64_t *out, size_t n, uint64_t *scratch, hipStream_t s)
{
    if (n == 0) return fill<uint64_t>(out, 0, 1, s);
    if (n <= kSingleScan) {
        GD_LAUNCH(k_scan_single<Tin>, dim3(1), dim3(kBlock), 0, s, in, out, n);
        return hipGetLastError();
    }
    const size_t nb = (n + kTile - 1) / kTile;
    GD_LAUNCH(k_scan_reduce<Tin>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, scratch);
    if (nb <= kFusedBlocks) {
        GD_LAUNCH(k_scan_apply_fused<Tin>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                  (const uint64_t *)scratch, nb);
        return hipGetLastError();
    }
    GD_LAUNCH(k_scan_top, dim3(1), dim3(kBlock), 0, s, scratch, nb);
    GD_LAUNCH(k_scan_apply<Tin>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                       (const uint64_t *)scratch, nb);
    return hipGetLastError();
}

}  // namespace

hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) { return fill(p, v, n, s); }

size_t scan_scratch(size_t n) { return (n + kTile - 1) / kTile + 2; }

hipError_t exclusive_scan_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *scratch,
                              hipStream_t s)
{
    return scan<uint64_t>(in, out, n, scratch, s);
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint64_t *out, size_t n, uint64_t *scratch,
                              hipStream_t s)
{
    return scan<uint32_t>(in, out, n, scratch, s);
}

}  // namespace gd
