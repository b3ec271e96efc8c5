// Seeding kernels: exact-match lookups in the sorted index, pattern alignment (choice of
// the per-read shift) and anchor expansion.
//
// Lookups are independent dependent-gather chains (a binary search over the sorted
// keys, then a galloping search for the end of the run of equal keys), one lane per
// query, so the kernel is bound by memory latency and the number of lines in flight.
// Alignment and expansion run one wave64 per read: lanes stride over the read's
// minimizer records and combine with wave reductions/scans, so anchors of a read are
// written as one contiguous, coalesced run in (qpos, rpos) order.
#include "gd_internal.h"

namespace gd {

namespace {

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t *keys, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, len = n;
    while (len > 0) {
        const uint64_t half = len >> 1;
        if (keys[lo + half] < x) { lo += half + 1; len -= half + 1; }
        else len = half;
    }
    return lo;
}

// End of the run of keys equal to x that starts at l (keys[l] == x assumed when l < n).
__device__ __forceinline__ uint64_t run_end(const uint64_t *keys, uint64_t n, uint64_t l, uint64_t x)
{
    if (l >= n || keys[l] != x) return l;
    uint64_t lo = l, hi = l + 1, step = 1;        // keys[lo] == x
    while (hi < n && keys[hi] == x) { lo = hi; step <<= 1; hi = lo + step; }
    if (hi > n) hi = n;
    uint64_t a = lo + 1, b = hi;                  // first index != x lies in [a, b]
    while (a < b) {
        const uint64_t m = a + ((b - a) >> 1);
        if (keys[m] == x) a = m + 1; else b = m;
    }
    return a;
}

__global__ __launch_bounds__(kBlock) void k_lookup(const uint64_t *ikeys, uint64_t in,
                                                   const uint64_t *q, const uint64_t *n_q,
                                                   uint64_t q_cap, uint32_t *lb, uint32_t *occ)
{
    uint64_t n = *n_q;
    if (n > q_cap) n = q_cap;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t x = q[i];
        const uint64_t l = lower_bound_u64(ikeys, in, x);
        const uint64_t u = run_end(ikeys, in, l, x);
        lb[i] = (uint32_t)l;
        occ[i] = (uint32_t)(u - l);
    }
}

constexpr int kReadsPerBlock = kBlock / kWave;

__global__ __launch_bounds__(kBlock) void k_align(AlignArgs A, uint8_t *shift_out,
                                                  uint32_t *shift_slot, uint32_t *anchor_cnt)
{
    const uint32_t r = blockIdx.x * kReadsPerBlock + threadIdx.x / kWave;
    if (r >= A.n_reads) return;
    const int lane = threadIdx.x & (kWave - 1);
    const size_t mzs = (size_t)A.n_reads + 1;
    uint32_t slot = 0;
    if (A.n_shift > 1) {
        uint64_t nstar = kMax64;
        for (uint32_t s = 0; s < A.n_shift; s++) {
            const uint64_t c = A.mzofs[s * mzs + r + 1] - A.mzofs[s * mzs + r];
            nstar = c < nstar ? c : nstar;
        }
        if (A.align_t > 0 && (uint64_t)A.align_t < nstar) nstar = A.align_t;
        uint64_t best = 0;
        for (uint32_t s = 0; s < A.n_shift; s++) {
            const uint64_t beg = A.mzofs[s * mzs + r];
            const uint32_t *occ = A.occ + s * A.stride + beg;
            uint64_t sc = 0;
            for (uint64_t j = lane; j < nstar; j += kWave) {
                const uint32_t o = occ[j];
                if (A.max_occ == 0 || o < A.max_occ) sc += o;
            }
            sc = wave_sum<uint64_t>(sc);
            if (sc > best) { best = sc; slot = s; }
        }
    }
    const uint64_t beg = A.mzofs[slot * mzs + r], end = A.mzofs[slot * mzs + r + 1];
    const uint32_t *occ = A.occ + slot * A.stride;
    uint64_t cnt = 0;
    for (uint64_t j = beg + lane; j < end; j += kWave) {
        const uint32_t o = occ[j];
        if (A.max_occ == 0 || o < A.max_occ) cnt += o;
    }
    cnt = wave_sum<uint64_t>(cnt);
    if (lane == 0) {
        shift_slot[r] = slot;
        if (shift_out) shift_out[r] = (uint8_t)(A.fixed_shift >= 0 ? (uint32_t)A.fixed_shift : slot);
        anchor_cnt[r] = (uint32_t)cnt;
    }
}

__global__ __launch_bounds__(kBlock) void k_expand(AlignArgs A, const uint32_t *shift_slot,
                                                   const uint64_t *read_off, const uint32_t *ivals,
                                                   uint4 *anchors, uint64_t capacity,
                                                   uint32_t *status)
{
    const uint32_t r = blockIdx.x * kReadsPerBlock + threadIdx.x / kWave;
    if (r >= A.n_reads) return;
    const int lane = threadIdx.x & (kWave - 1);
    if (read_off[A.n_reads] > capacity) {
        if (r == 0 && lane == 0) set_status(status, 1u);
        return;
    }
    const size_t mzs = (size_t)A.n_reads + 1;
    const uint32_t slot = shift_slot[r];
    const uint64_t beg = A.mzofs[slot * mzs + r], end = A.mzofs[slot * mzs + r + 1];
    const uint32_t *occ = A.occ + slot * A.stride;
    const uint32_t *lb = A.lb + slot * A.stride;
    const uint32_t *qv = A.qval + slot * A.stride;
    uint64_t out = read_off[r];
    for (uint64_t j0 = beg; j0 < end; j0 += kWave) {
        const uint64_t j = j0 + lane;
        uint32_t o = 0, l = 0, q = 0;
        if (j < end) {
            o = occ[j];
            if (A.max_occ != 0 && o >= A.max_occ) o = 0;
            l = lb[j];
            q = qv[j];
        }
        const uint32_t incl = wave_incl_scan<uint32_t>(o);
        const uint64_t at = out + (incl - o);
        for (uint32_t e = 0; e < o; e++) {
            const uint32_t v = ivals[l + e];
            anchors[at + e] = make_uint4(r, q >> 1, v >> 1, (q ^ v) & 1u);
        }
        out += __shfl(incl, kWave - 1, kWave);
    }
}

}  // namespace

hipError_t launch_lookup(const uint64_t *ikeys, uint64_t in, const uint64_t *q,
                         const uint64_t *n_q, uint64_t q_cap, uint32_t *lb, uint32_t *occ,
                         hipStream_t s)
{
    uint64_t blocks = (q_cap + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    GD_LAUNCH(k_lookup, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, in, q, n_q,
                       q_cap, lb, occ);
    return hipGetLastError();
}

hipError_t launch_align(const AlignArgs &a, uint8_t *shift_out, uint32_t *shift_slot,
                        uint32_t *anchor_cnt, hipStream_t s)
{
    if (a.n_reads == 0) return hipSuccess;
    const unsigned blocks = (a.n_reads + kReadsPerBlock - 1) / kReadsPerBlock;
    GD_LAUNCH(k_align, dim3(blocks), dim3(kBlock), 0, s, a, shift_out, shift_slot,
                       anchor_cnt);
    return hipGetLastError();
}

hipError_t launch_expand(const AlignArgs &a, const uint32_t *shift_slot, const uint64_t *read_off,
                         const void *ivals, uint32_t *anchors, uint64_t capacity,
                         uint32_t *status, hipStream_t s)
{
    if (a.n_reads == 0) return hipSuccess;
    const unsigned blocks = (a.n_reads + kReadsPerBlock - 1) / kReadsPerBlock;
    GD_LAUNCH(k_expand, dim3(blocks), dim3(kBlock), 0, s, a, shift_slot, read_off,
                       (const uint32_t *)ivals, (uint4 *)anchors, capacity, status);
    return hipGetLastError();
}

}  // namespace gd
