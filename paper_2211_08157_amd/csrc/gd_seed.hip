// Seeding kernels: exact-match lookups in the sorted index, pattern alignment (choice of
// the per-read shift) and anchor expansion.
//
// Lookups are independent dependent-gather chains (a binary search over the sorted
// keys, then a galloping search for the end of the run of equal keys), one lane per
// query, so the kernel is bound by memory latency and the number of lines in flight.
// Alignment and expansion take one thread per read when the read has few minimizer
// records (short reads) and one wave64 per read from a device-built list otherwise (long
// reads: lanes stride over the records and combine with wave reductions and scans); the
// anchors of a read are written as one contiguous run in (qpos, rpos) order.
#include "gd_internal.h"
#include "gd_rmi_model.h"
#include "gd_table_model.h"

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

// Lower bound l and run end u of q through the learned index when the keys are 16-byte
// aligned.  The lookup is bound by the number of random memory requests, so the leaf is
// one 16-byte load and the key window [lo - 1, hi] (both brackets included) is read as
// up to kPairs independent 16-byte loads; both ends come from those keys.  The bracket
// check keeps the result exact whatever the model holds; a wider window is searched by
// bisection after the same check, and a failed check takes the plain searches.
constexpr int kPairs = 8;

__device__ __forceinline__ void rmi_find(const void *rmi, bool valid, const uint64_t *keys,
                                         uint64_t n, uint64_t q, uint64_t &l, uint64_t &u)
{
    const RmiHeader &H = *(const RmiHeader *)rmi;
    const RmiLeaf *leaves = (const RmiLeaf *)((const char *)rmi + sizeof(RmiHeader));
    if (valid) {
        const RmiLeaf lf = leaves[route(H, q)];
        const int64_t p = predict(lf, q);
        int64_t lo = p - lf.err_lo, hi = p + lf.err_hi + 1;
        if (lo < 0) lo = 0;
        if (hi > (int64_t)n) hi = (int64_t)n;
        const int64_t s0 = lo > 0 ? lo - 1 : 0;                     // first key read
        const int64_t s1 = hi < (int64_t)n ? hi : (int64_t)n - 1;   // last key read
        const int64_t e0 = s0 & ~(int64_t)1;                        // 16-byte aligned
        if (lo <= hi && s1 - e0 < 2 * kPairs) {
            ulonglong2 v[kPairs];
#pragma unroll
            for (int c = 0; c < kPairs; c++) {
                const int64_t e = e0 + 2 * c;
                if (e <= s1 && e + 1 < (int64_t)n) v[c] = *(const ulonglong2 *)(keys + e);
                else if (e <= s1) v[c] = make_ulonglong2(keys[e], kMax64);
                else v[c] = make_ulonglong2(kMax64, kMax64);
            }
            bool ok = true, hi_eq = false;
            uint32_t lt = 0, eq = 0;
#pragma unroll
            for (int c = 0; c < kPairs; c++) {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int64_t idx = e0 + 2 * c + h;
                    const uint64_t kv = h ? v[c].y : v[c].x;
                    if (idx < s0 || idx > s1) continue;
                    if (idx == lo - 1) {
                        ok = ok && kv < q;                  // left bracket
                    } else if (idx == hi) {                 // right bracket (hi < n)
                        ok = ok && kv >= q;
                        hi_eq = kv == q;
                        eq += hi_eq ? 1u : 0u;
                    } else {                                // window [lo, hi)
                        lt += kv < q ? 1u : 0u;
                        eq += kv == q ? 1u : 0u;
                    }
                }
            }
            if (ok) {
                l = (uint64_t)lo + lt;
                u = hi_eq ? run_end(keys, n, (uint64_t)hi, q) : l + eq;
                return;
            }
        } else if (lo <= hi && (lo == 0 || keys[lo - 1] < q) &&
                   (hi == (int64_t)n || keys[hi] >= q)) {
            // a wide window (few leaves for many keys): binary search inside it
            uint64_t a = (uint64_t)lo, len = (uint64_t)(hi - lo);
            while (len > 0) {
                const uint64_t half = len >> 1;
                if (keys[a + half] < q) { a += half + 1; len -= half + 1; }
                else len = half;
            }
            l = a;
            u = run_end(keys, n, l, q);
            return;
        }
    }
    l = lower_bound_u64(keys, n, q);
    u = run_end(keys, n, l, q);
}

// One lane per query.  kMode: 0 binary search, 1 learned index (scalar loads), 2 learned
// index (keys 16-byte aligned, windowed loads), 3 hash table (lb 0 for absent keys).
// The model (model_bytes bytes) is checked once per workgroup: a learned index whose
// leaves would lie outside its buffer, or a hash table that does not fit its buffer or
// was built over other keys, is not used (binary search instead).
template <int kMode>
__global__ __launch_bounds__(kBlock) void k_lookup(const uint64_t *ikeys, uint64_t in,
                                                   const uint64_t *q, const uint64_t *n_q,
                                                   uint64_t q_cap, uint32_t *lb, uint32_t *occ,
                                                   const void *model, size_t model_bytes)
{
    __shared__ int sh_valid;
    if (kMode != 0) {
        if (threadIdx.x == 0)
            sh_valid = kMode == 3 ? table_valid(model, model_bytes, in, table_keys_fp(ikeys, in))
                                  : rmi_valid(model, model_bytes, in);
        __syncthreads();
    }
    const bool valid = kMode != 0 && sh_valid != 0;
    uint64_t n = n_q ? *n_q : q_cap;
    if (n > q_cap) n = q_cap;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t x = q[i];
        uint64_t l, u;
        if (kMode == 3) {
            uint64_t c;
            if (valid && table_find(model, in, x, l, c)) {
                u = l + c;
            } else {
                l = lower_bound_u64(ikeys, in, x);
                u = run_end(ikeys, in, l, x);
            }
        } else if (kMode == 2) {
            rmi_find(model, valid, ikeys, in, x, l, u);
        } else {
            l = kMode == 1 ? rmi_lower_bound(model, valid, ikeys, in, x)
                           : lower_bound_u64(ikeys, in, x);
            u = run_end(ikeys, in, l, x);
        }
        lb[i] = (uint32_t)l;
        occ[i] = (uint32_t)(u - l);
    }
}

// Random-gather probe: four independent loads per lane per step.
__global__ __launch_bounds__(kBlock) void k_random_gather(const uint64_t *src, uint64_t n_src,
                                                          const uint64_t *idx, uint64_t n_idx,
                                                          uint64_t *out, uint32_t *status)
{
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i0 = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i0 < n_idx; i0 += stride * U) {
        uint64_t v[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t i = i0 + (uint64_t)u * stride;
            const uint64_t j = i < n_idx ? idx[i] : 0;
            ok[u] = i < n_idx && j < n_src;
            v[u] = ok[u] ? src[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t i = i0 + (uint64_t)u * stride;
            if (i < n_idx) {
                out[i] = v[u];
                if (!ok[u]) set_status(status, 2u);
            }
        }
    }
}

constexpr int kReadsPerBlock = kBlock / kWave;
constexpr int kHugeBlock = 1024;            // threads per read on the huge-read path
constexpr uint64_t kHugeRecords = 16384;    // reads with more records take that path
// Reads whose minimizer records (summed over the sketched shifts) exceed A.long_records are
// handled by one wave each; shorter reads by one thread each.

// Records of read r at shift slot s: [mzofs[s][r], mzofs[s][r+1]).
__device__ __forceinline__ uint64_t rec_beg(const AlignArgs &A, uint32_t s, uint32_t r)
{
    return A.mzofs[s * ((size_t)A.n_reads + 1) + r];
}

__device__ __forceinline__ uint64_t read_records(const AlignArgs &A, uint32_t r)
{
    uint64_t n = 0;
    for (uint32_t s = 0; s < A.n_shift; s++) n += rec_beg(A, s, r + 1) - rec_beg(A, s, r);
    return n;
}

__device__ __forceinline__ uint32_t keep_occ(const AlignArgs &A, uint32_t o)
{
    return (A.max_occ == 0 || o < A.max_occ) ? o : 0u;
}

// n* = min over the sketched shifts of the record count, capped at t.
__device__ __forceinline__ uint64_t align_nstar(const AlignArgs &A, uint32_t r)
{
    uint64_t nstar = kMax64;
    for (uint32_t s = 0; s < A.n_shift; s++) {
        const uint64_t c = rec_beg(A, s, r + 1) - rec_beg(A, s, r);
        nstar = c < nstar ? c : nstar;
    }
    if (A.align_t > 0 && (uint64_t)A.align_t < nstar) nstar = A.align_t;
    return nstar;
}

__device__ __forceinline__ void align_store(const AlignArgs &A, uint32_t r, uint32_t slot,
                                            uint64_t cnt, uint8_t *shift_out, uint32_t *shift_slot,
                                            uint32_t *anchor_cnt)
{
    shift_slot[r] = slot;
    if (shift_out) shift_out[r] = (uint8_t)(A.fixed_shift >= 0 ? (uint32_t)A.fixed_shift : slot);
    anchor_cnt[r] = (uint32_t)cnt;
}

// One thread per read; reads with many records are appended to long_ids instead.
__global__ __launch_bounds__(kBlock) void k_align(AlignArgs A, uint8_t *shift_out,
                                                  uint32_t *shift_slot, uint32_t *anchor_cnt,
                                                  uint32_t *long_ids, uint32_t *long_n)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= A.n_reads) return;
    const uint64_t recs = read_records(A, r);
    if (recs > kHugeRecords) {
        long_ids[A.n_reads - 1 - atomicAdd(long_n + 1, 1u)] = r;
        return;
    }
    if (recs > A.long_records) {
        long_ids[atomicAdd(long_n, 1u)] = r;
        return;
    }
    uint32_t slot = 0;
    if (A.n_shift > 1) {
        const uint64_t nstar = align_nstar(A, r);
        uint64_t best = 0;
        for (uint32_t s = 0; s < A.n_shift; s++) {
            const uint32_t *occ = A.occ + s * A.stride + rec_beg(A, s, r);
            uint64_t sc = 0;
            for (uint64_t j = 0; j < nstar; j++) sc += keep_occ(A, occ[j]);
            if (sc > best) { best = sc; slot = s; }
        }
    }
    const uint64_t beg = rec_beg(A, slot, r), end = rec_beg(A, slot, r + 1);
    const uint32_t *occ = A.occ + slot * A.stride;
    uint64_t cnt = 0;
    for (uint64_t j = beg; j < end; j++) cnt += keep_occ(A, occ[j]);
    align_store(A, r, slot, cnt, shift_out, shift_slot, anchor_cnt);
}

// One wave per read of the long list (grid-stride over the list).
__global__ __launch_bounds__(kBlock) void k_align_long(AlignArgs A, uint8_t *shift_out,
                                                       uint32_t *shift_slot, uint32_t *anchor_cnt,
                                                       const uint32_t *long_ids,
                                                       const uint32_t *long_n)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nl = *long_n;
    for (uint32_t li = blockIdx.x * kReadsPerBlock + threadIdx.x / kWave; li < nl;
         li += gridDim.x * kReadsPerBlock) {
        const uint32_t r = long_ids[li];
        uint32_t slot = 0;
        if (A.n_shift > 1) {
            const uint64_t nstar = align_nstar(A, r);
            uint64_t best = 0;
            for (uint32_t s = 0; s < A.n_shift; s++) {
                const uint32_t *occ = A.occ + s * A.stride + rec_beg(A, s, r);
                uint64_t sc = 0;
                for (uint64_t j0 = 0; j0 < nstar; j0 += 4 * kWave) {    // 4 loads in flight
                    uint32_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint64_t j = j0 + (uint64_t)(u * kWave + lane);
                        v[u] = j < nstar ? occ[j] : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) sc += keep_occ(A, v[u]);
                }
                sc = wave_sum<uint64_t>(sc);
                if (sc > best) { best = sc; slot = s; }
            }
        }
        const uint64_t beg = rec_beg(A, slot, r), end = rec_beg(A, slot, r + 1);
        const uint32_t *occ = A.occ + slot * A.stride;
        uint64_t cnt = 0;
        for (uint64_t j0 = beg; j0 < end; j0 += 4 * kWave) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint64_t j = j0 + (uint64_t)(u * kWave + lane);
                v[u] = j < end ? occ[j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) cnt += keep_occ(A, v[u]);
        }
        cnt = wave_sum<uint64_t>(cnt);
        if (lane == 0) align_store(A, r, slot, cnt, shift_out, shift_slot, anchor_cnt);
    }
}

// Short reads: one wave per 64 consecutive reads (lane i holds read i's record range at
// its chosen shift).  The wave walks the group's records in (read, record) order, one
// record per lane, so neighbouring lanes read neighbouring records and write neighbouring
// anchors; a record's anchors start at its read's offset plus the anchors of the read's
// earlier records (a segmented wave scan, carried across chunks for the read that is
// still open at a chunk's end).  Long reads contribute no records here.
__global__ __launch_bounds__(kBlock) void k_expand(AlignArgs A, const uint32_t *shift_slot,
                                                   const uint64_t *read_off, const uint32_t *ivals,
                                                   uint4 *anchors, uint64_t capacity,
                                                   uint32_t *status)
{
    const uint64_t r64 = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (read_off[A.n_reads] > capacity) {
        if (r64 == 0) set_status(status, 1u);
        return;
    }
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t cnt = 0, slot = 0;
    uint64_t beg = 0, out = 0;
    if (r64 < A.n_reads) {
        const uint32_t r = (uint32_t)r64;
        if (read_records(A, r) <= A.long_records) {
            slot = shift_slot[r];
            beg = rec_beg(A, slot, r);
            cnt = (uint32_t)(rec_beg(A, slot, r + 1) - beg);
            out = read_off[r];
        }
    }
    const uint32_t incl = wave_incl_scan<uint32_t>(cnt);
    const uint32_t start = incl - cnt;                       // flat index of the first record
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    const uint64_t r_base = r64 - (uint64_t)lane;            // read id of lane 0
    int open_read = -1;                                      // read still open across chunks
    uint32_t open_sum = 0;                                   // its anchors so far
    for (uint32_t f0 = 0; f0 < total; f0 += kWave) {
        const uint32_t f = f0 + (uint32_t)lane;
        const bool valid = f < total;
        // read of flat record f: the last lane i with start_i <= f
        int i = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1) {
            const uint32_t st = __shfl(start, i + step, kWave);
            if (st <= f) i += step;
        }
        const uint32_t i_slot = __shfl(slot, i, kWave);
        const uint64_t i_beg = __shfl(beg, i, kWave);
        const uint32_t i_start = __shfl(start, i, kWave);
        const uint64_t i_out = __shfl(out, i, kWave);
        uint32_t o = 0, l = 0, q = 0;
        if (valid) {
            const size_t jj = (size_t)i_slot * A.stride + i_beg + (f - i_start);
            o = keep_occ(A, A.occ[jj]);
            l = A.lb[jj];
            q = A.qval[jj];
        }
        // segmented exclusive scan of o by read
        const uint32_t oi = wave_incl_scan<uint32_t>(o);
        const uint32_t oe = oi - o;
        const int prev_i = __shfl_up(i, 1, kWave);
        const bool head = lane == 0 || prev_i != i;
        const uint64_t heads = __ballot(head);
        const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
        const int hl = 63 - __clzll((long long)upto);
        const uint32_t seg = oe - __shfl(oe, hl, kWave) + (i == open_read ? open_sum : 0u);
        const uint32_t r = (uint32_t)(r_base + (uint64_t)i);
        const uint64_t pos = i_out + seg;
        for (uint32_t e = 0; e < o; e++) {
            const uint32_t v = ivals[l + e];
            anchors[pos + e] = make_uint4(r, q >> 1, v >> 1, (q ^ v) & 1u);
        }
        const int lv = (int)min((uint32_t)(kWave - 1), total - 1 - f0);
        open_read = __shfl(i, lv, kWave);
        open_sum = __shfl(seg + o, lv, kWave);
    }
}

// One wave per read of the long list: lanes stride over the records, a wave scan places
// each record's anchors.
__global__ __launch_bounds__(kBlock) void k_expand_long(AlignArgs A, const uint32_t *shift_slot,
                                                        const uint64_t *read_off,
                                                        const uint32_t *ivals, uint4 *anchors,
                                                        uint64_t capacity,
                                                        const uint32_t *long_ids,
                                                        const uint32_t *long_n)
{
    if (read_off[A.n_reads] > capacity) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nl = *long_n;
    for (uint32_t li = blockIdx.x * kReadsPerBlock + threadIdx.x / kWave; li < nl;
         li += gridDim.x * kReadsPerBlock) {
        const uint32_t r = long_ids[li];
        const uint32_t slot = shift_slot[r];
        const uint64_t beg = rec_beg(A, slot, r), end = rec_beg(A, slot, r + 1);
        const uint32_t *occ = A.occ + slot * A.stride;
        const uint32_t *lb = A.lb + slot * A.stride;
        const uint32_t *qv = A.qval + slot * A.stride;
        uint64_t out = read_off[r];
        // the next chunk's records are loaded before this chunk's gathers and writes
        uint32_t on = 0, ln = 0, qn = 0;
        if (beg + lane < end) {
            on = keep_occ(A, occ[beg + lane]);
            ln = lb[beg + lane];
            qn = qv[beg + lane];
        }
        for (uint64_t j0 = beg; j0 < end; j0 += kWave) {
            const uint32_t o = on, l = ln, q = qn;
            const uint64_t jn = j0 + kWave + lane;
            on = ln = qn = 0;
            if (jn < end) {
                on = keep_occ(A, occ[jn]);
                ln = lb[jn];
                qn = qv[jn];
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
}

// Reads with more than kHugeRecords records (the longest ONT reads) take one workgroup
// of kHugeBlock threads each, so the one or two longest reads of a batch do not leave a
// single wave working through their records while the rest of the GPU is idle.
__device__ __forceinline__ uint64_t huge_block_sum(uint64_t v, uint64_t *sh)
{
    v = wave_sum<uint64_t>(v);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < kHugeBlock / kWave; i++) t += sh[i];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kHugeBlock) void k_align_huge(AlignArgs A, uint8_t *shift_out,
                                                           uint32_t *shift_slot,
                                                           uint32_t *anchor_cnt,
                                                           const uint32_t *long_ids,
                                                           const uint32_t *long_n)
{
    __shared__ uint64_t sh[kHugeBlock / kWave];
    const uint32_t nh = long_n[1];
    for (uint32_t hi = blockIdx.x; hi < nh; hi += gridDim.x) {
        const uint32_t r = long_ids[A.n_reads - 1 - hi];
        uint32_t slot = 0;
        if (A.n_shift > 1) {
            const uint64_t nstar = align_nstar(A, r);
            uint64_t best = 0;
            for (uint32_t s = 0; s < A.n_shift; s++) {
                const uint32_t *occ = A.occ + s * A.stride + rec_beg(A, s, r);
                uint64_t sc = 0;
                for (uint64_t j0 = 0; j0 < nstar; j0 += 4 * kHugeBlock) {
                    uint32_t v[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint64_t j = j0 + (uint64_t)(u * kHugeBlock + threadIdx.x);
                        v[u] = j < nstar ? occ[j] : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) sc += keep_occ(A, v[u]);
                }
                sc = huge_block_sum(sc, sh);
                if (sc > best) { best = sc; slot = s; }
            }
        }
        const uint64_t beg = rec_beg(A, slot, r), end = rec_beg(A, slot, r + 1);
        const uint32_t *occ = A.occ + slot * A.stride;
        uint64_t cnt = 0;
        for (uint64_t j0 = beg; j0 < end; j0 += 4 * kHugeBlock) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint64_t j = j0 + (uint64_t)(u * kHugeBlock + threadIdx.x);
                v[u] = j < end ? occ[j] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) cnt += keep_occ(A, v[u]);
        }
        cnt = huge_block_sum(cnt, sh);
        if (threadIdx.x == 0) align_store(A, r, slot, cnt, shift_out, shift_slot, anchor_cnt);
    }
}

__global__ __launch_bounds__(kHugeBlock) void k_expand_huge(AlignArgs A, const uint32_t *shift_slot,
                                                            const uint64_t *read_off,
                                                            const uint32_t *ivals, uint4 *anchors,
                                                            uint64_t capacity,
                                                            const uint32_t *long_ids,
                                                            const uint32_t *long_n)
{
    __shared__ uint32_t sh[kHugeBlock / kWave];
    if (read_off[A.n_reads] > capacity) return;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t nh = long_n[1];
    for (uint32_t hi = blockIdx.x; hi < nh; hi += gridDim.x) {
        const uint32_t r = long_ids[A.n_reads - 1 - hi];
        const uint32_t slot = shift_slot[r];
        const uint64_t beg = rec_beg(A, slot, r), end = rec_beg(A, slot, r + 1);
        const uint32_t *occ = A.occ + slot * A.stride;
        const uint32_t *lb = A.lb + slot * A.stride;
        const uint32_t *qv = A.qval + slot * A.stride;
        uint64_t out = read_off[r];
        for (uint64_t j0 = beg; j0 < end; j0 += kHugeBlock) {
            const uint64_t j = j0 + threadIdx.x;
            uint32_t o = 0, l = 0, q = 0;
            if (j < end) {
                o = keep_occ(A, occ[j]);
                l = lb[j];
                q = qv[j];
            }
            const uint32_t incl = wave_incl_scan<uint32_t>(o);
            if (lane == kWave - 1) sh[wv] = incl;
            __syncthreads();
            uint32_t before = 0, total = 0;
#pragma unroll
            for (int i = 0; i < kHugeBlock / kWave; i++) {
                const uint32_t c = sh[i];
                before += i < wv ? c : 0u;
                total += c;
            }
            __syncthreads();
            const uint64_t at = out + before + (incl - o);
            for (uint32_t e = 0; e < o; e++) {
                const uint32_t v = ivals[l + e];
                anchors[at + e] = make_uint4(r, q >> 1, v >> 1, (q ^ v) & 1u);
            }
            out += total;
        }
    }
}

}  // namespace

hipError_t launch_random_gather(const uint64_t *src, uint64_t n_src, const uint64_t *idx,
                                uint64_t n_idx, uint64_t *out, uint32_t *status, hipStream_t s)
{
    hipError_t e = fill_u32(status, 0, 1, s);
    if (e != hipSuccess || n_idx == 0) return e;
    uint64_t blocks = (n_idx + 4 * kBlock - 1) / (4 * kBlock);
    if (blocks > 65536) blocks = 65536;
    GD_LAUNCH(k_random_gather, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, n_src, idx, n_idx,
              out, status);
    return hipGetLastError();
}

hipError_t launch_lookup(const uint64_t *ikeys, uint64_t in, const uint64_t *q,
                         const uint64_t *n_q, uint64_t q_cap, uint32_t *lb, uint32_t *occ,
                         const void *rmi, size_t rmi_bytes, const void *table,
                         size_t table_bytes, uint32_t max_blocks, hipStream_t s)
{
    uint64_t blocks = (q_cap + kBlock - 1) / kBlock;
    const uint64_t cap = max_blocks ? max_blocks : 8192;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    if (table)
        GD_LAUNCH(k_lookup<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, in, q, n_q,
                  q_cap, lb, occ, table, table_bytes);
    else if (rmi && ((uintptr_t)ikeys & 15) == 0)
        GD_LAUNCH(k_lookup<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, in, q, n_q,
                  q_cap, lb, occ, rmi, rmi_bytes);
    else if (rmi)
        GD_LAUNCH(k_lookup<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, in, q, n_q,
                  q_cap, lb, occ, rmi, rmi_bytes);
    else
        GD_LAUNCH(k_lookup<0>, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, in, q, n_q,
                  q_cap, lb, occ, rmi, (size_t)0);
    return hipGetLastError();
}

hipError_t launch_align(const AlignArgs &a, uint8_t *shift_out, uint32_t *shift_slot,
                        uint32_t *anchor_cnt, uint32_t *long_ids, uint32_t *long_n, hipStream_t s)
{
    if (a.n_reads == 0) return hipSuccess;
    hipError_t e = fill_u32(long_n, 0, 2, s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (a.n_reads + kBlock - 1) / kBlock;
    GD_LAUNCH(k_align, dim3(blocks), dim3(kBlock), 0, s, a, shift_out, shift_slot, anchor_cnt,
              long_ids, long_n);
    GD_LAUNCH(k_align_huge, dim3(64), dim3(kHugeBlock), 0, s, a, shift_out, shift_slot,
              anchor_cnt, (const uint32_t *)long_ids, (const uint32_t *)long_n);
    GD_LAUNCH(k_align_long, dim3(a.long_blocks), dim3(kBlock), 0, s, a, shift_out, shift_slot,
              anchor_cnt,
              (const uint32_t *)long_ids, (const uint32_t *)long_n);
    return hipGetLastError();
}

hipError_t launch_expand(const AlignArgs &a, const uint32_t *shift_slot, const uint64_t *read_off,
                         const void *ivals, uint32_t *anchors, uint64_t capacity,
                         uint32_t *status, const uint32_t *long_ids, const uint32_t *long_n,
                         hipStream_t s)
{
    if (a.n_reads == 0) return hipSuccess;
    const unsigned blocks = (a.n_reads + kBlock - 1) / kBlock;     // one lane per read
    GD_LAUNCH(k_expand, dim3(blocks), dim3(kBlock), 0, s, a, shift_slot, read_off,
              (const uint32_t *)ivals, (uint4 *)anchors, capacity, status);
    GD_LAUNCH(k_expand_long, dim3(a.long_blocks), dim3(kBlock), 0, s, a, shift_slot, read_off,
              (const uint32_t *)ivals, (uint4 *)anchors, capacity, long_ids, long_n);
    GD_LAUNCH(k_expand_huge, dim3(64), dim3(kHugeBlock), 0, s, a, shift_slot, read_off,
              (const uint32_t *)ivals, (uint4 *)anchors, capacity, long_ids, long_n);
    return hipGetLastError();
}

}  // namespace gd
