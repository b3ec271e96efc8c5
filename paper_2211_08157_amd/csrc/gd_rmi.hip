// Learned index over the sorted minimizer keys: a two-stage recursive model index with
// FP32 inference and a bounded, self-checking last-mile search.
//
// Model blob (device memory, godiet_rmi_size bytes):
//   RmiHeader                      magic, root kind, log2 of the leaf count, key count
//   root parameters                linear: leaf = a*x + b;  MLP: 1 -> 32 ReLU -> 1 with
//                                  hidden unit i = relu(x - t_i), out = c0 + sum c_i h_i,
//                                  x = key * 2^-64 (FP32), out = predicted rank / n
//   RmiLeaf[L]                     16 bytes: high half of the first key, base
//                                  position (intercept folded in), FP32 slope, 16-bit
//                                  error bounds
//
// Routing is monotone in the key (FP32 conversion, non-negative slopes, floor, and an
// MLP whose FP32 segments are made to agree in order at every knot), so each leaf owns
// a contiguous run of the sorted keys.  A leaf predicts
//     p = base + floor(slope * float((q >> 32) - khi))
// and the answer is searched in [p - err_lo, p + err_hi + 1].  The window is accepted
// only if keys[lo-1] < q <= keys[hi] (with the array ends as sentinels); otherwise the
// lookup falls back to a full binary search, so results never depend on the model or on
// floating-point details, only its speed does.
#include "gd_internal.h"
#include "gd_rmi_model.h"

namespace gd {

namespace {

// ---- training

// Make the FP32 MLP root non-decreasing in x, so that routing is monotone in the key.
// Each segment is monotone once its slope is non-negative (a fused multiply-add rounded
// to nearest preserves order); at a knot the two segments' FP32 values may disagree, so
// the first float above knot i must not evaluate below the knot itself: the intercept of
// its segment is raised by the deficit (at least one float step) until it does not.
// Knots are taken in ascending order, so a raise is seen by the next knot's check.
// Returns false if some knot could not be fixed (the caller then uses the linear root,
// monotone as it stands).
__device__ bool mlp_make_monotone(RmiHeader &h)
{
    for (int j = 0; j <= kKnots; j++)
        if (!(h.sb[j] >= 0.f)) h.sb[j] = 0.f;        // FP32 prefix sums of slopes >= 0
    for (int i = 0; i < kKnots; i++) {
        const float a = h.t[i];                      // knots are key * 2^-64: in [0, 1]
        if (i + 1 < kKnots && h.t[i + 1] == a) continue;   // the last of equal knots checks
        const float b = __int_as_float(__float_as_int(a) + 1);     // the next float up
        if (!(a >= 0.f) || !(b > a)) return false;
        // the knots ascend, so a lies on segment #(t < a) (the first knot equal to a) and
        // b, with no float between them, on segment #(t <= a) = i + 1
        int ja = i;
        while (ja > 0 && h.t[ja - 1] == a) ja--;
        const int jb = i + 1;
        bool ok = false;
        for (int it = 0; it < 64 && !ok; it++) {
            const float va = __builtin_fmaf(h.sb[ja], a, h.sa[ja]);
            const float vb = __builtin_fmaf(h.sb[jb], b, h.sa[jb]);
            ok = vb >= va;
            if (ok) break;
            // raise by the deficit; at least to the next float up
            const float cur = h.sa[jb];
            float up = (float)((double)cur + ((double)va - (double)vb));
            if (!(up > cur))
                up = cur == 0.f ? __int_as_float(1)
                                : __int_as_float(__float_as_int(cur) + (cur > 0.f ? 1 : -1));
            h.sa[jb] = up;
        }
        if (!ok || !(h.sa[jb] == h.sa[jb])) return false;
    }
    return true;
}

// One workgroup: root parameters from the sorted keys (knots at key quantiles; the
// network interpolates the rank/n curve linearly between them).
__global__ __launch_bounds__(kBlock) void k_rmi_root(const uint64_t *keys, uint64_t n, int kind,
                                                     uint32_t log2_leaves, RmiHeader *H)
{
    if (threadIdx.x != 0) return;
    RmiHeader h;
    for (size_t i = 0; i < sizeof(h) / 4; i++) ((uint32_t *)&h)[i] = 0;
    h.magic = kRmiMagic;
    h.kind = (uint32_t)kind;
    h.log2_leaves = log2_leaves;
    h.n_keys = n;
    const double L = (double)(1u << log2_leaves);
    if (n > 0) {
        const double x0 = (double)keys[0] * 0x1p-64, x1 = (double)keys[n - 1] * 0x1p-64;
        const double a = x1 > x0 ? L / (x1 - x0) : 0.0;
        h.a = (float)a;
        h.b = (float)(-a * x0);
        // knots at ranks j*n/32 and the rank/n value at each knot
        double tx[kKnots + 1], ty[kKnots + 1];
        for (int j = 0; j <= kKnots; j++) {
            const uint64_t r = j == kKnots ? n - 1 : (uint64_t)((double)n * j / kKnots);
            tx[j] = (double)keys[r] * 0x1p-64;
            ty[j] = (double)r / (double)n;
        }
        // slope of each segment; hidden unit i switches on at knot i
        double prev = 0.0;
        h.c[0] = (float)ty[0];
        for (int i = 0; i < kKnots; i++) {
            const double dx = tx[i + 1] - tx[i];
            const double s = dx > 0 ? (ty[i + 1] - ty[i]) / dx : 0.0;
            h.t[i] = (float)tx[i];
            h.c[i + 1] = (float)(s - prev);
            prev = s;
        }
        // the network per segment (FP32 prefix sums of the output weights)
        h.sa[0] = h.c[0];
        h.sb[0] = 0.f;
        for (int j = 1; j <= kKnots; j++) {
            h.sb[j] = __fadd_rn(h.sb[j - 1], h.c[j]);
            h.sa[j] = __builtin_fmaf(-h.c[j], h.t[j - 1], h.sa[j - 1]);
        }
        if (kind == 1 && !mlp_make_monotone(h)) h.kind = 0;
    }
    *H = h;
}

// Leaf boundaries: leaf l starts at the first key routed to a leaf >= l (index n routes
// past the last leaf), stored in its base field.  Routing is monotone in the key (the root
// is made so in training), so the indices where the routed leaf steps up partition the
// leaves: each leaf's start is written by exactly one lane, with a plain store, and every
// leaf is written (so no atomics, and no clearing of the leaves beforehand).  k_rmi_ends
// then copies each leaf's end (the next leaf's start) into its own slope field, so the
// fitting pass reads and rewrites only its own leaf.
__global__ __launch_bounds__(kBlock) void k_rmi_bounds(const uint64_t *keys, uint64_t n,
                                                       const RmiHeader *Hp, RmiLeaf *leaves)
{
    // The header's fields are read into registers once: the leaves share the model's
    // buffer, so a field read after a store to a leaf would be loaded again.  Lane i < 32
    // holds knot i, lane j <= 32 segment j's intercept and slope.
    const uint32_t kind = Hp->kind;
    const uint32_t L = 1u << Hp->log2_leaves;
    const float ra = Hp->a, rb = Hp->b;
    const int lane = threadIdx.x & (kWave - 1);
    const float knot = Hp->t[lane & (kKnots - 1)];
    const int seg = lane <= kKnots ? lane : kKnots;
    const float seg_a = Hp->sa[seg], seg_b = Hp->sb[seg];
    const uint64_t gtid = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    if (n == 0) {                         // no keys: index 0 routes past the end
        for (uint64_t l = gtid; l < L; l += (uint64_t)gridDim.x * kBlock) leaves[l].base = 0;
        return;
    }
    // A wave takes 63 new indices per group: lane t routes index s - 1 + t, so every lane
    // but the first finds its predecessor's leaf in the lane below (each key is routed
    // about once instead of twice).  Indices run to n inclusive (index n routes past the
    // end, to L).  A wave loads the keys of kGroups consecutive groups before routing
    // them, at clamped indices so that the loads need no branch and are all in flight.
    constexpr int kGroups = 4;
    constexpr uint64_t kStep = (uint64_t)(kWave - 1) * kGroups;
    const uint64_t wave = gtid / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / kWave);
    for (uint64_t s0 = wave * kStep; s0 <= n; s0 += waves * kStep) {   // wave-uniform
        uint64_t kvs[kGroups];
#pragma unroll
        for (int g = 0; g < kGroups; g++) {
            const uint64_t i = s0 + (uint64_t)g * (kWave - 1) + lane - 1;   // wraps for s = 0
            kvs[g] = keys[i < n ? i : n - 1];
        }
#pragma unroll
        for (int g = 0; g < kGroups; g++) {
            const uint64_t s = s0 + (uint64_t)g * (kWave - 1);
            if (s > n) break;                            // wave-uniform
            const uint64_t i = s + lane - 1;             // s - 1 for lane 0 (wraps at s = 0)
            const bool key = !(lane == 0 && s == 0) && i < n;
            const float x = key_x(kvs[g]);
            uint32_t cur = 0;
            if (kind == 0) {
                cur = leaf_of(__builtin_fmaf(ra, x, rb), L);
            } else {
                // the keys are sorted, so a wave's keys usually share the root's segment:
                // it is then the number of knots below the first and the last key, which
                // 32 lanes compare at once (route() gives the same leaves)
                const uint64_t m = __ballot(key);
                uint32_t j = 0;
                if (m != 0) {
                    const int first = __ffsll((unsigned long long)m) - 1;
                    const int last = 63 - __clzll((long long)m);
                    const float x0 = __shfl(x, first), x1 = __shfl(x, last);
                    j = (uint32_t)__popcll(__ballot(lane < kKnots && knot < x0));
                    const uint32_t j1 =
                        (uint32_t)__popcll(__ballot(lane < kKnots && knot < x1));
                    if (j != j1) {                       // wave-uniform test
                        // per lane, as root_segment(), with knot t read from lane t
                        j = 0;
#pragma unroll
                        for (int t = 0; t < kKnots; t++) {
                            const float tk = __int_as_float(
                                __builtin_amdgcn_readlane(__float_as_int(knot), t));
                            j += tk < x ? 1u : 0u;
                        }
                    }
                }
                cur = leaf_of(root_value(__shfl(seg_a, (int)j), __shfl(seg_b, (int)j), x, L), L);
            }
            if (!key) cur = (lane == 0 && s == 0) ? 0u : L;   // index n and past it: L
            const uint32_t prv = __shfl_up(cur, 1);
            if (lane == 0 || i > n) continue;
            const uint32_t from = i > 0 ? prv + 1 : 0;
            for (uint32_t l = from; l <= cur && l < L; l++) leaves[l].base = (uint32_t)i;
        }
    }
}

// One thread per leaf: its end is the next leaf's start (n for the last leaf).
__global__ __launch_bounds__(kBlock) void k_rmi_ends(uint64_t n, uint32_t L, RmiLeaf *leaves)
{
    const uint32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l < L) leaves[l].end = l + 1 < L ? leaves[l + 1].base : (uint32_t)n;
}

// Four lanes per leaf (a group never straddles a wave; leaves hold about 20 keys, so more
// lanes would mostly idle): least-squares line through ((key >> 32) - khi, position) in
// FP64, the lanes taking every fourth key so that a group reads consecutive keys; the
// intercept's integer part moves into the leaf's base position; then the largest under-
// and over-prediction over the leaf's keys with the lookup's own prediction function
// (saturated at 65535: a larger miss only sends those lookups to the binary-search
// fallback).  The butterfly sums add the same pairs in every lane, so all four lanes hold
// identical totals.
constexpr int kFitLanes = 4;

__global__ __launch_bounds__(kBlock) void k_rmi_fit(const uint64_t *keys, uint64_t n,
                                                    const RmiHeader *Hp, RmiLeaf *leaves)
{
    const uint32_t L = 1u << Hp->log2_leaves;
    const uint64_t g = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    const uint64_t l = g / kFitLanes;
    const int j = (int)(g % kFitLanes);
    if (l >= L) return;                       // whole groups only
    const uint64_t lo = leaves[l].base;
    const uint64_t hi = leaves[l].end;
    RmiLeaf lf;
    lf.base = (uint32_t)lo;
    lf.khi = lo < n ? (uint32_t)(keys[lo] >> 32) : 0xffffffffu;
    lf.slope = 0.f;
    lf.err_lo = 0;
    lf.err_hi = 0;
    const uint64_t m = hi > lo ? hi - lo : 0;
    // the group's first kHold * kFitLanes keys stay in registers for the error pass;
    // longer leaves read the rest twice
    constexpr int kHold = 8;
    unsigned long long held[kHold];
#pragma unroll
    for (int c = 0; c < kHold; c++) {
        const uint64_t i = lo + j + (uint64_t)c * kFitLanes;
        held[c] = i < hi ? keys[i] : 0;
    }
    const uint64_t rest = lo + (uint64_t)kHold * kFitLanes;      // first key not held
    if (m >= 2) {
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        auto add = [&](uint64_t i, unsigned long long k) {
            const double x = (double)((uint32_t)(k >> 32) - lf.khi), y = (double)(i - lo);
            sx += x; sy += y; sxx += x * x; sxy += x * y;
        };
#pragma unroll
        for (int c = 0; c < kHold; c++) {
            const uint64_t i = lo + j + (uint64_t)c * kFitLanes;
            if (i < hi) add(i, held[c]);
        }
        for (uint64_t i = rest + j; i < hi; i += kFitLanes) add(i, keys[i]);
#pragma unroll
        for (int o = 1; o < kFitLanes; o <<= 1) {
            sx += __shfl_xor(sx, o, kFitLanes);
            sy += __shfl_xor(sy, o, kFitLanes);
            sxx += __shfl_xor(sxx, o, kFitLanes);
            sxy += __shfl_xor(sxy, o, kFitLanes);
        }
        const double var = sxx - sx * sx / (double)m;
        const double sl = var > 0 ? (sxy - sx * sy / (double)m) / var : 0.0;
        const double ic = (sy - sl * sx) / (double)m;
        lf.slope = (float)(sl > 0 ? sl : 0.0);
        // base = lo + floor(intercept), kept inside [0, n]
        const double b = (double)lo + floor(ic);
        lf.base = b <= 0.0 ? 0u : (b >= (double)n ? (uint32_t)n : (uint32_t)b);
    }
    // errors: keep every key's first occurrence inside [p - err_lo, p + err_hi]; a lane's
    // previous key is the lane below's (lane 0: the last key of the group's previous step)
    long long elo = 0, ehi = 0;
    unsigned long long carry = 0;
    auto step = [&](uint64_t i, unsigned long long k) {
        unsigned long long prev = __shfl_up(k, 1, kFitLanes);
        if (j == 0) prev = carry;
        if (i < hi && (i == lo || k != prev)) {
            const long long d = (long long)i - (long long)predict(lf, k);
            if (d > ehi) ehi = d;
            if (-d > elo) elo = -d;
        }
        carry = __shfl(k, kFitLanes - 1, kFitLanes);
    };
#pragma unroll
    for (int c = 0; c < kHold; c++)
        if (lo + (uint64_t)c * kFitLanes < hi) step(lo + j + (uint64_t)c * kFitLanes, held[c]);
    for (uint64_t i0 = rest; i0 < hi; i0 += kFitLanes) {         // uniform in the group
        const uint64_t i = i0 + j;
        step(i, i < hi ? keys[i] : 0);
    }
#pragma unroll
    for (int o = 1; o < kFitLanes; o <<= 1) {
        const long long a = __shfl_xor(elo, o, kFitLanes), b = __shfl_xor(ehi, o, kFitLanes);
        elo = a > elo ? a : elo;
        ehi = b > ehi ? b : ehi;
    }
    lf.err_lo = (uint16_t)(elo < 65535 ? elo : 65535);
    lf.err_hi = (uint16_t)(ehi < 65535 ? ehi : 65535);
    if (j == 0) leaves[l] = lf;
}

// Diagnostics: per query, whether the model's window brackets it (else the lookups fall
// back to binary search) and how many keys the window spans with its brackets, counted in
// LDS per workgroup.  stats: [0] queries, [1] fallbacks, [2 + b] windows of w keys with
// 2^(b-1) < w <= 2^b (b = 0..kRmiStatBins - 1, the last bin open-ended).
constexpr int kRmiStatBins = 18;

__global__ __launch_bounds__(kBlock) void k_rmi_stats(const uint64_t *keys, uint64_t n,
                                                      const void *rmi, size_t rmi_bytes_,
                                                      const uint64_t *q, uint64_t n_q,
                                                      unsigned long long *stats)
{
    __shared__ unsigned long long h[2 + kRmiStatBins];
    __shared__ int sh_valid;
    for (int i = threadIdx.x; i < 2 + kRmiStatBins; i += kBlock) h[i] = 0;
    if (threadIdx.x == 0) sh_valid = rmi_valid(rmi, rmi_bytes_, n);
    __syncthreads();
    const bool valid = sh_valid != 0;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n_q;
         i += (uint64_t)gridDim.x * kBlock) {
        int64_t lo = 0, hi = 0;
        if (!valid || !rmi_window(rmi, keys, n, q[i], lo, hi)) {
            atomicAdd(&h[1], 1ull);
            continue;
        }
        const uint64_t w = (uint64_t)(hi - lo) + 2;
        int b = 0;
        while (b < kRmiStatBins - 1 && (1ull << b) < w) b++;
        atomicAdd(&h[2 + b], 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 + kRmiStatBins; i += kBlock)
        if (h[i]) atomicAdd(&stats[i], h[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&stats[0], (unsigned long long)n_q);
}

}  // namespace

int rmi_stat_words() { return 2 + kRmiStatBins; }

hipError_t launch_rmi_stats(const uint64_t *keys, uint64_t n, const void *rmi, size_t rmi_bytes_,
                            const uint64_t *q, uint64_t n_q, uint64_t *stats, hipStream_t s)
{
    hipError_t e = fill_u64(stats, 0, (size_t)rmi_stat_words(), s);
    if (e != hipSuccess) return e;
    uint64_t blocks = (n_q + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    GD_LAUNCH(k_rmi_stats, dim3((unsigned)blocks), dim3(kBlock), 0, s, keys, n, rmi, rmi_bytes_, q,
              n_q, (unsigned long long *)stats);
    return hipGetLastError();
}

size_t rmi_bytes(uint32_t log2_leaves)
{
    return sizeof(RmiHeader) + ((size_t)1 << log2_leaves) * sizeof(RmiLeaf);
}

hipError_t launch_rmi_train(const uint64_t *keys, uint64_t n, int kind, uint32_t log2_leaves,
                            void *rmi, hipStream_t s)
{
    RmiHeader *H = (RmiHeader *)rmi;
    RmiLeaf *leaves = (RmiLeaf *)((char *)rmi + sizeof(RmiHeader));
    const uint32_t L = 1u << log2_leaves;
    GD_LAUNCH(k_rmi_root, dim3(1), dim3(kBlock), 0, s, keys, n, kind, log2_leaves, H);
    uint64_t blocks = (n + 1 + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    GD_LAUNCH(k_rmi_bounds, dim3((unsigned)blocks), dim3(kBlock), 0, s, keys, n,
              (const RmiHeader *)H, leaves);
    GD_LAUNCH(k_rmi_ends, dim3((L + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, L, leaves);
    GD_LAUNCH(k_rmi_fit, dim3((unsigned)(((uint64_t)L * kFitLanes + kBlock - 1) / kBlock)),
              dim3(kBlock), 0, s, keys, n,
              (const RmiHeader *)H, leaves);
    return hipGetLastError();
}

}  // namespace gd
