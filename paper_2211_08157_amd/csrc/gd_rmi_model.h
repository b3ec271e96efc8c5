// Learned-index model layout and its device inference (shared by the training kernels and
// the lookup kernels, which live in different translation units).
#pragma once
#include "gd_common.h"

namespace gd {

constexpr uint32_t kRmiMagic = 0x524d4932u;   // "RMI2"
constexpr int kKnots = 32;

// The MLP root y = c[0] + sum_i c[i + 1] * relu(x - t[i]) is evaluated per segment: with
// knots ascending and j of them below x, y = sa[j] + sb[j] * x, where sb[j] sums the first
// j output weights and sa[j] = c[0] minus the same weights times their knots (prefix
// sums in FP32, written once by the training, which also makes the segments agree in
// order at every knot; training and lookups evaluate sb[j] * x + sa[j] as one fused
// multiply-add, so they route identically).
struct RmiHeader {
    uint32_t magic, kind, log2_leaves, pad;
    uint64_t n_keys;
    float a, b;                 // linear root
    float t[kKnots];            // MLP knots (ascending)
    float c[kKnots + 1];        // MLP output weights (c[0] is the bias)
    float sa[kKnots + 1];       // per-segment intercept
    float sb[kKnots + 1];       // per-segment slope
    float pad2[5];
};

// 16 bytes, so that a leaf is one load.  The prediction works on the key's high 32 bits:
// a leaf spans about 2^64 / 2^log2_leaves of key space, so dropping the low half costs
// far less than one position.  The fitted line's intercept is folded into base (its
// integer part; the fraction is absorbed by the error bounds), so the model holds only a
// position, an FP32 slope and the bounds.
struct RmiLeaf {
    uint32_t khi;              // high 32 bits of the leaf's first key
    uint32_t base;             // predicted position of a key with high bits khi
    union {
        float slope;           // positions per unit of (key >> 32)
        uint32_t end;          // during training only: one past the leaf's last key
    };
    uint16_t err_lo, err_hi;   // largest under- and over-prediction, saturated at 65535
};
static_assert(sizeof(RmiLeaf) == 16, "leaf record is 16 bytes");
static_assert(sizeof(RmiHeader) == 576, "header keeps the leaves 64-byte aligned");

// Whether `rmi` (rmi_bytes bytes) is a model of an index of n keys whose leaves all lie
// inside the buffer (the model's content is never trusted beyond that: every lookup
// checks its window against the keys).
__device__ __forceinline__ bool rmi_valid(const void *rmi, size_t rmi_bytes, uint64_t n)
{
    if (rmi_bytes < sizeof(RmiHeader)) return false;
    const RmiHeader &H = *(const RmiHeader *)rmi;
    return H.magic == kRmiMagic && H.n_keys == n && n > 0 && H.log2_leaves >= 1 &&
           H.log2_leaves <= 24 && H.kind <= 1 &&
           sizeof(RmiHeader) + ((size_t)1 << H.log2_leaves) * sizeof(RmiLeaf) <= rmi_bytes;
}

__device__ __forceinline__ float key_x(uint64_t k)
{
    return __fmul_rn(__ull2float_rn(k), 5.421010862427522e-20f);   // k * 2^-64
}

// Leaf of a root value y (in leaves, before clamping).
__device__ __forceinline__ uint32_t leaf_of(float y, uint32_t L)
{
    if (!(y > 0.f)) return 0;            // also catches NaN
    if (y >= (float)L) return L - 1;
    const uint32_t l = (uint32_t)y;
    return l < L ? l : L - 1;
}

// Number of MLP knots below x (the segment of the root's piecewise-linear function).
__device__ __forceinline__ uint32_t root_segment(const RmiHeader &H, float x)
{
    uint32_t j = 0;
#pragma unroll
    for (int i = 0; i < kKnots; i++) j += H.t[i] < x ? 1u : 0u;
    return j;
}

// Root value of x, in leaves, from its segment's intercept and slope: one fused
// multiply-add (a single rounding, written out so that no compiler contraction choice can
// make two callers differ), then the exact scaling by the power of two L.
__device__ __forceinline__ float root_value(float sa, float sb, float x, uint32_t L)
{
    return __builtin_fmaf(sb, x, sa) * (float)L;
}

// Root value of x on segment j, in leaves.
__device__ __forceinline__ float root_on_segment(const RmiHeader &H, uint32_t j, float x)
{
    return root_value(H.sa[j], H.sb[j], x, 1u << H.log2_leaves);
}

__device__ __forceinline__ uint32_t route(const RmiHeader &H, uint64_t k)
{
    const float x = key_x(k);
    const uint32_t L = 1u << H.log2_leaves;
    const float y = H.kind == 0 ? __builtin_fmaf(H.a, x, H.b)
                                : root_on_segment(H, root_segment(H, x), x);
    return leaf_of(y, L);
}

__device__ __forceinline__ int64_t predict(const RmiLeaf &lf, uint64_t k)
{
    const uint32_t kh = (uint32_t)(k >> 32);
    const float d = kh >= lf.khi ? __uint2float_rn(kh - lf.khi) : 0.f;
    return (int64_t)lf.base + (int64_t)floorf(__fmul_rn(lf.slope, d));
}

// The key window the model gives q: [lo, hi) with lo = p - err_lo and hi = p + err_hi + 1
// clamped to the keys.  Returns whether it brackets q (keys[lo - 1] < q <= keys[hi], the
// array ends counting as brackets); the lookups fall back to binary search otherwise.
__device__ __forceinline__ bool rmi_window(const void *rmi, const uint64_t *keys, uint64_t n,
                                           uint64_t q, int64_t &lo, int64_t &hi)
{
    const RmiHeader &H = *(const RmiHeader *)rmi;
    const RmiLeaf *leaves = (const RmiLeaf *)((const char *)rmi + sizeof(RmiHeader));
    const RmiLeaf lf = leaves[route(H, q)];
    const int64_t p = predict(lf, q);
    lo = p - lf.err_lo;
    hi = p + lf.err_hi + 1;
    if (lo < 0) lo = 0;
    if (hi > (int64_t)n) hi = (int64_t)n;
    return lo <= hi && (lo == 0 || keys[lo - 1] < q) && (hi == (int64_t)n || keys[hi] >= q);
}

// lower_bound of q in the sorted keys through the model (valid: rmi_valid held); exact
// whatever the model holds.
__device__ __forceinline__ uint64_t rmi_lower_bound(const void *rmi, bool valid,
                                                    const uint64_t *keys, uint64_t n, uint64_t q)
{
    const RmiHeader &H = *(const RmiHeader *)rmi;
    const RmiLeaf *leaves = (const RmiLeaf *)((const char *)rmi + sizeof(RmiHeader));
    if (valid) {
        const RmiLeaf lf = leaves[route(H, q)];
        const int64_t p = predict(lf, q);
        int64_t lo = p - lf.err_lo, hi = p + lf.err_hi + 1;
        if (lo < 0) lo = 0;
        if (hi > (int64_t)n) hi = (int64_t)n;
        if (lo <= hi && (lo == 0 || keys[lo - 1] < q) && (hi == (int64_t)n || keys[hi] >= q)) {
            uint64_t a = (uint64_t)lo, len = (uint64_t)(hi - lo);
            while (len > 0) {
                const uint64_t half = len >> 1;
                if (keys[a + half] < q) { a += half + 1; len -= half + 1; }
                else len = half;
            }
            return a;
        }
    }
    uint64_t a = 0, len = n;                  // fallback: plain binary search
    while (len > 0) {
        const uint64_t half = len >> 1;
        if (keys[a + half] < q) { a += half + 1; len -= half + 1; }
        else len = half;
    }
    return a;
}

}  // namespace gd
