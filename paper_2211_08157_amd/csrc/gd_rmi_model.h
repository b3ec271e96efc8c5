// Learned-index model layout and its device inference (shared by the training kernels and
// the lookup kernels, which live in different translation units).
#pragma once
#include "gd_common.h"

namespace gd {

constexpr uint32_t kRmiMagic = 0x524d4931u;   // "RMI1"
constexpr int kKnots = 32;

struct RmiHeader {
    uint32_t magic, kind, log2_leaves, pad;
    uint64_t n_keys;
    float a, b;                 // linear root
    float t[kKnots];            // MLP knots
    float c[kKnots + 1];        // MLP output weights (c[0] is the bias)
    float pad2[7];
};

// 16 bytes, so that a leaf is one load.  The prediction works on the key's high 32 bits:
// a leaf spans about 2^64 / 2^log2_leaves of key space, so dropping the low half costs
// far less than one position.
struct RmiLeaf {
    uint32_t khi;              // high 32 bits of the leaf's first key
    uint32_t base;             // index of the leaf's first key
    float slope;               // positions per unit of (key >> 32)
    _Float16 icpt;             // intercept in positions
    uint8_t err_lo, err_hi;    // largest under- and over-prediction, saturated at 255
};
static_assert(sizeof(RmiLeaf) == 16, "leaf record is 16 bytes");
static_assert(sizeof(RmiHeader) == 320, "header keeps the leaves 64-byte aligned");

__device__ __forceinline__ float key_x(uint64_t k)
{
    return __fmul_rn(__ull2float_rn(k), 5.421010862427522e-20f);   // k * 2^-64
}

__device__ __forceinline__ uint32_t route(const RmiHeader &H, uint64_t k)
{
    const float x = key_x(k);
    const uint32_t L = 1u << H.log2_leaves;
    float y;
    if (H.kind == 0) {
        y = __fadd_rn(__fmul_rn(H.a, x), H.b);
    } else {
        float acc = H.c[0];
#pragma unroll
        for (int i = 0; i < kKnots; i++) acc = __fadd_rn(acc, __fmul_rn(H.c[i + 1], fmaxf(__fsub_rn(x, H.t[i]), 0.f)));
        y = __fmul_rn(acc, (float)L);
    }
    if (!(y > 0.f)) return 0;            // also catches NaN
    if (y >= (float)L) return L - 1;
    const uint32_t l = (uint32_t)y;
    return l < L ? l : L - 1;
}

__device__ __forceinline__ int64_t predict(const RmiLeaf &lf, uint64_t k)
{
    const uint32_t kh = (uint32_t)(k >> 32);
    const float d = kh >= lf.khi ? __uint2float_rn(kh - lf.khi) : 0.f;
    const float f = __fadd_rn((float)lf.icpt, __fmul_rn(lf.slope, d));
    return (int64_t)lf.base + (int64_t)floorf(f);
}

// lower_bound of q in the sorted keys through the model; exact whatever the model holds.
__device__ __forceinline__ uint64_t rmi_lower_bound(const void *rmi, const uint64_t *keys,
                                                    uint64_t n, uint64_t q)
{
    const RmiHeader &H = *(const RmiHeader *)rmi;
    const RmiLeaf *leaves = (const RmiLeaf *)((const char *)rmi + sizeof(RmiHeader));
    if (H.magic == kRmiMagic && H.n_keys == n && n > 0) {
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
