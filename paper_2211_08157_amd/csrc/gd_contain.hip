// Containment-style counts: for every genome g of a multi-genome index (64-bit values,
// genome id in the top 32 bits), the number of distinct minimizer hashes g shares with a
// read sample, and the number of distinct hashes g has.
//
// The sample's minimizers (each read at its aligned shift) are looked up as for seeding;
// every index position holding a sample hash is marked (plain byte stores: all writers
// store the same value).  One pass over the index then finds the first record of every
// (hash, genome) pair -- records are sorted by (hash, genome << 32 | ...) -- and adds it to
// the genome's size and, when marked, to its shared count, through per-workgroup LDS
// histograms flushed with one atomic per genome and workgroup.
#include "gd_internal.h"

namespace gd {

namespace {

__device__ __forceinline__ uint64_t rec_at(const AlignArgs &A, uint32_t s, uint32_t r)
{
    return A.mzofs[s * ((size_t)A.n_reads + 1) + r];
}

// One thread per read: mark the index runs of its minimizers at the chosen shift.
__global__ __launch_bounds__(kBlock) void k_mark(AlignArgs A, const uint32_t *shift_slot,
                                                 uint8_t *mark)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= A.n_reads) return;
    const uint32_t slot = shift_slot[r];
    const uint64_t beg = rec_at(A, slot, r), end = rec_at(A, slot, r + 1);
    const uint32_t *occ = A.occ + slot * A.stride;
    const uint32_t *lb = A.lb + slot * A.stride;
    for (uint64_t j = beg; j < end; j++) {
        const uint32_t o = occ[j], l = lb[j];
        for (uint32_t e = 0; e < o; e++) mark[l + e] = 1;
    }
}

constexpr uint32_t kLdsGenomes = 4096;

__global__ __launch_bounds__(kBlock) void k_contain_count(const uint64_t *keys, const uint64_t *vals,
                                                          uint64_t n, const uint8_t *mark,
                                                          uint32_t n_genomes, uint32_t *counts,
                                                          uint32_t *sizes, uint32_t *status)
{
    __shared__ uint32_t hc[kLdsGenomes], hs[kLdsGenomes];
    const bool lds = n_genomes <= kLdsGenomes;
    if (lds)
        for (uint32_t g = threadIdx.x; g < n_genomes; g += kBlock) { hc[g] = 0; hs[g] = 0; }
    __syncthreads();
    for (uint64_t e = blockIdx.x * (uint64_t)kBlock + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * kBlock) {
        const uint64_t g = vals[e] >> 32;
        if (e > 0 && keys[e] == keys[e - 1] && (vals[e - 1] >> 32) == g) continue;
        if (g >= n_genomes) { set_status(status, 2u); continue; }
        const uint32_t m = mark[e];
        if (lds) {
            atomicAdd(&hs[g], 1u);
            if (m) atomicAdd(&hc[g], 1u);
        } else {
            atomicAdd(&sizes[g], 1u);
            if (m) atomicAdd(&counts[g], 1u);
        }
    }
    if (!lds) return;
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < n_genomes; g += kBlock) {
        if (hs[g]) atomicAdd(&sizes[g], hs[g]);
        if (hc[g]) atomicAdd(&counts[g], hc[g]);
    }
}

}  // namespace

hipError_t launch_contain(const AlignArgs &a, const uint32_t *shift_slot, const uint64_t *ikeys,
                          const uint64_t *ivals, uint64_t in, uint8_t *mark, uint32_t n_genomes,
                          uint32_t *counts, uint32_t *sizes, uint32_t *status, hipStream_t s)
{
    hipError_t e;
    if ((e = fill_u32((uint32_t *)mark, 0, (in + 3) / 4, s)) != hipSuccess) return e;
    if ((e = fill_u32(counts, 0, n_genomes, s)) != hipSuccess) return e;
    if ((e = fill_u32(sizes, 0, n_genomes, s)) != hipSuccess) return e;
    if (a.n_reads > 0)
        GD_LAUNCH(k_mark, dim3((a.n_reads + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a,
                  shift_slot, mark);
    if (in > 0) {
        uint64_t blocks = (in + kBlock - 1) / kBlock;
        if (blocks > 2048) blocks = 2048;
        GD_LAUNCH(k_contain_count, dim3((unsigned)blocks), dim3(kBlock), 0, s, ikeys, ivals, in,
                  (const uint8_t *)mark, n_genomes, counts, sizes, status);
    }
    return hipGetLastError();
}

}  // namespace gd
