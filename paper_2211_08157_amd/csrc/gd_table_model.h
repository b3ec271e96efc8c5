// Hash-table form of the seed index (shared by its build kernels and the lookup kernels).
//
// The paper's index maps every distinct minimizer hash to its sorted location list
// (Section 3.1).  The lists are the runs of equal keys in the sorted arrays, so a slot
// holds {key, start, count}: the run is [start, start + count) of the sorted keys/vals.
// Open addressing with linear probing over 2^b slots (2^b >= 2 n, load factor <= 1/2);
// the home slot of a key is its low b bits (minimizer hashes are skewed toward small
// values in their high bits only).  count == 0 marks an empty slot (every run has one or
// more records; a key of 0 is a real hash, so keys cannot mark emptiness).
#pragma once
#include "gd_common.h"

namespace gd {

constexpr uint32_t kTableMagic = 0x48544231u;   // "HTB1"

struct TableHeader {
    uint32_t magic, log2_slots;
    uint64_t n_keys;
    uint64_t pad[6];
};
static_assert(sizeof(TableHeader) == 64, "slots start 64 bytes in");

struct TableSlot {
    uint64_t key;
    uint32_t start, count;
};
static_assert(sizeof(TableSlot) == 16, "a slot is one 16-byte load");

// (start, count) of q; count 0 when q is absent.  Returns false when the table does not
// belong to an index of n keys (the caller then searches the sorted keys).
__device__ __forceinline__ bool table_find(const void *table, uint64_t n, uint64_t q,
                                           uint64_t &start, uint64_t &count)
{
    const TableHeader &H = *(const TableHeader *)table;
    if (H.magic != kTableMagic || H.n_keys != n || H.log2_slots > 40) return false;
    const uint64_t mask = (1ull << H.log2_slots) - 1;
    const ulonglong2 *slots = (const ulonglong2 *)((const char *)table + sizeof(TableHeader));
    uint64_t s = q & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        const ulonglong2 v = slots[s];
        const uint32_t cnt = (uint32_t)(v.y >> 32);
        if (cnt == 0) { start = 0; count = 0; return true; }
        if (v.x == q) { start = (uint32_t)v.y; count = cnt; return true; }
        s = (s + 1) & mask;
    }
    start = 0;
    count = 0;
    return true;
}

}  // namespace gd
