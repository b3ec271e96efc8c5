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
    uint64_t keys_fp;       // table_keys_fp of the keys the table was built over
    uint64_t pad[5];
};
static_assert(sizeof(TableHeader) == 64, "slots start 64 bytes in");

struct TableSlot {
    uint64_t key;
    uint32_t start, count;
};
static_assert(sizeof(TableSlot) == 16, "a slot is one 16-byte load");

// Fingerprint of a sorted key array: its size and eight keys spread over it, mixed.  A
// table whose fingerprint differs was built over other keys.
__device__ __forceinline__ uint64_t table_keys_fp(const uint64_t *keys, uint64_t n)
{
    uint64_t h = n * 0x9e3779b97f4a7c15ull;
    for (int i = 0; i < 8 && n > 0; i++) {
        h ^= keys[(n - 1) * (uint64_t)i / 7];
        h = (h ^ (h >> 29)) * 0xbf58476d1ce4e5b9ull;
    }
    return h ^ (h >> 32);
}

// Whether `table` (table_bytes bytes) is a hash table of the n keys with fingerprint fp
// whose slots all lie inside the buffer.
__device__ __forceinline__ bool table_valid(const void *table, size_t table_bytes, uint64_t n,
                                            uint64_t fp)
{
    if (table_bytes < sizeof(TableHeader)) return false;
    const TableHeader &H = *(const TableHeader *)table;
    return H.magic == kTableMagic && H.n_keys == n && H.keys_fp == fp && H.log2_slots <= 40 &&
           sizeof(TableHeader) + (((size_t)1 << H.log2_slots) * sizeof(TableSlot)) <= table_bytes;
}

// (start, count) of q; count 0 when q is absent.  The caller has checked table_valid.
// Returns false when a slot's run does not lie inside the n keys (the caller then
// searches the sorted keys).
__device__ __forceinline__ bool table_find(const void *table, uint64_t n, uint64_t q,
                                           uint64_t &start, uint64_t &count)
{
    const TableHeader &H = *(const TableHeader *)table;
    const uint64_t mask = (1ull << H.log2_slots) - 1;
    const ulonglong2 *slots = (const ulonglong2 *)((const char *)table + sizeof(TableHeader));
    uint64_t s = q & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        const ulonglong2 v = slots[s];
        const uint32_t cnt = (uint32_t)(v.y >> 32);
        if (cnt == 0) { start = 0; count = 0; return true; }
        if (v.x == q) {
            start = (uint32_t)v.y;
            count = cnt;
            return start + count <= n;
        }
        s = (s + 1) & mask;
    }
    start = 0;
    count = 0;
    return true;
}

}  // namespace gd
