// Build of the hash-table form of a sorted seed index (layout in gd_table_model.h):
// clear the slots, write the header, then one thread per record inserts the run that
// starts at it (the first record of each distinct key) by claiming the first empty slot
// from the key's home slot with a compare-and-swap on the count word.  Keys are distinct
// per insertion, so no key comparison is needed while inserting; the slot a key lands in
// depends on the order of the claims, its (start, count) and every lookup's result do
// not.
#include "gd_internal.h"
#include "gd_table_model.h"

namespace gd {

namespace {

__global__ void k_table_header(const uint64_t *keys, void *table, uint32_t log2_slots, uint64_t n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    TableHeader h;
    h.magic = kTableMagic;
    h.log2_slots = log2_slots;
    h.n_keys = n;
    h.keys_fp = table_keys_fp(keys, n);
    for (int i = 0; i < 5; i++) h.pad[i] = 0;
    *(TableHeader *)table = h;
}

__global__ __launch_bounds__(kBlock) void k_table_insert(const uint64_t *keys, uint64_t n,
                                                         uint32_t log2_slots, void *table)
{
    const uint64_t mask = (1ull << log2_slots) - 1;
    TableSlot *slots = (TableSlot *)((char *)table + sizeof(TableHeader));
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kBlock) {
        const uint64_t key = keys[i];
        if (i > 0 && keys[i - 1] == key) continue;       // not the first of its run
        uint64_t e = i + 1;                               // run end by galloping
        uint64_t step = 1;
        while (e < n && keys[e] == key) { e += step; step <<= 1; }
        uint64_t lo = e - (step >> 1), hi = e < n ? e : n;      // end in (lo, hi]
        if (lo <= i) lo = i + 1;
        while (lo < hi) {
            const uint64_t m = lo + ((hi - lo) >> 1);
            if (keys[m] == key) lo = m + 1; else hi = m;
        }
        const uint32_t count = (uint32_t)(lo - i);
        uint64_t s = key & mask;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            if (atomicCAS(&slots[s].count, 0u, count) == 0u) {
                slots[s].key = key;
                slots[s].start = (uint32_t)i;
                break;
            }
            s = (s + 1) & mask;
        }
    }
}

}  // namespace

uint32_t table_log2_slots(uint64_t n)
{
    uint32_t b = 4;
    while (b < 40 && (1ull << b) < 2 * n) b++;
    return b;
}

size_t table_bytes(uint64_t n)
{
    return sizeof(TableHeader) + ((size_t)1 << table_log2_slots(n)) * sizeof(TableSlot);
}

hipError_t launch_table_build(const uint64_t *keys, uint64_t n, void *table, hipStream_t s)
{
    const uint32_t b = table_log2_slots(n);
    hipError_t e = fill_u32((uint32_t *)table, 0, table_bytes(n) / 4, s);
    if (e != hipSuccess) return e;
    GD_LAUNCH(k_table_header, dim3(1), dim3(64), 0, s, keys, table, b, n);
    if (n > 0) {
        uint64_t blocks = (n + kBlock - 1) / kBlock;
        if (blocks > 16384) blocks = 16384;
        GD_LAUNCH(k_table_insert, dim3((unsigned)blocks), dim3(kBlock), 0, s, keys, n, b, table);
    }
    return hipGetLastError();
}

}  // namespace gd
