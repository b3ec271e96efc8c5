// Host-side launchers shared between the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gd_common.h"
#include "godiet.h"

namespace gd {

namespace trace {
bool enabled();
// Records HIP events on stream s around the kernel launched during its lifetime.
class Scope {
  public:
    Scope(const char *name, hipStream_t s);
    ~Scope();

  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_, b_;
};
}  // namespace trace

// Launch a kernel on stream s, bracketed by trace events when tracing is on.
// Launches a kernel (traced when tracing is on) and returns from the calling function
// with the error if the launch failed (every caller returns hipError_t).
#define GD_LAUNCH(kernel, grid, block, shmem, s, ...)                        \
    do {                                                                      \
        ::gd::trace::Scope gd_scope_(#kernel, s);                             \
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, __VA_ARGS__);       \
        const hipError_t gd_err_ = hipGetLastError();                         \
        if (gd_err_ != hipSuccess) return gd_err_;                            \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves sub-buffers out of the caller's workspace.  With base == nullptr it only
// measures, so the same plan code sizes and lays out the workspace.
struct Bump {
    char *base;
    size_t off = 0;
    explicit Bump(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count)
    {
        off = align_up(off, 256);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T) + 16;   // +16: vector loads may touch a little beyond
        return p;
    }
};

// ---- fill / scan (gd_scan.hip) ----
hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);
// Scratch (in uint64 elements) that exclusive_scan needs for n inputs.
size_t scan_scratch(size_t n);
// out[i] = sum_{j<i} in[j] for i in [0, n]; in is uint32 or uint64.
hipError_t exclusive_scan_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *scratch,
                              hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t *in, uint64_t *out, size_t n, uint64_t *scratch,
                              hipStream_t s);

// ---- sparsify / sketch (gd_sketch.hip) ----
enum ValMode : int { VAL_LOCAL32 = 0, VAL_GLOBAL32 = 1, VAL_SEQ64 = 2 };

// Geometry of the sketch tiles for a given w.
constexpr int kSkBlock = 512;   // threads per sketch tile, 16 positions each
struct TileGeom {
    int H;   // halo k-mers on each side (multiple of 16, >= w - 1)
    int T;   // output k-mers per tile
};
TileGeom tile_geom(int w);

// Device batch view used by the launchers.
struct Batch {
    const uint8_t *bases;
    const uint64_t *offsets;
    uint32_t n_seq;
    uint64_t n_bases;
    const uint32_t *nmask;   // N bit per base, or null
};

// Per-sequence kept counts (shift from shift[] or the uniform value) -> out[n_seq].
hipError_t launch_kept(const Batch &b, const Pattern &P, const uint32_t *shift,
                       uint32_t uniform_shift, uint64_t *kept, uint32_t *status, hipStream_t s);
// Patterned stream (uint32 words, 16 bases each) of `words` words from pofs; with b.nmask
// and pnw set, also the N bits of the kept bases (pnw: `words` 16-bit halves).
// lohi: per-workgroup sequence ranges, computed here unless ranges_ready.
hipError_t launch_sparsify(const Batch &b, const Pattern &P, const uint32_t *shift,
                           uint32_t uniform_shift, const uint64_t *pofs, uint32_t *psw,
                           uint32_t *pnw, size_t words, uint32_t *lohi, bool ranges_ready,
                           hipStream_t s);
// Sequence ranges of the sparsify workgroups (sparsify_lohi(words) entries) and of the
// sketch tiles for window w (2 * sketch_tiles_bound(np_bound, w) entries) in one launch.
hipError_t launch_window_ranges(const uint64_t *pofs, uint32_t n_seq, size_t words,
                                uint64_t np_bound, int w, uint32_t *lohi_sp, uint32_t *lohi_sk,
                                hipStream_t s);
// Text to 2-bit codes and N bits (godiet_pack_ascii).
hipError_t launch_pack_ascii(const char *text, uint64_t n, uint32_t *bases, uint16_t *nmask,
                             hipStream_t s);
// A sparsify workgroup of kBlock threads writes kSpWords output words per thread (16 kept
// bases each): its range of the patterned stream is kSpSpan positions.
constexpr int kSpWords = 4;
constexpr uint64_t kSpSpan = (uint64_t)kBlock * kSpWords * 16;
inline size_t sparsify_blocks(size_t words)
{
    return (words + (size_t)kBlock * kSpWords - 1) / ((size_t)kBlock * kSpWords);
}
// Entries of the lohi scratch a sparsify of `words` output words needs.
inline size_t sparsify_lohi(size_t words) { return 2 * sparsify_blocks(words) + 2; }

struct SketchOut {
    uint64_t *keys;
    void *vals;
    int val_mode;
    uint64_t *mz_offsets;   // n_seq + 1, may be null
    uint64_t capacity;
    uint64_t *n_out;        // may be null
};
// Minimizers of the patterned stream; tile_state holds sketch_tiles_bound(np_bound) + 1
// words (the last one is the tile ticket counter).
size_t sketch_tiles_bound(uint64_t np_bound, int w);
hipError_t launch_sketch(const Batch &b, const Pattern &P, const uint32_t *shift,
                         uint32_t uniform_shift, const uint64_t *pofs, const uint32_t *psw,
                         const uint32_t *pnw, uint64_t np_bound, int k, int w, int hash,
                         const SketchOut &o, uint64_t *tile_state, uint32_t *lohi,
                         bool ranges_ready, uint32_t *status, hipStream_t s);

// Words of the patterned stream buffer for an upper bound on kept bases.
inline size_t psw_words(uint64_t np_bound) { return (size_t)(np_bound / 16) + 8; }
// 32-bit words of its N mask (16 bits per stream word).
inline size_t pnw_words(uint64_t np_bound) { return (psw_words(np_bound) + 1) / 2; }

// ---- index sort (gd_sort.hip) ----
struct SortPlan {
    int Bf;                // fine-histogram bits (top bits of the key)
    size_t nfine;          // 2^Bf fine bins
    size_t target;         // records per coarse bucket
    size_t ncoarse;        // coarse buckets launched
    bool digits;           // counting pass of balanced digits with workgroup-local counters
    bool two_level;        // digits mode through a coarse then a fine scatter (large indexes)
    size_t nchunks;        // digits mode: record chunks (one workgroup each)
    size_t chunk;          // digits mode: records per chunk
};
SortPlan sort_plan(uint64_t expected_records, uint64_t capacity, int val_bytes);
size_t sort_top_bins();    // slices of the digits mode's key histogram
// Scratch pieces the sort needs.
struct SortWs {
    uint32_t *hist;        // nfine (digits mode: nchunks * nfine per-chunk digit counts)
    uint32_t *tot;         // digits mode: nfine digit totals
    uint32_t *top;         // digits mode: sort_top_bins() key-slice counts
    uint64_t *cdf;         // digits mode: sort_top_bins() + 1 cumulative slice counts
    uint64_t *fofs;        // nfine + 1
    uint32_t *rank;        // capacity: rank of each record inside its fine bin
    uint64_t *scan_tmp;    // scan_scratch(max(nfine, sort_top_bins()))
    ulonglong2 *trec;      // capacity: (key, value) records grouped by fine bin
    ulonglong2 *tmp;       // two-level: capacity records grouped by coarse digit
    uint32_t *cmat;        // two-level: nchunks * 256 per-chunk coarse-digit counts
    uint32_t *cstart;      // ncoarse + 1: first fine bin of each coarse bucket
    uint32_t *overflow;    // ncoarse
    uint32_t *blist;       // ncoarse: buckets for the digits mode's largest bucket launch
    uint32_t *overflow_n;  // 2: entries of overflow, then of blist
};
hipError_t launch_sort(const SortPlan &sp, const SortWs &w, uint64_t *keys, void *vals,
                       int val_bytes, const uint64_t *n_ptr, uint64_t capacity, hipStream_t s);

// ---- location voting (gd_vote.hip) ----
struct VoteArgs {
    uint32_t max_dist, min_votes, max_win;
    int lz;                 // key shift that puts the read id at the top of the key
    int sort;               // 0 adaptive, 1 batch digit sort, 2 per-read merge, 3 per-read heap
};
hipError_t launch_vote(const VoteArgs &A, const uint4 *anchors, const uint64_t *read_off,
                       uint32_t n_reads, uint64_t capacity, const SortPlan &sp,
                       const SortWs &sw, uint64_t *keys, uint32_t *vals, uint32_t *long_ids,
                       uint32_t *long_n, godiet_winner *out, uint32_t *n_win,
                       uint32_t *status, hipStream_t s);

// ---- lookups, alignment, anchors (gd_seed.hip) ----
// lb/occ of min(*n_q, q_cap) queries (n_q may be null: q_cap queries); rmi nullable.
// table (nullable, seeding only): hash-table lookups, whose lb is 0 for absent keys
hipError_t launch_random_gather(const uint64_t *src, uint64_t n_src, const uint64_t *idx,
                                uint64_t n_idx, uint64_t *out, uint32_t *status, hipStream_t s);
hipError_t launch_lookup(const uint64_t *ikeys, uint64_t in, const uint64_t *q,
                         const uint64_t *n_q, uint64_t q_cap, uint32_t *lb, uint32_t *occ,
                         const void *rmi, size_t rmi_bytes, const void *table,
                         size_t table_bytes, uint32_t max_blocks, hipStream_t s);

// ---- hash-table index form (gd_table.hip) ----
uint32_t table_log2_slots(uint64_t n);
size_t table_bytes(uint64_t n);
hipError_t launch_table_build(const uint64_t *keys, uint64_t n, void *table, hipStream_t s);

// ---- learned index (gd_rmi.hip)
size_t rmi_bytes(uint32_t log2_leaves);
int rmi_stat_words();
hipError_t launch_rmi_stats(const uint64_t *keys, uint64_t n, const void *rmi, size_t rmi_bytes,
                            const uint64_t *q, uint64_t n_q, uint64_t *stats, hipStream_t s);
hipError_t launch_rmi_train(const uint64_t *keys, uint64_t n, int kind, uint32_t log2_leaves,
                            void *rmi, hipStream_t s);

struct AlignArgs {
    const uint64_t *mzofs;   // shift-major: [n_shift][n_reads + 1]
    const uint32_t *occ;     // shift-major: [n_shift][stride]
    const uint32_t *lb;
    const uint32_t *qval;
    size_t stride;           // records per shift slot
    uint32_t n_reads;
    uint32_t n_shift;        // sketched shifts (p, or 1 for a fixed shift)
    int32_t fixed_shift;     // -1 when the shifts 0..p-1 were sketched
    uint32_t align_t, max_occ;
    uint32_t long_records;   // reads with more records go to the wave-per-read kernels
    uint32_t long_blocks;    // workgroups of those kernels
};
// Shift choice and per-read anchor counts; reads with many records go to long_ids
// (n_reads entries) for a wave-per-read pass (from the front, count long_n[0]), reads with
// very many to its back for a workgroup-per-read pass (count long_n[1]).
hipError_t launch_align(const AlignArgs &a, uint8_t *shift_out, uint32_t *shift_slot,
                        uint32_t *anchor_cnt, uint32_t *long_ids, uint32_t *long_n, hipStream_t s);
hipError_t launch_expand(const AlignArgs &a, const uint32_t *shift_slot,
                         const uint64_t *read_off, const void *ivals, uint32_t *anchors,
                         uint64_t capacity, uint32_t *status, const uint32_t *long_ids,
                         const uint32_t *long_n, hipStream_t s);

// ---- containment counts (gd_contain.hip); mark holds ceil(in / 4) * 4 bytes
hipError_t launch_contain(const AlignArgs &a, const uint32_t *shift_slot, const uint64_t *ikeys,
                          const uint64_t *ivals, uint64_t in, uint8_t *mark, uint32_t n_genomes,
                          uint32_t *counts, uint32_t *sizes, uint32_t *status, hipStream_t s);

// ---- seed-matching experiment (gd_fig4.hip) ----
hipError_t launch_seed_match(const godiet_seqs *a, const godiet_seqs *b, const Pattern &P, int k,
                             int w, int hash, uint32_t *counts, uint32_t *status, hipStream_t s);
hipError_t launch_edit_distance(const godiet_seqs *a, const godiet_seqs *b, uint32_t *dist,
                                uint32_t *status, hipStream_t s);
hipError_t launch_accepted(const uint32_t *dist, const uint32_t *counts, uint32_t n, int g,
                           uint32_t max_e, uint64_t *minkey, uint32_t *acc, hipStream_t s);

}  // namespace gd
