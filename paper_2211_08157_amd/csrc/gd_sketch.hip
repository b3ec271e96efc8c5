// Sparsification and minimizer sketching on gfx950.
//
// Layout: a batch of sequences is first sparsified into one "patterned stream" (2-bit
// packed, 16 bases per uint32 word, sequences back to back, boundaries pofs[]).  The
// sketch kernel then tiles the patterned positions of the whole batch: a workgroup of
// 256 threads owns T consecutive positions (k-mer starts) plus a halo of H positions on
// each side, so that every window touching an owned position lies in its LDS.  A
// position whose k-mer would cross the end of its sequence gets an "empty" hash, and a
// window is valid only when its w k-mers lie in one sequence, so tiles may span any
// number of sequences (reads) or cover part of one (a chromosome).
//
// Minimizer selection uses the identity: position i is a minimizer iff its hash equals
// max over the valid windows containing i of the window minimum (every window minimum
// is <= h_i, and equality holds exactly for the windows where i attains the minimum).
// Both sliding reductions run by doubling in LDS.  The output is compacted in position
// order with a single-pass decoupled look-back across tiles.
#include "gd_internal.h"

namespace gd {

TileGeom tile_geom(int w)
{
    TileGeom g;
    g.H = ((w - 1 + 15) / 16) * 16;
    if (g.H == 0) g.H = 16;
    g.T = kBlock * 16 - 2 * g.H;
    return g;
}

size_t sketch_tiles_bound(uint64_t np_bound, int w)
{
    const TileGeom g = tile_geom(w);
    return (size_t)(np_bound / (uint64_t)g.T) + 2;
}

namespace {

__device__ __forceinline__ uint32_t seq_shift(const uint32_t *shift, uint32_t uniform, uint32_t s)
{
    return shift ? shift[s] : uniform;
}

// ---------------------------------------------------------------- kept counts

__global__ __launch_bounds__(kBlock) void k_kept(const uint64_t *offsets, uint32_t n_seq,
                                                 Pattern P, const uint32_t *shift,
                                                 uint32_t uniform, uint64_t *kept,
                                                 uint32_t *status)
{
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_seq) return;
    uint32_t a = seq_shift(shift, uniform, s);
    if (a >= P.p) { set_status(status, 4u); a = 0; }
    kept[s] = kept_count(P, offsets[s + 1] - offsets[s], a);
}

// ---------------------------------------------------------------- sparsify

__device__ __forceinline__ uint32_t base_at(const uint8_t *bases, uint64_t g)
{
    return (bases[g >> 2] >> ((g & 3) * 2)) & 3u;
}

// One thread per output word: gathers the 16 kept bases [16q, 16q+16) of the batch.
__global__ __launch_bounds__(kBlock) void k_sparsify(const uint8_t *bases, const uint64_t *offsets,
                                                     uint32_t n_seq, Pattern P,
                                                     const uint32_t *shift, uint32_t uniform,
                                                     const uint64_t *pofs, uint32_t *psw,
                                                     size_t words)
{
    const size_t q = blockIdx.x * (size_t)kBlock + threadIdx.x;
    if (q >= words) return;
    const uint64_t np = pofs[n_seq];
    const uint64_t j0 = (uint64_t)q * 16;
    uint32_t word = 0;
    if (j0 < np) {
        uint32_t s = last_le(pofs, n_seq, j0);
        uint64_t end = pofs[s + 1];
        while (j0 >= end) { s++; end = pofs[s + 1]; }
        uint32_t a = seq_shift(shift, uniform, s);
        if (a >= P.p) a = 0;
        uint64_t li = j0 - pofs[s];
        uint64_t per = li / P.x;                 // period index
        uint32_t r = (uint32_t)(li - per * P.x); // rank within the period
        uint64_t obase = offsets[s];
        for (int u = 0; u < 16; u++) {
            const uint64_t j = j0 + u;
            if (j >= np) break;
            if (j >= end) {
                while (j >= end) { s++; end = pofs[s + 1]; }
                a = seq_shift(shift, uniform, s);
                if (a >= P.p) a = 0;
                per = 0;
                r = 0;
                obase = offsets[s];
            }
            const uint64_t o = obase + per * P.p + kept_phase(P, a, r);
            word |= base_at(bases, o) << (2 * u);
            if (++r == P.x) { r = 0; per++; }
        }
    }
    psw[q] = word;
}

// ---------------------------------------------------------------- sketch

constexpr int kE = kBlock * 16;     // LDS positions per tile (T + 2H)
constexpr uint64_t kFlagA = 1ull << 62, kFlagP = 2ull << 62, kValMask = (1ull << 62) - 1;

struct SketchArgs {
    const uint32_t *psw;
    const uint64_t *pofs;
    const uint64_t *offsets;
    const uint32_t *shift;
    uint32_t uniform;
    uint32_t n_seq;
    Pattern P;
    int k, w, H, T;
    uint64_t kmask;
    uint64_t *keys;
    void *vals;
    int val_mode;
    uint64_t *mz_offsets;
    uint64_t capacity;
    uint64_t *n_out;
    uint64_t *tile_state;
    uint32_t *tile_counter;
    uint32_t *status;
};

// Reverse the order of the 2-bit groups of a 64-bit word.
__device__ __forceinline__ uint64_t rev_groups(uint64_t x)
{
    x = __builtin_bitreverse64(x);
    return ((x >> 1) & 0x5555555555555555ull) | ((x & 0x5555555555555555ull) << 1);
}

__global__ __launch_bounds__(kBlock) void k_sketch(SketchArgs A)
{
    __shared__ uint64_t sh_m[kE];     // work array of the sliding reductions
    __shared__ uint64_t sh_scan[kBlock / kWave];
    __shared__ uint32_t sh_tile;
    __shared__ uint64_t sh_base;

    const int t = threadIdx.x;
    const int H = A.H, T = A.T, w = A.w, k = A.k;
    const uint64_t np = A.pofs[A.n_seq];
    const uint64_t n_tiles = np / (uint64_t)T + 1;     // the last tile covers position np

    if (t == 0) sh_tile = atomicAdd(A.tile_counter, 1u);
    __syncthreads();
    const uint64_t tile = sh_tile;
    if (tile >= n_tiles) return;

    const int64_t j0 = (int64_t)(tile * (uint64_t)T);
    const int64_t jc = j0 - H + 16 * t;                  // first position of this chunk

    // ---- stage 1: canonical k-mer hashes and flags of the 16 positions of the chunk.
    // hv = hash (kMax64 where there is no k-mer or it is a palindrome);
    // fv bit0 = may be selected, bit1 = a valid window starts here, bit2 = strand.
    uint64_t hv[16];
    uint32_t fv[16];
#pragma unroll
    for (int u = 0; u < 16; u++) { hv[u] = kMax64; fv[u] = 0; }
    uint32_t seq0 = 0;
    uint64_t beg0 = 0, end0 = 0;
    if (jc >= 0 && (uint64_t)jc < np) {
        uint32_t seq = last_le(A.pofs, A.n_seq, (uint64_t)jc);
        uint64_t seq_beg = A.pofs[seq], seq_end = A.pofs[seq + 1];
        while ((uint64_t)jc >= seq_end) { seq++; seq_beg = seq_end; seq_end = A.pofs[seq + 1]; }
        seq0 = seq; beg0 = seq_beg; end0 = seq_end;
        const size_t wi = (size_t)jc / 16;
        const uint64_t lo64 = (uint64_t)A.psw[wi] | ((uint64_t)A.psw[wi + 1] << 32);
        const uint64_t w2 = A.psw[wi + 2];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const uint64_t j = (uint64_t)jc + u;
            if (j < np) {
                while (j >= seq_end) { seq++; seq_beg = seq_end; seq_end = A.pofs[seq + 1]; }
                const bool kvalid = j + (uint64_t)k <= seq_end;
                const bool wvalid = j + (uint64_t)(k + w - 1) <= seq_end;
                const bool seq_ok = seq_end - seq_beg >= (uint64_t)(k + w - 1);
                if (kvalid) {
                    // bits [2u, 2u + 64) of the stream: base u of the chunk in the low bits
                    const uint64_t X = u == 0 ? lo64 : ((lo64 >> (2 * u)) | (w2 << (64 - 2 * u)));
                    const uint64_t rc = (~X) & A.kmask;
                    const uint64_t fwd = rev_groups(X) >> (64 - 2 * k);
                    if (fwd == rc) {
                        fv[u] = wvalid ? 2u : 0u;
                    } else {
                        const bool strand = rc < fwd;
                        hv[u] = mix64(strand ? rc : fwd);
                        fv[u] = (seq_ok ? 1u : 0u) | (wvalid ? 2u : 0u) | (strand ? 4u : 0u);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 16; u++) sh_m[16 * t + u] = hv[u];
    __syncthreads();

    // ---- stage 2: window minima (forward doubling), then the opening (backward doubling)
    int q2 = 1;                       // largest power of two <= w
    while (q2 * 2 <= w) q2 *= 2;
    const int r2 = w - q2;
    for (int d = 1; d < q2; d *= 2) {
        uint64_t v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int x = 16 * t + u;
            const uint64_t o = x + d < kE ? sh_m[x + d] : kMax64;
            v[u] = min(sh_m[x], o);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) sh_m[16 * t + u] = v[u];
        __syncthreads();
    }
    {
        uint64_t v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int x = 16 * t + u;
            const uint64_t o = x + r2 < kE ? sh_m[x + r2] : kMax64;
            v[u] = (fv[u] & 2u) ? min(sh_m[x], o) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) sh_m[16 * t + u] = v[u];
        __syncthreads();
    }
    for (int d = 1; d < q2; d *= 2) {
        uint64_t v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int x = 16 * t + u;
            const uint64_t o = x - d >= 0 ? sh_m[x - d] : 0;
            v[u] = max(sh_m[x], o);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; u++) sh_m[16 * t + u] = v[u];
        __syncthreads();
    }
    const bool owner = 16 * t >= H && 16 * t < H + T;
    uint32_t sel = 0;
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int x = 16 * t + u;
        const uint64_t o = x - r2 >= 0 ? sh_m[x - r2] : 0;
        const uint64_t opened = max(sh_m[x], o);
        if (owner && (fv[u] & 1u) && hv[u] == opened) sel |= 1u << u;
    }

    // ---- stage 3: position-ordered compaction across tiles (decoupled look-back)
    uint64_t total;
    const uint64_t excl = block_excl_scan<uint64_t>((uint64_t)__popc(sel), sh_scan, &total);
    // Wave 0 publishes this tile's aggregate, then looks back over 64 predecessors per
    // step: it adds every aggregate up to the nearest tile that already carries its
    // inclusive prefix, and waits only while one of the tiles in between has not
    // published yet.  The flag and the value share one 64-bit word, so relaxed atomics
    // suffice (no other data of a predecessor is read).
    if (t < kWave) {
        uint64_t before = 0;
        if (t == 0)
            __hip_atomic_store(&A.tile_state[tile], (tile == 0 ? kFlagP : kFlagA) | total,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t end = (int64_t)tile - 1;          // newest predecessor not yet added
        while (end >= 0) {
            const int64_t idx = end - t;
            const uint64_t st = idx >= 0 ? __hip_atomic_load(&A.tile_state[idx], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                                         : kFlagP;
            const uint64_t f = st & ~kValMask;
            const uint64_t pmask = __ballot(f == kFlagP);
            const uint64_t zmask = __ballot(f == 0);
            const int first_p = pmask ? __ffsll((unsigned long long)pmask) - 1 : kWave;
            const int first_z = zmask ? __ffsll((unsigned long long)zmask) - 1 : kWave;
            if (first_z < first_p) {              // a nearer predecessor is not ready yet
                __builtin_amdgcn_s_sleep(2);
                continue;
            }
            uint64_t v = t <= first_p ? (st & kValMask) : 0;
            v = wave_sum<uint64_t>(v);
            before += v;
            if (first_p < kWave) break;
            end -= kWave;
        }
        if (t == 0) {
            if (tile != 0)
                __hip_atomic_store(&A.tile_state[tile], kFlagP | (before + total),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh_base = before;
            if (tile == n_tiles - 1) {
                if (A.n_out) *A.n_out = before + total;
                if (before + total > A.capacity) set_status(A.status, 1u);
            }
        }
    }
    __syncthreads();
    const uint64_t base = sh_base + excl;

    if (!owner || (uint64_t)jc > np) return;

    // per-sequence record offsets of the sequences that start inside this chunk
    if (A.mz_offsets) {
        uint32_t s = first_ge(A.pofs, A.n_seq, (uint64_t)jc);
        while (s <= A.n_seq && A.pofs[s] < (uint64_t)jc + 16) {
            const uint32_t below = (uint32_t)(A.pofs[s] - (uint64_t)jc);
            A.mz_offsets[s] = base + __popc(sel & ((1u << below) - 1u));
            s++;
        }
    }
    if (sel == 0) return;

    // records, in position order: walk the chunk's positions keeping the original
    // coordinate as (period, rank within period)
    uint32_t seq = seq0;
    uint64_t seq_beg = beg0, seq_end = end0;
    uint32_t a = seq_shift(A.shift, A.uniform, seq);
    if (a >= A.P.p) a = 0;
    const uint64_t li0 = (uint64_t)jc - seq_beg;
    uint64_t per = li0 / A.P.x;
    uint32_t rk = (uint32_t)(li0 - per * A.P.x);
    uint64_t idx = base;
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const uint64_t j = (uint64_t)jc + u;
        if (j < np) {
            if (j >= seq_end) {
                while (j >= seq_end) { seq++; seq_beg = seq_end; seq_end = A.pofs[seq + 1]; }
                a = seq_shift(A.shift, A.uniform, seq);
                if (a >= A.P.p) a = 0;
                per = 0;
                rk = 0;
            }
            if ((sel >> u) & 1u) {
                const uint64_t local = per * A.P.p + kept_phase(A.P, a, rk);
                const uint32_t strand = (fv[u] >> 2) & 1u;
                if (idx < A.capacity) {
                    A.keys[idx] = hv[u];
                    if (A.val_mode == VAL_SEQ64) {
                        if (local >= (1ull << 31)) set_status(A.status, 2u);
                        ((uint64_t *)A.vals)[idx] = ((uint64_t)seq << 32) | (local << 1) | strand;
                    } else {
                        const uint64_t pos =
                            A.val_mode == VAL_GLOBAL32 ? A.offsets[seq] + local : local;
                        if (pos >= (1ull << 31)) set_status(A.status, 2u);
                        ((uint32_t *)A.vals)[idx] = (uint32_t)((pos << 1) | strand);
                    }
                }
                idx++;
            }
            if (++rk == A.P.x) { rk = 0; per++; }
        }
    }
}

}  // namespace

hipError_t launch_kept(const Batch &b, const Pattern &P, const uint32_t *shift,
                       uint32_t uniform_shift, uint64_t *kept, uint32_t *status, hipStream_t s)
{
    if (b.n_seq == 0) return hipSuccess;
    const unsigned blocks = (b.n_seq + kBlock - 1) / kBlock;
    GD_LAUNCH(k_kept, dim3(blocks), dim3(kBlock), 0, s, b.offsets, b.n_seq, P, shift,
                       uniform_shift, kept, status);
    return hipGetLastError();
}

hipError_t launch_sparsify(const Batch &b, const Pattern &P, const uint32_t *shift,
                           uint32_t uniform_shift, const uint64_t *pofs, uint32_t *psw,
                           size_t words, hipStream_t s)
{
    const size_t blocks = (words + kBlock - 1) / kBlock;
    GD_LAUNCH(k_sparsify, dim3((unsigned)blocks), dim3(kBlock), 0, s, b.bases, b.offsets,
                       b.n_seq, P, shift, uniform_shift, pofs, psw, words);
    return hipGetLastError();
}

hipError_t launch_sketch(const Batch &b, const Pattern &P, const uint32_t *shift,
                         uint32_t uniform_shift, const uint64_t *pofs, const uint32_t *psw,
                         uint64_t np_bound, int k, int w, const SketchOut &o,
                         uint64_t *tile_state, uint32_t *tile_counter, uint32_t *status,
                         hipStream_t s)
{
    const TileGeom g = tile_geom(w);
    const size_t tiles = sketch_tiles_bound(np_bound, w);
    hipError_t e = fill_u64(tile_state, 0, tiles, s);
    if (e != hipSuccess) return e;
    e = fill_u32(tile_counter, 0, 1, s);
    if (e != hipSuccess) return e;
    SketchArgs A;
    A.psw = psw;
    A.pofs = pofs;
    A.offsets = b.offsets;
    A.shift = shift;
    A.uniform = uniform_shift;
    A.n_seq = b.n_seq;
    A.P = P;
    A.k = k;
    A.w = w;
    A.H = g.H;
    A.T = g.T;
    A.kmask = k == 32 ? kMax64 : ((1ull << (2 * k)) - 1);
    A.keys = o.keys;
    A.vals = o.vals;
    A.val_mode = o.val_mode;
    A.mz_offsets = o.mz_offsets;
    A.capacity = o.capacity;
    A.n_out = o.n_out;
    A.tile_state = tile_state;
    A.tile_counter = tile_counter;
    A.status = status;
    GD_LAUNCH(k_sketch, dim3((unsigned)tiles), dim3(kBlock), 0, s, A);
    return hipGetLastError();
}

}  // namespace gd
