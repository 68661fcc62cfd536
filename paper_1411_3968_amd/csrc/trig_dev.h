// Device-side data structures and helpers of the trigger pipeline (gfx950).
//
// Pipeline of one batch of slices (every kernel covers all slices of the batch):
//   k_ingest     per 1024-hit chunk: min/max time, max PMT, run starts
//   k_psum       (slices of more than 1024 chunks) partial sums per block of chunks
//   k_plan       per slice: validation, t_min, run count, segment width, path and
//                ordering-kernel kind
//   k_bounds     per chunk: run start and segment-boundary positions of every run
//                (one extra block builds the segment work lists of both
//                ordering kernels from the plans)
//   k_segsort_w  persistent, one wave per time segment of at most WAVE_CAP hits:
//                gather the segment's stretch of every run into LDS, order it by
//                (t, pmt, input index), write the ordered structure-of-arrays
//                (slices with more runs than a wave merges: first per group of
//                runs, then k_bounds and k_segsort_w again over the groups'
//                ordered outputs)
//   k_segsort    the same with one block per segment, for wider segments
//   k_seed       per ordered tile of TILE hits: L1 seeds, compacted per tile
//   k_fold       per group of tiles: causal folds of every seed over its window,
//                fires to a per-tile scratch slot, a summary of the tile's fires
//                and their event structure
//   k_tsum/k_tscan  per slice: scan of the tile summaries (each tile's place in
//                the fire and event lists), counts, the last event's end, the
//                plan to host-mapped staging
//   k_place      per tile with fires: fire records and event halves at their
//                places, also to host-mapped staging
// (the seed menu and level 0 use k_tile, k_l0_ok and k_l0_pass instead of or
// before k_seed)
// A slice with a tile whose time window reaches past its staged halo (a burst far
// denser than the slice's mean) reruns the trigger stage after k_dseed has
// written the seed bit of every ordered hit.
// A slice whose input is not a concatenation of a modest number of time-ordered
// runs (or whose time density overflows a segment) is re-ordered by a general
// LSD radix sort (k_g*) and then runs the trigger stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/trig.h"

namespace trigdev {

constexpr int CHUNK = 1024;       // hits per ingest / bounds item
constexpr int TILE = 1024;        // ordered hits per trigger tile
constexpr uint32_t TS_CH = 1024;  // tiles per chunk of the tile scan
constexpr int HALO_SMALL = 256;   // ordered hits staged on each side of a tile (first pass)
constexpr int HALO_BIG = 1024;    // the same in the dense-window rerun
constexpr int GTILE = 4096;       // elements per block of the general radix sort
constexpr int LDS_THR_MAX_PMT = 128;  // thr table kept in LDS up to this many PMTs
constexpr int WAVE_CAP = 512;     // hits per segment of the wave-per-segment ordering (largest variant)
constexpr int WAVE_CAP_SMALL = 256;   // its smaller variant (half the registers and LDS per wave)
constexpr int WAVE_RUNS = 256;    // most runs a wave-per-segment slice may have

enum State : uint32_t {
    ST_SKIP = 0,          // error or empty: nothing to do
    ST_FAST = 1,          // run-merge ordering
    ST_NEED_GENERIC = 2,  // needs the general radix ordering
    ST_GENERIC_DONE = 3,  // ordered by the general path
    ST_DENSE = 4,         // trigger stage rerun with a precomputed seed mask
};

// Slots in BatchDev::counters (written by k_bounds, read by the ordering kernels).
enum Counter : int {
    Q_SEG_TOTAL = 0,     // number of segment items of the wave-per-segment kernel
    Q_SEG_TOTAL_B = 1,   // number of segment items of the block-per-segment kernel
    Q_SEG_TOTAL2 = 2,    // number of segment items of the second level (two-level slices)
    N_COUNTERS = 16,
};

constexpr uint32_t NO_START = 0xFFFFFFFFu;

// Summary of a run of consecutive tiles of one slice: its fires (in
// ordered-hit order) and the event structure among them.  A fire "starts" an
// event when it comes more than 2H after the previous fire; the first fire of
// the run is not counted as a start here (that depends on what precedes it).
struct TileAgg {
    uint32_t F;          // fires
    uint32_t S;          // seeds
    uint32_t E_int;      // starts among the fires after the first
    uint32_t first_t, last_t;   // t - t_min of the first and the last fire
    uint32_t m_head;     // largest fold before the first start (all fires if none)
    uint32_t m_tail;     // largest fold from the last start on (all fires if none)
    uint32_t ls_idx;     // index within the run of the last start, NO_START if none
    uint32_t ls_t;       // its t - t_min
};

// Per tile: its own summary, and the summary of all tiles of the slice before it.
struct TileStat {
    TileAgg agg;
    TileAgg pre;
};

// One fire in a tile's scratch slot, before it is placed.
struct FireRec {
    uint32_t t;          // t - t_min
    uint32_t hit;        // input index
    uint32_t fold;
    uint32_t pmt;
};

// The plan's partial sums over a block of PL_CH chunks of one slice: time range,
// largest PMT id and chunk density, run starts, and (written by the plan) the runs
// started before the block.
constexpr uint32_t PL_CH = 1024;
struct PlanPart {
    int64_t t_min, t_max;
    uint32_t pmt_max;
    uint32_t runs;
    float dmax;
    uint32_t run_off;
};

struct ChunkPart {
    int64_t t_min, t_max;
    uint32_t pmt_max;
    uint32_t n_start;    // run starts in the chunk
    uint32_t run_base;   // runs started before the chunk
    uint32_t pad;
};

struct Plan {
    int64_t t_min, t_max;
    int32_t status;
    uint32_t state;
    uint32_t n_runs;
    uint32_t shift;          // segment width 2^shift ns
    uint32_t n_seg;
    uint32_t n_seeds;
    uint32_t n_fires;
    uint32_t n_events;
    uint32_t seg_item_base;
    uint32_t overflow;       // a segment exceeded the LDS capacity
    uint32_t seg_item_base_b;  // base in the block-kernel segment work list
    uint32_t seg_kind;       // 0: wave-per-segment ordering, 1: block-per-segment ordering
    uint32_t dense;          // a trigger tile's window outran its staged halo: rerun with a seed mask
    uint32_t generic;        // ordered by the general path
    uint32_t n_tagged;       // hits inside the event windows (slices that ask for the tagged list)
    // two-level ordering (slices with more runs than a wave merges): level 1 orders
    // groups of run_grp consecutive runs over segments of 2^shift ns (n_grp * n_seg
    // work items), level 2 merges the n_runs2 = n_grp time-ordered stretches that
    // level 1 leaves (one per group) over segments of 2^shift2 ns
    uint32_t tl;
    uint32_t n_grp, run_grp;
    uint32_t n_runs2, shift2, n_seg2, seg_item_base2;
    uint32_t seed_halo;      // hits staged on each side of a seed-kernel tile (before its cap)
};

struct SliceDev {
    const uint16_t *pmt;
    const int64_t *t;
    const uint16_t *q;
    uint64_t n;
    const int32_t *floor_id;
    const uint16_t *floor16; // dense floor index per PMT (equal iff floor_id equal)
    const uint32_t *thr32;
    const uint16_t *thr16;   // min(thr, 65535)
    uint32_t n_pmt, pbits;
    uint32_t chunk_base, n_chunks;
    uint32_t tile_base, n_tiles;   // k_trig tiles: max(1, chunks) (an empty slice has one)
    uint32_t group_base;     // first fold-kernel group of the slice (groups of BatchDev::tile_group tiles)
    uint32_t group_pad;
    uint32_t seg_target, seg_cap;
    uint64_t pos_cap;
    ChunkPart *part;
    PlanPart *ppart;         // per block of PL_CH chunks: the plan's partial sums
    uint32_t *pos;           // run-major: pos[r * (n_seg + 1) + j]
    uint32_t *o_t, *o_pq, *o_idx;   // ordered: t - t_min, pmt << 16 | q, input index
    TileStat *tstat;         // per trigger tile
    TileAgg *cagg;           // per chunk of TS_CH tiles: their combined summary (tile scan)
    FireRec *fsc;            // per trigger tile, TILE fire slots
    uint64_t *dmask;         // seed bits by ordered position (dense-window rerun only)
    trig_fire *fires;
    trig_event *events;
    uint8_t *seed_flags;     // optional, by input index
    Plan *plan;
    trig_fire *x_fires;      // host-mapped staging of the results (null: none)
    trig_event *x_events;
    uint32_t x_fire_cap, x_event_cap;
    uint32_t *tagc;          // per tile: tagged-hit count, then its exclusive prefix
    uint32_t *tagged;        // tagged hits' input indices (the fire-scratch area)
    uint32_t tag_on;         // the caller asked for the tagged list
    uint32_t x_tag_cap;      // capacity of its host-mapped staging
    uint32_t *x_tagged;      // host-mapped staging of the tagged list (null: none)
    uint64_t *l0m;           // level-0 pass bits by ordered position (level 0 on)
    const uint32_t *adj32;   // per PMT: adjacency group (SC)
    const uint32_t *afl32;   // per PMT: floor rank, 1 apart exactly for consecutive floors (AFC)
    const uint16_t *tbnd;    // table bounds per pair of 32-PMT blocks, nbk x nbk: lower | upper << 8 in
                             // 16 ns units (upper 255: none)
    const uint32_t *rmax;    // per PMT: the largest entry of its row of the table
    uint32_t nbk;            // blocks per side, 0: no bounds
    uint32_t thr_max;        // the largest entry of the table
};

constexpr int TBND_SHIFT = 5;   // 32 PMTs per block of the table bounds
constexpr uint32_t TBND_MIN_PMT = 256;   // bounds only for detectors with more PMTs
constexpr int TBND_LDS_MAX = 128;   // bounds staged in LDS up to 128 x 128 blocks (32 KB)

struct BatchDev {
    SliceDev *slices;
    const uint32_t *chunk_bases, *tile_bases;   // per slice: first chunk / first tile (dense copies)
    Plan *plans;
    uint32_t n_slices;
    uint32_t total_chunks;
    uint32_t total_tiles;
    uint32_t tail_state;     // the tail kernels process slices in this state
    uint32_t sort_kernels;   // ordering kernels launched: bit 0 wave-per-segment, bit 1 block-per-segment,
                             // bit 2 the second level of the two-level ordering
    uint32_t block_cap, block_target;   // block kernel capacity / target for slices it takes over
    uint32_t *counters;
    Plan *x_plans;           // host-mapped copy of the plans written at the end of the tail
    trig_params prm;
    // fold kernel: groups of tile_group consecutive tiles of one slice per
    // workgroup, window_cap window seeds staged in LDS at most; group_slice
    // maps every group to its slice (written by k_plan; unused for one slice)
    uint32_t tile_group, window_cap;
    uint32_t total_groups;
    uint32_t max_tiles;      // the most tiles of one slice (the tile scan's grid)
    uint32_t tbnd_lds;       // table-bound entries the fold kernel stages in LDS (0: none)
    uint32_t any_bounds;     // some slice has table bounds (the fold kernel's variant)
    uint32_t *group_slice;
    // the slice of every tile and of every chunk of the launch (written by k_plan
    // for the kernels after it; a one-slice launch reads none)
    uint32_t *tile_slice, *chunk_slice;
};

// ------------------------------------------------------------------ helpers

// Global-memory views of pointers read from descriptors.  Pointers loaded from
// memory are generic, and generic (flat) accesses count against the LDS wait
// counter too; through these views loads and stores compile to global
// instructions, so waiting on LDS does not wait on HBM.
#define TRIG_GAS __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ TRIG_GAS T *gmem(T *p) { return (TRIG_GAS T *)p; }
template <class T> __device__ __forceinline__ const TRIG_GAS T *gmem(const T *p) { return (const TRIG_GAS T *)p; }
// Device memory that no kernel of the launch writes (filled by an earlier
// kernel): uniform loads from it can go through the scalar cache.
#define TRIG_CAS __attribute__((address_space(4)))
template <class T> __device__ __forceinline__ const TRIG_CAS T *cmem(const T *p) { return (const TRIG_CAS T *)p; }
// Whole-struct copies through such pointers, a word at a time.
template <class T> __device__ __forceinline__ T gload(const TRIG_GAS T *p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
    T v;
    uint32_t *d = (uint32_t *)&v;
    const TRIG_GAS uint32_t *s = (const TRIG_GAS uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
    return v;
}
template <class T> __device__ __forceinline__ void gstore(TRIG_GAS T *p, const T &v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
    const uint32_t *s = (const uint32_t *)&v;
    TRIG_GAS uint32_t *d = (TRIG_GAS uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// ---- wave-wide scans on DPP lane moves (VALU, no LDS round trip).  A move
// reads a 32-bit word from another lane of the wave; lanes whose source is out
// of range, or whose 16-lane row is masked off, receive `id`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t id, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_words(const T &id, const T &v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized values only");
    T r;
    const uint32_t *pi = (const uint32_t *)&id;
    const uint32_t *pv = (const uint32_t *)&v;
    uint32_t *pr = (uint32_t *)&r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) pr[i] = dpp_u32<CTRL, ROW_MASK>(pi[i], pv[i]);
    return r;
}

// Inclusive scan over the 64 lanes under an associative `op(earlier, later)`
// with left identity `id`: shifts by 1, 2, 4 and 8 lanes within each row, then
// the last lane of row 0 (2) into row 1 (3), then lane 31 into rows 2 and 3.
template <class T, class Op>
__device__ __forceinline__ T wave_scan(T v, const T &id, Op op) {
    v = op(dpp_words<0x111, 0xF>(id, v), v);   // row_shr:1
    v = op(dpp_words<0x112, 0xF>(id, v), v);   // row_shr:2
    v = op(dpp_words<0x114, 0xF>(id, v), v);   // row_shr:4
    v = op(dpp_words<0x118, 0xF>(id, v), v);   // row_shr:8
    v = op(dpp_words<0x142, 0xA>(id, v), v);   // row_bcast:15 into rows 1, 3
    v = op(dpp_words<0x143, 0xC>(id, v), v);   // row_bcast:31 into rows 2, 3
    return v;
}

// Value of the lane below (lane 0 receives id).  Like every lane move here it
// must run with all lanes active: a lane masked off reads as id.
template <class T>
__device__ __forceinline__ T wave_shr1(const T &v, const T &id) { return dpp_words<0x138, 0xF>(id, v); }
// Value of the lane above (lane 63 receives id); all lanes active, as above.
template <class T>
__device__ __forceinline__ T wave_shl1(const T &v, const T &id) { return dpp_words<0x130, 0xF>(id, v); }

// Value of lane `src` (uniform) in every lane.
__device__ __forceinline__ uint32_t lane_read(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

// A word-sized struct of lane `src` (uniform) in every lane.
template <class T>
__device__ __forceinline__ T lane_read_all(const T &v, int src) {
    static_assert(sizeof(T) % 4 == 0, "word-sized values only");
    T r;
    const uint32_t *pv = (const uint32_t *)&v;
    uint32_t *pr = (uint32_t *)&r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) pr[i] = lane_read(pv[i], src);
    return r;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    return wave_scan(v, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
    return wave_scan(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

__device__ __forceinline__ uint32_t wave_total(uint32_t v) { return lane_read(wave_incl_scan(v), 63); }
__device__ __forceinline__ uint32_t wave_max_all(uint32_t v) { return lane_read(wave_incl_max_u32(v), 63); }

// Exclusive scan over the block; sh needs NT/64 + 1 words.  Ends with a barrier.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total, uint32_t *sh) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < NT / 64; ++i) {
            uint32_t x = sh[i];
            sh[i] = acc;
            acc += x;
        }
        sh[NT / 64] = acc;
    }
    __syncthreads();
    uint32_t r = sh[w] + inc - v;
    total = sh[NT / 64];
    __syncthreads();
    return r;
}

// In-place exclusive scan of a[0..len) by one block (4 consecutive items per
// thread per round); returns the total.
template <int NT>
__device__ __forceinline__ uint32_t block_scan_array(uint32_t *a, uint32_t len, uint32_t *sh) {
    constexpr uint32_t PT = 4;
    uint32_t acc = 0;
    for (uint32_t i0 = 0; i0 < len; i0 += NT * PT) {
        const uint32_t b = i0 + threadIdx.x * PT;
        uint32_t v[PT], sum = 0;
#pragma unroll
        for (uint32_t p = 0; p < PT; ++p) {
            v[p] = (b + p < len) ? a[b + p] : 0u;
            sum += v[p];
        }
        uint32_t tot;
        uint32_t run = acc + block_excl_scan<NT>(sum, tot, sh);
#pragma unroll
        for (uint32_t p = 0; p < PT; ++p) {
            if (b + p < len) a[b + p] = run;
            run += v[p];
        }
        acc += tot;
    }
    return acc;
}

// Cooperative copy src[0..n) -> dst[0..n) by one block with U loads in flight
// per thread before any store (a plain strided loop waits for every load).
template <int NT, int U, class T, class Tr>
__device__ __forceinline__ void stage_copy(T *dst, const TRIG_GAS T *src, uint32_t n, Tr tr) {
    for (uint32_t b0 = 0; b0 < n; b0 += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = b0 + u * NT + threadIdx.x;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = b0 + u * NT + threadIdx.x;
            if (i < n) dst[i] = tr(v[u]);
        }
    }
}

template <int NT, int U, class T>
__device__ __forceinline__ void stage_copy(T *dst, const TRIG_GAS T *src, uint32_t n) {
    stage_copy<NT, U>(dst, src, n, [](T x) { return x; });
}

template <int NT>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *sh) {
    uint32_t tot;
    block_excl_scan<NT>(v, tot, sh);
    return tot;
}

// Slice owning work item `item` given per-slice non-decreasing bases: the last
// slice whose base is <= item.
template <class BaseOf>
__device__ __forceinline__ uint32_t find_slice(uint32_t n_slices, uint32_t item, BaseOf base_of) {
    if (n_slices <= 1) return 0;      // no load on the single-slice path
    uint32_t lo = 0, hi = n_slices;   // first index with base > item, in [lo, hi]
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (base_of(mid) <= item) lo = mid + 1; else hi = mid;
    }
    return lo ? lo - 1 : 0;
}

// The same for work items met in increasing order, from slice `from` (at or
// before the item's): a few steps forward, then a binary search over the rest.
template <class BaseOf>
__device__ __forceinline__ uint32_t find_slice_from(uint32_t n_slices, uint32_t from, uint32_t item, BaseOf base_of) {
    if (n_slices <= 1) return 0;
    uint32_t s = from;
    for (int k = 0; k < 4; ++k) {
        if (s + 1 >= n_slices || base_of(s + 1) > item) return s;
        ++s;
    }
    uint32_t lo = s + 1, hi = n_slices;   // first index with base > item, in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base_of(mid) <= item) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

// First tile / chunk of slice si in the launch's numbering: a one-slice launch
// (one slice of a larger batch rerun on its own) numbers from 0.
__device__ __forceinline__ uint32_t tile_base_of(const BatchDev &b, uint32_t si) {
    return b.n_slices <= 1 ? 0u : b.tile_bases[si];
}
__device__ __forceinline__ uint32_t chunk_base_of(const BatchDev &b, uint32_t si) {
    return b.n_slices <= 1 ? 0u : b.chunk_bases[si];
}
// Boundary table of the ordering stage: entry (j, r) = the first position of run
// r at or after segment boundary j.  Rows j come in tiles of TJ consecutive
// boundaries, run-major inside a tile.  With TJ = BND_TJ one run's entries for 16
// consecutive boundaries are one 64-byte stretch, written whole by the chunk that
// crosses them (neighbouring segments read the same lines): the single-level and
// level-1 tables.  The level-2 table of the two-level ordering (a few dozen long
// runs, written by level 1, each level-1 segment a run of consecutive rows of
// its group) takes 8 rows a tile: on the 2688-PMT block the two levels took
// 329 + 265 us with 1 row (each entry a partial line of its own), 280 + 271 us
// with 8 and 278 + 286 us with 32 (a level-2 segment's entries over more lines).
constexpr uint32_t BND_TJ = 16;
constexpr uint32_t BND_TJ2 = 8;
template <uint32_t TJ>
__host__ __device__ __forceinline__ uint64_t bnd_at(uint32_t j, uint32_t r, uint64_t R) {
    return (uint64_t)(j / TJ) * R * TJ + (uint64_t)r * TJ + (j % TJ);
}
// Entries of a table of `rows` boundaries over R runs.
template <uint32_t TJ>
__host__ __device__ __forceinline__ uint64_t bnd_entries(uint64_t rows, uint64_t R) {
    return ((rows + TJ - 1) / TJ) * TJ * R;
}

// The slice of tile / chunk `item` of a launch that k_plan has mapped.
__device__ __forceinline__ uint32_t slice_of_tile(const BatchDev &b, uint32_t item) {
    return b.n_slices <= 1 ? 0u : gmem(b.tile_slice)[item];
}
__device__ __forceinline__ uint32_t slice_of_chunk(const BatchDev &b, uint32_t item) {
    return b.n_slices <= 1 ? 0u : gmem(b.chunk_slice)[item];
}

// Groups of the fold kernel of a slice with n_tiles tiles.
__host__ __device__ __forceinline__ uint32_t groups_of(uint32_t n_tiles, uint32_t tile_group) {
    return (n_tiles + tile_group - 1) / tile_group;
}

// Packed copy of the input hits for the ordering stage, one word per input hit:
// low 32 bits the low 32 bits of t (t - t_min is then their difference modulo
// 2^32, exact since the span is below 2^31), high 32 bits pmt << 16 | charge.  It
// lives in the fire-record area, which is unused until the trigger stage (16
// bytes per hit there, 8 needed).
__device__ __forceinline__ TRIG_GAS uint64_t *packed_hits(const SliceDev &S) {
    return (TRIG_GAS uint64_t *)gmem(S.fsc);
}

// Two-level ordering: level 1 writes each group's ordered hits as packed words
// (same format as packed_hits) into the second half of the fire-record area, and
// their input indices into the fire area (both unused until the trigger stage).
__device__ __forceinline__ TRIG_GAS uint64_t *level1_hits(const SliceDev &S) {
    return (TRIG_GAS uint64_t *)gmem(S.fsc) + (uint64_t)S.n_tiles * TILE;
}
__device__ __forceinline__ TRIG_GAS uint32_t *level1_index(const SliceDev &S) {
    return (TRIG_GAS uint32_t *)gmem(S.fires);
}
// Two-level slices: the level-2 boundary table (rows 0 .. n_seg2 over the n_grp
// groups, whose ordered level-1 outputs are the runs of level 2; written by
// level 1 as it orders them) at the end of the table area, after the level-1
// table that level 1 still reads.
__host__ __device__ __forceinline__ uint64_t level2_entries(const Plan &P) {
    return bnd_entries<BND_TJ2>((uint64_t)P.n_seg2 + 1, P.n_grp);
}
__device__ __forceinline__ TRIG_GAS uint32_t *level2_table(const SliceDev &S, const Plan &P) {
    return gmem(S.pos) + (S.pos_cap - level2_entries(P));
}

// Plain rule: every tile's seeds, compacted in time order by the seed kernel and
// read by the fold kernel: time (t - t_min) and pmt << 16 | position in the tile,
// TILE slots per tile each, then a record per tile (seed count, first and last
// seed time).  They live in the boundary-table area, unused once the ordering is
// done (3n + 65536 words hold 2 TILE n_tiles + 4 n_tiles).
struct SeedRec {
    uint32_t n;          // seeds of the tile
    uint32_t first_t;    // t - t_min of its first and last seed (n > 0)
    uint32_t last_t;
    uint32_t pad;
};
__device__ __forceinline__ TRIG_GAS uint32_t *seed_t(const SliceDev &S) { return gmem(S.pos); }
__device__ __forceinline__ TRIG_GAS uint32_t *seed_p(const SliceDev &S) {
    return gmem(S.pos) + (uint64_t)S.n_tiles * TILE;
}
__device__ __forceinline__ TRIG_GAS SeedRec *seed_rec(const SliceDev &S) {
    return (TRIG_GAS SeedRec *)(gmem(S.pos) + 2ull * S.n_tiles * TILE);
}

__device__ __forceinline__ bool slice_in_tail(const BatchDev &b, uint32_t state) {
    return state == b.tail_state;
}

}  // namespace trigdev

// ------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.  All work goes on `stream`.
struct TrigLaunchCfg {
    int n_cu;
    int persist_per_cu;
};

hipError_t trig_launch_tag(const trigdev::BatchDev &b, hipStream_t s, void (*mark)(void *, const char *, int),
                           void *mark_ctx);
hipError_t trig_launch_l0(const trigdev::BatchDev &b, hipStream_t s, void (*mark)(void *, const char *, int),
                          void *mark_ctx);
hipError_t trig_launch_front(const trigdev::BatchDev &b, uint32_t seg_cap, uint32_t wave_cap, int wave_wgs_per_cu,
                             const TrigLaunchCfg &cfg, hipStream_t s, void (*mark)(void *, const char *, int),
                             void *mark_ctx);
// max_pmt: the largest PMT count of the batch's geometries (sizes the LDS table).
hipError_t trig_launch_tail(const trigdev::BatchDev &b, const TrigLaunchCfg &cfg, uint32_t max_pmt, hipStream_t s,
                            void (*mark)(void *, const char *, int), void *mark_ctx);
// Dense-window rerun of the slices whose plan has `dense` set: seed mask, then
// the trigger stage reading it (b.tail_state must be ST_DENSE).
hipError_t trig_launch_dense(const trigdev::BatchDev &b, const TrigLaunchCfg &cfg, uint32_t max_pmt, hipStream_t s,
                             void (*mark)(void *, const char *, int), void *mark_ctx);
// General path for one slice: device-wide stable LSD radix sort over key_bits
// bits; scratch holds trig_generic_scratch_bytes(n) bytes.
hipError_t trig_launch_generic_slice(const trigdev::SliceDev &S, const trigdev::Plan &P, uint32_t key_bits,
                                     void *scratch, hipStream_t s,
                                     void (*mark)(void *, const char *, int), void *mark_ctx);
size_t trig_generic_scratch_bytes(uint64_t n);
