// Device-side data structures and helpers of the trigger pipeline (gfx950).
//
// Pipeline of one batch of slices (every kernel covers all slices of the batch):
//   k_reset      clear work-queue counters
//   k_ingest     per 4096-hit chunk: min/max time, max PMT, run starts
//   k_plan       per slice: validation, t_min, run count, segment width, path
//   k_seg_prefix one block: work-list bases of the ordering stage
//   k_bounds     per chunk: run start and segment-boundary positions of every run
//   k_segsort    persistent: gather one time segment from all runs into LDS,
//                radix-sort it by (t, pmt) with input-position tie-break, write the
//                ordered structure-of-arrays
//   k_seed       per 4096-hit ordered tile: L1 seed bits (charge or floor coincidence)
//   k_seed_scan  per slice: tile offsets of the seed list
//   k_seed_emit  per tile: compact seed list (t, pmt|q, input index)
//   k_count_prefix one block: work-list bases of the counting stage
//   k_count      persistent: causal fold of every seed, fire counts per seed tile
//   k_fire_scan  per slice: fire offsets
//   k_fire_emit  per seed tile: ordered fire records
//   k_events     per slice: merged event windows
// A slice whose input is not a concatenation of a modest number of time-ordered
// runs (or whose time density overflows a segment) is re-ordered by a general
// LSD radix sort (k_g*) and then runs the same tail (k_seed ... k_events).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/trig.h"

namespace trigdev {

constexpr int CHUNK = 1024;       // hits per ingest / bounds item
constexpr int TILE = 1024;        // ordered hits per seed tile
constexpr int SHALO = 64;         // ordered neighbours staged on each side of a seed tile
constexpr int CT1 = 256;          // seeds per counting tile (table in LDS)
constexpr int CT8 = 2048;         // seeds per counting tile (row-grouped table in L2)
constexpr int CHALO = 256;        // seeds staged on each side of a counting tile
constexpr int GTILE = 4096;       // elements per block of the general radix sort
constexpr int LDS_THR_MAX_PMT = 128;  // thr table kept in LDS up to this many PMTs
constexpr int SEED_LDS_FLOORS = 8192; // dense floor ids kept in LDS up to this many PMTs
constexpr int ROWGROUPS = 8;      // counting rows split over the 8 XCDs for large tables
constexpr int WAVE_CAP = 512;     // hits per segment of the wave-per-segment ordering
constexpr int WAVE_RUNS = 256;    // most runs a wave-per-segment slice may have

enum State : uint32_t {
    ST_SKIP = 0,          // error or empty: nothing to do
    ST_FAST = 1,          // run-merge ordering
    ST_NEED_GENERIC = 2,  // needs the general radix ordering
    ST_GENERIC_DONE = 3,  // ordered by the general path
};

// Work-queue / counter slots in BatchDev::counters.
enum Counter : int {
    Q_SEG = 0,           // dequeue counter of k_segsort
    Q_SEG_TOTAL = 1,     // number of segment items
    Q_COUNT_TOTAL = 2,   // number of counting items
    C_PLAN_DONE = 3,     // slices planned so far (the last block builds the segment work list)
    C_SCAN_DONE = 4,     // slices whose seed list is scanned (the last block builds the count work list)
    Q_SEG_TOTAL_B = 5,   // number of segment items of the block-per-segment kernel
    N_COUNTERS = 16,
};

__host__ __device__ constexpr uint32_t count_tile(uint32_t groups) { return groups > 1 ? CT8 : CT1; }

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
    uint32_t n_ctiles;
    uint32_t count_item_base;
    uint32_t groups;         // counting row groups (1 or ROWGROUPS)
    uint32_t overflow;       // a segment exceeded the LDS capacity
    uint32_t seg_item_base_b;  // base in the block-kernel segment work list
    uint32_t seg_kind;       // 0: wave-per-segment ordering, 1: block-per-segment ordering
    uint32_t pad;
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
    uint32_t tile_base, n_tiles;
    uint32_t seg_target, seg_cap;
    uint64_t pos_cap;
    ChunkPart *part;
    uint32_t *pos;           // run-major: pos[r * (n_seg + 1) + j]
    uint32_t *o_t, *o_pq, *o_idx;   // ordered: t - t_min, pmt << 16 | q, input index
    uint64_t *seed_mask;     // one bit per ordered hit
    uint32_t *tile_seeds;    // per tile: count, then offset
    uint32_t *s_t, *s_pq, *s_idx, *s_fold;   // seed list
    uint32_t *ctile_fires;   // per seed tile: count, then offset
    uint32_t *fire_ev, *ev_first, *ev_max;
    trig_fire *fires;
    trig_event *events;
    uint8_t *seed_flags;     // optional, by input index
    Plan *plan;
    trig_fire *x_fires;      // host-mapped staging of the results (null: none)
    trig_event *x_events;
    uint32_t x_fire_cap, x_event_cap;
};

struct BatchDev {
    SliceDev *slices;
    Plan *plans;
    uint32_t n_slices;
    uint32_t total_chunks;
    uint32_t total_tiles;
    uint32_t tail_state;     // the tail kernels process slices in this state
    uint32_t sort_kernels;   // ordering kernels launched: bit 0 wave-per-segment, bit 1 block-per-segment
    uint32_t block_cap, block_target;   // block kernel capacity / target for slices it takes over
    uint32_t *counters;
    Plan *x_plans;           // host-mapped copy of the plans written at the end of the tail
    trig_params prm;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

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
__device__ __forceinline__ void stage_copy(T *dst, const T *src, uint32_t n, Tr tr) {
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
__device__ __forceinline__ void stage_copy(T *dst, const T *src, uint32_t n) {
    stage_copy<NT, U>(dst, src, n, [](T x) { return x; });
}

// Device-scope load that bypasses a possibly stale L1 line (data written by
// other workgroups of the same kernel before a release fence).
__device__ __forceinline__ uint32_t load_acquire(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    uint32_t lo = 0, hi = n_slices;   // first index with base > item, in [lo, hi]
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (base_of(mid) <= item) lo = mid + 1; else hi = mid;
    }
    return lo ? lo - 1 : 0;
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

hipError_t trig_launch_front(const trigdev::BatchDev &b, uint32_t seg_cap, int wave_wgs_per_cu,
                             const TrigLaunchCfg &cfg, hipStream_t s, void (*mark)(void *, const char *, int),
                             void *mark_ctx);
hipError_t trig_launch_tail(const trigdev::BatchDev &b, const TrigLaunchCfg &cfg, hipStream_t s,
                            void (*mark)(void *, const char *, int), void *mark_ctx);
// General path for one slice: device-wide stable LSD radix sort over key_bits
// bits; scratch holds trig_generic_scratch_bytes(n) bytes.
hipError_t trig_launch_generic_slice(const trigdev::SliceDev &S, const trigdev::Plan &P, uint32_t key_bits,
                                     void *scratch, hipStream_t s,
                                     void (*mark)(void *, const char *, int), void *mark_ctx);
size_t trig_generic_scratch_bytes(uint64_t n);
