// Tail of the pipeline on the time-ordered hits of each slice:
//   L1 seeds (paper Sec. 3 and Sec. 4.2: charge over threshold, floor coincidence),
//   causal N-fold count (Sec. 3: Cherenkov hits of one muon are correlated in
//   space and time within less than 3 us), fires, and the merged event windows
//   (Sec. 2: 6 us window centred on the trigger seed; Sec. 4.2: +-3 us tagging).
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NT = 256;

__device__ __forceinline__ uint32_t wave_sumu(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Seed bits of one tile of 4096 ordered hits.  Element e*256 + tid of the tile is
// handled by thread tid in iteration e, so every wave's ballot covers one aligned
// 64-hit word of the seed mask.  A floor partner is searched among the ordered
// neighbours within t_floor_ns on both sides.
__global__ __launch_bounds__(NT) void k_seed(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].tile_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t tile = item - S.tile_base;
    if (tile >= S.n_tiles) return;
    const uint32_t state = S.plan->state;
    if (!slice_in_tail(b, state)) return;
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t n = S.n;
    const uint32_t Q = b.prm.q_seed;
    const int32_t tau = b.prm.t_floor_ns;
    uint32_t cnt = 0;
    for (int e = 0; e < TILE / NT; ++e) {
        const uint64_t k = base + (uint64_t)e * NT + threadIdx.x;
        bool seed = false;
        if (k < n) {
            const uint32_t t = S.o_t[k];
            const uint32_t pq = S.o_pq[k];
            const uint32_t p = pq >> 16;
            seed = (pq & 0xFFFFu) >= Q;
            if (!seed && tau >= 0) {
                const int32_t f = S.floor_id[p];
                for (uint64_t m = k; m > 0;) {
                    --m;
                    const uint32_t tm = S.o_t[m];
                    if (t - tm > (uint32_t)tau) break;
                    const uint32_t pm = S.o_pq[m] >> 16;
                    if (pm != p && S.floor_id[pm] == f) { seed = true; break; }
                }
                for (uint64_t m = k + 1; !seed && m < n; ++m) {
                    const uint32_t tm = S.o_t[m];
                    if (tm - t > (uint32_t)tau) break;
                    const uint32_t pm = S.o_pq[m] >> 16;
                    if (pm != p && S.floor_id[pm] == f) seed = true;
                }
            }
            if (S.seed_flags) S.seed_flags[S.o_idx[k]] = seed ? 1 : 0;
        }
        const uint64_t bal = __ballot(seed);
        if (lane_id() == 0 && base + (uint64_t)e * NT + (threadIdx.x & ~63u) < n)
            S.seed_mask[(base + (uint64_t)e * NT + (threadIdx.x & ~63u)) >> 6] = bal;
        cnt += seed;
    }
    const uint32_t tot = block_sum<NT>(cnt, sh);
    if (threadIdx.x == 0) S.tile_seeds[tile] = tot;
}

// Per slice: exclusive scan of the per-tile seed counts.
__global__ __launch_bounds__(NT) void k_seed_scan(BatchDev b) {
    const SliceDev &S = b.slices[blockIdx.x];
    Plan *P = S.plan;
    if (!slice_in_tail(b, P->state)) return;
    __shared__ uint32_t sh[NT / 64 + 1];
    uint32_t acc = 0;
    for (uint32_t i0 = 0; i0 < S.n_tiles; i0 += NT) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t v = i < S.n_tiles ? S.tile_seeds[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NT>(v, tot, sh);
        if (i < S.n_tiles) S.tile_seeds[i] = acc + ex;
        acc += tot;
    }
    const uint32_t nct = (acc + CTILE - 1) / CTILE;
    for (uint32_t i = threadIdx.x; i < nct; i += NT) S.ctile_fires[i] = 0;
    if (threadIdx.x == 0) {
        P->n_seeds = acc;
        P->n_ctiles = nct;
        P->groups = (S.n_pmt > (uint32_t)LDS_THR_MAX_PMT) ? ROWGROUPS : 1u;
    }
}

// Compact seed list of one tile, in ordered-hit order.
__global__ __launch_bounds__(NT) void k_seed_emit(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].tile_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t tile = item - S.tile_base;
    if (tile >= S.n_tiles) return;
    if (!slice_in_tail(b, S.plan->state)) return;
    __shared__ uint32_t wpre[TILE / 64];
    __shared__ uint64_t wmask[TILE / 64];
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t n = S.n;
    const uint32_t nwords = (uint32_t)(((n - base < (uint64_t)TILE ? n - base : (uint64_t)TILE) + 63) / 64);
    if (threadIdx.x < 64) {
        const uint64_t wv = threadIdx.x < nwords ? S.seed_mask[(base >> 6) + threadIdx.x] : 0ull;
        const uint32_t c = (uint32_t)__popcll(wv);
        const uint32_t inc = wave_incl_scan(c);
        wpre[threadIdx.x] = inc - c;
        wmask[threadIdx.x] = wv;
    }
    __syncthreads();
    const uint32_t off = S.tile_seeds[tile];
    for (int e = 0; e < TILE / NT; ++e) {
        const uint32_t i = (uint32_t)e * NT + threadIdx.x;
        const uint64_t k = base + i;
        if (k >= n) break;
        const uint64_t wv = wmask[i >> 6];
        const uint32_t bit = i & 63u;
        if ((wv >> bit) & 1ull) {
            const uint64_t below = bit ? (wv & (~0ull >> (64 - bit))) : 0ull;
            const uint32_t rank = off + wpre[i >> 6] + (uint32_t)__popcll(below);
            S.s_t[rank] = S.o_t[k];
            S.s_pq[rank] = S.o_pq[k];
            S.s_idx[rank] = S.o_idx[k];
        }
    }
}

// One block: work-list bases of the counting stage.  Slices with a large table
// use ROWGROUPS items per tile (item % 8 == row group) and start at a multiple of 8.
__global__ __launch_bounds__(NT) void k_count_prefix(BatchDev b) {
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (uint32_t i = 0; i < b.n_slices; ++i) {
        Plan *P = &b.plans[i];
        uint32_t items = 0;
        if (slice_in_tail(b, P->state)) {
            if (P->groups > 1) acc = (acc + ROWGROUPS - 1) / ROWGROUPS * ROWGROUPS;
            items = P->n_ctiles * P->groups;
        }
        P->count_item_base = acc;
        acc += items;
    }
    b.counters[Q_COUNT_TOTAL] = acc;
}

// Causal fold of every seed: 1 + the other seeds j with
// |t_i - t_j| <= min(thr[p_i][p_j], w_ns), scanned outwards over the time-ordered
// seed list until the time difference exceeds w_ns.  Static grid-stride over items
// (grid a multiple of 8): for large tables each workgroup keeps one row group, so the
// rows it reads stay in one L2.
__global__ __launch_bounds__(NT) void k_count(BatchDev b) {
    __shared__ uint16_t lthr[LDS_THR_MAX_PMT * LDS_THR_MAX_PMT];
    __shared__ uint32_t sh[NT / 64 + 1];
    __shared__ const uint32_t *loaded_thr;
    if (threadIdx.x == 0) loaded_thr = nullptr;
    __syncthreads();
    const uint32_t total = b.counters[Q_COUNT_TOTAL];
    const uint32_t W = b.prm.w_ns;
    const uint32_t N = b.prm.min_fold;
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.plans[i].count_item_base; });
        const SliceDev &S = b.slices[si];
        const Plan P = b.plans[si];
        if (!slice_in_tail(b, P.state)) continue;
        const uint32_t local = item - P.count_item_base;
        const uint32_t G = P.groups;
        const uint32_t tile = local / G, g = local % G;
        if (tile >= P.n_ctiles) continue;
        const uint32_t np = S.n_pmt;
        const bool use_lds = (G == 1) && (W <= 65535u);
        if (use_lds && loaded_thr != S.thr32) {
            __syncthreads();
            for (uint32_t x = threadIdx.x; x < np * np; x += NT) {
                const uint32_t v = S.thr32[x];
                lthr[x] = (uint16_t)(v < W ? v : W);
            }
            __syncthreads();
            if (threadIdx.x == 0) loaded_thr = S.thr32;
            __syncthreads();
        }
        const uint32_t ns = P.n_seeds;
        const uint32_t i0 = tile * CTILE;
        const uint32_t i1 = (i0 + CTILE < ns) ? i0 + CTILE : ns;
        uint32_t fires = 0;
        for (uint32_t i = i0 + threadIdx.x; i < i1; i += NT) {
            const uint32_t p = S.s_pq[i] >> 16;
            if (G > 1 && (p * G) / np != g) continue;
            const uint32_t t = S.s_t[i];
            uint32_t c = 1;
            if (use_lds) {
                const uint16_t *row = lthr + p * np;
                for (uint32_t j = i; j > 0;) {
                    --j;
                    const uint32_t d = t - S.s_t[j];
                    if (d > W) break;
                    c += d <= row[S.s_pq[j] >> 16];
                }
                for (uint32_t j = i + 1; j < ns; ++j) {
                    const uint32_t d = S.s_t[j] - t;
                    if (d > W) break;
                    c += d <= row[S.s_pq[j] >> 16];
                }
            } else {
                const uint64_t rb = (uint64_t)p * np;
                for (uint32_t j = i; j > 0;) {
                    --j;
                    const uint32_t d = t - S.s_t[j];
                    if (d > W) break;
                    uint32_t lim;
                    if (W <= 65535u) lim = S.thr16[rb + (S.s_pq[j] >> 16)];
                    else lim = S.thr32[rb + (S.s_pq[j] >> 16)];
                    lim = lim < W ? lim : W;
                    c += d <= lim;
                }
                for (uint32_t j = i + 1; j < ns; ++j) {
                    const uint32_t d = S.s_t[j] - t;
                    if (d > W) break;
                    uint32_t lim;
                    if (W <= 65535u) lim = S.thr16[rb + (S.s_pq[j] >> 16)];
                    else lim = S.thr32[rb + (S.s_pq[j] >> 16)];
                    lim = lim < W ? lim : W;
                    c += d <= lim;
                }
            }
            S.s_fold[i] = c;
            fires += c >= N;
        }
        const uint32_t tot = block_sum<NT>(fires, sh);
        if (threadIdx.x == 0 && tot) atomicAdd(&S.ctile_fires[tile], tot);
    }
}

// Per slice: exclusive scan of fires per seed tile.
__global__ __launch_bounds__(NT) void k_fire_scan(BatchDev b) {
    const SliceDev &S = b.slices[blockIdx.x];
    Plan *P = S.plan;
    if (!slice_in_tail(b, P->state)) return;
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint32_t nct = P->n_ctiles;
    uint32_t acc = 0;
    for (uint32_t i0 = 0; i0 < nct; i0 += NT) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t v = i < nct ? S.ctile_fires[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NT>(v, tot, sh);
        if (i < nct) S.ctile_fires[i] = acc + ex;
        acc += tot;
    }
    if (threadIdx.x == 0) P->n_fires = acc;
}

// Ordered fire records of one seed tile (row group 0 items only).
__global__ __launch_bounds__(NT) void k_fire_emit(BatchDev b) {
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint32_t total = b.counters[Q_COUNT_TOTAL];
    const uint32_t N = b.prm.min_fold;
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.plans[i].count_item_base; });
        const SliceDev &S = b.slices[si];
        const Plan P = b.plans[si];
        if (!slice_in_tail(b, P.state)) continue;
        const uint32_t local = item - P.count_item_base;
        const uint32_t tile = local / P.groups;
        if (local % P.groups != 0 || tile >= P.n_ctiles) continue;
        const uint32_t ns = P.n_seeds;
        const uint32_t i0 = tile * CTILE;
        uint32_t off = S.ctile_fires[tile];
        for (uint32_t c0 = i0; c0 < i0 + CTILE && c0 < ns; c0 += NT) {
            const uint32_t i = c0 + threadIdx.x;
            const bool f = i < ns && i < i0 + CTILE && S.s_fold[i] >= N;
            uint32_t tot;
            const uint32_t ex = block_excl_scan<NT>(f ? 1u : 0u, tot, sh);
            if (f) {
                trig_fire r;
                r.t_ns = P.t_min + (int64_t)S.s_t[i];
                r.hit_index = S.s_idx[i];
                r.fold = S.s_fold[i];
                r.pmt_id = (uint16_t)(S.s_pq[i] >> 16);
                r.pad[0] = r.pad[1] = r.pad[2] = 0;
                S.fires[off + ex] = r;
            }
            off += tot;
        }
    }
}

// Per slice: merge the +-H windows of the ordered fires.  A fire starts a new event
// when its window begins after the previous fire's window ends (t_i - t_{i-1} > 2H);
// the largest fold per event comes from a segmented max within each 1024-fire chunk.
__global__ __launch_bounds__(1024) void k_events(BatchDev b) {
    constexpr int NE = 1024;
    const SliceDev &S = b.slices[blockIdx.x];
    Plan *P = S.plan;
    if (!slice_in_tail(b, P->state)) return;
    __shared__ uint32_t sh[NE / 64 + 1];
    __shared__ uint32_t smax[NE];
    __shared__ uint32_t sev[NE];
    const uint32_t nf = P->n_fires;
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const int64_t H = (int64_t)b.prm.half_event_ns;
    uint32_t ne = 0;
    for (uint32_t c0 = 0; c0 < nf; c0 += NE) {
        const uint32_t i = c0 + threadIdx.x;
        const bool act = i < nf;
        bool start = false;
        uint32_t fold = 0;
        if (act) {
            const int64_t t = S.fires[i].t_ns;
            fold = S.fires[i].fold;
            start = (i == 0) || ((uint64_t)(t - S.fires[i - 1].t_ns) > twoH);
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NE>(start ? 1u : 0u, tot, sh);
        const uint32_t ev = ne + ex + (start ? 1u : 0u) - 1u;   // event of fire i
        if (act) {
            S.fire_ev[i] = ev;
            if (start) { S.ev_first[ev] = i; atomicExch(&S.ev_max[ev], 0u); }
        }
        sev[threadIdx.x] = act ? ev : 0xFFFFFFFFu;
        smax[threadIdx.x] = fold;
        __syncthreads();
        // segmented inclusive max within the chunk (segments = equal event id)
        for (int d = 1; d < NE; d <<= 1) {
            uint32_t v = smax[threadIdx.x];
            if ((int)threadIdx.x >= d && sev[threadIdx.x - d] == sev[threadIdx.x]) {
                const uint32_t u = smax[threadIdx.x - d];
                v = u > v ? u : v;
            }
            __syncthreads();
            smax[threadIdx.x] = v;
            __syncthreads();
        }
        if (act) {
            const bool last_in_chunk = (threadIdx.x + 1 == NE) || (i + 1 >= nf) || sev[threadIdx.x + 1] != ev;
            if (last_in_chunk) atomicMax(&S.ev_max[ev], smax[threadIdx.x]);
        }
        ne += tot;
        __syncthreads();
    }
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < ne; e += NE) {
        const uint32_t first = S.ev_first[e];
        const uint32_t last = (e + 1 < ne ? S.ev_first[e + 1] : nf) - 1;
        trig_event r;
        r.t_trig = S.fires[first].t_ns;
        r.t_begin = r.t_trig - H;
        r.t_end = S.fires[last].t_ns + H;
        r.n_fire = last - first + 1;
        r.max_fold = S.ev_max[e];
        S.events[e] = r;
    }
    if (threadIdx.x == 0) P->n_events = ne;
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t trig_launch_tail(const BatchDev &b, const TrigLaunchCfg &cfg, hipStream_t s,
                            void (*mark)(void *, const char *, int), void *mark_ctx) {
    const int grid = ((cfg.n_cu * cfg.persist_per_cu + 7) / 8) * 8;
    if (b.total_tiles) {
        TRIG_MARK("k_seed", 0);
        hipLaunchKernelGGL(k_seed, dim3(b.total_tiles), dim3(NT), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_seed", 1);
    }
    TRIG_MARK("k_seed_scan", 0);
    hipLaunchKernelGGL(k_seed_scan, dim3(b.n_slices), dim3(NT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_seed_scan", 1);
    if (b.total_tiles) {
        TRIG_MARK("k_seed_emit", 0);
        hipLaunchKernelGGL(k_seed_emit, dim3(b.total_tiles), dim3(NT), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_seed_emit", 1);
    }
    TRIG_MARK("k_count_prefix", 0);
    hipLaunchKernelGGL(k_count_prefix, dim3(1), dim3(64), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_count_prefix", 1);
    TRIG_MARK("k_count", 0);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(NT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_count", 1);
    TRIG_MARK("k_fire_scan", 0);
    hipLaunchKernelGGL(k_fire_scan, dim3(b.n_slices), dim3(NT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_fire_scan", 1);
    TRIG_MARK("k_fire_emit", 0);
    hipLaunchKernelGGL(k_fire_emit, dim3(grid), dim3(NT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_fire_emit", 1);
    TRIG_MARK("k_events", 0);
    hipLaunchKernelGGL(k_events, dim3(b.n_slices), dim3(1024), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_events", 1);
    return hipSuccess;
}
