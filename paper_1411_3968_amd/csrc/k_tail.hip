// Tail of the pipeline on the time-ordered hits of each slice:
//   L1 seeds (paper Sec. 3 and Sec. 4.2: charge over threshold, floor coincidence),
//   causal N-fold count (Sec. 3: Cherenkov hits of one muon are correlated in
//   space and time within less than 3 us), fires, and the merged event windows
//   (Sec. 2: 6 us window centred on the trigger seed; Sec. 4.2: +-3 us tagging).
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NT = 256;

// Seed bits of one tile of 1024 ordered hits.  The tile and SHALO neighbours on
// each side are staged in LDS with coalesced loads; a floor partner is searched
// among the ordered neighbours within t_floor_ns on both sides (reading global
// memory only when a search runs past the staged halo).  Element e*256 + tid of
// the tile is handled by thread tid in round e, so every wave's ballot is one
// aligned 64-hit word of the seed mask.
__global__ __launch_bounds__(NT) void k_seed(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].tile_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t tile = item - S.tile_base;
    if (tile >= S.n_tiles) return;
    if (!slice_in_tail(b, S.plan->state)) return;
    __shared__ uint32_t lt[TILE + 2 * SHALO], lpq[TILE + 2 * SHALO];
    __shared__ uint16_t lfloor[SEED_LDS_FLOORS];
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint32_t *o_t = S.o_t, *o_pq = S.o_pq;
    const uint64_t n = S.n;
    const uint32_t np = S.n_pmt;
    const uint16_t *floor16 = S.floor16;
    const bool lds_floor = np <= (uint32_t)SEED_LDS_FLOORS;
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t lo = base >= (uint64_t)SHALO ? base - SHALO : 0;
    const uint64_t hi = (base + TILE + SHALO < n) ? base + TILE + SHALO : n;
    stage_copy<NT, 5>(lt, o_t + lo, (uint32_t)(hi - lo));
    stage_copy<NT, 5>(lpq, o_pq + lo, (uint32_t)(hi - lo));
    if (lds_floor) stage_copy<NT, 8>(lfloor, floor16, np);
    __syncthreads();
    auto T_at = [&](uint64_t m) -> uint32_t { return (m >= lo && m < hi) ? lt[m - lo] : o_t[m]; };
    auto P_at = [&](uint64_t m) -> uint32_t { return ((m >= lo && m < hi) ? lpq[m - lo] : o_pq[m]) >> 16; };
    auto F_of = [&](uint32_t p) -> uint32_t { return lds_floor ? lfloor[p] : floor16[p]; };
    const uint32_t Q = b.prm.q_seed;
    const int32_t tau = b.prm.t_floor_ns;
    uint8_t *flags = S.seed_flags;
    uint32_t cnt = 0;
#pragma unroll
    for (int e = 0; e < TILE / NT; ++e) {
        const uint64_t k = base + (uint64_t)e * NT + threadIdx.x;
        bool seed = false;
        if (k < n) {
            const uint32_t t = lt[k - lo];
            const uint32_t pq = lpq[k - lo];
            const uint32_t p = pq >> 16;
            seed = (pq & 0xFFFFu) >= Q;
            if (!seed && tau >= 0) {
                const uint32_t f = F_of(p);
                for (uint64_t m = k; m > 0;) {
                    --m;
                    if (t - T_at(m) > (uint32_t)tau) break;
                    const uint32_t pm = P_at(m);
                    if (pm != p && F_of(pm) == f) { seed = true; break; }
                }
                for (uint64_t m = k + 1; !seed && m < n; ++m) {
                    if (T_at(m) - t > (uint32_t)tau) break;
                    const uint32_t pm = P_at(m);
                    if (pm != p && F_of(pm) == f) seed = true;
                }
            }
            if (flags) flags[S.o_idx[k]] = seed ? 1 : 0;
        }
        const uint64_t bal = __ballot(seed);
        const uint64_t w0 = base + (uint64_t)e * NT + (threadIdx.x & ~63u);
        if (lane_id() == 0 && w0 < n) S.seed_mask[w0 >> 6] = bal;
        cnt += seed;
    }
    const uint32_t tot = block_sum<NT>(cnt, sh);
    if (threadIdx.x == 0) S.tile_seeds[tile] = tot;
}

// Per slice: exclusive scan of the per-tile seed counts.  The last slice to
// finish builds the work list of the counting stage (slices with a large table
// use ROWGROUPS items per tile, item % 8 == row group, starting at a multiple of 8).
__global__ __launch_bounds__(1024) void k_seed_scan(BatchDev b) {
    const SliceDev &S = b.slices[blockIdx.x];
    Plan *P = S.plan;
    __shared__ uint32_t sh[1024 / 64 + 1];
    __shared__ bool last;
    if (slice_in_tail(b, P->state)) {
        const uint32_t ns = block_scan_array<1024>(S.tile_seeds, S.n_tiles, sh);
        const uint32_t groups = (S.n_pmt > (uint32_t)LDS_THR_MAX_PMT) ? ROWGROUPS : 1u;
        const uint32_t nct = (ns + count_tile(groups) - 1) / count_tile(groups);
        for (uint32_t i = threadIdx.x; i < nct; i += 1024) S.ctile_fires[i] = 0;
        if (threadIdx.x == 0) {
            P->n_seeds = ns;
            P->n_ctiles = nct;
            P->groups = groups;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&b.counters[C_SCAN_DONE], 1u) == b.n_slices - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    uint32_t acc = 0;
    for (uint32_t i = 0; i < b.n_slices; ++i) {
        Plan *Pi = &b.plans[i];
        uint32_t items = 0;
        if (slice_in_tail(b, load_acquire(&Pi->state))) {
            const uint32_t g = load_acquire(&Pi->groups);
            if (g > 1) acc = (acc + ROWGROUPS - 1) / ROWGROUPS * ROWGROUPS;
            items = load_acquire(&Pi->n_ctiles) * g;
        }
        Pi->count_item_base = acc;
        acc += items;
    }
    b.counters[Q_COUNT_TOTAL] = acc;
    b.counters[C_SCAN_DONE] = 0;
}

// Compact seed list of one tile, in ordered-hit order.
__global__ __launch_bounds__(NT) void k_seed_emit(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].tile_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t tile = item - S.tile_base;
    if (tile >= S.n_tiles) return;
    if (!slice_in_tail(b, S.plan->state)) return;
    constexpr int NWORD = TILE / 64;
    __shared__ uint32_t wpre[NWORD];
    __shared__ uint64_t wmask[NWORD];
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t n = S.n;
    const uint32_t nwords = (uint32_t)(((n - base < (uint64_t)TILE ? n - base : (uint64_t)TILE) + 63) / 64);
    if (threadIdx.x < 64) {
        const uint64_t wv = threadIdx.x < nwords ? S.seed_mask[(base >> 6) + threadIdx.x] : 0ull;
        const uint32_t c = (uint32_t)__popcll(wv);
        const uint32_t inc = wave_incl_scan(c);
        if (threadIdx.x < NWORD) {
            wpre[threadIdx.x] = inc - c;
            wmask[threadIdx.x] = wv;
        }
    }
    __syncthreads();
    const uint32_t off = S.tile_seeds[tile];
#pragma unroll
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

// Causal fold of every seed: 1 + the other seeds j with
// |t_i - t_j| <= min(thr[p_i][p_j], w_ns), scanned outwards over the time-ordered
// seed list until the time difference exceeds w_ns.  A counting tile and CHALO
// seeds on each side are staged in LDS.  Tables of up to 128 PMTs are kept in LDS
// as u16 min(thr, w_ns).  Larger tables are read from L2: such a slice has 8 items
// per tile (row groups), the grid is a multiple of 8 and items are taken with a
// grid stride, so workgroup b (dispatched to XCD b mod 8) only reads the rows of
// group b mod 8 and that 1/8 of the table stays in one XCD's L2.
__global__ __launch_bounds__(NT) void k_count(BatchDev b) {
    constexpr int LTHR_BYTES = LDS_THR_MAX_PMT * LDS_THR_MAX_PMT * 2;
    constexpr int STAGE = CT8 + 2 * CHALO;
    __shared__ __align__(16) unsigned char raw[LTHR_BYTES + (CT1 + 2 * CHALO) * 8 > STAGE * 8 + CT8 * 2
                                                   ? LTHR_BYTES + (CT1 + 2 * CHALO) * 8
                                                   : STAGE * 8 + CT8 * 2];
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
        const uint32_t TS = count_tile(G);
        const bool use_lds = (G == 1) && (W <= 65535u);
        uint16_t *lthr = (uint16_t *)raw;
        uint32_t *st = (uint32_t *)(raw + (G == 1 ? LTHR_BYTES : 0));
        const uint32_t stage_cap = G == 1 ? CT1 + 2 * CHALO : STAGE;
        uint32_t *sp = st + stage_cap;
        uint16_t *mine = (uint16_t *)(sp + stage_cap);
        if (use_lds && loaded_thr != S.thr32) {
            __syncthreads();
            // the u16 copy min(thr, 65535) moves as 32-bit pairs; min(., W) at use
            stage_copy<NT, 8>((uint32_t *)lthr, (const uint32_t *)S.thr16, (np * np + 1) / 2);
            __syncthreads();
            if (threadIdx.x == 0) loaded_thr = S.thr32;
            __syncthreads();
        } else if (!use_lds && G > 1 && loaded_thr != nullptr) {
            __syncthreads();
            if (threadIdx.x == 0) loaded_thr = nullptr;   // the staging area overwrites the table
            __syncthreads();
        }
        const uint32_t ns = P.n_seeds;
        const uint32_t i0 = tile * TS;
        const uint32_t i1 = (i0 + TS < ns) ? i0 + TS : ns;
        const uint32_t lo = i0 >= (uint32_t)CHALO ? i0 - CHALO : 0u;
        const uint32_t hi = (i1 + CHALO < ns) ? i1 + CHALO : ns;
        stage_copy<NT, 6>(st, S.s_t + lo, hi - lo);
        stage_copy<NT, 6>(sp, S.s_pq + lo, hi - lo, [](uint32_t v) { return v >> 16; });
        __syncthreads();
        // the seeds of this item: the whole tile, or those whose PMT is in row group g
        uint32_t m = i1 - i0;
        if (G > 1) {
            uint32_t tot_all = 0;
            for (uint32_t c0 = 0; c0 < i1 - i0; c0 += NT) {
                const uint32_t x = c0 + threadIdx.x;
                const bool mineflag = x < i1 - i0 && (sp[i0 - lo + x] * G) / np == g;
                uint32_t tot;
                const uint32_t ex = block_excl_scan<NT>(mineflag ? 1u : 0u, tot, sh);
                if (mineflag) mine[tot_all + ex] = (uint16_t)x;
                tot_all += tot;
            }
            m = tot_all;
            __syncthreads();
        }
        auto T_at = [&](uint32_t j) -> uint32_t { return (j >= lo && j < hi) ? st[j - lo] : S.s_t[j]; };
        auto P_at = [&](uint32_t j) -> uint32_t { return (j >= lo && j < hi) ? sp[j - lo] : (S.s_pq[j] >> 16); };
        uint32_t fires = 0;
        for (uint32_t x = threadIdx.x; x < m; x += NT) {
            const uint32_t i = i0 + (G > 1 ? (uint32_t)mine[x] : x);
            const uint32_t p = sp[i - lo];
            const uint32_t t = st[i - lo];
            // the window: seeds [jl, jr) within w_ns of seed i
            uint32_t jl = i, jr = i + 1;
            while (jl > 0 && t - T_at(jl - 1) <= W) --jl;
            while (jr < ns && T_at(jr) - t <= W) ++jr;
            uint32_t c = 1;
            if (use_lds) {
                const uint16_t *row = lthr + p * np;
                for (uint32_t j = jl; j < jr; ++j) {
                    if (j == i) continue;
                    const uint32_t tj = T_at(j);
                    const uint32_t d = tj > t ? tj - t : t - tj;
                    c += d <= row[P_at(j)];
                }
            } else {
                // table rows from L2: issue CB lookups before using any of them
                constexpr int CB = 8;
                const uint64_t rb = (uint64_t)p * np;
                for (uint32_t j0 = jl; j0 < jr; j0 += CB) {
                    uint32_t lim[CB], dd[CB];
#pragma unroll
                    for (int u = 0; u < CB; ++u) {
                        const uint32_t j = j0 + u;
                        dd[u] = 0xFFFFFFFFu;
                        lim[u] = 0;
                        if (j < jr && j != i) {
                            const uint32_t tj = T_at(j);
                            dd[u] = tj > t ? tj - t : t - tj;
                            const uint32_t pj = P_at(j);
                            lim[u] = (W <= 65535u) ? (uint32_t)S.thr16[rb + pj] : S.thr32[rb + pj];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < CB; ++u) {
                        const uint32_t l = lim[u] < W ? lim[u] : W;
                        c += dd[u] != 0xFFFFFFFFu && dd[u] <= l;
                    }
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
__global__ __launch_bounds__(1024) void k_fire_scan(BatchDev b) {
    const SliceDev &S = b.slices[blockIdx.x];
    Plan *P = S.plan;
    if (!slice_in_tail(b, P->state)) return;
    __shared__ uint32_t sh[1024 / 64 + 1];
    const uint32_t nf = block_scan_array<1024>(S.ctile_fires, P->n_ctiles, sh);
    if (threadIdx.x == 0) P->n_fires = nf;
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
        const uint32_t TS = count_tile(P.groups);
        const uint32_t ns = P.n_seeds;
        const uint32_t i0 = tile * TS;
        const uint32_t i1 = (i0 + TS < ns) ? i0 + TS : ns;
        uint32_t off = S.ctile_fires[tile];
        for (uint32_t c0 = i0; c0 < i1; c0 += NT) {
            const uint32_t i = c0 + threadIdx.x;
            const bool f = i < i1 && S.s_fold[i] >= N;
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

// Results to host-mapped staging: every plan, and the fires and events of each
// slice of this tail that fit its staging capacity (the host copies larger lists
// from device memory).  One sync then delivers the whole batch.
__global__ __launch_bounds__(NT) void k_export(BatchDev b) {
    const uint32_t gt = blockIdx.x * NT + threadIdx.x;
    const uint32_t gs = gridDim.x * NT;
    for (uint32_t i = gt; i < b.n_slices; i += gs) b.x_plans[i] = b.plans[i];
    for (uint32_t si = 0; si < b.n_slices; ++si) {
        const SliceDev &S = b.slices[si];
        const Plan &P = b.plans[si];
        if (!slice_in_tail(b, P.state)) continue;
        if (S.x_fires && P.n_fires <= S.x_fire_cap)
            for (uint32_t i = gt; i < P.n_fires; i += gs) S.x_fires[i] = S.fires[i];
        if (S.x_events && P.n_events <= S.x_event_cap)
            for (uint32_t i = gt; i < P.n_events; i += gs) S.x_events[i] = S.events[i];
    }
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
    hipLaunchKernelGGL(k_seed_scan, dim3(b.n_slices), dim3(1024), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_seed_scan", 1);
    if (b.total_tiles) {
        TRIG_MARK("k_seed_emit", 0);
        hipLaunchKernelGGL(k_seed_emit, dim3(b.total_tiles), dim3(NT), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_seed_emit", 1);
    }
    TRIG_MARK("k_count", 0);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(NT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_count", 1);
    TRIG_MARK("k_fire_scan", 0);
    hipLaunchKernelGGL(k_fire_scan, dim3(b.n_slices), dim3(1024), 0, s, b);
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
    if (b.x_plans) {
        TRIG_MARK("k_export", 0);
        hipLaunchKernelGGL(k_export, dim3(64), dim3(NT), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_export", 1);
    }
    return hipSuccess;
}
