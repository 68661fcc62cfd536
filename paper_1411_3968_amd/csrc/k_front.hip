// Front of the pipeline: ingest, plan, segment boundaries and the run-merge
// ordering of each time slice (paper Sec. 4.2: hits are time-sorted before the
// triggers; each PMT's stream arrives time-ordered, which the ordering uses).
#include "radix_lds.h"
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NT_ING = 256;

__device__ __forceinline__ int64_t wave_min64(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { int64_t u = __shfl_xor(v, d, 64); v = u < v ? u : v; }
    return v;
}
__device__ __forceinline__ int64_t wave_max64(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { int64_t u = __shfl_xor(v, d, 64); v = u > v ? u : v; }
    return v;
}
__device__ __forceinline__ uint32_t wave_maxu(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) { uint32_t u = __shfl_xor(v, d, 64); v = u > v ? u : v; }
    return v;
}
__device__ __forceinline__ uint32_t wave_sumu(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__global__ void k_reset(uint32_t *counters) {
    if (threadIdx.x < N_COUNTERS) counters[threadIdx.x] = 0;
}

// Per chunk of 4096 input hits: time range, largest PMT id, run starts
// (position 0 and every position whose time is below its predecessor's).
__global__ __launch_bounds__(NT_ING) void k_ingest(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].chunk_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t c = item - S.chunk_base;
    if (c >= S.n_chunks) return;
    const uint64_t k0 = (uint64_t)c * CHUNK;
    const uint64_t k1 = (k0 + CHUNK < S.n) ? k0 + CHUNK : S.n;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    uint32_t pmax = 0, ns = 0;
    for (uint64_t k = k0 + threadIdx.x; k < k1; k += NT_ING) {
        const int64_t t = S.t[k];
        lo = t < lo ? t : lo;
        hi = t > hi ? t : hi;
        const uint32_t p = S.pmt[k];
        pmax = p > pmax ? p : pmax;
        ns += (k == 0) || (t < S.t[k - 1]);
    }
    __shared__ int64_t slo[NT_ING / 64], shi[NT_ING / 64];
    __shared__ uint32_t sp[NT_ING / 64], sn[NT_ING / 64];
    lo = wave_min64(lo); hi = wave_max64(hi); pmax = wave_maxu(pmax); ns = wave_sumu(ns);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { slo[w] = lo; shi[w] = hi; sp[w] = pmax; sn[w] = ns; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NT_ING / 64; ++i) {
            lo = slo[i] < lo ? slo[i] : lo;
            hi = shi[i] > hi ? shi[i] : hi;
            pmax = sp[i] > pmax ? sp[i] : pmax;
            ns += sn[i];
        }
        ChunkPart cp;
        cp.t_min = lo; cp.t_max = hi; cp.pmt_max = pmax; cp.n_start = ns; cp.run_base = 0; cp.pad = 0;
        S.part[c] = cp;
    }
}

// Per slice: reduce the chunks, validate the input range, number the runs and
// choose the segment width of the ordering stage.
__global__ __launch_bounds__(256) void k_plan(BatchDev b) {
    const uint32_t si = blockIdx.x;
    const SliceDev &S = b.slices[si];
    Plan *P = S.plan;
    __shared__ uint32_t sh[256 / 64 + 1];
    __shared__ int64_t slo[4], shi[4];
    __shared__ uint32_t spm[4];
    if (S.n == 0) {
        if (threadIdx.x == 0) {
            Plan p = {};
            p.status = TRIG_OK; p.state = ST_SKIP;
            *P = p;
        }
        return;
    }
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    uint32_t pmax = 0;
    for (uint32_t c = threadIdx.x; c < S.n_chunks; c += 256) {
        const ChunkPart cp = S.part[c];
        lo = cp.t_min < lo ? cp.t_min : lo;
        hi = cp.t_max > hi ? cp.t_max : hi;
        pmax = cp.pmt_max > pmax ? cp.pmt_max : pmax;
    }
    lo = wave_min64(lo); hi = wave_max64(hi); pmax = wave_maxu(pmax);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { slo[w] = lo; shi[w] = hi; spm[w] = pmax; }
    __syncthreads();
    lo = slo[0]; hi = shi[0]; pmax = spm[0];
    for (int i = 1; i < 4; ++i) {
        lo = slo[i] < lo ? slo[i] : lo;
        hi = shi[i] > hi ? shi[i] : hi;
        pmax = spm[i] > pmax ? spm[i] : pmax;
    }
    // run numbering: exclusive scan of run starts over the chunks
    uint32_t runs = 0;
    for (uint32_t c0 = 0; c0 < S.n_chunks; c0 += 256) {
        const uint32_t c = c0 + threadIdx.x;
        const uint32_t v = c < S.n_chunks ? S.part[c].n_start : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<256>(v, tot, sh);
        if (c < S.n_chunks) S.part[c].run_base = runs + ex;
        runs += tot;
    }
    if (threadIdx.x != 0) return;
    Plan p = {};
    p.t_min = lo; p.t_max = hi; p.n_runs = runs;
    const uint64_t span = (uint64_t)hi - (uint64_t)lo;
    const int64_t H = (int64_t)b.prm.half_event_ns;
    if (pmax >= S.n_pmt || span >= (1ull << 31) || lo < INT64_MIN + H || hi > INT64_MAX - H) {
        p.status = TRIG_ERANGE; p.state = ST_SKIP;
        *P = p;
        return;
    }
    // segment width: the largest power of two with expected occupancy <= seg_target
    const uint64_t x = ((uint64_t)S.seg_target * (span + 1)) / S.n;
    uint32_t sft = x ? 63u - (uint32_t)__clzll(x) : 0u;
    if (sft > 31) sft = 31;
    const uint64_t nseg = (span >> sft) + 1;
    p.shift = sft; p.n_seg = (uint32_t)nseg;
    p.status = TRIG_OK;
    const bool fits = (uint64_t)runs * (nseg + 1) <= S.pos_cap;
    p.state = fits ? ST_FAST : ST_NEED_GENERIC;
    *P = p;
}

// One block: work-list bases of the ordering stage (segments of fast slices).
__global__ __launch_bounds__(256) void k_seg_prefix(BatchDev b) {
    __shared__ uint32_t sh[256 / 64 + 1];
    uint32_t acc = 0;
    for (uint32_t i0 = 0; i0 < b.n_slices; i0 += 256) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t v = 0;
        if (i < b.n_slices) v = (b.plans[i].state == ST_FAST) ? b.plans[i].n_seg : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<256>(v, tot, sh);
        if (i < b.n_slices) b.plans[i].seg_item_base = acc + ex;
        acc += tot;
    }
    if (threadIdx.x == 0) { b.counters[Q_SEG_TOTAL] = acc; b.counters[Q_SEG] = 0; }
}

// Per chunk: for every run r and segment boundary j (time j << shift relative to
// t_min), pos[r][j] = first position of run r whose time is at or after the boundary;
// pos[r][n_seg] = end of run r.  Runs are maximal time-non-decreasing stretches.
__global__ __launch_bounds__(256) void k_bounds(BatchDev b) {
    constexpr int NT = 256, PER = CHUNK / NT;
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.slices[i].chunk_base; });
    const SliceDev &S = b.slices[si];
    const uint32_t c = item - S.chunk_base;
    if (c >= S.n_chunks) return;
    const Plan P = *S.plan;
    if (P.state != ST_FAST) return;
    __shared__ int64_t st[CHUNK + 2];
    __shared__ uint32_t sh[NT / 64 + 1];
    const uint64_t k0 = (uint64_t)c * CHUNK;
    const uint32_t len = (uint32_t)((k0 + CHUNK < S.n) ? CHUNK : S.n - k0);
    for (uint32_t i = threadIdx.x; i < len; i += NT) st[i + 1] = S.t[k0 + i];
    if (threadIdx.x == 0) {
        st[0] = k0 ? S.t[k0 - 1] : INT64_MIN;
        st[len + 1] = (k0 + len < S.n) ? S.t[k0 + len] : INT64_MIN;
    }
    __syncthreads();
    const uint32_t a = threadIdx.x * PER;
    uint32_t starts = 0;
    for (int e = 0; e < PER; ++e) {
        const uint32_t i = a + e;
        if (i < len) starts += (k0 + i == 0) || (st[i + 1] < st[i]);
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<NT>(starts, tot, sh);
    const uint32_t row_len = P.n_seg + 1;
    const uint32_t sft = P.shift;
    const int64_t tmin = P.t_min;
    int64_t r = (int64_t)S.part[c].run_base + ex - 1;   // run of the element before a
    for (int e = 0; e < PER; ++e) {
        const uint32_t i = a + e;
        if (i >= len) break;
        const uint64_t k = k0 + i;
        const int64_t t = st[i + 1];
        const bool is_start = (k == 0) || (t < st[i]);
        const bool is_end = (k + 1 == S.n) || (st[i + 2] < t);
        if (is_start) ++r;
        uint32_t *row = S.pos + (uint64_t)r * row_len;
        const uint32_t g = (uint32_t)((uint64_t)(t - tmin) >> sft);
        if (is_start) {
            for (uint32_t j = 0; j <= g; ++j) row[j] = (uint32_t)k;
        } else {
            const uint32_t gp = (uint32_t)((uint64_t)(st[i] - tmin) >> sft);
            for (uint32_t j = gp + 1; j <= g; ++j) row[j] = (uint32_t)k;
        }
        if (is_end)
            for (uint32_t j = g + 1; j <= P.n_seg; ++j) row[j] = (uint32_t)(k + 1);
    }
}

// Persistent ordering of time segments.  Segment j of a slice holds the hits with
// t - t_min in [j << shift, (j + 1) << shift); each run contributes the stretch
// [pos[r][j], pos[r][j + 1]).  The segment is gathered into LDS, ranked by the key
// ((t - segment start) << pbits | pmt) with a stable LSD radix over 8-bit digits,
// ties of equal (t, pmt) are put in input-position order, and the ordered
// structure-of-arrays is written at the segment's global offset.
template <int NT, int CAP>
struct SegShared {
    uint32_t dt[CAP], dpq[CAP], didx[CAP];
    uint16_t perm[2][CAP];
    uint32_t run_lo[NT], run_base[NT];
    RankScratch<NT> rs;
    uint32_t misc[8];
};

template <int NT, int CAP>
__global__ __launch_bounds__(NT) void k_segsort(BatchDev b) {
    constexpr int E = CAP / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SegShared<NT, CAP> &sm = *reinterpret_cast<SegShared<NT, CAP> *>(smem_raw);
    const uint32_t total = b.counters[Q_SEG_TOTAL];
    for (;;) {
        if (threadIdx.x == 0) sm.misc[0] = atomicAdd(&b.counters[Q_SEG], 1u);
        __syncthreads();
        const uint32_t item = sm.misc[0];
        __syncthreads();
        if (item >= total) break;
        const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.plans[i].seg_item_base; });
        const SliceDev &S = b.slices[si];
        const Plan P = b.plans[si];
        const uint32_t j = item - P.seg_item_base;
        const uint32_t row_len = P.n_seg + 1;
        const uint64_t seg_lo = (uint64_t)j << P.shift;
        // gather the segment's stretch of every run
        uint32_t m = 0;
        uint32_t goff_part = 0;   // this thread's share of the global offset
        bool over = false;
        for (uint32_t r0 = 0; r0 < P.n_runs; r0 += NT) {
            const uint32_t r = r0 + threadIdx.x;
            uint32_t lo = 0, hi = 0;
            if (r < P.n_runs) {
                const uint32_t *row = S.pos + (uint64_t)r * row_len;
                lo = row[j];
                hi = row[j + 1];
                goff_part += lo - row[0];
            }
            uint32_t cnt_tot;
            const uint32_t ex = block_excl_scan<NT>(hi - lo, cnt_tot, sm.rs.scan);
            if (m + cnt_tot > (uint32_t)CAP) { over = true; break; }
            sm.run_lo[threadIdx.x] = lo;
            sm.run_base[threadIdx.x] = ex;
            __syncthreads();
            const uint32_t nr = (P.n_runs - r0 < (uint32_t)NT) ? P.n_runs - r0 : (uint32_t)NT;
            for (uint32_t k = threadIdx.x; k < cnt_tot; k += NT) {
                // run of element k: last run whose base is <= k
                uint32_t a = 0, z = nr;
                while (a < z) {
                    const uint32_t mid = (a + z) >> 1;
                    if (sm.run_base[mid] <= k) a = mid + 1; else z = mid;
                }
                const uint32_t rr = a - 1;
                const uint32_t src = sm.run_lo[rr] + (k - sm.run_base[rr]);
                sm.dt[m + k] = (uint32_t)(S.t[src] - P.t_min);
                sm.dpq[m + k] = ((uint32_t)S.pmt[src] << 16) | (uint32_t)S.q[src];
                sm.didx[m + k] = src;
            }
            m += cnt_tot;
            __syncthreads();
        }
        if (over) {
            if (threadIdx.x == 0) { S.plan->overflow = 1u; S.plan->state = ST_NEED_GENERIC; }
            __syncthreads();
            continue;
        }
        const uint32_t goff = block_sum<NT>(goff_part, sm.rs.scan);
        // stable LSD radix over the key bits
        const uint32_t pbits = S.pbits;
        const uint32_t key_bits = P.shift + pbits;
        const int passes = (int)((key_bits + 7) / 8);
        for (int k = threadIdx.x; k < (int)m; k += NT) sm.perm[0][k] = (uint16_t)k;
        __syncthreads();
        int cur = 0;
        for (int ps = 0; ps < passes; ++ps) {
            const uint32_t sh8 = 8u * (uint32_t)ps;
            uint32_t rk[E], dg[E];
            auto digit_of = [&](int k) -> uint32_t {
                const uint32_t v = sm.perm[cur][k];
                const uint64_t key = ((uint64_t)(sm.dt[v] - (uint32_t)seg_lo) << pbits) | (uint64_t)(sm.dpq[v] >> 16);
                return (uint32_t)(key >> sh8) & 255u;
            };
            block_rank8<NT, E>((int)m, digit_of, sm.rs, rk, dg);
            const int w = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = (w * E + e) * 64 + lane;
                if (k < (int)m) sm.perm[cur ^ 1][sm.rs.dbase[dg[e]] + rk[e]] = sm.perm[cur][k];
            }
            __syncthreads();
            cur ^= 1;
        }
        // equal (t, pmt): order by input position
        auto keyof = [&](uint32_t v) -> uint64_t {
            return ((uint64_t)(sm.dt[v] - (uint32_t)seg_lo) << pbits) | (uint64_t)(sm.dpq[v] >> 16);
        };
        for (int k = threadIdx.x; k < (int)m; k += NT) {
            const uint32_t v = sm.perm[cur][k];
            const uint64_t kv = keyof(v);
            const bool tie_prev = k > 0 && keyof(sm.perm[cur][k - 1]) == kv;
            const bool tie_next = k + 1 < (int)m && keyof(sm.perm[cur][k + 1]) == kv;
            if (!tie_prev && !tie_next) { sm.perm[cur ^ 1][k] = (uint16_t)v; continue; }
            int a = k, z = k + 1;
            while (a > 0 && keyof(sm.perm[cur][a - 1]) == kv) --a;
            while (z < (int)m && keyof(sm.perm[cur][z]) == kv) ++z;
            int rank = 0;
            for (int u = a; u < z; ++u) rank += sm.didx[sm.perm[cur][u]] < sm.didx[v];
            sm.perm[cur ^ 1][a + rank] = (uint16_t)v;
        }
        __syncthreads();
        cur ^= 1;
        for (int k = threadIdx.x; k < (int)m; k += NT) {
            const uint32_t v = sm.perm[cur][k];
            S.o_t[goff + k] = sm.dt[v];
            S.o_pq[goff + k] = sm.dpq[v];
            S.o_idx[goff + k] = sm.didx[v];
        }
        __syncthreads();
    }
}

template <int NT, int CAP>
hipError_t launch_segsort(const BatchDev &b, const TrigLaunchCfg &cfg, hipStream_t s) {
    const size_t shm = sizeof(SegShared<NT, CAP>);
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_segsort<NT, CAP>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    const int grid = cfg.n_cu * cfg.persist_per_cu;
    hipLaunchKernelGGL((k_segsort<NT, CAP>), dim3(grid), dim3(NT), shm, s, b);
    return hipGetLastError();
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t trig_launch_front(const BatchDev &b, uint32_t seg_cap, const TrigLaunchCfg &cfg, hipStream_t s,
                             void (*mark)(void *, const char *, int), void *mark_ctx) {
    TRIG_MARK("k_reset", 0);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, b.counters);
    TRIG_CHECK();
    TRIG_MARK("k_reset", 1);
    if (b.total_chunks) {
        TRIG_MARK("k_ingest", 0);
        hipLaunchKernelGGL(k_ingest, dim3(b.total_chunks), dim3(NT_ING), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_ingest", 1);
    }
    TRIG_MARK("k_plan", 0);
    hipLaunchKernelGGL(k_plan, dim3(b.n_slices), dim3(256), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_plan", 1);
    TRIG_MARK("k_seg_prefix", 0);
    hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(256), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_seg_prefix", 1);
    if (b.total_chunks) {
        TRIG_MARK("k_bounds", 0);
        hipLaunchKernelGGL(k_bounds, dim3(b.total_chunks), dim3(256), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_bounds", 1);
    }
    TRIG_MARK("k_segsort", 0);
    hipError_t e;
    if (seg_cap <= 2048) e = launch_segsort<256, 2048>(b, cfg, s);
    else if (seg_cap <= 4096) e = launch_segsort<256, 4096>(b, cfg, s);
    else e = launch_segsort<512, 8192>(b, cfg, s);
    if (e != hipSuccess) return e;
    TRIG_MARK("k_segsort", 1);
    return hipSuccess;
}
