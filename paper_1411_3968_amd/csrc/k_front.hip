// Front of the pipeline: ingest, plan, segment boundaries and the run-merge
// ordering of each time slice (paper Sec. 4.2: hits are time-sorted before the
// triggers; each PMT's stream arrives time-ordered, which the ordering uses).
#include "radix_lds.h"
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NT_ING = 256;

__device__ __forceinline__ int64_t lane_read_i64(int64_t v, int src) {
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)lane_read((uint32_t)(u >> 32), src) << 32) | lane_read((uint32_t)u, src));
}
__device__ __forceinline__ int64_t wave_min64(int64_t v) {
    return lane_read_i64(wave_scan(v, (int64_t)INT64_MAX, [](int64_t a, int64_t b) { return a < b ? a : b; }), 63);
}
__device__ __forceinline__ int64_t wave_max64(int64_t v) {
    return lane_read_i64(wave_scan(v, (int64_t)INT64_MIN, [](int64_t a, int64_t b) { return a > b ? a : b; }), 63);
}
__device__ __forceinline__ uint32_t wave_maxu(uint32_t v) { return wave_max_all(v); }
__device__ __forceinline__ uint32_t wave_sumu(uint32_t v) { return wave_total(v); }

typedef int64_t i64x2 __attribute__((ext_vector_type(2)));    // 16-byte loads
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));   // 16-byte stores
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));   // 8-byte loads

// Per chunk of CHUNK input hits: time range, largest PMT id, run starts
// (position 0 and every position whose time is below its predecessor's), and
// the packed copy of the chunk's hits that the wave ordering kernel gathers.
// A thread takes four consecutive hits: two 16-byte loads of times, one 8-byte
// load each of PMT ids and charges, two 16-byte stores (scalar accesses at the
// slice's end or when the caller's arrays are not aligned for them).
__global__ __launch_bounds__(NT_ING) void k_ingest(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = find_slice(b.n_slices, item, [&](uint32_t i) { return b.chunk_bases[i]; });
    const SliceDev &S = b.slices[si];
    const uint32_t c = item - chunk_base_of(b, si);
    if (c >= S.n_chunks) return;
    const uint64_t k0 = (uint64_t)c * CHUNK;
    const uint64_t k1 = (k0 + CHUNK < S.n) ? k0 + CHUNK : S.n;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    uint32_t pmax = 0, ns = 0;
    const TRIG_GAS int64_t *tin = gmem(S.t);
    const TRIG_GAS uint16_t *pin = gmem(S.pmt);
    const TRIG_GAS uint16_t *qin = gmem(S.q);
    TRIG_GAS uint64_t *pk = packed_hits(S);
    constexpr int PER = CHUNK / NT_ING;
    static_assert(PER == 4, "four consecutive hits per thread");
    const uint64_t ka = k0 + (uint64_t)threadIdx.x * PER;   // (a multiple of 4)
    const uint32_t own = ka < k1 ? (uint32_t)min(k1 - ka, (uint64_t)PER) : 0u;
    const bool aligned = (((uintptr_t)S.t | (uintptr_t)pk) & 15) == 0 && (((uintptr_t)S.pmt | (uintptr_t)S.q) & 7) == 0;
    int64_t tv[PER];
    uint32_t pv[PER], qv[PER];
    if (own == PER && aligned) {
        const i64x2 t01 = *(const TRIG_GAS i64x2 *)(tin + ka), t23 = *(const TRIG_GAS i64x2 *)(tin + ka + 2);
        const u16x4 p4 = *(const TRIG_GAS u16x4 *)(pin + ka), q4 = *(const TRIG_GAS u16x4 *)(qin + ka);
        tv[0] = t01.x; tv[1] = t01.y; tv[2] = t23.x; tv[3] = t23.y;
        pv[0] = p4.x; pv[1] = p4.y; pv[2] = p4.z; pv[3] = p4.w;
        qv[0] = q4.x; qv[1] = q4.y; qv[2] = q4.z; qv[3] = q4.w;
    } else {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            tv[e] = 0; pv[e] = qv[e] = 0;
            if ((uint32_t)e < own) { tv[e] = tin[ka + e]; pv[e] = pin[ka + e]; qv[e] = qin[ka + e]; }
        }
    }
    const int64_t tprev = (own && ka) ? tin[ka - 1] : INT64_MIN;   // the hit before the thread's first
    uint64_t w4[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        w4[e] = ((uint64_t)((pv[e] << 16) | qv[e]) << 32) | (uint32_t)(uint64_t)tv[e];
        if ((uint32_t)e < own) {
            const int64_t t = tv[e];
            lo = t < lo ? t : lo;
            hi = t > hi ? t : hi;
            pmax = pv[e] > pmax ? pv[e] : pmax;
            ns += (ka + e == 0) || (t < (e ? tv[e - 1] : tprev));
        }
    }
    if (own == PER && aligned) {
        *(TRIG_GAS u64x2 *)(pk + ka) = u64x2{w4[0], w4[1]};
        *(TRIG_GAS u64x2 *)(pk + ka + 2) = u64x2{w4[2], w4[3]};
    } else {
#pragma unroll
        for (int e = 0; e < PER; ++e)
            if ((uint32_t)e < own) pk[ka + e] = w4[e];
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
        gstore(gmem(S.part) + c, cp);
    }
}

// The sums of block blk of PL_CH chunks of slice S, a chunk per thread of a
// 1024-thread workgroup; every thread ends with them.
__device__ __forceinline__ void block_sums(const SliceDev &S, uint32_t blk, int64_t &lo, int64_t &hi, uint32_t &pmax,
                                           float &dmax, uint32_t &runs) {
    constexpr int NT = 1024, NW = NT / 64;
    static_assert(PL_CH == (uint32_t)NT, "a chunk per thread");
    const uint32_t nch = S.n_chunks;
    const uint64_t n = S.n;
    TRIG_GAS ChunkPart *part = gmem(S.part);
    const uint32_t c = blk * PL_CH + threadIdx.x;
    const bool in = c < nch;
    lo = INT64_MAX;
    hi = INT64_MIN;
    pmax = 0;
    dmax = 0.f;
    uint32_t ns = 0;
    if (in) {
        const ChunkPart cp = gload(part + c);
        ns = cp.n_start;
        lo = cp.t_min;
        hi = cp.t_max;
        pmax = cp.pmt_max;
        const uint64_t cnt = (c + 1 < nch) ? (uint64_t)CHUNK : n - (uint64_t)c * CHUNK;
        dmax = (float)cnt / ((float)(uint64_t)(cp.t_max - cp.t_min) + 1.0f);
    }
    __shared__ uint32_t sh[NW + 1];
    __shared__ int64_t slo[NW], shi[NW];
    __shared__ uint32_t spm[NW];
    __shared__ float sdm[NW];
    const uint32_t ex = block_excl_scan<NT>(ns, runs, sh);
    if (in) part[c].run_base = ex;
    lo = wave_min64(lo); hi = wave_max64(hi); pmax = wave_maxu(pmax);
    // (densities are non-negative: their bit patterns order as unsigned integers)
    dmax = __uint_as_float(wave_maxu(__float_as_uint(dmax)));
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { slo[w] = lo; shi[w] = hi; spm[w] = pmax; sdm[w] = dmax; }
    __syncthreads();
    lo = slo[0]; hi = shi[0]; pmax = spm[0]; dmax = sdm[0];
    for (int i = 1; i < NW; ++i) {
        lo = slo[i] < lo ? slo[i] : lo;
        hi = shi[i] > hi ? shi[i] : hi;
        pmax = spm[i] > pmax ? spm[i] : pmax;
        dmax = sdm[i] > dmax ? sdm[i] : dmax;
    }
}

// Partial sums of the plan over a block of PL_CH chunks of a slice (grid: blocks x
// slices; many CUs instead of one workgroup per slice), launched when a slice has
// more than one block: the time range, largest PMT id, the largest chunk density
// in hits per ns (a chunk is mostly one run: a burst on one PMT shows as a short
// chunk), and the run numbering within the block (each chunk's run_base from a
// block scan of the run starts; the plan adds the runs before the block).
__global__ __launch_bounds__(1024) void k_psum(BatchDev b) {
    const uint32_t si = blockIdx.y, blk = blockIdx.x;
    const SliceDev &S = b.slices[si];
    if ((uint64_t)blk * PL_CH >= S.n_chunks) return;
    int64_t lo, hi;
    uint32_t pmax, runs;
    float dmax;
    block_sums(S, blk, lo, hi, pmax, dmax, runs);
    if (threadIdx.x == 0) gstore(gmem(S.ppart) + blk, PlanPart{lo, hi, pmax, runs, dmax, 0u});
}

// The runs started before each block of chunks (from the blocks' run counts),
// their total, and the blocks' time range, largest PMT id and density.
template <int NT>
__device__ __forceinline__ void plan_blocks(const SliceDev &S, int64_t &lo, int64_t &hi, uint32_t &pmax,
                                            uint32_t &runs, float &dmax, uint32_t *sh) {
    TRIG_GAS PlanPart *pp = gmem(S.ppart);
    const uint32_t nb = (S.n_chunks + PL_CH - 1) / PL_CH;
    for (uint32_t i0 = 0; i0 < nb; i0 += NT) {
        const uint32_t i = i0 + threadIdx.x;
        PlanPart q = PlanPart{INT64_MAX, INT64_MIN, 0u, 0u, 0.f, 0u};
        if (i < nb) q = gload(pp + i);
        lo = q.t_min < lo ? q.t_min : lo;
        hi = q.t_max > hi ? q.t_max : hi;
        pmax = q.pmt_max > pmax ? q.pmt_max : pmax;
        dmax = q.dmax > dmax ? q.dmax : dmax;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NT>(q.runs, tot, sh);
        if (i < nb) pp[i].run_off = runs + ex;
        runs += tot;
    }
}

// Per slice: combine the chunk blocks' partial sums, validate the input range,
// number the runs and choose the segment width and the ordering kernel of the
// slice.
__global__ __launch_bounds__(1024) void k_plan(BatchDev b) {
    constexpr int NT = 1024, NW = NT / 64;
    const uint32_t si = blockIdx.x;
    const SliceDev &S = b.slices[si];
    Plan *P = S.plan;
    __shared__ uint32_t sh[NW + 1];
    __shared__ int64_t slo[NW], shi[NW];
    __shared__ uint32_t spm[NW];
    __shared__ float sdm[NW];
    Plan p = {};
    p.status = TRIG_OK;
    p.state = ST_SKIP;
    if (S.n > 0) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        uint32_t pmax = 0, runs = 0;
        float dmax = 0.f;
        if (b.max_tiles > PL_CH) {
            plan_blocks<NT>(S, lo, hi, pmax, runs, dmax, sh);   // k_psum's blocks
        } else {
            block_sums(S, 0, lo, hi, pmax, dmax, runs);         // the one block, here
            if (threadIdx.x == 0) gmem(S.ppart)[0].run_off = 0u;
        }
        lo = wave_min64(lo); hi = wave_max64(hi); pmax = wave_maxu(pmax);
        // (densities are non-negative: their bit patterns order as unsigned integers)
        dmax = __uint_as_float(wave_maxu(__float_as_uint(dmax)));
        const int w = threadIdx.x >> 6;
        if (lane_id() == 0) { slo[w] = lo; shi[w] = hi; spm[w] = pmax; sdm[w] = dmax; }
        __syncthreads();
        lo = slo[0]; hi = shi[0]; pmax = spm[0]; dmax = sdm[0];
        for (int i = 1; i < NW; ++i) {
            lo = slo[i] < lo ? slo[i] : lo;
            hi = shi[i] > hi ? shi[i] : hi;
            pmax = spm[i] > pmax ? spm[i] : pmax;
            dmax = sdm[i] > dmax ? sdm[i] : dmax;
        }
        p.t_min = lo; p.t_max = hi; p.n_runs = runs;
        const uint64_t span = (uint64_t)hi - (uint64_t)lo;
        const int64_t H = (int64_t)b.prm.half_event_ns;
        // the seed kernel's halo: four times the mean number of hits in t_floor_ns,
        // at least one 64-hit word, in whole words (none for a negative t_floor_ns)
        {
            const int32_t tau = b.prm.t_floor_ns;
            const double hf = tau < 0 ? 0.0 : 4.0 * (double)S.n * ((double)tau + 1.0) / ((double)span + 1.0);
            const uint32_t h = hf >= 1048576.0 ? 1048576u : (uint32_t)hf;
            p.seed_halo = tau < 0 ? 0u : (h < 64 ? 64u : (h + 63) & ~63u);
        }
        if (pmax >= S.n_pmt || span >= (1ull << 31) || lo < INT64_MIN + H || hi > INT64_MAX - H) {
            p.status = TRIG_ERANGE;
        } else {
            // ordering kernel: wave per segment for few runs; for more runs than a
            // wave merges, two levels of wave merges (groups of runs, then the
            // groups' ordered stretches) or, when tuned to it, block per segment
            uint32_t cap = S.seg_cap, target = S.seg_target;
            bool ok = true;
            const bool many = cap <= (uint32_t)WAVE_CAP && runs > (uint32_t)WAVE_RUNS;
            const bool tl = many && (b.sort_kernels & 4u) != 0 && runs <= (uint32_t)(WAVE_RUNS * WAVE_RUNS);
            if (many && !tl) {
                cap = b.block_cap;
                target = b.block_target;
                ok = (b.sort_kernels & 2u) != 0;
            }
            p.seg_kind = cap <= (uint32_t)WAVE_CAP ? 0u : 1u;
            // segment width: the largest power of two with expected occupancy <= target
            // at the slice's mean density plus its densest chunk's (a burst on one
            // PMT would otherwise overflow the segments it crosses)
            auto shift_for = [&](float dens) -> uint32_t {
                const float xf = (float)target / dens;
                const uint64_t x = xf >= 1.0f ? (uint64_t)fminf(xf, 4.0e18f) : 0ull;
                const uint32_t sf = x ? 63u - (uint32_t)__clzll(x) : 0u;
                return sf > 31 ? 31u : sf;
            };
            const float mean = (float)S.n / ((float)span + 1.0f);
            uint32_t sft = shift_for(mean + dmax);
            uint64_t tcap = S.pos_cap;   // entries of the (level-1) boundary table at most
            if (tl) {
                // level 2 merges the groups' stretches at the slice's density; level 1
                // orders each group of rg runs at its share of it (a burst stays in
                // its own group), widened while the level-1 table is over budget
                const uint32_t rg = max((uint32_t)64, (runs + WAVE_RUNS - 1) / WAVE_RUNS);
                const uint32_t ngrp = (runs + rg - 1) / rg;
                p.tl = 1;
                p.run_grp = rg;
                p.n_grp = ngrp;
                p.n_runs2 = ngrp;
                p.shift2 = sft;
                p.n_seg2 = (uint32_t)((span >> sft) + 1);
                // (the level-2 table takes the end of the area)
                const uint64_t l2e = level2_entries(p);
                tcap = l2e < S.pos_cap ? S.pos_cap - l2e : 0;
                uint32_t s1 = shift_for(mean / (float)ngrp + dmax);
                while (s1 < 31 && bnd_entries<BND_TJ>((span >> s1) + 2, runs) > tcap &&
                       2 * ((S.n << (s1 + 1)) / ((span + 1) * ngrp)) <= (uint64_t)cap)
                    ++s1;
                sft = s1;
            } else {
                // many runs: widen the segments (up to half the LDS capacity expected)
                // until the boundary table fits its budget
                while (sft < 31 && bnd_entries<BND_TJ>((span >> sft) + 2, runs) > tcap &&
                       2 * ((S.n << (sft + 1)) / (span + 1)) <= (uint64_t)cap)
                    ++sft;
            }
            const uint64_t nseg = (span >> sft) + 1;
            p.shift = sft;
            p.n_seg = (uint32_t)nseg;
            const bool fits = ok && bnd_entries<BND_TJ>(nseg + 1, runs) <= tcap;
            p.state = fits ? ST_FAST : ST_NEED_GENERIC;
        }
    }
    if (threadIdx.x == 0) *P = p;
    // the maps from the fold kernel's groups, from tiles and from chunks to their
    // slice (every slice, whatever its state: each work item looks its slice up
    // there)
    if (b.n_slices > 1 && b.group_slice) {
        const uint32_t ng = groups_of(S.n_tiles, b.tile_group);
        for (uint32_t g = threadIdx.x; g < ng; g += NT) b.group_slice[S.group_base + g] = si;
        for (uint32_t t = threadIdx.x; t < S.n_tiles; t += NT) b.tile_slice[S.tile_base + t] = si;
        for (uint32_t c = threadIdx.x; c < S.n_chunks; c += NT) b.chunk_slice[S.chunk_base + c] = si;
    }
}

// Work lists of the two ordering kernels (run-merge slices' segments), by one
// extra block of k_bounds: every plan is final once k_plan has finished.  (A last-block
// pattern inside k_plan would need a device-scope fence per block, which costs
// microseconds each on this chip.)
__device__ void build_segment_lists(const BatchDev &b) {
    constexpr int NT = 256;
    __shared__ uint32_t sh[NT / 64 + 1];
    uint32_t acc = 0, acc_b = 0, acc_2 = 0;
    for (uint32_t i0 = 0; i0 < b.n_slices; i0 += NT) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t nw = 0, nb = 0, n2 = 0;
        if (i < b.n_slices) {
            const Plan &P = b.plans[i];
            if (P.state == ST_FAST) {
                if (P.seg_kind == 0) nw = P.tl ? P.n_grp * P.n_seg : P.n_seg; else nb = P.n_seg;
                if (P.tl) n2 = P.n_seg2;   // (the second level skips a slice that level 1 gave up)
            }
        }
        uint32_t tw, tbk, t2;
        const uint32_t ew = block_excl_scan<NT>(nw, tw, sh);
        const uint32_t eb = block_excl_scan<NT>(nb, tbk, sh);
        const uint32_t e2 = block_excl_scan<NT>(n2, t2, sh);
        if (i < b.n_slices) {
            b.plans[i].seg_item_base = acc + ew;
            b.plans[i].seg_item_base_b = acc_b + eb;
            b.plans[i].seg_item_base2 = acc_2 + e2;
        }
        acc += tw;
        acc_b += tbk;
        acc_2 += t2;
    }
    if (threadIdx.x == 0) {
        b.counters[Q_SEG_TOTAL] = acc;
        b.counters[Q_SEG_TOTAL_B] = acc_b;
        b.counters[Q_SEG_TOTAL2] = acc_2;
    }
}

// Per chunk: for every run r and segment boundary j (time j << shift relative to
// t_min), pos[j][r] = first position of run r whose time is at or after the
// boundary; pos[n_seg][r] = end of run r.  Runs are maximal time-non-decreasing
// stretches.  The table comes in tiles of BND_TJ consecutive boundaries,
// run-major inside a tile (bnd_at), so a chunk writes whole 64-byte stretches of
// its run's entries (segment-major, every entry was a partial cache line of its
// own, written by a chunk far in time from the ones that share the line: 760
// against 544 us on the 256-slice batch).  (The second level's table of
// two-level slices is written by level 1 itself.)
__global__ __launch_bounds__(256) void k_bounds(BatchDev b) {
    constexpr int NT = 256, PER = CHUNK / NT;
    const uint32_t item = blockIdx.x;
    if (item == b.total_chunks) {   // one extra block
        build_segment_lists(b);
        return;
    }
    const uint32_t si = slice_of_chunk(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t c = item - chunk_base_of(b, si);
    if (c >= S.n_chunks) return;
    const Plan P = gload(gmem(b.plans + si));
    if (P.state != ST_FAST) return;
    const TRIG_GAS int64_t *tin = gmem(S.t);
    // the chunk's times at st[2 ..], its predecessor's at st[1] and its
    // successor's after them (a thread stages its four with two 16-byte loads
    // and stores when the caller's array allows)
    __shared__ __align__(16) int64_t st[CHUNK + 4];
    __shared__ uint32_t sh[NT / 64 + 1];
    static_assert(PER == 4, "four consecutive hits per thread");
    const uint64_t k0 = (uint64_t)c * CHUNK;
    const uint32_t len = (uint32_t)((k0 + CHUNK < S.n) ? CHUNK : S.n - k0);
    const uint32_t a = threadIdx.x * PER;
    if (a + PER <= len && ((uintptr_t)S.t & 15) == 0) {
        typedef int64_t i64x2 __attribute__((ext_vector_type(2)));
        const i64x2 t01 = *(const TRIG_GAS i64x2 *)(tin + k0 + a), t23 = *(const TRIG_GAS i64x2 *)(tin + k0 + a + 2);
        *(i64x2 *)(st + 2 + a) = t01;
        *(i64x2 *)(st + 4 + a) = t23;
    } else {
        for (uint32_t e = 0; e < (uint32_t)PER; ++e)
            if (a + e < len) st[2 + a + e] = tin[k0 + a + e];
    }
    if (threadIdx.x == 0) {
        st[1] = k0 ? tin[k0 - 1] : INT64_MIN;
        st[len + 2] = (k0 + len < S.n) ? tin[k0 + len] : INT64_MIN;
    }
    __syncthreads();
    uint32_t starts = 0;
    for (int e = 0; e < PER; ++e) {
        const uint32_t i = a + e;
        if (i < len) starts += (k0 + i == 0) || (st[i + 2] < st[i + 1]);
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<NT>(starts, tot, sh);
    const uint64_t R = P.n_runs;
    // run of the element before a: the runs before the chunk's block, before the chunk in it, before a in it
    int64_t r = (int64_t)gmem(S.ppart)[c / PL_CH].run_off + gmem(S.part)[c].run_base + ex - 1;
    TRIG_GAS uint32_t *pos = gmem(S.pos);
    for (int e = 0; e < PER; ++e) {
        const uint32_t i = a + e;
        if (i >= len) break;
        const uint64_t k = k0 + i;
        const int64_t t = st[i + 2];
        const bool is_start = (k == 0) || (t < st[i + 1]);
        const bool is_end = (k + 1 == S.n) || (st[i + 3] < t);
        if (is_start) ++r;
        const uint32_t g = (uint32_t)((uint64_t)(t - P.t_min) >> P.shift);
        if (is_start) {
            for (uint32_t j = 0; j <= g; ++j) pos[bnd_at<BND_TJ>(j, (uint32_t)r, R)] = (uint32_t)k;
        } else {
            const uint32_t gp = (uint32_t)((uint64_t)(st[i + 1] - P.t_min) >> P.shift);
            for (uint32_t j = gp + 1; j <= g; ++j) pos[bnd_at<BND_TJ>(j, (uint32_t)r, R)] = (uint32_t)k;
        }
        if (is_end)
            for (uint32_t j = g + 1; j <= P.n_seg; ++j) pos[bnd_at<BND_TJ>(j, (uint32_t)r, R)] = (uint32_t)(k + 1);
    }
}

// Ordering of time segments.  Segment j of a slice holds the hits with
// t - t_min in [j << shift, (j + 1) << shift); each run contributes the stretch
// [pos[r][j], pos[r][j + 1]).  Workgroup b owns a contiguous range of the
// segment work list (consecutive segments share boundary rows in cache).  A
// segment is gathered into LDS, scattered into 256 buckets by the top 8 bits of
// its local time (LDS atomics give each hit a slot; the order within a bucket is
// then fixed by an insertion sort on (t, pmt, input index)), and written as the
// ordered structure-of-arrays at the segment's global offset.  A segment with a
// crowded bucket (a dense burst) is ordered by a stable LSD radix over 8-bit
// digits of (t << pbits | pmt) instead, then equal (t, pmt) keys are put in
// input order.
template <int NT, int CAP>
struct SegShared {
    uint32_t dt[CAP], dpq[CAP], didx[CAP];
    uint16_t perm[2][CAP];
    uint32_t run_lo[NT], run_base[NT];
    uint32_t bcount[256], bbase[256];
    RankScratch<NT> rs;
};

constexpr uint32_t BUCKET_MAX = 48;   // larger buckets take the radix path

template <int NT, int CAP>
__global__ __launch_bounds__(NT) void k_segsort(BatchDev b) {
    constexpr int E = CAP / NT;
    constexpr int GU = 4;   // gathered hits in flight per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SegShared<NT, CAP> &sm = *reinterpret_cast<SegShared<NT, CAP> *>(smem_raw);
    const uint32_t total = b.counters[Q_SEG_TOTAL_B];
    // as in the wave kernel: each XCD a contiguous eighth of the segments,
    // interleaved over its workgroups
    const uint32_t xcd = blockIdx.x % 8, wg_in_xcd = blockIdx.x / 8, wg_per_xcd = gridDim.x / 8;
    const uint32_t x0 = (uint32_t)(((uint64_t)total * xcd) / 8), x1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / 8);
    uint32_t si = 0, s_base = 1, s_end = 0;
    const TRIG_GAS uint64_t *in_pk = nullptr;
    const TRIG_GAS uint32_t *pos = nullptr;
    TRIG_GAS uint32_t *o_t = nullptr, *o_pq = nullptr, *o_idx = nullptr;
    uint32_t pbits = 0;
    Plan P = {};
    for (uint32_t item = x0 + wg_in_xcd; item < x1; item += wg_per_xcd) {
        if (item < s_base || item >= s_end) {
            si = find_slice_from(b.n_slices, si, item, [&](uint32_t i) { return b.plans[i].seg_item_base_b; });
            P = b.plans[si];
            const SliceDev &S = b.slices[si];
            in_pk = packed_hits(S); pos = gmem(S.pos);
            o_t = gmem(S.o_t); o_pq = gmem(S.o_pq); o_idx = gmem(S.o_idx); pbits = S.pbits;
            s_base = P.seg_item_base_b;
            s_end = s_base + P.n_seg;
        }
        const uint32_t j = item - s_base;
        const uint64_t R = P.n_runs;
        const uint32_t seg_lo = (uint32_t)((uint64_t)j << P.shift);
        // gather the segment's stretch of every run
        uint32_t m = 0;
        uint32_t goff_part = 0;   // this thread's share of the segment's global offset
        bool over = false;
        for (uint32_t r0 = 0; r0 < P.n_runs; r0 += NT) {
            const uint32_t r = r0 + threadIdx.x;
            uint32_t lo = 0, hi = 0;
            if (r < P.n_runs) {
                lo = pos[bnd_at<BND_TJ>(j, r, R)];
                hi = pos[bnd_at<BND_TJ>(j + 1, r, R)];
                goff_part += lo - pos[bnd_at<BND_TJ>(0, r, R)];
            }
            uint32_t cnt_tot;
            const uint32_t ex = block_excl_scan<NT>(hi - lo, cnt_tot, sm.rs.scan);
            if (m + cnt_tot > (uint32_t)CAP) { over = true; break; }
            sm.run_lo[threadIdx.x] = lo;
            sm.run_base[threadIdx.x] = ex;
            __syncthreads();
            const uint32_t nr = (P.n_runs - r0 < (uint32_t)NT) ? P.n_runs - r0 : (uint32_t)NT;
            for (uint32_t k0 = 0; k0 < cnt_tot; k0 += NT * GU) {
                uint32_t src[GU];
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const uint32_t k = k0 + u * NT + threadIdx.x;
                    src[u] = 0xFFFFFFFFu;
                    if (k < cnt_tot) {
                        uint32_t a = 0, z = nr;   // last run whose base is <= k
                        while (a < z) {
                            const uint32_t mid = (a + z) >> 1;
                            if (sm.run_base[mid] <= k) a = mid + 1; else z = mid;
                        }
                        src[u] = sm.run_lo[a - 1] + (k - sm.run_base[a - 1]);
                    }
                }
                // one packed word per hit (one stream of lines per run stretch)
                uint64_t hv[GU];
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    if (src[u] != 0xFFFFFFFFu) hv[u] = in_pk[src[u]];
                }
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    if (src[u] != 0xFFFFFFFFu) {
                        const uint32_t k = m + k0 + u * NT + threadIdx.x;
                        sm.dt[k] = (uint32_t)hv[u] - (uint32_t)(uint64_t)P.t_min;
                        sm.dpq[k] = (uint32_t)(hv[u] >> 32);
                        sm.didx[k] = src[u];
                    }
                }
            }
            m += cnt_tot;
            __syncthreads();
        }
        if (over) {
            if (threadIdx.x == 0) { b.slices[si].plan->overflow = 1u; b.slices[si].plan->state = ST_NEED_GENERIC; }
            __syncthreads();
            continue;
        }
        const uint32_t goff = block_sum<NT>(goff_part, sm.rs.scan);
        auto less = [&](uint32_t a, uint32_t c) -> bool {
            if (sm.dt[a] != sm.dt[c]) return sm.dt[a] < sm.dt[c];
            const uint32_t pa = sm.dpq[a] >> 16, pc = sm.dpq[c] >> 16;
            if (pa != pc) return pa < pc;
            return sm.didx[a] < sm.didx[c];
        };
        // bucket scatter by the top 8 bits of the local time
        const uint32_t tb = P.shift > 8 ? P.shift - 8 : 0u;
        if (threadIdx.x < 256) sm.bcount[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < m; k += NT) {
            const uint32_t d = (sm.dt[k] - seg_lo) >> tb;
            sm.perm[1][k] = (uint16_t)atomicAdd(&sm.bcount[d], 1u);
        }
        __syncthreads();
        uint32_t bc = threadIdx.x < 256 ? sm.bcount[threadIdx.x] : 0u;
        uint32_t btot;
        const uint32_t bex = block_excl_scan<NT>(bc, btot, sm.rs.scan);
        if (threadIdx.x < 256) sm.bbase[threadIdx.x] = bex;
        const int crowd = __syncthreads_or(bc > BUCKET_MAX);
        if (!crowd) {
            for (uint32_t k = threadIdx.x; k < m; k += NT) {
                const uint32_t d = (sm.dt[k] - seg_lo) >> tb;
                sm.perm[0][sm.bbase[d] + sm.perm[1][k]] = (uint16_t)k;
            }
            __syncthreads();
            if (threadIdx.x < 256 && bc > 1) {
                uint16_t *bk = sm.perm[0] + bex;
                for (uint32_t x = 1; x < bc; ++x) {
                    const uint16_t v = bk[x];
                    uint32_t y = x;
                    while (y > 0 && less(v, bk[y - 1])) { bk[y] = bk[y - 1]; --y; }
                    bk[y] = v;
                }
            }
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < m; k += NT) {
                const uint32_t v = sm.perm[0][k];
                o_t[goff + k] = sm.dt[v];
                o_pq[goff + k] = sm.dpq[v];
                o_idx[goff + k] = sm.didx[v];
            }
            __syncthreads();
            continue;
        }
        // crowded segment: stable LSD radix over the key bits
        auto keyof = [&](uint32_t v) -> uint64_t {
            return ((uint64_t)(sm.dt[v] - seg_lo) << pbits) | (uint64_t)(sm.dpq[v] >> 16);
        };
        const uint32_t key_bits = P.shift + pbits;
        const int passes = (int)((key_bits + 7) / 8);
        for (uint32_t k = threadIdx.x; k < m; k += NT) sm.perm[0][k] = (uint16_t)k;
        __syncthreads();
        int cur = 0;
        for (int ps = 0; ps < passes; ++ps) {
            const uint32_t sh8 = 8u * (uint32_t)ps;
            uint32_t rk[E], dg[E];
            block_rank8<NT, E>((int)m, [&](int k) -> uint32_t { return (uint32_t)(keyof(sm.perm[cur][k]) >> sh8) & 255u; },
                               sm.rs, rk, dg);
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
        for (uint32_t k = threadIdx.x; k < m; k += NT) {
            const uint32_t v = sm.perm[cur][k];
            const uint64_t kv = keyof(v);
            const bool tie_prev = k > 0 && keyof(sm.perm[cur][k - 1]) == kv;
            const bool tie_next = k + 1 < m && keyof(sm.perm[cur][k + 1]) == kv;
            if (!tie_prev && !tie_next) { sm.perm[cur ^ 1][k] = (uint16_t)v; continue; }
            uint32_t a = k, z = k + 1;
            while (a > 0 && keyof(sm.perm[cur][a - 1]) == kv) --a;
            while (z < m && keyof(sm.perm[cur][z]) == kv) ++z;
            uint32_t rank = 0;
            for (uint32_t u = a; u < z; ++u) rank += sm.didx[sm.perm[cur][u]] < sm.didx[v];
            sm.perm[cur ^ 1][a + rank] = (uint16_t)v;
        }
        __syncthreads();
        cur ^= 1;
        for (uint32_t k = threadIdx.x; k < m; k += NT) {
            const uint32_t v = sm.perm[cur][k];
            o_t[goff + k] = sm.dt[v];
            o_pq[goff + k] = sm.dpq[v];
            o_idx[goff + k] = sm.didx[v];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ wave per segment
// Same ordering with one wave per time segment (slices with at most WAVE_RUNS
// runs, segments of at most WAVE_CAP hits).  A wave owns a contiguous range of
// the segment work list and needs no workgroup barrier, so the waves of a CU
// overlap each other's memory latency.
//
// Gathered element k of a segment comes from run r (runs in input order, each
// run's stretch in input order), so k increases with the input index among
// hits of equal (t, pmt).  The segment is split into 256 buckets by its local
// time; the rank of element k in the segment is its bucket's base plus the
// number of bucket members that precede it in (t, pmt, k) order.

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sort key of a gathered element: local time, PMT, gather position.
constexpr int KEY_P_SHIFT = 9, KEY_T_SHIFT = 25;   // gather positions < 512, PMT ids < 2^16
constexpr uint32_t KEY_K_MASK = (1u << KEY_P_SHIFT) - 1;
static_assert(WAVE_CAP <= (1 << KEY_P_SHIFT), "gather positions must fit the key");

template <int CAP>
struct WaveSeg {
    uint64_t key[CAP];           // keys grouped by bucket, then in output order
    uint16_t dq[CAP];            // charge of each gathered element
    uint16_t aux[CAP];           // run marks while gathering, then the run of each element
    uint32_t roff[WAVE_RUNS];    // per run: its first gathered input position minus its first gathered index
    uint32_t bkt[256];           // per bucket: members counted, then base << 16 | count
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) { return wave_total(v); }

// L2 = false: single-level slices, and level 1 of two-level slices (a work item is
// a segment of one group of run_grp consecutive runs; the group's ordered hits
// go, as packed words with their input indices, to the level-1 output at the
// group's own input range).  L2 = true: level 2 of two-level slices (the
// level-1 output's stretches merged; the input index of each hit comes from the
// level-1 output).
template <int CAP, bool L2>
__global__ __launch_bounds__(256, 4) void k_segsort_w(BatchDev b) {   // 4 waves per SIMD (at most 128 VGPRs)
    constexpr int EG = CAP / 64;
    constexpr int RI = WAVE_RUNS / 64;
    static_assert((CAP & (CAP - 1)) == 0 && (WAVE_RUNS & (WAVE_RUNS - 1)) == 0, "masks below need powers of two");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int w = threadIdx.x >> 6, lane = lane_id();
    WaveSeg<CAP> &sm = reinterpret_cast<WaveSeg<CAP> *>(smem_raw)[w];
    const uint32_t total = b.counters[L2 ? Q_SEG_TOTAL2 : Q_SEG_TOTAL];
    // XCD-aware split: workgroup b runs on XCD b % 8 (round-robin dispatch), and
    // each XCD takes one contiguous eighth of the segment list, its items
    // interleaved over the XCD's waves: the segments in flight on an XCD at any
    // time are neighbours, so the cache lines they share in every run are fetched
    // into its L2 once
    const uint32_t xcd = blockIdx.x % 8, wg_in_xcd = blockIdx.x / 8, wg_per_xcd = gridDim.x / 8;
    const uint32_t x0 = (uint32_t)(((uint64_t)total * xcd) / 8), x1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / 8);
    const uint32_t nwv = wg_per_xcd * 4;
    const uint32_t gw = wg_in_xcd * 4 + (uint32_t)w;
    uint32_t si = 0, s_base = 1, s_end = 0;
    const TRIG_GAS uint64_t *in_pk = nullptr;
    const TRIG_GAS uint32_t *pos = nullptr;
    TRIG_GAS uint32_t *o_t = nullptr, *o_pq = nullptr, *o_idx = nullptr;
    TRIG_GAS uint64_t *l1_out = nullptr;
    TRIG_GAS uint32_t *l1_idx = nullptr;
    TRIG_GAS uint32_t *t2 = nullptr;   // (level 1 of a two-level slice) the level-2 table
    Plan P = {};
    // the plan fields of this launch's level
    uint32_t n_runs = 0, shift = 0, n_seg = 1;
    bool tl1 = false;   // level 1 of a two-level slice
    for (uint32_t item = x0 + gw; item < x1; item += nwv) {
        if (item < s_base || item >= s_end) {
            si = find_slice_from(b.n_slices, si, item,
                                 [&](uint32_t i) { return L2 ? b.plans[i].seg_item_base2 : b.plans[i].seg_item_base; });
            P = b.plans[si];
            const SliceDev &S = b.slices[si];
            in_pk = L2 ? level1_hits(S) : packed_hits(S);
            pos = L2 ? level2_table(S, P) : gmem(S.pos);
            o_t = gmem(S.o_t); o_pq = gmem(S.o_pq); o_idx = gmem(S.o_idx);
            l1_out = level1_hits(S);
            l1_idx = level1_index(S);
            tl1 = !L2 && P.tl;
            t2 = tl1 ? level2_table(S, P) : nullptr;
            n_runs = L2 ? P.n_runs2 : P.n_runs;
            shift = L2 ? P.shift2 : P.shift;
            n_seg = L2 ? P.n_seg2 : P.n_seg;
            s_base = L2 ? P.seg_item_base2 : P.seg_item_base;
            s_end = s_base + (tl1 ? P.n_grp * n_seg : n_seg);
        }
        if (L2 && P.state != ST_FAST) continue;   // (level 1 gave the slice up)
        const uint32_t jj = item - s_base;
        // the segment and (level 1 of a two-level slice) the group of runs
        const uint32_t grp = tl1 ? jj / n_seg : 0u;
        const uint32_t j = tl1 ? jj - grp * n_seg : jj;
        const uint32_t r_lo = tl1 ? grp * P.run_grp : 0u;
        const uint32_t r_hi = tl1 ? min(r_lo + P.run_grp, n_runs) : n_runs;
        const uint64_t R = n_runs;
        const uint32_t seg_lo = (uint32_t)((uint64_t)j << shift);
        // the segment's stretch of every run (run r = r_lo + i * 64 + lane), from
        // the segment's bounds j and j + 1 and the run starts (row 0)
        uint32_t lo[RI], hi[RI], st[RI];
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const uint32_t r = r_lo + (uint32_t)(i * 64 + lane);
            lo[i] = hi[i] = st[i] = 0;
            if (r < r_hi) {
                lo[i] = pos[bnd_at<L2 ? BND_TJ2 : BND_TJ>(j, r, R)];
                hi[i] = pos[bnd_at<L2 ? BND_TJ2 : BND_TJ>(j + 1, r, R)];
                st[i] = pos[bnd_at<L2 ? BND_TJ2 : BND_TJ>(0, r, R)];
            }
        }
        uint32_t m = 0, gpart = 0, rb[RI];
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            rb[i] = 0;
            if ((uint32_t)(i * 64) >= r_hi - r_lo) continue;   // (no run of the item in this group of 64)
            const uint32_t c = hi[i] - lo[i];
            const uint32_t incl = wave_incl_scan(c);
            const uint32_t rl = (uint32_t)(i * 64 + lane);   // run index within the item
            rb[i] = m + incl - c;
            if (r_lo + rl < r_hi) {
                sm.roff[rl] = lo[i] - rb[i];
            }
            m += lane_read(incl, 63);
            gpart += lo[i] - st[i];
        }
        // output offset: hits of the item's runs before the segment (level 1: after
        // the group's first input position, where its ordered hits go)
        const uint32_t goff = wave_sum_u32(gpart) + (tl1 ? lane_read(st[0], 0) : 0u);
        if (m > (uint32_t)CAP) {
            if (lane == 0) { b.slices[si].plan->overflow = 1u; b.slices[si].plan->state = ST_NEED_GENERIC; }
            continue;
        }
        // Every phase below reads LDS unconditionally at in-range addresses and
        // selects the result, so that the reads of a lane's EG elements are in
        // flight together rather than one round trip each.
        //
        // run marks: each non-empty run's index at its first gathered position
        // (positions past m stay 0)
#pragma unroll
        for (int e = 0; e < EG; ++e) sm.aux[e * 64 + lane] = 0;
        wave_sync();
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const uint32_t rl = (uint32_t)(i * 64 + lane);
            if (r_lo + rl < r_hi && hi[i] > lo[i]) sm.aux[rb[i]] = (uint16_t)rl;
        }
        wave_sync();
        // gather: run of element k = the largest mark at or before k (the EG
        // scans are independent; their carries are a max over earlier groups)
        uint32_t src[EG], rr[EG];
#pragma unroll
        for (int e = 0; e < EG; ++e) rr[e] = sm.aux[e * 64 + lane];
#pragma unroll
        for (int e = 0; e < EG; ++e) rr[e] = wave_incl_max_u32(rr[e]);
        {
            uint32_t carry = 0;
#pragma unroll
            for (int e = 0; e < EG; ++e) {
                const uint32_t last = lane_read(rr[e], 63);
                rr[e] = rr[e] > carry ? rr[e] : carry;
                carry = last > carry ? last : carry;
            }
        }
        // (each lane rewrites only its own marks: the run of element k, from which
        // the output recomputes the input index; rr < WAVE_RUNS for every k)
        {
            uint32_t ro[EG];
#pragma unroll
            for (int e = 0; e < EG; ++e) ro[e] = sm.roff[rr[e]];
#pragma unroll
            for (int e = 0; e < EG; ++e) {
                const uint32_t k = (uint32_t)(e * 64 + lane);
                src[e] = k < m ? ro[e] + k : 0xFFFFFFFFu;
            }
        }
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t k = (uint32_t)(e * 64 + lane);
            if (k < m) sm.aux[k] = (uint16_t)rr[e];
        }
        // one packed word per hit: a single stream of lines per run stretch
        uint64_t hv[EG];
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            hv[e] = 0;
            if (src[e] != 0xFFFFFFFFu) hv[e] = in_pk[src[e]];
        }
        // key of each element: (local time, PMT, gather position), unique and in
        // the output order; bucket by the top 8 bits of the local time
        const uint32_t tb = shift > 8 ? shift - 8 : 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) sm.bkt[lane * 4 + i] = 0;
        wave_sync();
        uint64_t key[EG];
        uint32_t slot[EG];
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t k = (uint32_t)(e * 64 + lane);
            key[e] = 0;
            slot[e] = 0;
            if (src[e] != 0xFFFFFFFFu) {
                const uint32_t tl = ((uint32_t)hv[e] - (uint32_t)(uint64_t)P.t_min) - seg_lo;
                key[e] = ((uint64_t)tl << KEY_T_SHIFT) | ((hv[e] >> 48) << KEY_P_SHIFT) | k;
                sm.dq[k] = (uint16_t)(hv[e] >> 32);
                slot[e] = atomicAdd(&sm.bkt[tl >> tb], 1u);
            }
        }
        wave_sync();
        {
            uint32_t v[4], sum = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) { v[i] = sm.bkt[lane * 4 + i]; sum += v[i]; }
            const uint32_t incl = wave_incl_scan(sum);
            uint32_t run = incl - sum;
#pragma unroll
            for (int i = 0; i < 4; ++i) { sm.bkt[lane * 4 + i] = (run << 16) | v[i]; run += v[i]; }
        }
        wave_sync();
        // keys grouped by bucket (an element without a hit reads bucket 0 and
        // takes no part: its count is 0)
        uint32_t ebase[EG], ecnt[EG], rank[EG];
        uint32_t most = 0;
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t bk = (uint32_t)(key[e] >> KEY_T_SHIFT) >> tb;
            const uint32_t wb = sm.bkt[bk];
            ebase[e] = wb >> 16;
            ecnt[e] = wb & 0xFFFFu;
        }
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            rank[e] = 0;
            if (src[e] == 0xFFFFFFFFu) ecnt[e] = 0;
            else sm.key[ebase[e] + slot[e]] = key[e];
            most = ecnt[e] > most ? ecnt[e] : most;
        }
        wave_sync();
        // rank within the bucket: the members with a smaller key (the EG reads
        // of a step are independent; past its bucket an element reads a clamped
        // address and counts nothing)
        for (uint32_t x = 0; x < most; ++x) {
            uint64_t kx[EG];
#pragma unroll
            for (int e = 0; e < EG; ++e) kx[e] = sm.key[min(ebase[e] + x, (uint32_t)CAP - 1u)];
#pragma unroll
            for (int e = 0; e < EG; ++e) rank[e] += (x < ecnt[e] && kx[e] < key[e]) ? 1u : 0u;
        }
        wave_sync();
        // keys in output order (each bucket's range rewritten by its own members)
#pragma unroll
        for (int e = 0; e < EG; ++e)
            if (ecnt[e] != 0) sm.key[ebase[e] + rank[e]] = key[e];
        wave_sync();
        // output in order: key, then the element's charge and run, then the
        // run's stretch (positions past m read stale entries, masked in range,
        // and store nothing)
        const uint32_t tm32 = (uint32_t)(uint64_t)P.t_min;
        uint64_t kk[EG];
        uint32_t dqv[EG], rv[EG], from[EG];
#pragma unroll
        for (int e = 0; e < EG; ++e) kk[e] = sm.key[e * 64 + lane];
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t k = (uint32_t)kk[e] & (uint32_t)(CAP - 1);
            dqv[e] = sm.dq[k];
            rv[e] = sm.aux[k] & (uint32_t)(WAVE_RUNS - 1);
        }
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t k = (uint32_t)kk[e] & (uint32_t)(CAP - 1);
            from[e] = sm.roff[rv[e]] + k;   // gathered position
        }
#pragma unroll
        for (int e = 0; e < EG; ++e) {
            const uint32_t i = (uint32_t)(e * 64 + lane);
            if (i < m) {
                const uint32_t p = (uint32_t)(kk[e] >> KEY_P_SHIFT) & 0xFFFFu;
                const uint32_t t_loc = seg_lo + (uint32_t)(kk[e] >> KEY_T_SHIFT);
                const uint32_t pq = (p << 16) | dqv[e];
                if (tl1) {
                    l1_out[goff + i] = ((uint64_t)pq << 32) | (uint32_t)(t_loc + tm32);
                    l1_idx[goff + i] = from[e];
                } else {
                    o_t[goff + i] = t_loc;
                    o_pq[goff + i] = pq;
                    o_idx[goff + i] = L2 ? l1_idx[from[e]] : from[e];
                }
            }
        }
        if (tl1) {
            // the level-2 boundary rows of this group that fall in the segment
            // (rows q for times q << shift2 from j << d on, through n_seg2 in the
            // last segment): row q = the first output position at or after its time
            const uint32_t d = shift - P.shift2;
            const uint32_t q_lo = j << d;
            const uint32_t q_hi = j + 1 == n_seg ? P.n_seg2 : min(((j + 1) << d) - 1u, P.n_seg2);
            const uint64_t R2 = P.n_grp;
            uint32_t carry = q_lo - 1u;   // the row of the element before (wraps for q_lo = 0)
            uint32_t last = q_lo - 1u;    // the row of the last element
#pragma unroll
            for (int e = 0; e < EG; ++e) {
                const uint32_t i = (uint32_t)(e * 64 + lane);
                const uint32_t g2 = (seg_lo + (uint32_t)(kk[e] >> KEY_T_SHIFT)) >> P.shift2;
                const uint32_t pv = wave_shr1(g2, carry);
                carry = lane_read(g2, 63);
                if (i < m)
                    for (uint32_t q = pv + 1u; q <= g2; ++q) t2[bnd_at<BND_TJ2>(q, grp, R2)] = goff + i;
                if (m && (uint32_t)e == (m - 1u) >> 6) last = lane_read(g2, (int)((m - 1u) & 63u));
            }
            for (uint32_t q = last + 1u + (uint32_t)lane; q <= q_hi; q += 64) t2[bnd_at<BND_TJ2>(q, grp, R2)] = goff + m;
        }
        wave_sync();
    }
}

template <int CAP, bool L2>
hipError_t launch_segsort_w(const BatchDev &b, const TrigLaunchCfg &cfg, hipStream_t s) {
    const size_t shm = 4 * sizeof(WaveSeg<CAP>);
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_segsort_w<CAP, L2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    const int grid = ((cfg.n_cu * cfg.persist_per_cu + 7) / 8) * 8;   // a multiple of the 8 XCDs
    hipLaunchKernelGGL((k_segsort_w<CAP, L2>), dim3(grid), dim3(256), shm, s, b);
    return hipGetLastError();
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
    const int grid = ((cfg.n_cu * cfg.persist_per_cu + 7) / 8) * 8;   // a multiple of the 8 XCDs
    hipLaunchKernelGGL((k_segsort<NT, CAP>), dim3(grid), dim3(NT), shm, s, b);
    return hipGetLastError();
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t trig_launch_front(const BatchDev &b, uint32_t seg_cap, uint32_t wave_cap, int wave_wgs_per_cu,
                             const TrigLaunchCfg &cfg,
                             hipStream_t s, void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (b.total_chunks) {
        TRIG_MARK("k_ingest", 0);
        hipLaunchKernelGGL(k_ingest, dim3(b.total_chunks), dim3(NT_ING), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_ingest", 1);
    }
    if (b.max_tiles > PL_CH) {   // (else each slice is one block, summed by k_plan itself)
        TRIG_MARK("k_psum", 0);
        hipLaunchKernelGGL(k_psum, dim3((b.max_tiles + PL_CH - 1) / PL_CH, b.n_slices), dim3(1024), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_psum", 1);
    }
    TRIG_MARK("k_plan", 0);
    hipLaunchKernelGGL(k_plan, dim3(b.n_slices), dim3(1024), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_plan", 1);
    // always launched: its extra block writes the segment counts the ordering kernels read
    TRIG_MARK("k_bounds", 0);
    hipLaunchKernelGGL(k_bounds, dim3(b.total_chunks + 1), dim3(256), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_bounds", 1);
    hipError_t e;
    TrigLaunchCfg wc = cfg;
    wc.persist_per_cu = wave_wgs_per_cu;
    if (b.sort_kernels & 1u) {
        TRIG_MARK("k_segsort_w", 0);
        // segments of slices tuned for the small variant also fit the large one
        e = wave_cap <= (uint32_t)WAVE_CAP_SMALL ? launch_segsort_w<WAVE_CAP_SMALL, false>(b, wc, s)
                                                 : launch_segsort_w<WAVE_CAP, false>(b, wc, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_segsort_w", 1);
    }
    if (b.sort_kernels & 4u) {
        // second level of the two-level slices: the merge of the groups' ordered
        // outputs (level 1 has written their boundary table)
        TRIG_MARK("k_segsort_w2", 0);
        e = wave_cap <= (uint32_t)WAVE_CAP_SMALL ? launch_segsort_w<WAVE_CAP_SMALL, true>(b, wc, s)
                                                 : launch_segsort_w<WAVE_CAP, true>(b, wc, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_segsort_w2", 1);
    }
    if (b.sort_kernels & 2u) {
        TRIG_MARK("k_segsort", 0);
        if (seg_cap <= 2048) e = launch_segsort<256, 2048>(b, cfg, s);
        else if (seg_cap <= 4096) e = launch_segsort<256, 4096>(b, cfg, s);
        else e = launch_segsort<512, 8192>(b, cfg, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_segsort", 1);
    }
    return hipSuccess;
}
