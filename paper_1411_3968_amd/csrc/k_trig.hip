// Trigger stage on the time-ordered hits of each slice:
//   L1 seeds (paper Sec. 3 and Sec. 4.2: charge over threshold, floor coincidence),
//   causal N-fold count (Sec. 3: the Cherenkov hits of one muon are correlated in
//   space and time, within less than 3 us across a tower), fires, and the merged
//   event windows (Sec. 2: a 6 us window centred on the trigger seed; Sec. 4.2:
//   +-3 us tagging around each seed).
//
// k_tile: one workgroup per ordered tile of TILE hits.  The tile and a halo of
// ordered neighbours on both sides are staged in LDS; the halo is sized from the
// slice's mean hit density so that it spans w_ns + t_floor_ns of time.  Seeds are
// marked for the whole stage, the stage's seeds are compacted in LDS, and the
// fold of each seed of the tile is counted over the compacted seeds within w_ns.
// The tile's fires go to its scratch slot, and a summary of them (TileAgg: count,
// first and last time, event starts among them, largest folds around the starts)
// to its status.  A tile whose halo does not span the window (a local burst far
// above the mean density) flags its slice for a rerun with a precomputed seed
// mask and a wider halo, where such tiles are counted from global memory.
// k_tscan: per slice, the scan of the tile summaries gives every tile the
// summary of the tiles before it.  k_place: every tile with fires writes them at
// their place in the slice's list, and writes event records in two halves: the
// tile of an event's first fire writes its start, the tile of the next event's
// first fire (or k_tscan, for the slice's last event) its end, fire count and
// largest fold.  No workgroup waits on another.
#include <algorithm>

#include "trig_dev.h"

using namespace trigdev;

namespace {

// k_tile workgroups: 512 threads when the tiles fit the GPU in one wave of
// workgroups (lower latency per tile), else 256 (more tiles per CU in flight)
constexpr int NT_ONE_WAVE = 512, NT_MANY = 256;
constexpr int FLOOR_LDS_MAX = 4096;   // floor numbering kept in LDS up to this many PMTs

// Seeds of one stage that the compacted lists hold: a fraction of the stage in
// the first pass (seeds are a few per cent of the hits; a stage with more is
// rerun with the mask), every hit in the rerun.
__host__ __device__ constexpr int compact_cap(int hmax, bool mask) { return mask ? TILE + 2 * hmax : 512; }

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) { return wave_max_all(v); }

// LDS written by some lanes of a wave, then read by others of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ TileAgg agg_empty() {
    TileAgg a;
    a.F = a.S = a.E_int = a.first_t = a.last_t = a.m_head = a.m_tail = a.ls_t = 0;
    a.ls_idx = NO_START;
    return a;
}

// Summary of run A followed by run B (twoH: the merge distance 2H).  Associative.
__device__ __forceinline__ TileAgg agg_combine(const TileAgg &A, const TileAgg &B, uint64_t twoH) {
    // field by field, with selects: a branch between whole summaries makes the
    // compiler pick one of the two addresses, which sends the summaries to
    // private memory when one lives in LDS
    const bool a0 = A.F == 0, b0 = B.F == 0;   // A empty: B; B empty: A (seed counts add)
    const bool bs = !a0 && !b0 && (uint64_t)(B.first_t - A.last_t) > twoH;
    TileAgg r;
    r.F = A.F + B.F;
    r.S = A.S + B.S;
    r.first_t = a0 ? B.first_t : A.first_t;
    r.last_t = (b0 && !a0) ? A.last_t : B.last_t;
    const uint32_t e_int = A.E_int + B.E_int + (bs ? 1u : 0u);
    const uint32_t m_head = (A.E_int > 0 || bs) ? A.m_head : umax(A.m_head, B.m_head);
    const uint32_t m_tail = (B.E_int > 0 || bs) ? B.m_tail : umax(A.m_tail, B.m_tail);
    const uint32_t ls_idx = B.E_int > 0 ? A.F + B.ls_idx : bs ? A.F : A.ls_idx;
    const uint32_t ls_t = B.E_int > 0 ? B.ls_t : bs ? B.first_t : A.ls_t;
    r.E_int = a0 ? B.E_int : b0 ? A.E_int : e_int;
    r.m_head = a0 ? B.m_head : b0 ? A.m_head : m_head;
    r.m_tail = a0 ? B.m_tail : b0 ? A.m_tail : m_tail;
    r.ls_idx = a0 ? B.ls_idx : b0 ? A.ls_idx : ls_idx;
    r.ls_t = a0 ? B.ls_t : b0 ? A.ls_t : ls_t;
    return r;
}

// Index (within the slice's fire list) of the first fire of the last event of
// a prefix summary.
__device__ __forceinline__ uint32_t open_start(const TileAgg &P) { return P.ls_idx == NO_START ? 0u : P.ls_idx; }


// Staged words pmt << 16 | floor: another PMT on the same floor.
__device__ __forceinline__ bool floor_partner(uint32_t a, uint32_t b) {
    return (a >> 16) != (b >> 16) && (a & 0xFFFFu) == (b & 0xFFFFu);
}

__device__ __forceinline__ bool mask_bit(const SliceDev &S, uint64_t j) { return (S.dmask[j >> 6] >> (j & 63)) & 1ull; }

__device__ __forceinline__ uint32_t lim_global(const SliceDev &S, uint32_t W, uint32_t p, uint32_t q) {
    const uint64_t x = (uint64_t)p * S.n_pmt + q;
    const uint32_t v = (W <= 65535u) ? (uint32_t)S.thr16[x] : S.thr32[x];
    return v < W ? v : W;
}

// Fold of seed j (time t, PMT p) counted from global memory with the seed mask.
__device__ uint32_t fold_global(const SliceDev &S, uint32_t W, uint64_t j, uint32_t t, uint32_t p) {
    uint32_t c = 1;
    for (uint64_t m = j; m > 0;) {
        --m;
        const uint32_t d = t - S.o_t[m];
        if (d > W) break;
        const uint32_t q = S.o_pq[m] >> 16;
        if (d <= lim_global(S, W, p, q) && mask_bit(S, m)) ++c;
    }
    for (uint64_t m = j + 1; m < S.n; ++m) {
        const uint32_t d = S.o_t[m] - t;
        if (d > W) break;
        const uint32_t q = S.o_pq[m] >> 16;
        if (d <= lim_global(S, W, p, q) && mask_bit(S, m)) ++c;
    }
    return c;
}

// Plans of slices whose trigger stage does not run in this pass (errors, empty
// slices, general ordering pending) go to the host as they are.
__device__ __forceinline__ bool export_as_is(uint32_t state) {
    return state != ST_FAST && state != ST_GENERIC_DONE && state != ST_DENSE;
}

// LDS bytes of a tile's stage and lists (the per-PMT tables come after them).
template <int HMAX, bool MASK>
constexpr size_t tile_lds_bytes() {
    constexpr size_t STG = TILE + 2 * HMAX, CS = compact_cap(HMAX, MASK);
    return STG * 4 * 2 + CS * 4 * 2 + (STG / 64) * 8 * 2 + (STG / 64 + 1) * 4 + CS * 2 * 3;
}

template <int NT, int HMAX, bool MASK, bool MENU>
__global__ __launch_bounds__(NT) void k_tile(BatchDev b, uint32_t floor_lds) {
    constexpr int NW = NT / 64;
    constexpr int STG = TILE + 2 * HMAX;
    constexpr int CS = compact_cap(HMAX, MASK);      // seeds of a stage the compacted lists hold
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *st = (uint32_t *)smem;                 // staged t - t_min
    uint32_t *spf = st + STG;                        // staged pmt << 16 | dense floor index
    uint32_t *ct = spf + STG;                        // compacted seeds: time
    uint32_t *fold = ct + CS;                        // fold of each seed of the tile
    uint64_t *sbits = (uint64_t *)(fold + CS);       // seed bits of the stage
    uint64_t *l0w = sbits + STG / 64;                // level-0 pass bits of the stage (level 0 on)
    uint32_t *wpre = (uint32_t *)(l0w + STG / 64);   // seeds before each 64-hit word
    uint16_t *cp = (uint16_t *)(wpre + STG / 64 + 1);   // compacted seeds: PMT
    uint16_t *cidx = cp + CS;                        // compacted seeds: stage position
    uint16_t *fci = cidx + CS;                       // fires: compacted index
    uint16_t *lfl = fci + CS;                        // dense floor index of every PMT (floor_lds of them)
    // seed menu: adjacency group and floor rank of every PMT (floor_lds of each)
    uint32_t *ladj = (uint32_t *)(smem + tile_lds_bytes<HMAX, MASK>() + ((floor_lds * 2 + 15) & ~15u));
    uint32_t *lafl = ladj + floor_lds;
    // seed menu: the same two per staged hit, so the partner search reads no table
    uint32_t *hadj = lafl + floor_lds;
    uint32_t *hafl = hadj + STG;
    __shared__ uint32_t sh[NW + 1];
    __shared__ uint32_t s_ncs, s_ca, s_cb;

    // XCD-aware order: workgroup b runs on XCD b % 8 and takes tiles from that
    // XCD's contiguous eighth of the list, so neighbouring tiles share their halos
    // in one L2
    const uint32_t per_xcd = (b.total_tiles + 7) / 8;
    const uint32_t item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (item >= b.total_tiles) return;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return;
    // (the plan by its index, in flight with the descriptor; generic: the flag
    // updates below are atomics)
    Plan *Pp = b.plans + si;
    const TRIG_GAS Plan *Pg = gmem(Pp);
    if (!slice_in_tail(b, Pg->state)) return;
    // descriptor fields read once, as global-memory pointers
    const TRIG_GAS uint32_t *o_t = gmem(S.o_t);
    const TRIG_GAS uint32_t *o_pq = gmem(S.o_pq);
    const TRIG_GAS uint32_t *o_idx = gmem(S.o_idx);
    const TRIG_GAS uint16_t *thr16 = gmem(S.thr16);
    const TRIG_GAS uint32_t *thr32 = gmem(S.thr32);
    const TRIG_GAS uint16_t *floor16 = gmem(S.floor16);
    TRIG_GAS uint8_t *seed_flags = gmem(S.seed_flags);
    const TRIG_GAS uint32_t *adj32 = gmem(S.adj32);
    const TRIG_GAS uint32_t *afl32 = gmem(S.afl32);
    const uint32_t n_pmt = S.n_pmt;
    const uint64_t n = S.n;
    const int64_t t_min = Pg->t_min;
    const uint64_t span = (uint64_t)(Pg->t_max - t_min);
    const uint32_t W = b.prm.w_ns;
    const uint32_t N = b.prm.min_fold;
    const int32_t tau = b.prm.t_floor_ns;
    // the seed menu (adjacent PMTs, consecutive floors, the combination): its
    // widest window sets the reach of the partner search
    const int32_t t_sc = b.prm.t_adj_ns, t_afc = b.prm.t_afloor_ns;
    constexpr bool menu = MENU && !MASK;   // a variant of its own: the plain rule keeps its registers
    const bool mode1 = b.prm.seed_mode == 1;
    const int32_t tmax = menu ? max(tau, max(t_sc, t_afc)) : tau;
    const uint32_t tau_u = tmax > 0 ? (uint32_t)tmax : 0u;
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const int lane = lane_id(), w = threadIdx.x >> 6;

    const uint64_t a = (uint64_t)k * TILE;
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    // halo: twice the mean number of hits in w_ns + t_floor_ns, plus a margin
    const uint64_t reach = (uint64_t)W + tau_u;
    uint64_t halo = (2ull * n * reach) / (span + 1) + 64;
    if (halo > (uint64_t)HMAX) halo = HMAX;
    const uint64_t sl = a > halo ? a - halo : 0;
    const uint64_t sh_end = (e + halo < n) ? e + halo : n;
    const uint32_t len = (uint32_t)(sh_end - sl);
    const uint32_t q_seed = b.prm.q_seed;
    // level 0 on: only hits that pass it may be seeds or floor partners
    const bool L0 = !MASK && b.prm.l0_n > 0;
    const TRIG_GAS uint64_t *l0m = gmem(S.l0m);
    {
        // stage the times and PMTs with all loads of a thread in flight
        constexpr int U = (STG + NT - 1) / NT;
        uint32_t vt[U], vp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = u * NT + threadIdx.x;
            if (x < len) {
                vt[u] = o_t[sl + x];
                vp[u] = o_pq[sl + x];
            }
        }
        // the floor numbering (independent of the staged hits, so in flight with them)
        if (!MASK && n_pmt <= floor_lds)
            for (uint32_t x = threadIdx.x; x < n_pmt; x += NT) {
                lfl[x] = floor16[x];
                if (MENU) {
                    ladj[x] = adj32[x];
                    lafl[x] = afl32[x];
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = u * NT + threadIdx.x;
            if (x < len) st[x] = vt[u];
            if (!MASK) {
                // charge seeds of the stage, a word per wave (the floor coincidences
                // are added below); x / 64 is this wave's word
                bool l0x = x < len;
                if (L0 && x < len) {
                    const uint64_t j = sl + x;
                    l0x = (l0m[j >> 6] >> (j & 63)) & 1ull;
                }
                const uint64_t lb = __ballot(l0x);
                const uint64_t qb = __ballot(x < len && (vp[u] & 0xFFFFu) >= q_seed) & lb;
                if (lane == 0 && u * NT + w * 64 < len) {
                    sbits[(u * NT) / 64 + w] = qb;
                    l0w[(u * NT) / 64 + w] = lb;
                }
            }
        }
        if (!MASK) __syncthreads();   // floor numbering complete
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = u * NT + threadIdx.x;
            if (x < len) {
                const uint32_t p = vp[u] >> 16;
                uint32_t f = 0;
                if (!MASK) f = n_pmt <= floor_lds ? (uint32_t)lfl[p] : (uint32_t)floor16[p];
                spf[x] = (p << 16) | f;
                if (menu) {
                    if (n_pmt <= floor_lds) {
                        hadj[x] = ladj[p];
                        hafl[x] = lafl[p];
                    } else {
                        hadj[x] = adj32[p];
                        hafl[x] = afl32[p];
                    }
                }
            }
        }
    }
    __syncthreads();
    const uint32_t ta = st[a - sl], te = st[e - 1 - sl];
    // the stage spans the window of every seed of the tile when the halo reaches
    // past w_ns + t_floor_ns on both sides (or the slice ends there)
    const bool cover_l = sl == 0 || (uint64_t)st[0] + reach < (uint64_t)ta;
    const bool cover_r = sh_end == n || (uint64_t)st[len - 1] > (uint64_t)te + reach;
    uint32_t ca = 0, cb = 0;
    uint64_t cbase = a;
    const bool covered = cover_l && cover_r;
    bool fits = true;
    if (covered) {
        cbase = sl;
        // seed bits of the whole stage
        // (level 0 on: a partner must pass it, and so must the hit)
        auto l0b = [&](uint32_t y) -> bool { return !L0 || ((l0w[y >> 6] >> (y & 63)) & 1ull); };
        for (uint32_t x0 = 0; x0 < len; x0 += NT) {
            const uint32_t x = x0 + threadIdx.x;
            bool seed = false;
            if (MASK) {
                seed = x < len && mask_bit(S, sl + x);
            } else if (menu) {
                if (x < len && tmax >= 0 && l0b(x)) {   // (a hit failing level 0 is no seed)
                    // FC, SC and AFC partners within the widest window, both sides
                    const uint32_t t = st[x], f = spf[x], p = f >> 16, fl = f & 0xFFFFu;
                    const uint32_t ak = hadj[x], rk = hafl[x];
                    // found rules as bits (1 FC, 2 SC, 4 AFC), kept in a register: a
                    // window below zero is off (its limit 0 admits nothing)
                    const uint32_t lim_fc = tau >= 0 ? (uint32_t)tau + 1u : 0u;
                    const uint32_t lim_sc = t_sc >= 0 ? (uint32_t)t_sc + 1u : 0u;
                    const uint32_t lim_afc = t_afc >= 0 ? (uint32_t)t_afc + 1u : 0u;
                    auto look = [&](bool in, uint32_t dt, uint32_t g, uint32_t y, uint32_t am, uint32_t rm) -> uint32_t {
                        const bool ok = in & ((g >> 16) != p) & l0b(y);
                        const bool same = (g & 0xFFFFu) == fl;
                        const bool nb = (rm == rk + 1u) | (rm + 1u == rk);
                        return (uint32_t)(ok & same & (dt < lim_fc)) | ((uint32_t)(ok & same & (dt < lim_sc) & (am == ak)) << 1) |
                               ((uint32_t)(ok & !same & (dt < lim_afc) & nb) << 2);
                    };
                    auto done = [&](uint32_t m) -> bool { return mode1 ? ((m & 3u) != 0u && (m & 4u) != 0u) : m != 0u; };
                    uint32_t m = 0;
                    // one step looks at the neighbours d positions away on both sides;
                    // every read of a step is issued together (clamped positions)
                    for (uint32_t d = 1;; ++d) {
                        const uint32_t yl = x >= d ? x - d : x, yr = x + d < len ? x + d : x;
                        const uint32_t tl = st[yl], tr = st[yr], gl = spf[yl], gr = spf[yr];
                        const uint32_t al = hadj[yl], ar = hadj[yr], rl = hafl[yl], rr_ = hafl[yr];
                        const bool ll = (x >= d) & (t - tl <= tau_u);
                        const bool rr = (x + d < len) & (tr - t <= tau_u);
                        if (!ll && !rr) break;
                        m |= look(ll, t - tl, gl, yl, al, rl) | look(rr, tr - t, gr, yr, ar, rr_);
                        if (done(m)) break;
                    }
                    seed = done(m);
                }
            } else if (tau >= 0 && x < len) {
                // floor coincidence: a hit of another PMT on the same floor within
                // t_floor_ns.  The nearest neighbours on both sides are read together;
                // a hit with a closer non-partner looks further.
                const uint32_t xl = x ? x - 1 : 0, xr = x + 1 < len ? x + 1 : x;
                const uint32_t t = st[x], f = spf[x];
                const uint32_t tl = st[xl], fl = spf[xl], tr = st[xr], fr = spf[xr];
                // (bitwise operators: no branch between the reads and their use)
                const bool l_in = (x >= 1) & (t - tl <= tau_u);
                const bool r_in = (x + 1 < len) & (tr - t <= tau_u);
                seed = (l_in & floor_partner(fl, f) & l0b(xl)) | (r_in & floor_partner(fr, f) & l0b(xr));
                if (!seed && (l_in || r_in)) {
                    for (uint32_t d = 2;; ++d) {
                        const bool ll = x >= d && t - st[x - d] <= tau_u;
                        const bool rr = x + d < len && st[x + d] - t <= tau_u;
                        if (!ll && !rr) break;
                        if ((ll && floor_partner(spf[x - d], f) && l0b(x - d)) ||
                            (rr && floor_partner(spf[x + d], f) && l0b(x + d))) {
                            seed = true;
                            break;
                        }
                    }
                }
                seed = seed && l0b(x);
            }
            const uint64_t bal = __ballot(seed);
            if (lane == 0 && x0 + w * 64 < len) {
                if (MASK) sbits[x0 / 64 + w] = bal;
                else sbits[x0 / 64 + w] |= bal;
            }
        }
        __syncthreads();
        const uint32_t nwords = (len + 63) / 64;
        if (w == 0) {
            // word prefixes (one lane per word)
            uint32_t tot = 0;
            for (uint32_t w0 = 0; w0 < nwords; w0 += 64) {
                const uint32_t wd = w0 + lane;
                const uint32_t c = wd < nwords ? (uint32_t)__popcll(sbits[wd]) : 0u;
                const uint32_t inc = wave_incl_scan(c);
                if (wd < nwords) wpre[wd] = tot + inc - c;
                tot += lane_read(inc, 63);
            }
            if (lane == 0) {
                wpre[nwords] = tot;
                s_ncs = tot;
            }
        }
        __syncthreads();
        fits = s_ncs <= (uint32_t)CS;
    }
    if (covered && !fits) {
        // more seeds in the stage than the compacted lists hold: rerun with a mask
        if (threadIdx.x == 0) atomicOr(&Pp->dense, 1u);
    } else if (covered) {
        const uint32_t nwords = (len + 63) / 64;
        // seeds before the tile and before its end
        if (threadIdx.x < 2) {
            const uint32_t x = (uint32_t)((threadIdx.x == 0 ? a : e) - sl);
            const uint32_t wd = x / 64, bit = x % 64;
            const uint64_t word = wd < nwords ? sbits[wd] : 0ull;
            const uint32_t v = wpre[wd] + (uint32_t)__popcll(bit ? word & (~0ull >> (64 - bit)) : 0ull);
            if (threadIdx.x == 0) s_ca = v; else s_cb = v;
        }
        // compacted seeds of the stage (time order kept)
        for (uint32_t x = threadIdx.x; x < len; x += NT) {
            const uint64_t word = sbits[x / 64];
            const uint32_t bit = x % 64;
            if ((word >> bit) & 1ull) {
                const uint32_t r = wpre[x / 64] + (uint32_t)__popcll(bit ? word & (~0ull >> (64 - bit)) : 0ull);
                ct[r] = st[x];
                cp[r] = (uint16_t)(spf[x] >> 16);
                cidx[r] = (uint16_t)x;
            }
        }
        __syncthreads();
        ca = s_ca;
        cb = s_cb;
        const uint32_t ncs = s_ncs;
        // causal fold of each seed of the tile over the compacted seeds within
        // w_ns: G lanes per seed split its window (bounds by binary search in the
        // time-ordered seeds), each with CB table lookups in flight (the thr table
        // is read through the caches)
        constexpr int G = 4, CB = 8;
        const bool t16 = W <= 65535u;
        const uint32_t sub = threadIdx.x % G;
        for (uint32_t ci = ca + threadIdx.x / G; ci < cb; ci += NT / G) {
            const uint32_t t = ct[ci];
            const uint64_t row = (uint64_t)cp[ci] * n_pmt;
            const uint32_t t_lo = t > W ? t - W : 0u;
            const uint64_t t_hi = (uint64_t)t + W;
            uint32_t jl = 0, z = ci;          // first seed with time >= t - W
            while (jl < z) {
                const uint32_t mid = (jl + z) >> 1;
                if (ct[mid] < t_lo) jl = mid + 1; else z = mid;
            }
            uint32_t jr = ci + 1;
            z = ncs;                          // first seed with time > t + W
            while (jr < z) {
                const uint32_t mid = (jr + z) >> 1;
                if ((uint64_t)ct[mid] <= t_hi) jr = mid + 1; else z = mid;
            }
            uint32_t c = 0;
            for (uint32_t j0 = jl + sub; j0 < jr; j0 += G * CB) {
                uint32_t lim[CB], dd[CB];
#pragma unroll
                for (int u = 0; u < CB; ++u) {
                    const uint32_t j = j0 + u * G;
                    dd[u] = 0xFFFFFFFFu;
                    lim[u] = 0;
                    if (j < jr && j != ci) {
                        const uint32_t tj = ct[j];
                        dd[u] = tj > t ? tj - t : t - tj;
                        lim[u] = t16 ? (uint32_t)thr16[row + cp[j]] : thr32[row + cp[j]];
                    }
                }
#pragma unroll
                for (int u = 0; u < CB; ++u) c += dd[u] <= (lim[u] < W ? lim[u] : W);
            }
            // sum over the G = 4 lanes of the seed (quad permutations: lane ^ 1, lane ^ 2)
            c += dpp_u32<0xB1, 0xF>(0u, c);
            c += dpp_u32<0x4E, 0xF>(0u, c);
            if (sub == 0) fold[ci - ca] = c + 1;
        }
        if (seed_flags) {
            for (uint64_t j = a + threadIdx.x; j < e; j += NT) {
                const uint32_t x = (uint32_t)(j - sl);
                seed_flags[o_idx[j]] = (uint8_t)((sbits[x / 64] >> (x % 64)) & 1ull);
            }
        }
    } else if (!MASK) {
        // a window beyond the staged halo: this pass leaves the tile empty and the
        // slice is rerun with a seed mask
        if (threadIdx.x == 0) atomicOr(&Pp->dense, 1u);
    } else if (!covered) {
        // seeds from the mask, folds of the tile from global memory
        uint32_t acc = 0;
        for (uint64_t j0 = a; j0 < e; j0 += NT) {
            const uint64_t j = j0 + threadIdx.x;
            const bool seed = j < e && mask_bit(S, j);
            uint32_t tot;
            const uint32_t ex = block_excl_scan<NT>(seed ? 1u : 0u, tot, sh);
            if (seed) {
                ct[acc + ex] = o_t[j];
                cp[acc + ex] = (uint16_t)(o_pq[j] >> 16);
                cidx[acc + ex] = (uint16_t)(j - a);
            }
            if (j < e && seed_flags) seed_flags[o_idx[j]] = seed ? 1 : 0;
            acc += tot;
        }
        __syncthreads();
        cb = acc;
        for (uint32_t ci = threadIdx.x; ci < cb; ci += NT)
            fold[ci] = fold_global(S, W, a + cidx[ci], ct[ci], cp[ci]);
    }
    __syncthreads();
    // fires of the tile in order, to the tile's scratch slot
    uint32_t nf = 0;
    TRIG_GAS FireRec *slot = gmem(S.fsc) + (uint64_t)k * TILE;
    for (uint32_t c0 = ca; c0 < cb; c0 += NT) {
        const uint32_t ci = c0 + threadIdx.x;
        const bool f = ci < cb && fold[ci - ca] >= N;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NT>(f ? 1u : 0u, tot, sh);
        if (f) {
            fci[nf + ex] = (uint16_t)ci;
            FireRec fr;
            fr.t = ct[ci];
            fr.hit = o_idx[cbase + cidx[ci]];
            fr.fold = fold[ci - ca];
            fr.pmt = cp[ci];
            gstore(slot + nf + ex, fr);
        }
        nf += tot;
    }
    __syncthreads();
    if (w != 0) return;
    // summary of this tile's fires (wave 0)
    TileAgg A = agg_empty();
    A.S = cb - ca;
    A.F = nf;
    uint32_t prev_t = 0, first_int = NO_START, last_int = NO_START, m_head = 0, m_tail = 0;
    for (uint32_t r0 = 0; r0 < nf; r0 += 64) {
        const uint32_t r = r0 + lane;
        const bool v = r < nf;
        uint32_t t = 0, fd = 0;
        if (v) {
            const uint32_t ci = fci[r];
            t = ct[ci];
            fd = fold[ci - ca];
        }
        // the lane move runs in every lane (under a select it would run with lane 0
        // masked off, and lane 1 would read the fill value)
        const uint32_t t_below = wave_shr1(t, 0u);
        const uint32_t tp = lane == 0 ? prev_t : t_below;
        const bool is_int = v && r > 0 && (uint64_t)(t - tp) > twoH;
        const uint64_t ib = __ballot(is_int);
        if (r0 == 0) A.first_t = lane_read(t, 0);
        prev_t = lane_read(t, 63);
        if (ib) {
            const int lo = __ffsll((unsigned long long)ib) - 1;
            const int hi = 63 - __clzll((long long)ib);
            if (first_int == NO_START) {
                first_int = r0 + lo;
                m_head = umax(m_head, wave_max_u32(v && lane < lo ? fd : 0u));
            }
            last_int = r0 + hi;
            m_tail = wave_max_u32(v && lane >= hi ? fd : 0u);
            A.ls_t = lane_read(t, hi);
        } else {
            const uint32_t mx = wave_max_u32(v ? fd : 0u);
            if (first_int == NO_START) m_head = umax(m_head, mx);
            m_tail = umax(m_tail, mx);
        }
        A.E_int += (uint32_t)__popcll(ib);
    }
    if (nf) A.last_t = ct[fci[nf - 1]];
    A.m_tail = m_tail;
    A.m_head = first_int == NO_START ? m_tail : m_head;
    A.ls_idx = last_int;
    if (last_int == NO_START) A.ls_t = 0;
    if (lane == 0) gstore(&gmem(S.tstat)[k].agg, A);
}

// Tile scan, in chunks of TS_CH tiles of one slice (grid: chunks x slices), 256
// threads of four tiles each.  k_tsum (launched when a slice has more than one
// chunk): each chunk's combined summary.  k_tscan: each chunk combines the
// summaries of the chunks before it, then scans its tiles: every tile gets the
// summary of the tiles of the slice before it; the last chunk ends with the whole
// slice: its counts, the end of its last event, and the plan to host-mapped
// staging.
constexpr int TS_NT = 256;
constexpr int TS_PT = (int)TS_CH / TS_NT;   // tiles per thread

// Summary of this thread's tiles of chunk c, with the tiles' own summaries.
__device__ __forceinline__ TileAgg tscan_thread(const TRIG_GAS TileStat *tstat, uint32_t t0, uint32_t nt,
                                                uint64_t twoH, TileAgg (&x)[TS_PT]) {
    TileAgg mine = agg_empty();
#pragma unroll
    for (int u = 0; u < TS_PT; ++u) x[u] = t0 + u < nt ? gload(&tstat[t0 + u].agg) : agg_empty();
#pragma unroll
    for (int u = 0; u < TS_PT; ++u) mine = agg_combine(mine, x[u], twoH);
    return mine;
}

__global__ __launch_bounds__(TS_NT) void k_tsum(BatchDev b) {
    constexpr int NW = TS_NT / 64;
    const uint32_t si = blockIdx.y, c = blockIdx.x;
    const SliceDev &S = b.slices[si];
    const uint32_t nt = S.n_tiles;
    if ((uint64_t)c * TS_CH >= nt) return;
    if (!slice_in_tail(b, gmem(b.plans + si)->state)) return;
    __shared__ TileAgg wsum[NW];
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    TileAgg x[TS_PT];
    const TileAgg mine = tscan_thread(gmem(S.tstat), c * TS_CH + threadIdx.x * TS_PT, nt, twoH, x);
    const TileAgg inc = wave_scan(mine, agg_empty(), [&](const TileAgg &p, const TileAgg &q) { return agg_combine(p, q, twoH); });
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        TileAgg t = wsum[0];
        for (int i = 1; i < NW; ++i) t = agg_combine(t, wsum[i], twoH);
        gstore(gmem(S.cagg) + c, t);
    }
}

__global__ __launch_bounds__(TS_NT) void k_tscan(BatchDev b) {
    constexpr int NW = TS_NT / 64;
    const uint32_t si = blockIdx.y, c = blockIdx.x;
    const SliceDev &S = b.slices[si];
    const uint32_t nt = S.n_tiles;
    if ((uint64_t)c * TS_CH >= nt) return;
    TRIG_GAS Plan *Pp = gmem(b.plans + si);
    TRIG_GAS TileStat *tstat = gmem(S.tstat);
    __shared__ TileAgg wpre[NW + 1];
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t nch = (nt + TS_CH - 1) / TS_CH;
    // the tile summaries are read in flight with the plan state (they are only
    // used when the slice is in this pass)
    TileAgg x[TS_PT];
    const uint32_t t0 = c * TS_CH + threadIdx.x * TS_PT;
    const TileAgg mine = tscan_thread(tstat, t0, nt, twoH, x);
    const uint32_t state = Pp->state;
    if (!slice_in_tail(b, state)) {
        if (c == 0 && threadIdx.x == 0 && b.x_plans && export_as_is(state)) gstore(gmem(b.x_plans) + si, gload(Pp));
        return;
    }
    // the chunks before this one, combined in order by the first wave (64 at a time)
    if (w == 0) {
        TileAgg P0 = agg_empty();
        for (uint32_t c0 = 0; c0 < c; c0 += 64) {
            const uint32_t ci = c0 + (uint32_t)lane;
            const TileAgg v = ci < c ? gload(gmem(S.cagg) + ci) : agg_empty();
            const TileAgg vi = wave_scan(v, agg_empty(), [&](const TileAgg &p, const TileAgg &q) { return agg_combine(p, q, twoH); });
            P0 = agg_combine(P0, lane_read_all(vi, 63), twoH);
        }
        if (lane == 0) wpre[NW] = P0;
    }
    // inclusive scan within the wave
    const TileAgg inc = wave_scan(mine, agg_empty(), [&](const TileAgg &p, const TileAgg &q) { return agg_combine(p, q, twoH); });
    if (lane == 63) wpre[w] = inc;
    __syncthreads();
    // the waves before this one, after the chunks before this one
    TileAgg before = wpre[NW];
    for (int i = 0; i < w; ++i) before = agg_combine(before, wpre[i], twoH);
    TileAgg P = agg_combine(before, wave_shr1(inc, agg_empty()), twoH);
#pragma unroll
    for (int u = 0; u < TS_PT; ++u) {
        if (t0 + u < nt) gstore(&tstat[t0 + u].pre, P);
        P = agg_combine(P, x[u], twoH);
    }
    if (c != nch - 1 || threadIdx.x != TS_NT - 1) return;
    const TileAgg I = P;   // the last thread of the last chunk ends with the whole slice
    const uint32_t n_ev = I.F ? 1 + I.E_int : 0u;
    const int64_t H = (int64_t)b.prm.half_event_ns;
    const int64_t t_min = Pp->t_min;
    if (I.F && !(Pp->dense && b.tail_state != ST_DENSE)) {
        // the slice's last event ends at its last fire
        const uint32_t le = n_ev - 1, s0 = open_start(I);
        const int64_t tend = t_min + (int64_t)I.last_t + H;
        TRIG_GAS trig_event *events = gmem(S.events);
        events[le].t_end = tend;
        events[le].n_fire = I.F - s0;
        events[le].max_fold = I.m_tail;
        if (S.x_events && n_ev <= S.x_event_cap) {
            TRIG_GAS trig_event *xe = gmem(S.x_events);
            xe[le].t_end = tend;
            xe[le].n_fire = I.F - s0;
            xe[le].max_fold = I.m_tail;
        }
    }
    Pp->n_seeds = I.S;
    Pp->n_fires = I.F;
    Pp->n_events = n_ev;
    if (b.x_plans) gstore(gmem(b.x_plans) + si, gload(Pp));
}

// Segmented max: (a segment starts here, running max since the last start).
struct SegMax {
    uint32_t f, v;
};

// One tile with fires (nf of them), by one wave with every lane active: fire
// records and event halves at their places.
__device__ void place_tile(const BatchDev &b, const SliceDev &S, const TRIG_GAS Plan *Pp, uint32_t k, uint32_t nf) {
    const TRIG_GAS TileStat *tstat = gmem(S.tstat);
    const TileAgg P = gload(&tstat[k].pre);
    const TRIG_GAS FireRec *slot = gmem(S.fsc) + (uint64_t)k * TILE;
    TRIG_GAS trig_fire *fires = gmem(S.fires);
    TRIG_GAS trig_event *events = gmem(S.events);
    const int lane = lane_id();
    const int64_t t_min = Pp->t_min;
    const int64_t H = (int64_t)b.prm.half_event_ns;
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const uint32_t EP = P.F ? 1 + P.E_int : 0u;       // events begun before this tile
    const uint32_t p_open = open_start(P);
    // host-mapped staging only when the whole list fits it (else the host copies
    // the list from device memory)
    TRIG_GAS trig_fire *xf = (S.x_fires && Pp->n_fires <= S.x_fire_cap) ? gmem(S.x_fires) : nullptr;
    TRIG_GAS trig_event *xe = (S.x_events && Pp->n_events <= S.x_event_cap) ? gmem(S.x_events) : nullptr;
    uint32_t carry_starts = 0;                       // starts among earlier fires of the tile
    int32_t carry_latest = -1;                       // local index of the latest start, -1: none
    uint32_t carry_max = P.F ? P.m_tail : 0u;        // largest fold of the open event so far
    uint32_t prev_t = P.F ? P.last_t : 0u;
    for (uint32_t r0 = 0; r0 < nf; r0 += 64) {
        const uint32_t r = r0 + lane;
        const bool v = r < nf;
        FireRec fr = {0, 0, 0, 0};
        if (v) fr = gload(slot + r);
        // (lane 63) the next round's first fire time, read with this round's fires
        const uint32_t t_after = (lane == 63 && r + 1 < nf) ? slot[r + 1].t : 0u;
        const uint32_t t = fr.t, fd = fr.fold;
        // the lane moves run in every lane (under a select they would run with
        // lanes masked off, and their neighbours would read the fill value)
        const uint32_t t_below = wave_shr1(t, 0u);
        const uint32_t t_next = wave_shl1(t, t_after);   // the next fire's time
        const uint32_t tp = lane == 0 ? prev_t : t_below;
        const bool first_of_slice = r == 0 && P.F == 0;
        const bool st = v && (first_of_slice || (uint64_t)(t - tp) > twoH);
        const uint64_t sb = __ballot(st);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const uint32_t starts_incl = carry_starts + (uint32_t)__popcll(sb & upto);
        const uint64_t sbu = sb & upto;
        const int32_t latest = sbu ? (int32_t)(r0 + 63 - __clzll((long long)sbu)) : carry_latest;
        // segmented inclusive max of the folds (segments begin at starts)
        SegMax sm0;
        sm0.f = st ? 1u : 0u;
        sm0.v = fd;
        SegMax id0;
        id0.f = id0.v = 0;
        const SegMax sx = wave_scan(sm0, id0, [](const SegMax &x, const SegMax &y) {
            SegMax z;
            z.f = x.f | y.f;
            z.v = y.f ? y.v : umax(x.v, y.v);
            return z;
        });
        uint32_t mv = sx.v;
        if (!sx.f) mv = umax(mv, carry_max);
        const uint32_t ev = EP + starts_incl - 1;   // event of fire r
        if (v) {
            trig_fire out;
            out.t_ns = t_min + (int64_t)t;
            out.hit_index = fr.hit;
            out.fold = fd;
            out.pmt_id = (uint16_t)fr.pmt;
            out.pad[0] = out.pad[1] = out.pad[2] = 0;
            const uint32_t g = P.F + r;
            gstore(fires + g, out);
            if (xf) gstore(xf + g, out);
            if (st) {
                events[ev].t_trig = out.t_ns;
                events[ev].t_begin = out.t_ns - H;
                if (xe) {
                    xe[ev].t_trig = out.t_ns;
                    xe[ev].t_begin = out.t_ns - H;
                }
                if (r == 0 && P.F) {
                    // this fire ends the event left open by the preceding tiles
                    const uint32_t pe = EP - 1;
                    const int64_t tend = t_min + (int64_t)P.last_t + H;
                    events[pe].t_end = tend;
                    events[pe].n_fire = P.F - p_open;
                    events[pe].max_fold = P.m_tail;
                    if (xe) {
                        xe[pe].t_end = tend;
                        xe[pe].n_fire = P.F - p_open;
                        xe[pe].max_fold = P.m_tail;
                    }
                }
            }
            // the next fire of the tile starts a new event: this one ends its event
            if (r + 1 < nf && (uint64_t)(t_next - t) > twoH) {
                const uint32_t sg = latest >= 0 ? P.F + (uint32_t)latest : p_open;
                const int64_t tend = out.t_ns + H;
                events[ev].t_end = tend;
                events[ev].n_fire = P.F + r - sg + 1;
                events[ev].max_fold = mv;
                if (xe) {
                    xe[ev].t_end = tend;
                    xe[ev].n_fire = P.F + r - sg + 1;
                    xe[ev].max_fold = mv;
                }
            }
        }
        carry_starts = lane_read(starts_incl, 63);
        carry_latest = (int32_t)lane_read((uint32_t)latest, 63);
        carry_max = lane_read(mv, 63);
        prev_t = lane_read(t, 63);
    }
}

// Persistent: each wave owns a contiguous stretch of the tile list (XCD-aware as
// in the ordering kernel), looks its slice up once per slice, reads the fire
// counts of 64 tiles at a time and places only the tiles that have fires.
__global__ __launch_bounds__(64) void k_place(BatchDev b) {
    const uint32_t total = b.total_tiles;
    const uint32_t xcd = blockIdx.x % 8, g = blockIdx.x / 8, per_xcd = gridDim.x / 8;
    const uint32_t x0 = (uint32_t)(((uint64_t)total * xcd) / 8), x1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / 8);
    const uint32_t per = (x1 - x0 + per_xcd - 1) / per_xcd;
    uint32_t item = x0 + g * per;
    const uint32_t end = (item + per < x1) ? item + per : x1;
    const int lane = lane_id();
    while (item < end) {
        const uint32_t si = slice_of_tile(b, item);
        const SliceDev &S = b.slices[si];
        const uint32_t base = tile_base_of(b, si);
        uint32_t s_end = base + S.n_tiles;          // first item past this slice
        if (s_end > end) s_end = end;
        if (s_end <= item) { ++item; continue; }    // (an empty slice shares its base)
        const TRIG_GAS Plan *Pp = gmem(b.plans + si);
        // slices outside this pass, and slices that are rerun, place nothing
        const bool live = slice_in_tail(b, Pp->state) && !(Pp->dense && b.tail_state != ST_DENSE);
        if (live) {
            const TRIG_GAS TileStat *tstat = gmem(S.tstat);
            for (uint32_t i0 = item; i0 < s_end; i0 += 64) {
                const uint32_t it = i0 + (uint32_t)lane;
                const uint32_t nf = it < s_end ? tstat[it - base].agg.F : 0u;
                uint64_t m = __ballot(nf != 0);
                while (m) {
                    const int l = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    place_tile(b, S, Pp, i0 + (uint32_t)l - base, lane_read(nf, l));
                }
            }
        }
        item = s_end;
    }
}

// Seed mask of the slices being rerun (plan.dense), one tile per workgroup: the
// tile and DSH ordered neighbours on each side are staged in LDS; a floor partner
// search that runs past them reads global memory.  Also moves the slice to
// ST_DENSE for the rerun.
constexpr int DSH = 64;
constexpr int NTD = 256;

__global__ __launch_bounds__(NTD) void k_dseed(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return;
    Plan *Pp = S.plan;
    if (!Pp->dense || Pp->status != TRIG_OK) return;
    if (k == 0 && threadIdx.x == 0) Pp->state = ST_DENSE;
    __shared__ uint32_t lt[TILE + 2 * DSH], lpq[TILE + 2 * DSH];
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) return;
    const uint64_t lo = a >= (uint64_t)DSH ? a - DSH : 0;
    const uint64_t hi = (a + TILE + DSH < n) ? a + TILE + DSH : n;
    stage_copy<NTD, 5>(lt, gmem(S.o_t) + lo, (uint32_t)(hi - lo));
    stage_copy<NTD, 5>(lpq, gmem(S.o_pq) + lo, (uint32_t)(hi - lo));
    __syncthreads();
    auto T_at = [&](uint64_t m) -> uint32_t { return (m >= lo && m < hi) ? lt[m - lo] : S.o_t[m]; };
    auto P_at = [&](uint64_t m) -> uint32_t { return ((m >= lo && m < hi) ? lpq[m - lo] : S.o_pq[m]) >> 16; };
    const uint32_t Q = b.prm.q_seed;
    const int32_t tau = b.prm.t_floor_ns;
    // level 0 on: a seed and its floor partner must both pass it
    const bool L0 = b.prm.l0_n > 0;
    const TRIG_GAS uint64_t *l0m = gmem(S.l0m);
    auto l0_at = [&](uint64_t m) -> bool { return !L0 || ((l0m[m >> 6] >> (m & 63)) & 1ull); };
    // partner rules: FC (same floor, tau), SC (same floor and adjacency group),
    // AFC (consecutive floors); without the seed menu only FC is on
    const int32_t t_sc = b.prm.t_adj_ns, t_afc = b.prm.t_afloor_ns;
    const bool mode1 = b.prm.seed_mode == 1;
    const int32_t tmax = max(tau, max(t_sc, t_afc));
    const TRIG_GAS uint16_t *floor16 = gmem(S.floor16);
    const TRIG_GAS uint32_t *adj32 = gmem(S.adj32);
    const TRIG_GAS uint32_t *afl32 = gmem(S.afl32);
#pragma unroll
    for (int e = 0; e < TILE / NTD; ++e) {
        const uint64_t j = a + (uint64_t)e * NTD + threadIdx.x;
        bool seed = false;
        if (j < n && l0_at(j)) {
            const uint32_t t = lt[j - lo], pq = lpq[j - lo], p = pq >> 16;
            seed = (pq & 0xFFFFu) >= Q;
            if (!seed && tmax >= 0) {
                const uint32_t f = floor16[p], ak = adj32[p], rk = afl32[p];
                // found rules as bits (1 FC, 2 SC, 4 AFC), kept in a register
                const uint32_t lim_fc = tau >= 0 ? (uint32_t)tau + 1u : 0u;
                const uint32_t lim_sc = t_sc >= 0 ? (uint32_t)t_sc + 1u : 0u;
                const uint32_t lim_afc = t_afc >= 0 ? (uint32_t)t_afc + 1u : 0u;
                uint32_t found = 0;
                auto met = [&]() { return mode1 ? ((found & 3u) != 0u && (found & 4u) != 0u) : found != 0u; };
                auto visit = [&](uint64_t m, uint32_t dt) {
                    const uint32_t pm = P_at(m);
                    const bool ok = pm != p && l0_at(m);
                    const bool same = floor16[pm] == f;
                    const uint32_t rm = afl32[pm];
                    const bool nb = (rm == rk + 1u) | (rm + 1u == rk);
                    found |= (uint32_t)(ok & same & (dt < lim_fc)) | ((uint32_t)(ok & same & (dt < lim_sc) & (adj32[pm] == ak)) << 1) |
                             ((uint32_t)(ok & !same & (dt < lim_afc) & nb) << 2);
                };
                for (uint64_t m = j; m > 0 && !met();) {
                    --m;
                    const uint32_t dt = t - T_at(m);
                    if (dt > (uint32_t)tmax) break;
                    visit(m, dt);
                }
                for (uint64_t m = j + 1; m < n && !met(); ++m) {
                    const uint32_t dt = T_at(m) - t;
                    if (dt > (uint32_t)tmax) break;
                    visit(m, dt);
                }
                seed = met();
            }
        }
        const uint64_t bal = __ballot(seed);
        const uint64_t w0 = a + (uint64_t)e * NTD + (threadIdx.x & ~63u);
        if (lane_id() == 0 && w0 < n) S.dmask[w0 >> 6] = bal;
    }
}


template <int NT, int HMAX, bool MASK, bool MENU>
hipError_t launch_tile_nt(const BatchDev &b, uint32_t floor_lds, hipStream_t s) {
    constexpr size_t STG = TILE + 2 * HMAX;
    const size_t shm = tile_lds_bytes<HMAX, MASK>() + ((floor_lds * 2 + 15) & ~15u) + (MENU ? floor_lds * 8 + STG * 8 : 0);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_tile<NT, HMAX, MASK, MENU>, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)(tile_lds_bytes<HMAX, MASK>() + FLOOR_LDS_MAX * 2 + (MENU ? FLOOR_LDS_MAX * 8 + STG * 8 : 0)));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_tile<NT, HMAX, MASK, MENU>), dim3(((b.total_tiles + 7) / 8) * 8), dim3(NT), shm, s, b,
                       floor_lds);
    return hipGetLastError();
}

template <int HMAX, bool MASK, bool MENU>
hipError_t launch_tile(const BatchDev &b, uint32_t max_pmt, uint32_t n_cu, hipStream_t s) {
    // the floor numbering of the batch's largest geometry in LDS when it is small
    const uint32_t floor_lds = max_pmt <= (uint32_t)FLOOR_LDS_MAX ? max_pmt : 0u;
    if (b.total_tiles <= 4 * n_cu) return launch_tile_nt<NT_ONE_WAVE, HMAX, MASK, MENU>(b, floor_lds, s);
    return launch_tile_nt<NT_MANY, HMAX, MASK, MENU>(b, floor_lds, s);
}


// ------------------------------------------------------------------ k_seed
// L1 seeds of the plain rule (Sec. 3 and Sec. 4.2: charge over threshold, or
// another PMT of the same floor within t_floor_ns; with level 0 on, the hit and
// its partner must pass it), one 256-thread workgroup per ordered tile, each
// thread owning four consecutive hits of the tile (16-byte loads; their times,
// PMTs, floors, charges and level-0 bits stay in registers).  The tile and up to
// SD_HS ordered neighbours on each side (whole 64-hit words, sized from the
// slice's mean density to span t_floor_ns) are staged in LDS.  A thread checks
// the pairs of its four hits among themselves and with the next four staged hits
// (one 16-byte LDS read of times and one of floors: distances up to 7), and
// reads further blocks of four only while its last hit's successors are still
// within t_floor_ns; a pair of two PMTs of one floor marks both hits (a partner
// ahead of the thread's own hits through an LDS atomic: pairs are rare).  Hits
// within t_floor_ns of the tile's start also look back into the left halo.  A
// tile whose staged neighbours do not span t_floor_ns (a burst of near-equal
// times) searches each hit's partners on both sides instead, reading past the
// stage from global memory.  The tile's seeds are written compacted, in time
// order (one block scan of the threads' counts), to its seed list, with its
// record (count, first and last seed time).
constexpr int SD_NT = 256;
constexpr int SD_HS = 256;   // staged neighbours per side at most (whole words)
constexpr int SD_PL = 4;     // consecutive hits per thread
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte loads and stores

struct SeedShape {
    static constexpr int NT = SD_NT;
    static constexpr int STG = TILE + 2 * SD_HS;
    static constexpr int NWD = STG / 64;
    static constexpr size_t lds_bytes() { return (size_t)STG * 4 * 2 + (size_t)NWD * 8 * 2; }
    static_assert(TILE == NT * SD_PL && SD_HS % 64 == 0, "stage layout");
};

__global__ __launch_bounds__(SD_NT) void k_seed(BatchDev b) {
    using Sh = SeedShape;
    constexpr int NT = Sh::NT, NWD = Sh::NWD;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *st = (uint32_t *)smem;            // staged t - t_min
    uint32_t *spf = st + Sh::STG;               // staged dense floor index << 16 | pmt
    uint64_t *lw = (uint64_t *)(spf + Sh::STG); // level-0 pass bits per word (level 0 on)
    uint64_t *mk = lw + NWD;                    // partner marks per word
    __shared__ uint32_t wsum[NT / 64 + 1];

    // XCD-aware order: workgroup b runs on XCD b % 8 and takes tiles from that
    // XCD's contiguous eighth of the list (neighbouring tiles share halos in one L2)
    const uint32_t per_xcd = (b.total_tiles + 7) / 8;
    const uint32_t item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (item >= b.total_tiles) return;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return;
    const TRIG_GAS Plan *Pg = gmem(b.plans + si);
    // halo: from the plan (four times the mean number of hits in t_floor_ns, whole
    // words), at most SD_HS (a burst that outruns it takes the search past the
    // stage below)
    const uint64_t halo = min(cmem(b.plans + si)->seed_halo, (uint32_t)SD_HS);
    if (!slice_in_tail(b, Pg->state)) return;
    const TRIG_GAS uint32_t *o_t = gmem(S.o_t);
    const TRIG_GAS uint32_t *o_pq = gmem(S.o_pq);
    const TRIG_GAS uint32_t *o_idx = gmem(S.o_idx);
    const TRIG_GAS uint16_t *floor16 = gmem(S.floor16);
    TRIG_GAS uint8_t *seed_flags = gmem(S.seed_flags);
    const TRIG_GAS uint64_t *l0m = gmem(S.l0m);
    TRIG_GAS uint32_t *sd_t = seed_t(S) + (uint64_t)k * TILE;
    TRIG_GAS uint32_t *sd_p = seed_p(S) + (uint64_t)k * TILE;
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) {   // the one tile of an empty slice
        if (threadIdx.x == 0) gstore(seed_rec(S) + k, SeedRec{0u, 0u, 0u, 0u});
        return;
    }
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    const int32_t tau = b.prm.t_floor_ns;
    const uint32_t tau_u = tau > 0 ? (uint32_t)tau : 0u;
    const uint32_t q_seed = b.prm.q_seed;
    const bool L0 = b.prm.l0_n > 0;
    const uint32_t tid = threadIdx.x;
    const int lane = lane_id(), w = (int)(tid >> 6);


    const uint64_t sl = a >= halo ? a - halo : 0;   // (a is a multiple of TILE: sl = a - halo or 0)
    const uint64_t she = (e + halo < n) ? e + halo : n;
    const uint32_t len = (uint32_t)(she - sl);
    const uint32_t a_loc = (uint32_t)(a - sl), e_loc = (uint32_t)(e - sl);   // a_loc: whole words
    const uint32_t nwords = (len + 63) / 64;

    // 1. this thread's four hits (tile positions 4 tid .. 4 tid + 3), then the
    // halo's groups of four (by the first threads), all loads in flight; the
    // floor numbering gathered from the table in device memory (cache-resident)
    const uint32_t x0 = a_loc + SD_PL * tid;                 // stage position of the first own hit
    const uint32_t own = e_loc > x0 ? min(e_loc - x0, (uint32_t)SD_PL) : 0u;   // own hits in the tile
    uint32_t t4[SD_PL], p4[SD_PL];
    auto load4 = [&](uint32_t x, uint32_t (&tv)[SD_PL], uint32_t (&pv)[SD_PL]) {   // stage positions x .. x + 3
        if (x + SD_PL <= len) {
            const u32x4 tq = *(const TRIG_GAS u32x4 *)(o_t + sl + x);
            const u32x4 pq = *(const TRIG_GAS u32x4 *)(o_pq + sl + x);
            tv[0] = tq.x; tv[1] = tq.y; tv[2] = tq.z; tv[3] = tq.w;
            pv[0] = pq.x; pv[1] = pq.y; pv[2] = pq.z; pv[3] = pq.w;
        } else {
#pragma unroll
            for (int s = 0; s < SD_PL; ++s) {
                const uint32_t xc = min(x + (uint32_t)s, len - 1);
                tv[s] = o_t[sl + xc];
                pv[s] = o_pq[sl + xc];
            }
        }
    };
    load4(x0 < len ? x0 : len - 1, t4, p4);
    // halo groups: [0, a_loc) on the left, [e_loc, len) on the right
    const uint32_t nhl = a_loc / SD_PL, nh = nhl + (len - e_loc + SD_PL - 1) / SD_PL;
    const bool has_h = tid < nh;
    const uint32_t xh = tid < nhl ? SD_PL * tid : e_loc + SD_PL * (tid - nhl);
    uint32_t th[SD_PL], ph[SD_PL];
    if (has_h) load4(xh, th, ph);
    uint32_t q4 = 0;   // charge over threshold, bit s
#pragma unroll
    for (int s = 0; s < SD_PL; ++s) {
        q4 |= (uint32_t)((uint32_t)s < own && (p4[s] & 0xFFFFu) >= q_seed) << s;
        const uint32_t p = p4[s] >> 16;
        p4[s] = ((uint32_t)floor16[p] << 16) | p;
    }
    if (has_h) {
#pragma unroll
        for (int s = 0; s < SD_PL; ++s) {
            const uint32_t p = ph[s] >> 16;
            ph[s] = ((uint32_t)floor16[p] << 16) | p;
        }
    }
    if (x0 + SD_PL <= Sh::STG) {
        *(u32x4 *)(st + x0) = u32x4{t4[0], t4[1], t4[2], t4[3]};
        *(u32x4 *)(spf + x0) = u32x4{p4[0], p4[1], p4[2], p4[3]};
    }
    if (has_h) {
        *(u32x4 *)(st + xh) = u32x4{th[0], th[1], th[2], th[3]};
        *(u32x4 *)(spf + xh) = u32x4{ph[0], ph[1], ph[2], ph[3]};
    }
    if (tid < nwords) {
        mk[tid] = 0ull;
        if (L0) lw[tid] = l0m[(sl >> 6) + tid];   // (sl is a whole word)
    }
    __syncthreads();
    // level-0 pass bit of stage position x (level 0 on)
    auto l0_at = [&](uint32_t x) -> bool { return !L0 || ((lw[x >> 6] >> (x & 63)) & 1ull); };
    uint32_t l4 = (1u << SD_PL) - 1u;   // own hits passing level 0
    if (L0) {
        l4 = 0;
#pragma unroll
        for (int s = 0; s < SD_PL; ++s) l4 |= (uint32_t)l0_at(min(x0 + (uint32_t)s, len - 1)) << s;
    }
    q4 &= l4;

    const uint32_t ta = st[a_loc], te = st[e_loc - 1];
    // the stage spans t_floor_ns around the tile on both sides (or the slice ends there)
    const bool cover_l = sl == 0 || (uint64_t)st[0] + tau_u < (uint64_t)ta;
    const bool cover_r = she == n || (uint64_t)st[len - 1] > (uint64_t)te + tau_u;
    uint32_t f4 = 0;   // own hits with a floor partner, bit s
    // keys (floor << 16 | pmt): x ^ y - 1 < 0xFFFF iff one floor and two PMTs
    auto floor_pair = [](uint32_t kx, uint32_t ky) -> bool { return ((kx ^ ky) - 1u) < 0xFFFFu; };
    if (tau >= 0 && tau_u < 0xFFFEu && cover_l && cover_r) {
        // 2. the own hits among themselves and with the staged hits after them,
        // four at a time.  For own hit s and a later hit y (t_y >= t_s) let
        // m = max((k_s ^ k_y) - 1, t_y - (t_s + tau - 0xFFFE)): the pair counts iff
        // m < 0xFFFF (one floor, two PMTs, t_y - t_s <= tau).  An own hit that is
        // not there or fails level 0 takes t_s + tau - 0xFFFE = 2^31, a staged one
        // t_y = 3 * 2^30: m is then at least 2^30.  Each own hit keeps the least
        // m of its pairs; marks of partners after the own hits go to LDS.
        constexpr uint32_t A_NONE = 0x80000000u, T_NONE = 0xC0000000u;
        uint32_t as[SD_PL], tv[SD_PL], macc[SD_PL];
#pragma unroll
        for (int s = 0; s < SD_PL; ++s) {
            const bool ok = (uint32_t)s < own && ((l4 >> s) & 1u);
            as[s] = ok ? t4[s] + tau_u - 0xFFFEu : A_NONE;
            tv[s] = ok ? t4[s] : T_NONE;
            macc[s] = 0xFFFFFFFFu;
        }
#pragma unroll
        for (int s = 0; s < SD_PL; ++s)
#pragma unroll
            for (int s2 = s + 1; s2 < SD_PL; ++s2) {
                const uint32_t m = max(((p4[s] ^ p4[s2]) - 1u), tv[s2] - as[s]);
                macc[s] = min(macc[s], m);
                macc[s2] = min(macc[s2], m);
            }
        if (own) {
            const uint32_t tl = t4[own - 1];   // the last own hit: the one nearest what follows
            for (uint32_t y0 = x0 + SD_PL;; y0 += SD_PL) {
                if (y0 >= len || st[y0] - tl > tau_u) break;
                uint32_t ty[SD_PL], py[SD_PL];
                if (y0 + SD_PL <= len) {
                    const u32x4 tq = *(const u32x4 *)(st + y0);
                    const u32x4 pq = *(const u32x4 *)(spf + y0);
                    ty[0] = tq.x; ty[1] = tq.y; ty[2] = tq.z; ty[3] = tq.w;
                    py[0] = pq.x; py[1] = pq.y; py[2] = pq.z; py[3] = pq.w;
                } else {
#pragma unroll
                    for (int j = 0; j < SD_PL; ++j) {
                        const uint32_t yc = min(y0 + (uint32_t)j, len - 1);
                        ty[j] = y0 + (uint32_t)j < len ? st[yc] : T_NONE;
                        py[j] = spf[yc];
                    }
                }
                if (L0) {
#pragma unroll
                    for (int j = 0; j < SD_PL; ++j)
                        if (!l0_at(min(y0 + (uint32_t)j, len - 1))) ty[j] = T_NONE;
                }
                uint32_t hacc[SD_PL];   // the least m of each staged hit's pairs with the own hits
#pragma unroll
                for (int j = 0; j < SD_PL; ++j) {
                    uint32_t mj[SD_PL];
#pragma unroll
                    for (int s = 0; s < SD_PL; ++s) {
                        mj[s] = max(((p4[s] ^ py[j]) - 1u), ty[j] - as[s]);
                        macc[s] = min(macc[s], mj[s]);
                    }
                    hacc[j] = min(min(mj[0], mj[1]), min(mj[2], mj[3]));
                }
                if (min(min(hacc[0], hacc[1]), min(hacc[2], hacc[3])) < 0xFFFFu) {   // (rare)
#pragma unroll
                    for (int j = 0; j < SD_PL; ++j)
                        if (hacc[j] < 0xFFFFu) {
                            const uint32_t y = y0 + (uint32_t)j;
                            atomicOr((unsigned long long *)&mk[y >> 6], 1ull << (y & 63));
                        }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < SD_PL; ++s) f4 |= (uint32_t)(macc[s] < 0xFFFFu) << s;
        if (own) {
            // own hits within t_floor_ns of the tile's start: partners in the left halo
            if (a_loc > 0 && t4[0] - st[a_loc - 1] <= tau_u) {
#pragma unroll
                for (int s = 0; s < SD_PL; ++s) {
                    if ((uint32_t)s >= own || !((l4 >> s) & 1u)) continue;
                    for (uint32_t y = a_loc; y > 0;) {
                        --y;
                        if (t4[s] - st[y] > tau_u) break;
                        if (l0_at(y) && floor_pair(spf[y], p4[s])) {
                            f4 |= 1u << s;
                            break;
                        }
                    }
                }
            }
        }
    } else if (tau >= 0) {
        // the stage does not span t_floor_ns: each own hit searches its partners on
        // both sides, past the stage in global memory
        auto T_at = [&](uint64_t m) -> uint32_t { return (m >= sl && m < she) ? st[m - sl] : o_t[m]; };
        auto F_at = [&](uint64_t m) -> uint32_t {
            if (m >= sl && m < she) return spf[m - sl];
            const uint32_t p = o_pq[m] >> 16;
            return ((uint32_t)floor16[p] << 16) | p;
        };
        auto l0g = [&](uint64_t m) -> bool { return !L0 || ((l0m[m >> 6] >> (m & 63)) & 1ull); };
        for (int s = 0; s < SD_PL; ++s) {
            if ((uint32_t)s >= own || !((l4 >> s) & 1u)) continue;
            const uint64_t j = sl + x0 + (uint32_t)s;
            const uint32_t t = t4[s], f = p4[s];
            bool found = false;
            for (uint64_t m = j; m > 0 && !found;) {
                --m;
                if (t - T_at(m) > tau_u) break;
                found = floor_pair(F_at(m), f) && l0g(m);
            }
            for (uint64_t m = j + 1; m < n && !found; ++m) {
                if (T_at(m) - t > tau_u) break;
                found = floor_pair(F_at(m), f) && l0g(m);
            }
            f4 |= (uint32_t)found << s;
        }
    }
    __syncthreads();

    // 3. the own seeds (charge, partner found here, or marked by another thread),
    // their place among the tile's seeds (block scan), the compacted list
    uint32_t s4 = q4 | f4;
    if (own) s4 |= (uint32_t)(mk[x0 >> 6] >> (x0 & 63)) & ((1u << own) - 1u);   // (4 bits of one word)
    s4 &= (1u << own) - 1u;
    const uint32_t c = (uint32_t)__popc(s4);
    const uint32_t inc = wave_incl_scan(c);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const uint32_t v = wsum[i];
        before += i < w ? v : 0u;
        total += v;
    }
    uint32_t at = before + inc - c;
#pragma unroll
    for (int s = 0; s < SD_PL; ++s) {
        if ((s4 >> s) & 1u) {
            sd_t[at] = t4[s];
            sd_p[at] = (p4[s] << 16) | (SD_PL * tid + (uint32_t)s);
            if (at == 0) gstore(&seed_rec(S)[k].first_t, t4[s]);
            if (at + 1 == total) gstore(&seed_rec(S)[k].last_t, t4[s]);
            ++at;
        }
        if (seed_flags && (uint32_t)s < own) seed_flags[o_idx[a + SD_PL * tid + s]] = (uint8_t)((s4 >> s) & 1u);
    }
    if (tid == 0) gstore(&seed_rec(S)[k].n, total);
}

hipError_t launch_seed(const BatchDev &b, hipStream_t s) {
    const size_t shm = SeedShape::lds_bytes();
    static const hipError_t attr = hipFuncSetAttribute((const void *)k_seed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)shm);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_seed, dim3(((b.total_tiles + 7) / 8) * 8), dim3(SD_NT), shm, s, b);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_fold
// Causal folds of the plain rule's seeds (Sec. 3: the Cherenkov hits of one muon
// are correlated within min(thr, w_ns)) and the fires: one wave per tile, G tiles
// of one slice per workgroup (the group map written by k_plan; the table bounds
// of a large detector staged in LDS once for them).  A seed of PMT p counts the
// other seeds within R_p = min(w_ns, the largest entry of p's row of the table),
// so a tile's window reaches the tiles with seeds within min(w_ns, the table's
// largest entry) of its own: the records of the 32 tiles before it and the 31
// after it, read at once, give that window (further tiles are walked 64 at a
// time).  Its seeds, concatenated in time order, are staged in the wave's LDS (at
// most CAP; a larger window is read from the lists in device memory).  A lane per
// seed counts, over its stretch of the window (bounds by fixed-count binary
// searches), the other seeds within min(thr, w_ns), four or eight table reads in
// flight; for large detectors the pair of the two PMTs' 32-PMT blocks has a lower
// and an upper bound of thr (16 ns units) that decide most pairs, and the table
// is read only for the rest.  Each round of 64 seeds then writes its fires to the tile's
// slot and adds them to the tile's summary (TileAgg).
constexpr int FD_TMAX = 64;   // window tiles staged at most

template <int CAP>
struct FoldShape {
    static constexpr size_t wave_bytes() { return (size_t)CAP * 8; }   // per wave: time | (pmt << 16 | position) << 32
};

template <int G, int CAP, bool BOUNDS>
__global__ __launch_bounds__(64 * G) void k_fold(BatchDev b) {
    constexpr int NT = 64 * G;
    extern __shared__ __align__(16) unsigned char smem[];
    // LDS: the table bounds (large detectors), then each wave's window of seeds,
    // one 8-byte entry per seed (one LDS read per candidate)
    const size_t tb_bytes = ((size_t)(BOUNDS ? b.tbnd_lds : 0u) * 2 + 15) & ~(size_t)15;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint16_t *ltb = (uint16_t *)smem;                 // the table bounds (b.tbnd_lds of them)
    uint64_t *lwin = (uint64_t *)(smem + tb_bytes + (size_t)w * FoldShape<CAP>::wave_bytes());   // window seeds
    const uint32_t *lt = (const uint32_t *)lwin;      // their times: the low word of each entry (stride 2)
    __shared__ uint32_t woff_all[G][FD_TMAX + 1];     // window seeds before each window tile
    uint32_t *woff = woff_all[w];

    const uint32_t per_xcd = (b.total_groups + 7) / 8;
    const uint32_t item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (item >= b.total_groups) return;
    const uint32_t si = b.n_slices <= 1 ? 0u : gmem(b.group_slice)[item];
    const SliceDev &S = b.slices[si];
    const uint32_t g = item - (b.n_slices <= 1 ? 0u : S.group_base);
    const uint32_t k0 = g * (uint32_t)G;
    const uint32_t n_tiles = S.n_tiles;
    if (k0 >= n_tiles) return;
    const TRIG_GAS Plan *Pg = gmem(b.plans + si);
    if (!slice_in_tail(b, Pg->state)) return;
    const uint32_t W = b.prm.w_ns;
    const uint32_t nbk = S.nbk;
    const bool bounds = nbk != 0 && W <= 65535u;
    const bool tb_in_lds = bounds && nbk * nbk <= b.tbnd_lds;
    const TRIG_GAS uint16_t *tbnd = gmem(S.tbnd);
    if (tb_in_lds) {   // (16-byte pieces: the table's allocation is padded to them)
        const TRIG_GAS u32x4 *src = (const TRIG_GAS u32x4 *)tbnd;
        for (uint32_t x = threadIdx.x; x < (nbk * nbk + 7) / 8; x += NT) ((u32x4 *)ltb)[x] = src[x];
        __syncthreads();
    }
    const uint32_t kt = k0 + (uint32_t)w;
    if (kt >= n_tiles) return;
    const TRIG_GAS uint32_t *o_idx = gmem(S.o_idx);
    const TRIG_GAS uint16_t *thr16 = gmem(S.thr16);
    const TRIG_GAS uint32_t *thr32 = gmem(S.thr32);
    const TRIG_GAS uint32_t *rmax = gmem(S.rmax);
    const TRIG_GAS uint32_t *sdt = seed_t(S);
    const TRIG_GAS uint32_t *sdp = seed_p(S);
    const TRIG_GAS SeedRec *recs = seed_rec(S);
    const uint32_t n_pmt = S.n_pmt;
    const uint32_t N = b.prm.min_fold;
    const uint64_t twoH = 2ull * (uint64_t)b.prm.half_event_ns;
    const uint32_t Wr = W < S.thr_max ? W : S.thr_max;   // the reach of any seed

    // 1. the window: lane l holds the record of tile kt - 32 + l
    const int64_t jj = (int64_t)kt - 32 + lane;
    const bool vj = jj >= 0 && jj < (int64_t)n_tiles;
    SeedRec R = SeedRec{0u, 0u, 0u, 0u};
    if (vj) R = gload(recs + jj);
    const uint32_t cnt = lane_read(R.n, 32);
    TileAgg A = agg_empty();
    if (cnt == 0) {
        if (lane == 0) gstore(&gmem(S.tstat)[kt].agg, A);
        return;
    }
    const uint32_t t_first = lane_read(R.first_t, 32), t_last = lane_read(R.last_t, 32);
    const uint32_t t_lo_w = t_first > Wr ? t_first - Wr : 0u;
    const uint64_t t_hi_w = (uint64_t)t_last + Wr;
    // the nearest tile on each side whose seeds all lie outside: it and the tiles
    // beyond it hold none within reach
    const uint64_t stopL = __ballot(lane < 32 && vj && R.n > 0 && R.last_t < t_lo_w);
    const uint64_t stopR = __ballot(lane > 32 && vj && R.n > 0 && (uint64_t)R.first_t > t_hi_w);
    bool near = true;
    uint32_t jl, jr;
    if (stopL) {
        jl = kt - 32 + (uint32_t)(63 - __clzll((long long)stopL)) + 1;
    } else if (kt < 32) {
        jl = 0;
    } else {
        near = false;
        jl = kt - 32;
        for (;;) {
            const bool v = jl > (uint32_t)lane;
            SeedRec Rw = SeedRec{0u, 0u, 0u, 0u};
            if (v) Rw = gload(recs + (jl - 1 - (uint32_t)lane));
            const uint64_t M = __ballot(!v || (Rw.n > 0 && Rw.last_t < t_lo_w));
            if (M) {
                jl -= (uint32_t)(__ffsll((unsigned long long)M) - 1);
                break;
            }
            jl -= 64;
        }
    }
    if (stopR) {
        jr = kt - 32 + (uint32_t)(__ffsll((unsigned long long)stopR) - 1);
    } else if ((uint64_t)kt + 32 >= n_tiles) {
        jr = n_tiles;
    } else {
        near = false;
        jr = kt + 32;
        for (;;) {
            const uint32_t j = jr + (uint32_t)lane;
            const bool v = j < n_tiles;
            SeedRec Rw = SeedRec{0u, 0u, 0u, 0u};
            if (v) Rw = gload(recs + j);
            const uint64_t M = __ballot(!v || (Rw.n > 0 && (uint64_t)Rw.first_t > t_hi_w));
            if (M) {
                jr += (uint32_t)(__ffsll((unsigned long long)M) - 1);
                break;
            }
            jr += 64;
        }
    }
    const uint32_t nt = jr - jl;
    uint32_t tot = 0;
    bool staged = false;
    if (near || nt <= (uint32_t)FD_TMAX) {
        // window seeds before each window tile (the records already in the lanes
        // when the window lies within them)
        uint32_t c = 0, at = 0;
        bool in = false;
        if (near) {
            in = vj && jj >= (int64_t)jl && jj < (int64_t)jr;
            c = in ? R.n : 0u;
            at = (uint32_t)(jj - (int64_t)jl);
        } else {
            in = (uint32_t)lane < nt;
            c = in ? gload(recs + jl + lane).n : 0u;
            at = (uint32_t)lane;
        }
        const uint32_t inc = wave_incl_scan(c);
        tot = lane_read(inc, 63);
        if (in) woff[at] = inc - c;
        if (lane == 0) woff[nt] = tot;
        staged = tot <= (uint32_t)CAP;
        wave_lds_sync();
    }

    // 2. stage the window's seeds (UB loads in flight per lane)
    if (staged) {
        constexpr int UB = 8;
        for (uint32_t x0 = 0; x0 < tot; x0 += 64 * UB) {
            uint32_t vt[UB], vp[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const uint32_t x = x0 + u * 64 + (uint32_t)lane;
                if (x < tot) {
                    uint32_t lo = 0, hi = nt;   // window tile of x: the last with woff <= x
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (woff[mid] <= x) lo = mid; else hi = mid;
                    }
                    const uint64_t src = (uint64_t)(jl + lo) * TILE + (x - woff[lo]);
                    vt[u] = sdt[src];
                    vp[u] = sdp[src];
                }
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const uint32_t x = x0 + u * 64 + (uint32_t)lane;
                if (x < tot) {
                    lwin[x] = (uint64_t)vt[u] | ((uint64_t)vp[u] << 32);
                }
            }
        }
        wave_lds_sync();
    }

    // 3. folds and fires, 64 seeds per round
    const uint32_t own0 = staged ? woff[kt - jl] : 0u;   // the tile's first seed in the window
    TRIG_GAS FireRec *slot = gmem(S.fsc) + (uint64_t)kt * TILE;
    const bool t16 = W <= 65535u;
    uint32_t top = 1;   // the largest power of two <= tot
    while (top * 2 <= tot) top *= 2;
    // window entries per lane and step: twelve in the variant for batches with
    // large detectors (32-PMT block bounds decide most pairs of their dense
    // windows, and the rest read the table from far memory: on the block 8 took
    // 209 us, 12 200 us, 16 215 us; the slices without bounds in such a batch
    // share the loop), four in the one for towers only (every pair reads the
    // table; short windows)
    constexpr int CB = BOUNDS ? 12 : 4;

    // fold of one seed (time ti, PMT pi, window index self) over window entries
    // [jlo, jhi), each read through E_at as time | (pmt << 16 | position) << 32.
    // A step reads CB entries at indexes clamped to jmax (E_at's last readable
    // one) whatever their range, so the reads are in flight together; entries
    // past the range, the seed itself and those beyond its reach count nothing
    // and read the table at the seed's own row start.
    auto count_range = [&](uint32_t ti, uint32_t pi, uint32_t lim_w, uint32_t jlo, uint32_t jhi, uint32_t self,
                           uint32_t jmax, auto E_at) -> uint32_t {
        const uint64_t row = (uint64_t)pi * n_pmt;
        const uint32_t brow = (pi >> TBND_SHIFT) * nbk;
        uint32_t c = 0;
        // one step: the distances of CB entries (0xFFFFFFFF: out of range, the seed
        // itself or beyond its reach) and their PMTs
        auto load_step = [&](uint32_t j0, uint32_t (&dd)[CB], uint32_t (&pj)[CB]) {
            uint64_t ej[CB];
#pragma unroll
            for (int kk = 0; kk < CB; ++kk) ej[kk] = E_at(min(j0 + (uint32_t)kk, jmax));
#pragma unroll
            for (int kk = 0; kk < CB; ++kk) {
                const uint32_t j = j0 + (uint32_t)kk;
                const uint32_t tj = (uint32_t)ej[kk];
                const uint32_t dt = tj > ti ? tj - ti : ti - tj;
                const bool ok = j < jhi && j != self && dt <= lim_w;
                dd[kk] = ok ? dt : 0xFFFFFFFFu;
                pj[kk] = ok ? (uint32_t)(ej[kk] >> 48) : 0u;
            }
        };
        for (uint32_t j0 = jlo;; j0 += CB) {
            if (!__ballot(j0 < jhi)) break;
            uint32_t dd[CB], pj[CB], lim[CB];
            load_step(j0, dd, pj);
            if (BOUNDS && bounds) {
                uint32_t bb[CB];
#pragma unroll
                for (int kk = 0; kk < CB; ++kk) {
                    const uint32_t bx = brow + (pj[kk] >> TBND_SHIFT);
                    bb[kk] = tb_in_lds ? (uint32_t)ltb[bx] : (uint32_t)tbnd[bx];
                }
#pragma unroll
                for (int kk = 0; kk < CB; ++kk) {
                    const uint32_t hb = bb[kk] >> 8;
                    const uint32_t mn = min((bb[kk] & 0xFFu) * 16u, W), mx = hb == 255u ? W : min(hb * 16u, W);
                    lim[kk] = dd[kk] <= mn ? W : 0u;
                    if (dd[kk] != 0xFFFFFFFFu && dd[kk] > mn && dd[kk] <= mx) lim[kk] = (uint32_t)thr16[row + pj[kk]];
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < CB; ++kk) {
                    lim[kk] = 0;
                    if (dd[kk] != 0xFFFFFFFFu) {
                        const uint64_t x = row + pj[kk];
                        lim[kk] = t16 ? (uint32_t)thr16[x] : thr32[x];
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < CB; ++kk) c += dd[kk] <= (lim[kk] < W ? lim[kk] : W);
        }
        return c;
    };

    A.S = cnt;
    uint32_t nf = 0, prev_t = 0, first_int = NO_START, last_int = NO_START, m_head = 0, m_tail = 0;
    for (uint32_t r0 = 0; r0 < cnt; r0 += 64) {
        const uint32_t r = r0 + (uint32_t)lane;
        const bool v = r < cnt;
        const uint32_t rc = v ? r : cnt - 1;
        uint32_t ti, sp;
        if (staged) {
            const uint64_t ev = lwin[own0 + rc];
            ti = (uint32_t)ev;
            sp = (uint32_t)(ev >> 32);
        } else {
            ti = sdt[(uint64_t)kt * TILE + rc];
            sp = sdp[(uint64_t)kt * TILE + rc];
        }
        const uint32_t pi = sp >> 16;
        const uint32_t rm = rmax[pi];
        const uint32_t Ri = W < rm ? W : rm;   // this seed's reach
        const uint32_t t_lo = ti > Ri ? ti - Ri : 0u;
        const uint64_t t_hi = (uint64_t)ti + Ri;
        uint32_t c = 0;
        if (staged) {
            uint32_t jlo = 0, jhi = 0;   // window seeds with time < t_lo, with time <= t_hi
            for (uint32_t step = top; step; step >>= 1) {
                const uint32_t ml = jlo + step, mr = jhi + step;
                if (ml <= tot && lt[2 * (ml - 1)] < t_lo) jlo = ml;
                if (mr <= tot && (uint64_t)lt[2 * (mr - 1)] <= t_hi) jhi = mr;
            }
            if (!v) jhi = jlo;
            c = count_range(ti, pi, Ri, jlo, jhi, own0 + r, (uint32_t)CAP - 1u, [&](uint32_t j) { return lwin[j]; });
        } else {
            // the window tile by tile from the lists in device memory
            for (uint32_t jt = jl; jt < jr; ++jt) {
                const uint32_t cj = gload(recs + jt).n;
                const TRIG_GAS uint32_t *tj = sdt + (uint64_t)jt * TILE;
                const TRIG_GAS uint32_t *pj = sdp + (uint64_t)jt * TILE;
                uint32_t jlo, jhi;   // first with time >= t_lo, first with time > t_hi
                {
                    uint32_t lo = 0, hi = cj;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (tj[mid] < t_lo) lo = mid + 1; else hi = mid;
                    }
                    jlo = lo;
                    hi = cj;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if ((uint64_t)tj[mid] <= t_hi) lo = mid + 1; else hi = mid;
                    }
                    jhi = v ? lo : jlo;
                }
                c += count_range(ti, pi, Ri, jlo, jhi, jt == kt ? r : 0xFFFFFFFFu, (uint32_t)TILE - 1u,
                                 [&](uint32_t j) { return (uint64_t)tj[j] | ((uint64_t)pj[j] << 32); });
            }
        }
        const uint32_t fd = c + 1;
        const bool f = v && fd >= N;
        const uint64_t M = __ballot(f);
        const uint32_t below = (uint32_t)__popcll(M & ((1ull << lane) - 1ull));
        if (f) {
            FireRec fr;
            fr.t = ti;
            fr.hit = o_idx[(uint64_t)kt * TILE + (sp & 0xFFFFu)];
            fr.fold = fd;
            fr.pmt = pi;
            gstore(slot + nf + below, fr);
        }
        // the summary over this round's fires: the previous fire of each is the
        // latest fire below it in the round (times are ordered: a max-scan), or the
        // last fire of the rounds before
        const uint32_t incl = wave_incl_max_u32(f ? ti + 1u : 0u);   // (times < 2^31: ti + 1 does not wrap)
        const uint32_t excl = wave_shr1(incl, 0u);
        const bool has_prev = (nf + below) > 0;
        const uint32_t tp = excl ? excl - 1u : prev_t;
        const bool is_int = f && has_prev && (uint64_t)(ti - tp) > twoH;
        const uint64_t ib = __ballot(is_int);
        if (M) {
            if (nf == 0) A.first_t = lane_read(ti, __ffsll((unsigned long long)M) - 1);
            prev_t = lane_read(ti, 63 - __clzll((long long)M));
            A.last_t = prev_t;
        }
        if (ib) {
            const int lo = __ffsll((unsigned long long)ib) - 1;
            const int hi = 63 - __clzll((long long)ib);
            if (first_int == NO_START) {
                first_int = nf + (uint32_t)__popcll(M & ((1ull << lo) - 1ull));
                m_head = umax(m_head, wave_max_all(f && lane < lo ? fd : 0u));
            }
            last_int = nf + (uint32_t)__popcll(M & ((1ull << hi) - 1ull));
            m_tail = wave_max_all(f && lane >= hi ? fd : 0u);
            A.ls_t = lane_read(ti, hi);
        } else {
            const uint32_t mx = wave_max_all(f ? fd : 0u);
            if (first_int == NO_START) m_head = umax(m_head, mx);
            m_tail = umax(m_tail, mx);
        }
        A.E_int += (uint32_t)__popcll(ib);
        nf += (uint32_t)__popcll(M);
    }
    A.F = nf;
    A.m_tail = m_tail;
    A.m_head = first_int == NO_START ? m_tail : m_head;
    A.ls_idx = last_int;
    if (last_int == NO_START) A.ls_t = 0;
    if (lane == 0) gstore(&gmem(S.tstat)[kt].agg, A);
}

template <int G, int CAP, bool BOUNDS>
hipError_t launch_fold_v(const BatchDev &b, hipStream_t s) {
    const size_t tb_bytes = ((size_t)(BOUNDS ? b.tbnd_lds : 0u) * 2 + 15) & ~(size_t)15;
    const size_t shm = tb_bytes + (size_t)G * FoldShape<CAP>::wave_bytes();
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_fold<G, CAP, BOUNDS>, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)(TBND_LDS_MAX * TBND_LDS_MAX * 2 + 16 + (size_t)G * FoldShape<CAP>::wave_bytes()));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_fold<G, CAP, BOUNDS>), dim3(((b.total_groups + 7) / 8) * 8), dim3(64 * G), shm, s, b);
    return hipGetLastError();
}

template <bool BOUNDS>
hipError_t launch_fold_b(const BatchDev &b, hipStream_t s) {
    const bool wide = b.window_cap > 512;
    switch (b.tile_group) {
    case 4: return wide ? launch_fold_v<4, 2048, BOUNDS>(b, s) : launch_fold_v<4, 512, BOUNDS>(b, s);
    case 2: return wide ? launch_fold_v<2, 2048, BOUNDS>(b, s) : launch_fold_v<2, 512, BOUNDS>(b, s);
    default: return wide ? launch_fold_v<1, 2048, BOUNDS>(b, s) : launch_fold_v<1, 512, BOUNDS>(b, s);
    }
}

// The variant with table bounds when a slice of the batch has them.  (For towers
// only, a copy of the whole table in LDS per workgroup cost more than the reads
// it saved: 0.36 against 0.21 ms on the 256-slice batch.)
hipError_t launch_fold(const BatchDev &b, hipStream_t s) {
    return b.any_bounds ? launch_fold_b<true>(b, s) : launch_fold_b<false>(b, s);
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

static hipError_t launch_trigger(const BatchDev &b, uint32_t max_pmt, uint32_t n_cu, bool dense, hipStream_t s,
                                 void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (!dense) {
        // level-0 pass bits of the ordered hits (the dense rerun keeps the first pass's)
        hipError_t e0 = trig_launch_l0(b, s, mark, mark_ctx);
        if (e0 != hipSuccess) return e0;
    }
    // the seed menu (SC, AFC, their combination) and its dense rerun run in
    // variants of the tile-per-workgroup kernel; the plain rule in the seed and
    // fold kernels
    const bool menu = b.prm.t_adj_ns >= 0 || b.prm.t_afloor_ns >= 0 || b.prm.seed_mode != 0;
    if (dense || menu) {
        TRIG_MARK("k_tile", 0);
        hipError_t e = dense ? launch_tile<HALO_BIG, true, false>(b, max_pmt, n_cu, s)
                             : launch_tile<HALO_SMALL, false, true>(b, max_pmt, n_cu, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_tile", 1);
    } else {
        TRIG_MARK("k_seed", 0);
        hipError_t e = launch_seed(b, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_seed", 1);
        TRIG_MARK("k_fold", 0);
        e = launch_fold(b, s);
        if (e != hipSuccess) return e;
        TRIG_MARK("k_fold", 1);
    }
    {
        const uint32_t nch = (b.max_tiles + TS_CH - 1) / TS_CH;
        if (nch > 1) {
            TRIG_MARK("k_tsum", 0);
            hipLaunchKernelGGL(k_tsum, dim3(nch, b.n_slices), dim3(TS_NT), 0, s, b);
            TRIG_CHECK();
            TRIG_MARK("k_tsum", 1);
        }
        TRIG_MARK("k_tscan", 0);
        hipLaunchKernelGGL(k_tscan, dim3(nch, b.n_slices), dim3(TS_NT), 0, s, b);
        TRIG_CHECK();
        TRIG_MARK("k_tscan", 1);
    }
    TRIG_MARK("k_place", 0);
    {
        // one wave per tile up to 8 per CU, then persistent waves; a multiple of the 8 XCDs
        const uint32_t cap = 8u * (n_cu ? n_cu : 1u);
        const uint32_t waves = b.total_tiles < cap ? b.total_tiles : cap;
        hipLaunchKernelGGL(k_place, dim3(((waves + 7) / 8) * 8), dim3(64), 0, s, b);
    }
    TRIG_CHECK();
    TRIG_MARK("k_place", 1);
    return hipSuccess;
}

hipError_t trig_launch_tail(const BatchDev &b, const TrigLaunchCfg &cfg, uint32_t max_pmt, hipStream_t s,
                            void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (!b.total_tiles) return hipSuccess;
    return launch_trigger(b, max_pmt, (uint32_t)cfg.n_cu, false, s, mark, mark_ctx);
}

hipError_t trig_launch_dense(const BatchDev &b, const TrigLaunchCfg &cfg, uint32_t max_pmt, hipStream_t s,
                             void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (!b.total_tiles) return hipSuccess;
    TRIG_MARK("k_dseed", 0);
    hipLaunchKernelGGL(k_dseed, dim3(b.total_tiles), dim3(NTD), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_dseed", 1);
    return launch_trigger(b, max_pmt, (uint32_t)cfg.n_cu, true, s, mark, mark_ctx);
}
