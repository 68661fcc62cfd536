// Hit tagging and extraction (paper Sec. 4.2: once the trigger fires, the hits
// within +-3 us of a trigger seed are tagged and sent back to the host to be
// saved; Sec. 2: the 6 us window of tower data around the trigger is what the
// event manager stores).  A hit is tagged when it lies in one of the slice's
// merged event windows [t_begin, t_end], the union of the +-H windows of its
// fires.  The output is the tagged hits' input indices in the ordered-hit order
// (time, PMT, input index).  Runs after every pass that can change a slice's
// events, on the slices that asked for it:
//   k_tag_bits   per tile: tag bit of each ordered hit (one ballot word per 64
//                hits, in the seed-mask area) and the tile's count
//   k_tag_scan   per slice: exclusive scan of the tile counts, total to the plan
//   k_tag_write  per tile: input indices of its tagged hits at their places (in
//                the fire-scratch area, free once the fires are placed)
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NTT = 256;       // threads per tile workgroup
constexpr int EV_LDS = NTT;    // events over one tile's time range kept in LDS
static_assert(TILE % NTT == 0 && NTT % 64 == 0, "tile layout");

// A slice that asked for tags and whose events are final: ordered, triggered, and
// no dense-window rerun pending (that rerun replaces its events, then tags again).
__device__ __forceinline__ bool tag_slice(const SliceDev &S, const TRIG_GAS Plan *Pg) {
    const uint32_t st = Pg->state;
    const bool pending = Pg->dense && st != ST_DENSE;
    return S.tag_on && Pg->status == TRIG_OK && !pending && (st == ST_FAST || st == ST_GENERIC_DONE || st == ST_DENSE);
}

__global__ __launch_bounds__(NTT) void k_tag_bits(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return;
    const TRIG_GAS Plan *Pg = gmem(b.plans + si);
    if (!tag_slice(S, Pg)) return;
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) return;
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    const TRIG_GAS uint32_t *o_t = gmem(S.o_t);
    const TRIG_GAS trig_event *ev = gmem(S.events);
    const int64_t t_min = Pg->t_min;
    const uint32_t ne = Pg->n_events;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    __shared__ int64_t eb[EV_LDS], ee[EV_LDS];
    __shared__ uint32_t s_e0, s_cnt[NTT / 64];
    const int64_t lo = t_min + (int64_t)o_t[a], hi = t_min + (int64_t)o_t[e - 1];
    if (threadIdx.x == 0) {
        // events are disjoint and in time order: the first one ending at or after lo
        uint32_t l = 0, h = ne;
        while (l < h) {
            const uint32_t m = (l + h) >> 1;
            if (ev[m].t_end < lo) l = m + 1; else h = m;
        }
        s_e0 = l;
    }
    __syncthreads();
    const uint32_t e0 = s_e0;
    // the events from e0 on that begin at or before hi (a prefix), up to EV_LDS
    bool in = false;
    if (e0 + threadIdx.x < ne) {
        const int64_t tb = ev[e0 + threadIdx.x].t_begin;
        in = tb <= hi;
        eb[threadIdx.x] = tb;
        ee[threadIdx.x] = ev[e0 + threadIdx.x].t_end;
    }
    const uint32_t nl = (uint32_t)__syncthreads_count(in);
    // more of them than LDS holds (a sparse slice with many short events): each
    // hit searches the global list instead
    const bool spill = nl == (uint32_t)EV_LDS && e0 + EV_LDS < ne && ev[e0 + EV_LDS].t_begin <= hi;
    TRIG_GAS uint64_t *tbits = gmem(S.dmask);
    uint32_t cnt = 0;
    for (uint32_t x0 = 0; x0 < (uint32_t)TILE; x0 += NTT) {
        const uint64_t j = a + x0 + threadIdx.x;
        bool tg = false;
        if (j < e) {
            const int64_t t = t_min + (int64_t)o_t[j];
            if (!spill) {
                uint32_t l = 0, h = nl;
                while (l < h) {
                    const uint32_t m = (l + h) >> 1;
                    if (ee[m] < t) l = m + 1; else h = m;
                }
                tg = l < nl && eb[l] <= t;
            } else {
                uint32_t l = e0, h = ne;
                while (l < h) {
                    const uint32_t m = (l + h) >> 1;
                    if (ev[m].t_end < t) l = m + 1; else h = m;
                }
                tg = l < ne && ev[l].t_begin <= t;
            }
        }
        const uint64_t bal = __ballot(tg);
        if (lane == 0 && a + x0 + (uint32_t)w * 64 < e) tbits[(a + x0) / 64 + w] = bal;
        cnt += (uint32_t)__popcll(bal);
    }
    if (lane == 0) s_cnt[w] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < NTT / 64; ++i) tot += s_cnt[i];
        gmem(S.tagc)[k] = tot;
    }
}

// Per slice: tile counts -> exclusive prefixes (in place), total to the plan,
// and the plan once more to the host-mapped staging.
__global__ __launch_bounds__(1024) void k_tag_scan(BatchDev b) {
    constexpr int NTS = 1024;
    const uint32_t si = blockIdx.x;
    const SliceDev &S = b.slices[si];
    TRIG_GAS Plan *Pp = gmem(b.plans + si);
    if (!tag_slice(S, Pp) || S.n == 0) return;
    __shared__ uint32_t sh[NTS / 64 + 1];
    const uint32_t total = block_scan_array<NTS>(S.tagc, S.n_tiles, sh);
    if (threadIdx.x == 0) {
        Pp->n_tagged = total;
        if (b.x_plans) gstore(gmem(b.x_plans) + si, gload(Pp));
    }
}

__global__ __launch_bounds__(NTT) void k_tag_write(BatchDev b) {
    constexpr int WPT = TILE / 64;   // tag words per tile
    const uint32_t item = blockIdx.x;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    const uint32_t k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return;
    const TRIG_GAS Plan *Pg = gmem(b.plans + si);
    if (!tag_slice(S, Pg)) return;
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) return;
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    const uint32_t nw = (uint32_t)((e - a + 63) / 64);
    const TRIG_GAS uint64_t *tbits = gmem(S.dmask);
    __shared__ uint64_t sw[WPT];
    __shared__ uint32_t spre[WPT];
    if (threadIdx.x < (unsigned)WPT) sw[threadIdx.x] = threadIdx.x < nw ? tbits[a / 64 + threadIdx.x] : 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < WPT; ++i) {
            spre[i] = acc;
            acc += (uint32_t)__popcll(sw[i]);
        }
    }
    __syncthreads();
    const uint32_t base = gmem(S.tagc)[k];
    const TRIG_GAS uint32_t *o_idx = gmem(S.o_idx);
    TRIG_GAS uint32_t *out = gmem(S.tagged);
    // host-mapped staging too when the whole list fits it (else the host copies
    // the list from device memory)
    TRIG_GAS uint32_t *xout = (S.x_tagged && Pg->n_tagged <= S.x_tag_cap) ? gmem(S.x_tagged) : nullptr;
    const int lane = lane_id();
    for (uint32_t x = threadIdx.x; x < (uint32_t)TILE; x += NTT) {
        const uint64_t j = a + x;
        if (j >= e) break;
        const uint64_t word = sw[x / 64];
        if ((word >> lane) & 1ull) {
            const uint32_t r = spre[x / 64] + (uint32_t)__popcll(lane ? word & (~0ull >> (64 - lane)) : 0ull);
            const uint32_t v = o_idx[j];
            out[base + r] = v;
            if (xout) xout[base + r] = v;
        }
    }
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t trig_launch_tag(const BatchDev &b, hipStream_t s, void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (!b.total_tiles) return hipSuccess;
    TRIG_MARK("k_tag_bits", 0);
    hipLaunchKernelGGL(k_tag_bits, dim3(b.total_tiles), dim3(NTT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_tag_bits", 1);
    TRIG_MARK("k_tag_scan", 0);
    hipLaunchKernelGGL(k_tag_scan, dim3(b.n_slices), dim3(1024), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_tag_scan", 1);
    TRIG_MARK("k_tag_write", 0);
    hipLaunchKernelGGL(k_tag_write, dim3(b.total_tiles), dim3(NTT), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_tag_write", 1);
    return hipSuccess;
}
