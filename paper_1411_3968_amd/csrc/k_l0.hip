// Level-0 prefilter (paper Sec. 3: a level-0 trigger of N hits in a fixed time
// window TW, N7TW1000, and N7TW500 for the 84-PMT tower; Sec. 4.1: DN7TW1000
// asks for hits of N different PMTs).  On the time-ordered hits of a slice, a
// hit passes when some window [t_i, t_i + TW) that starts at a hit i and holds
// the hit also holds >= N hits (>= N distinct PMTs for the DN form).  The seed
// rule then runs on the hits that pass.
//   k_l0_ok    per ordered position i: the window starting at i holds enough
//              (counting hits: t[i + N - 1] - t[i] < TW)
//   k_l0_pass  per ordered position x: some start i <= x within TW of it is ok
//              (counting hits, the starts x - N + 1 .. x suffice)
// Both write one ballot word per 64 positions; the ok words live in the seed
// mask area, which the dense rerun overwrites later, the pass words in their own.
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NTL = 256;
static_assert(TILE % NTL == 0, "tile layout");

__device__ __forceinline__ bool l0_slice(const BatchDev &b, const SliceDev &S, uint32_t &k, uint32_t si,
                                         uint32_t item) {
    k = item - tile_base_of(b, si);
    if (k >= S.n_tiles) return false;
    return slice_in_tail(b, gmem(b.plans + si)->state);
}

// The distinct-PMT form stages its tile and DN_HALO ordered neighbours (after
// the tile for the windows that start in it, before it for the starts that hold
// its hits) in LDS; a window reaching past them reads global memory.
constexpr int DN_HALO = 512;

__global__ __launch_bounds__(NTL) void k_l0_ok(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    uint32_t k;
    if (!l0_slice(b, S, k, si, item)) return;
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) return;
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    const TRIG_GAS uint32_t *o_t = gmem(S.o_t);
    const TRIG_GAS uint32_t *o_pq = gmem(S.o_pq);
    TRIG_GAS uint64_t *okw = gmem(S.dmask);
    const uint32_t N = b.prm.l0_n, TW = b.prm.l0_tw_ns;
    const bool distinct = b.prm.l0_distinct != 0;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    __shared__ uint32_t lt[TILE + DN_HALO];
    __shared__ uint16_t lp[TILE + DN_HALO];
    const uint64_t se = distinct ? ((e + DN_HALO < n) ? e + DN_HALO : n) : a;   // staged [a, se)
    if (distinct) {
        for (uint32_t x = threadIdx.x; x < (uint32_t)(se - a); x += NTL) {
            lt[x] = o_t[a + x];
            lp[x] = (uint16_t)(o_pq[a + x] >> 16);
        }
        __syncthreads();
    }
    auto t_at = [&](uint64_t m) -> uint32_t { return m < se ? lt[m - a] : o_t[m]; };
    auto p_at = [&](uint64_t m) -> uint32_t { return m < se ? (uint32_t)lp[m - a] : (o_pq[m] >> 16); };
    for (uint32_t x0 = 0; x0 < (uint32_t)TILE; x0 += NTL) {
        const uint64_t i = a + x0 + threadIdx.x;
        bool ok = false;
        if (i < e) {
            if (!distinct) {
                ok = i + N - 1 < n && o_t[i + N - 1] - o_t[i] < TW;
            } else {
                // distinct PMTs among the hits from i on within TW (stop at N)
                const uint32_t ti = t_at(i);
                uint32_t c = 0;
                for (uint64_t m = i; m < n && t_at(m) - ti < TW && c < N; ++m) {
                    const uint32_t pm = p_at(m);
                    bool dup = false;
                    for (uint64_t u = i; u < m && !dup; ++u) dup = p_at(u) == pm;
                    c += dup ? 0u : 1u;
                }
                ok = c >= N;
            }
        }
        const uint64_t bal = __ballot(ok);
        if (lane == 0 && a + x0 + (uint32_t)w * 64 < e) okw[(a + x0) / 64 + w] = bal;
    }
}

__device__ __forceinline__ bool bit_at(const TRIG_GAS uint64_t *wv, uint64_t j) { return (wv[j >> 6] >> (j & 63)) & 1ull; }

__global__ __launch_bounds__(NTL) void k_l0_pass(BatchDev b) {
    const uint32_t item = blockIdx.x;
    const uint32_t si = slice_of_tile(b, item);
    const SliceDev &S = b.slices[si];
    uint32_t k;
    if (!l0_slice(b, S, k, si, item)) return;
    const uint64_t n = S.n;
    const uint64_t a = (uint64_t)k * TILE;
    if (a >= n) return;
    const uint64_t e = (a + TILE < n) ? a + TILE : n;
    const TRIG_GAS uint32_t *o_t = gmem(S.o_t);
    const TRIG_GAS uint64_t *okw = gmem(S.dmask);
    TRIG_GAS uint64_t *pw = gmem(S.l0m);
    const uint32_t N = b.prm.l0_n, TW = b.prm.l0_tw_ns;
    const bool distinct = b.prm.l0_distinct != 0;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    // the distinct-PMT form: times of the tile and DN_HALO positions before it in LDS
    __shared__ uint32_t lt[TILE + DN_HALO];
    const uint64_t s0 = distinct ? (a > (uint64_t)DN_HALO ? a - DN_HALO : 0) : a;   // staged [s0, e)
    if (distinct) {
        for (uint32_t x = threadIdx.x; x < (uint32_t)(e - s0); x += NTL) lt[x] = o_t[s0 + x];
        __syncthreads();
    }
    auto t_at = [&](uint64_t m) -> uint32_t { return m >= s0 && m < e ? lt[m - s0] : o_t[m]; };
    for (uint32_t x0 = 0; x0 < (uint32_t)TILE; x0 += NTL) {
        const uint64_t x = a + x0 + threadIdx.x;
        bool pass = false;
        if (x < e && !distinct) {
            // counting hits: an ok start i in x - N + 1 .. x holds x (t_x <= t_{i+N-1}
            // < t_i + TW), and a start before that is matched by a later one, so x
            // passes exactly when one of those N bits is set (N <= 64: two words)
            const uint64_t lo = x + 1 >= N ? x + 1 - N : 0;
            const uint64_t wx = okw[x >> 6], hi_mask = (x & 63) == 63 ? ~0ull : ((2ull << (x & 63)) - 1ull);
            if ((lo >> 6) == (x >> 6)) {
                pass = (wx & hi_mask & (~0ull << (lo & 63))) != 0;
            } else {
                pass = (wx & hi_mask) != 0 || (okw[lo >> 6] & (~0ull << (lo & 63))) != 0;
            }
        } else if (x < e) {
            // counting PMTs: every start at or before x (in time order) that still holds x
            const uint32_t tx = t_at(x);
            for (uint64_t i = x + 1; i-- > 0 && !pass;) {
                if (tx - t_at(i) >= TW) break;
                pass = bit_at(okw, i);
            }
        }
        const uint64_t bal = __ballot(pass);
        if (lane == 0 && a + x0 + (uint32_t)w * 64 < e) pw[(a + x0) / 64 + w] = bal;
    }
}

}  // namespace

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t trig_launch_l0(const BatchDev &b, hipStream_t s, void (*mark)(void *, const char *, int), void *mark_ctx) {
    if (!b.total_tiles || b.prm.l0_n == 0) return hipSuccess;
    TRIG_MARK("k_l0_ok", 0);
    hipLaunchKernelGGL(k_l0_ok, dim3(b.total_tiles), dim3(NTL), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_l0_ok", 1);
    TRIG_MARK("k_l0_pass", 0);
    hipLaunchKernelGGL(k_l0_pass, dim3(b.total_tiles), dim3(NTL), 0, s, b);
    TRIG_CHECK();
    TRIG_MARK("k_l0_pass", 1);
    return hipSuccess;
}
