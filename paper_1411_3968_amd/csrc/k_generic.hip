// General ordering path: a device-wide stable LSD radix sort of one slice by the
// key ((t - t_min) << pbits | pmt), starting from input order, so that equal
// (t, pmt) keys stay in input-position order.  Used when the input is not a
// concatenation of a modest number of time-ordered runs, or when one time segment
// of the run-merge path is denser than its LDS capacity.
#include "radix_lds.h"
#include "trig_dev.h"

using namespace trigdev;

namespace {

constexpr int NT = 256;
constexpr int E = GTILE / NT;

__global__ __launch_bounds__(NT) void k_gkeys(SliceDev S, Plan P, uint64_t *key, uint32_t *val) {
    const uint64_t k = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (k >= S.n) return;
    key[k] = ((uint64_t)(S.t[k] - P.t_min) << S.pbits) | (uint64_t)S.pmt[k];
    val[k] = (uint32_t)k;
}

// Digit counts of one 4096-element block, stored digit-major: hist[d * nblk + blk].
__global__ __launch_bounds__(NT) void k_ghist(uint64_t n, const uint64_t *key, uint32_t shift, uint32_t nblk,
                                              uint32_t *hist) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * GTILE;
    for (int e = 0; e < E; ++e) {
        const uint64_t k = b0 + (uint64_t)e * NT + threadIdx.x;
        if (k < n) atomicAdd(&cnt[(uint32_t)(key[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of the whole histogram (one block, chunked).
__global__ __launch_bounds__(1024) void k_gscan(uint32_t *hist, uint64_t len) {
    __shared__ uint32_t sh[1024 / 64 + 1];
    uint32_t acc = 0;
    for (uint64_t i0 = 0; i0 < len; i0 += 1024) {
        const uint64_t i = i0 + threadIdx.x;
        const uint32_t v = i < len ? hist[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(v, tot, sh);
        if (i < len) hist[i] = acc + ex;
        acc += tot;
    }
}

// Stable scatter of one block: block-local rank within the digit plus the digit's
// global offset for this block.
__global__ __launch_bounds__(NT) void k_gscatter(uint64_t n, const uint64_t *key, const uint32_t *val,
                                                 uint64_t *key2, uint32_t *val2, uint32_t shift, uint32_t nblk,
                                                 const uint32_t *hist) {
    __shared__ RankScratch<NT> rs;
    const uint64_t b0 = (uint64_t)blockIdx.x * GTILE;
    const int m = (int)((n - b0) < (uint64_t)GTILE ? (n - b0) : (uint64_t)GTILE);
    uint64_t kk[E];
    uint32_t vv[E];
    const int w = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = (w * E + e) * 64 + lane;
        if (k < m) { kk[e] = key[b0 + k]; vv[e] = val[b0 + k]; }
    }
    uint32_t rk[E], dg[E];
    auto digit_of = [&](int k) -> uint32_t {
        return (uint32_t)(key[b0 + k] >> shift) & 255u;
    };
    block_rank8<NT, E>(m, digit_of, rs, rk, dg);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = (w * E + e) * 64 + lane;
        if (k < m) {
            const uint64_t dst = (uint64_t)hist[(uint64_t)dg[e] * nblk + blockIdx.x] + rk[e];
            key2[dst] = kk[e];
            val2[dst] = vv[e];
        }
    }
}

__global__ __launch_bounds__(NT) void k_gfinish(SliceDev S, const uint64_t *key, const uint32_t *val) {
    const uint64_t k = (uint64_t)blockIdx.x * NT + threadIdx.x;
    if (k == 0) { S.plan->state = ST_GENERIC_DONE; S.plan->generic = 1; }
    if (k >= S.n) return;
    const uint64_t kv = key[k];
    const uint32_t v = val[k];
    const uint32_t pmask = (S.pbits >= 32) ? 0xFFFFFFFFu : ((1u << S.pbits) - 1u);
    S.o_t[k] = (uint32_t)(kv >> S.pbits);
    S.o_pq[k] = (((uint32_t)kv & pmask) << 16) | (uint32_t)S.q[v];
    S.o_idx[k] = v;
}

}  // namespace

size_t trig_generic_scratch_bytes(uint64_t n) {
    const uint64_t nblk = (n + GTILE - 1) / GTILE;
    return 2 * n * sizeof(uint64_t) + 2 * n * sizeof(uint32_t) + 256 * nblk * sizeof(uint32_t) + 1024;
}

#define TRIG_MARK(name, ph) do { if (mark) mark(mark_ctx, name, ph); } while (0)
#define TRIG_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

// The slice descriptor and plan are read back by the host before this call
// (the general path is chosen from the plan), so they arrive by value.
hipError_t trig_launch_generic_slice(const SliceDev &S, const Plan &P, uint32_t key_bits, void *scratch,
                                     hipStream_t s, void (*mark)(void *, const char *, int), void *mark_ctx) {
    const uint64_t n = S.n;
    if (n == 0) return hipSuccess;
    const uint64_t nblk = (n + GTILE - 1) / GTILE;
    uint64_t *key0 = (uint64_t *)scratch;
    uint64_t *key1 = key0 + n;
    uint32_t *val0 = (uint32_t *)(key1 + n);
    uint32_t *val1 = val0 + n;
    uint32_t *hist = val1 + n;
    const uint32_t g1 = (uint32_t)((n + NT - 1) / NT);
    TRIG_MARK("k_gkeys", 0);
    hipLaunchKernelGGL(k_gkeys, dim3(g1), dim3(NT), 0, s, S, P, key0, val0);
    TRIG_CHECK();
    TRIG_MARK("k_gkeys", 1);
    const int passes = (int)((key_bits + 7) / 8);
    for (int ps = 0; ps < passes; ++ps) {
        const uint32_t sh = 8u * (uint32_t)ps;
        TRIG_MARK("k_gpass", 0);
        hipLaunchKernelGGL(k_ghist, dim3((uint32_t)nblk), dim3(NT), 0, s, n, key0, sh, (uint32_t)nblk, hist);
        TRIG_CHECK();
        hipLaunchKernelGGL(k_gscan, dim3(1), dim3(1024), 0, s, hist, (uint64_t)256 * nblk);
        TRIG_CHECK();
        hipLaunchKernelGGL(k_gscatter, dim3((uint32_t)nblk), dim3(NT), 0, s, n, key0, val0, key1, val1, sh,
                           (uint32_t)nblk, hist);
        TRIG_CHECK();
        TRIG_MARK("k_gpass", 1);
        uint64_t *tk = key0; key0 = key1; key1 = tk;
        uint32_t *tv = val0; val0 = val1; val1 = tv;
    }
    TRIG_MARK("k_gfinish", 0);
    hipLaunchKernelGGL(k_gfinish, dim3(g1), dim3(NT), 0, s, S, key0, val0);
    TRIG_CHECK();
    TRIG_MARK("k_gfinish", 1);
    return hipSuccess;
}
