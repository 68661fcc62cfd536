// Stable LDS ranking of up to NT*E elements by an 8-bit digit (one radix pass).
//
// Element k of a workgroup's set sits at wave w, iteration e, lane l with
//   k = (w * E + e) * 64 + l,
// so the order in which a wave walks its elements is k order and equal digits
// keep their relative order (the pass is stable).  Lanes holding the same
// digit in one iteration are found with eight ballots (one per digit bit);
// each wave keeps its running per-digit counts in its own LDS histogram row,
// and a digit-major prefix over (digit, wave) turns those into ranks.
#pragma once

#include "trig_dev.h"

namespace trigdev {

template <int NT>
struct RankScratch {
    uint32_t hist[(NT / 64) * 256];
    uint32_t dbase[256];
    uint32_t scan[NT / 64 + 1];
};

// digit_of(k) -> 0..255 for k < m.  On return rank_in_digit[e] holds, for each of the
// thread's active elements, the number of elements before it with the same digit;
// sc.dbase[d] holds the number of elements with a smaller digit.  dig[e] the digit.
template <int NT, int E, class DigitOf>
__device__ __forceinline__ void block_rank8(int m, DigitOf digit_of, RankScratch<NT> &sc,
                                            uint32_t (&rank_in_digit)[E], uint32_t (&dig)[E]) {
    constexpr int NW = NT / 64;
    static_assert(NT >= 256, "one thread per digit for the column scan");
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int i = threadIdx.x; i < NW * 256; i += NT) sc.hist[i] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = (w * E + e) * 64 + lane;
        const bool act = k < m;
        const uint32_t d = act ? digit_of(k) : 0u;
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t r = 0;
        if (act) {
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            const uint32_t base = sc.hist[w * 256 + d];
            r = base + below;
            __builtin_amdgcn_wave_barrier();
            if (below == 0) sc.hist[w * 256 + d] = base + (uint32_t)__popcll(peers);
        } else {
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
        rank_in_digit[e] = r;
        dig[e] = d;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, total
    uint32_t tot = 0;
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t acc = 0;
        for (int ww = 0; ww < NW; ++ww) {
            uint32_t x = sc.hist[ww * 256 + d];
            sc.hist[ww * 256 + d] = acc;
            acc += x;
        }
        tot = acc;
    }
    __syncthreads();
    uint32_t all;
    uint32_t ex = block_excl_scan<NT>(threadIdx.x < 256 ? tot : 0u, all, sc.scan);
    if (threadIdx.x < 256) sc.dbase[threadIdx.x] = ex;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = (w * E + e) * 64 + lane;
        if (k < m) rank_in_digit[e] += sc.hist[w * 256 + dig[e]];
    }
}

}  // namespace trigdev
