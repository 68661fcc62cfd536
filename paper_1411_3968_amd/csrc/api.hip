// Host side of libtrig: context, geometry upload, workspace layout, the
// synchronous slice / batch entry points, per-kernel timing and tuning.
// The serving loop (stream submit / poll) lives in serve.hip.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "api_internal.h"

using namespace trigdev;

// ------------------------------------------------------------------ errors

void ctx_set_error(trig_ctx *c, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> g(c->err_mu);
    c->err = buf;
}

int hip_fail(trig_ctx *c, hipError_t e, const char *where) {
    ctx_set_error(c, "%s: %s", where, hipGetErrorString(e));
    return TRIG_EHIP;
}

// ----------------------------------------------------------- device memory

int ctx_reserve(trig_ctx *c, uint64_t bytes) {
    std::lock_guard<std::mutex> g(c->mem_mu);
    if (c->bytes_in_use + bytes > c->budget) return TRIG_ENOMEM;
    c->bytes_in_use += bytes;
    c->bytes_peak = std::max(c->bytes_peak, c->bytes_in_use);
    return TRIG_OK;
}

void ctx_release(trig_ctx *c, uint64_t bytes) {
    std::lock_guard<std::mutex> g(c->mem_mu);
    c->bytes_in_use -= std::min(c->bytes_in_use, bytes);
}

int DevBuf::ensure(trig_ctx *c, size_t want, hipStream_t s) {
    if (want <= cap) return TRIG_OK;
    size_t nc = std::max(want, cap + cap / 2);
    nc = (nc + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    if (ctx_reserve(c, nc - cap) != TRIG_OK) {
        nc = want;
        if (ctx_reserve(c, nc - cap) != TRIG_OK) {
            ctx_set_error(c, "device budget of %llu bytes exceeded (need %llu more)",
                          (unsigned long long)c->budget, (unsigned long long)(nc - cap));
            return TRIG_ENOMEM;
        }
    }
    if (ptr) {
        hipStreamSynchronize(s);
        hipFree(ptr);
        ptr = nullptr;
    }
    hipError_t e = hipMalloc(&ptr, nc);
    if (e != hipSuccess) {
        ctx_release(c, nc);
        ctx_release(c, cap);
        cap = 0;
        ptr = nullptr;
        ctx_set_error(c, "hipMalloc(%zu): %s", nc, hipGetErrorString(e));
        return TRIG_ENOMEM;
    }
    cap = nc;
    return TRIG_OK;
}

void DevBuf::release(trig_ctx *c) {
    if (ptr) hipFree(ptr);
    ctx_release(c, cap);
    ptr = nullptr;
    cap = 0;
}

int PinBuf::ensure(size_t want) {
    if (want <= cap) return TRIG_OK;
    if (ptr) hipHostFree(ptr);
    ptr = nullptr;
    size_t nc = std::max(want, (size_t)4096);
    if (hipHostMalloc(&ptr, nc, hipHostMallocDefault) != hipSuccess) {
        ptr = nullptr;
        cap = 0;
        return TRIG_ENOMEM;
    }
    cap = nc;
    return TRIG_OK;
}

void PinBuf::release() {
    if (ptr) hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
}

// ------------------------------------------------------------------ tuning

trig_tune ctx_tune_for(const trig_ctx *c, uint32_t n_pmt) {
    for (const auto &t : c->tunes)
        if (n_pmt <= t.first) return t.second;
    return c->tunes.back().second;
}

static uint32_t pbits_of(uint32_t n_pmt) {
    return n_pmt <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(n_pmt - 1);
}

// ---------------------------------------------------------------- profiling

static void prof_mark(void *vc, const char *name, int phase) {
    trig_ctx *c = (trig_ctx *)vc;
    if (!c->prof_on) return;
    hipEvent_t ev;
    if (c->ev_pool.empty()) {
        if (hipEventCreate(&ev) != hipSuccess) return;
    } else {
        ev = c->ev_pool.back();
        c->ev_pool.pop_back();
    }
    hipEventRecord(ev, c->prof_stream);
    c->prof_pending.push_back({name, phase, ev});
}

// Called after the profiled stream was synchronised.
static void prof_collect(trig_ctx *c) {
    std::vector<ProfMark> &v = c->prof_pending;
    for (size_t i = 0; i < v.size(); ++i) {
        if (v[i].phase != 0) continue;
        for (size_t j = i + 1; j < v.size(); ++j) {
            if (v[j].phase == 1 && v[j].name == v[i].name) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, v[i].ev, v[j].ev) == hipSuccess) {
                    auto it = std::find_if(c->prof.begin(), c->prof.end(),
                                           [&](const trig_kernel_time &k) { return v[i].name == k.name; });
                    if (it == c->prof.end()) {
                        trig_kernel_time k = {};
                        snprintf(k.name, sizeof k.name, "%s", v[i].name.c_str());
                        c->prof.push_back(k);
                        it = c->prof.end() - 1;
                    }
                    it->launches += 1;
                    it->total_ms += ms;
                }
                break;
            }
        }
    }
    for (auto &m : v) c->ev_pool.push_back(m.ev);
    v.clear();
}

// ------------------------------------------------------------ one job

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte layout of one slice's workspace; returns the size.
static size_t slice_layout(uint64_t n, bool host_input, bool want_flags, SliceLayout &L) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    const uint64_t n_chunks = (n + CHUNK - 1) / CHUNK;
    const uint64_t n_tiles = (n + TILE - 1) / TILE;
    L.pos_cap = 3 * n + 65536;
    L.in_pmt = host_input ? take(n * 2) : SIZE_MAX;
    L.in_t = host_input ? take(n * 8) : SIZE_MAX;
    L.in_q = host_input ? take(n * 2) : SIZE_MAX;
    L.part = take(std::max<uint64_t>(n_chunks, 1) * sizeof(ChunkPart));
    L.ppart = take((std::max<uint64_t>(n_chunks, 1) + PL_CH - 1) / PL_CH * sizeof(PlanPart));
    L.pos = take(L.pos_cap * 4);
    L.o_t = take(n * 4 + 4);
    L.o_pq = take(n * 4 + 4);
    L.o_idx = take(n * 4 + 4);
    L.tstat = take(std::max<uint64_t>(n_tiles, 1) * sizeof(TileStat));
    L.cagg = take((std::max<uint64_t>(n_tiles, 1) + TS_CH - 1) / TS_CH * sizeof(TileAgg));
    L.dmask = take((n / 64 + 1) * 8);
    L.fsc = take(std::max<uint64_t>(n_tiles, 1) * TILE * sizeof(FireRec));
    L.fires = take(n * sizeof(trig_fire) + 32);
    L.events = take(n * sizeof(trig_event) + 32);
    L.flags = want_flags ? take(n + 4) : SIZE_MAX;
    L.tagc = take(std::max<uint64_t>(n_tiles, 1) * 4);
    L.l0m = take((n / 64 + 1) * 8);
    return o;
}

// Descriptors, then the per-slice chunk and tile bases (two dense arrays that the
// kernels binary-search), then plans and counters.
static size_t desc_upload_bytes(uint32_t n) { return n * sizeof(SliceDev) + 2 * (size_t)n * sizeof(uint32_t); }

size_t job_meta_bytes(uint32_t n, uint32_t total_tiles) {
    // descriptors, plans, counters, then the maps from groups, tiles and chunks
    // to their slice (at most total_tiles entries each)
    return align256(desc_upload_bytes(n)) + align256(n * sizeof(Plan)) + 256 + 3 * align256((size_t)total_tiles * 4);
}

// Fixed memory: descriptors, plans and counters, then the radix scratch of
// slices of at most 30 hits (a larger slice holds it in its own fire and event
// areas), then `ws_total` bytes of slice workspaces.
static constexpr size_t FIXED_GEN_BYTES = 4096;
static size_t fixed_layout_bytes(size_t ws_total, uint32_t n, uint32_t total_tiles) {
    return align256(job_meta_bytes(n, total_tiles)) + FIXED_GEN_BYTES + ws_total;
}

size_t slice_footprint(uint64_t n, bool host_input) {
    SliceLayout L;
    return slice_layout(n, host_input, false, L) + align256(sizeof(SliceDev)) + align256(sizeof(Plan));
}

// Device address of a caller's host buffer of `bytes` bytes when it is pinned
// (HIP host memory, so the kernels can write the results there directly), else
// null.  Asked only for lists worth it: below 1 MiB the copy from the staging
// costs less than the query.
static void *pinned_dev_ptr(const void *p, size_t bytes) {
    if (!p || bytes < (1u << 20)) return nullptr;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return at.type == hipMemoryTypeHost ? at.devicePointer : nullptr;
}

int Job::prepare(trig_ctx *c, uint32_t n, const trig_slice_desc *d, const trig_params *prm,
                 const uint8_t *want_flags, const uint64_t *fire_caps, const uint64_t *event_caps, hipStream_t s,
                 const uint8_t *want_tags, const uint64_t *tag_caps, const trig_result *res) {
    stream = s;
    params = *prm;
    slices.assign(n, SliceInfo{});
    any_tag = reran = false;
    size_t total = 0;
    uint32_t chunk_base = 0, tile_base = 0;
    uint32_t cap_max = 0;
    sort_kernels = 0;
    max_pmt = 0;
    wave_wgs = 0;
    wave_cap = 0;
    block_wgs = 0;
    for (uint32_t i = 0; i < n; ++i) {
        SliceInfo &si = slices[i];
        si.desc = d[i];
        si.host_status = TRIG_OK;
        if (d[i].geom_id >= c->geoms.size()) {
            si.host_status = TRIG_EINVAL;
            ctx_set_error(c, "slice %u: unknown geom_id %u", i, d[i].geom_id);
        } else if (d[i].n_hits >= (1ull << 32)) {
            si.host_status = TRIG_ERANGE;
            ctx_set_error(c, "slice %u: n_hits >= 2^32", i);
        } else if (d[i].n_hits && (!d[i].pmt_id || !d[i].t_ns || !d[i].charge)) {
            si.host_status = TRIG_EINVAL;
            ctx_set_error(c, "slice %u: null input array", i);
        } else if (d[i].mem != TRIG_MEM_HOST && d[i].mem != TRIG_MEM_DEVICE) {
            si.host_status = TRIG_EINVAL;
            ctx_set_error(c, "slice %u: bad mem kind", i);
        }
        const uint64_t nh = si.host_status == TRIG_OK ? d[i].n_hits : 0;
        si.n = nh;
        si.want_flags = want_flags && want_flags[i];
        si.want_tag = want_tags && want_tags[i];
        any_tag |= si.want_tag;
        si.ws_off = total;
        total += slice_layout(nh, d[i].mem == TRIG_MEM_HOST, si.want_flags, si.L);
        si.chunk_base = chunk_base;
        si.n_chunks = (uint32_t)((nh + CHUNK - 1) / CHUNK);
        si.tile_base = tile_base;
        si.n_tiles = std::max<uint32_t>(1, (uint32_t)((nh + TILE - 1) / TILE));
        chunk_base += si.n_chunks;
        tile_base += si.n_tiles;
        const uint32_t np = (d[i].geom_id < c->geoms.size()) ? c->geoms[d[i].geom_id].n_pmt : 1u;
        max_pmt = std::max(max_pmt, np);
        si.tune = ctx_tune_for(c, np);
        if (si.host_status == TRIG_OK && nh) {
            if (si.tune.seg_cap <= (uint32_t)WAVE_CAP) {
                sort_kernels |= 1u;
                wave_wgs = std::max(wave_wgs, si.tune.grid_per_cu);
                wave_cap = std::max(wave_cap, si.tune.seg_cap);
                if (np > (uint32_t)WAVE_RUNS) sort_kernels |= 4u;   // a slice may take the two-level merge
            } else {
                sort_kernels |= 2u;
                cap_max = std::max(cap_max, si.tune.seg_cap);
                block_wgs = std::max(block_wgs, si.tune.grid_per_cu);
            }
        }
    }
    seg_cap = cap_max ? cap_max : 4096;
    // pinned result staging: plans, then per slice min(n, cap) fires and events,
    // and the tagged list when asked for; a list whose caller buffer is pinned
    // host memory is written there directly instead
    size_t xs = align256(n * sizeof(Plan));
    for (uint32_t i = 0; i < n; ++i) {
        SliceInfo &si = slices[i];
        const uint64_t dflt = si.n / 16 + 4096;
        const uint64_t fc = std::min<uint64_t>(si.n, fire_caps ? fire_caps[i] : dflt);
        const uint64_t ec = std::min<uint64_t>(si.n, event_caps ? event_caps[i] : dflt);
        const uint64_t tc = si.want_tag ? std::min<uint64_t>(si.n, tag_caps ? tag_caps[i] : dflt) : 0;
        si.direct_f = nullptr;
        si.direct_e = nullptr;
        si.direct_t = nullptr;
        if (res && !fixed_ws && si.host_status == TRIG_OK) {
            si.direct_f = (trig_fire *)pinned_dev_ptr(res[i].fires, fc * sizeof(trig_fire));
            si.direct_e = (trig_event *)pinned_dev_ptr(res[i].events, ec * sizeof(trig_event));
            si.direct_t = si.want_tag ? (uint32_t *)pinned_dev_ptr(res[i].tagged, tc * sizeof(uint32_t)) : nullptr;
        }
        si.x_fcap = (uint32_t)fc;
        si.x_ecap = (uint32_t)ec;
        si.x_tcap = (uint32_t)tc;
        si.x_off_f = xs;
        if (!si.direct_f) xs = align256(xs + fc * sizeof(trig_fire));
        si.x_off_e = xs;
        if (!si.direct_e) xs = align256(xs + ec * sizeof(trig_event));
        si.x_off_t = xs;
        if (!si.direct_t) xs = align256(xs + tc * sizeof(uint32_t));
    }
    total_chunks = chunk_base;
    total_tiles = tile_base;
    // fold-kernel groups: the largest tile group and window capacity the slices'
    // classes ask for, fewer tiles per group while that would leave a compute unit
    // with less than two workgroups
    tile_group = 1;
    window_cap = 512;
    for (const SliceInfo &si : slices) {
        tile_group = std::max(tile_group, si.tune.tile_group);
        window_cap = std::max(window_cap, si.tune.window_cap);
    }
    auto count_groups = [&](uint32_t g) {
        uint32_t tot = 0;
        for (const SliceInfo &si : slices) tot += groups_of(si.n_tiles, g);
        return tot;
    };
    while (tile_group > 1 && count_groups(tile_group) < 2u * (uint32_t)std::max(1, c->cfg.n_cu)) tile_group /= 2;
    total_groups = 0;
    for (SliceInfo &si : slices) {
        si.group_base = total_groups;
        total_groups += groups_of(si.n_tiles, tile_group);
    }
    const size_t desc_bytes = job_meta_bytes(n, total_tiles);
    const bool fixed = fixed_ws != nullptr;
    if (fixed) {
        // one region for everything: descriptors, plans and counters first, then
        // the radix scratch of tiny slices, then the slices' workspaces
        const size_t need = fixed_layout_bytes(total, n, total_tiles);
        const size_t pin_need = align256(desc_upload_bytes(n)) + n * sizeof(Plan);
        if (need > fixed_cap || pin_need > fixed_pin_cap) {
            ctx_set_error(c, "slice needs %zu bytes of the fixed scratch, which holds %zu", need, fixed_cap);
            return TRIG_ENOMEM;
        }
        ext_ws.clear();
    }
    const bool own_ws = ext_ws.empty() && !fixed;
    if (!ext_ws.empty()) {
        bool bad = ext_ws.size() != n;
        for (uint32_t i = 0; !bad && i < n; ++i) bad = d[i].mem == TRIG_MEM_HOST && d[i].n_hits;
        if (bad) {   // caller-supplied workspaces hold no input staging
            ctx_set_error(c, "internal: workspace bases need %u device-resident slices", n);
            return TRIG_EINVAL;
        }
    }
    char *meta = nullptr, *base = nullptr;
    SliceDev *hs = nullptr;
    if (fixed) {
        meta = fixed_ws;
        fixed_gen = fixed_ws + align256(desc_bytes);
        base = fixed_gen + FIXED_GEN_BYTES;
        hs = (SliceDev *)fixed_pin;
        x_plans_dev = nullptr;   // results are read back by copies
        for (uint32_t i = 0; i < n; ++i) slices[i].x_fcap = slices[i].x_ecap = slices[i].x_tcap = 0;
    } else {
        int rc = own_ws ? ws.ensure(c, total, s) : TRIG_OK;
        if (rc) return rc;
        rc = dmeta.ensure(c, desc_bytes, s);
        if (rc) return rc;
        if (h_slices.ensure(desc_upload_bytes(n) + 64) || h_plans.ensure(xs + 64)) {
            ctx_set_error(c, "pinned host allocation failed");
            return TRIG_ENOMEM;
        }
        void *dp = nullptr;
        hipError_t e0 = hipHostGetDevicePointer(&dp, h_plans.ptr, 0);
        if (e0 != hipSuccess) return hip_fail(c, e0, "mapping the result staging");
        x_plans_dev = (Plan *)dp;
        meta = (char *)dmeta.ptr;
        base = (char *)ws.ptr;
        hs = (SliceDev *)h_slices.ptr;
    }
    d_slices = (SliceDev *)meta;
    d_plans = (Plan *)(meta + align256(desc_upload_bytes(n)));
    // (the counters are written by k_bounds before any kernel reads them)
    d_counters = (uint32_t *)((char *)d_plans + align256(n * sizeof(Plan)));
    // (the group, tile and chunk maps are written by k_plan before any kernel reads them)
    d_group_slice = (uint32_t *)((char *)d_counters + 256);
    d_tile_slice = (uint32_t *)((char *)d_group_slice + align256((size_t)total_tiles * 4));
    d_chunk_slice = (uint32_t *)((char *)d_tile_slice + align256((size_t)total_tiles * 4));
    for (uint32_t i = 0; i < n; ++i) {
        SliceInfo &si = slices[i];
        SliceDev S;
        std::memset(&S, 0, sizeof S);   // padding too: descriptors are compared bytewise
        char *b = ext_ws.empty() ? base + si.ws_off : ext_ws[i];   // (fixed memory: base is its workspace part)
        const SliceLayout &L = si.L;
        const uint64_t nh = si.n;
        if (si.host_status == TRIG_OK) {
            const GeomDev &g = c->geoms[si.desc.geom_id];
            S.floor_id = g.floor_id;
            S.floor16 = g.floor16;
            S.thr32 = g.thr32;
            S.thr16 = g.thr16;
            S.adj32 = g.adj32;
            S.afl32 = g.afl32;
            S.tbnd = g.tbnd;
            S.nbk = g.nbk;
            S.rmax = g.rmax;
            S.thr_max = g.thr_max;
            S.n_pmt = g.n_pmt;
            S.pbits = pbits_of(g.n_pmt);
        } else {
            const GeomDev &g = c->geoms.empty() ? GeomDev{} : c->geoms[0];
            S.floor_id = g.floor_id; S.thr32 = g.thr32; S.thr16 = g.thr16; S.n_pmt = std::max(1u, g.n_pmt);
        }
        if (si.desc.mem == TRIG_MEM_HOST && nh) {
            S.pmt = (const uint16_t *)(b + L.in_pmt);
            S.t = (const int64_t *)(b + L.in_t);
            S.q = (const uint16_t *)(b + L.in_q);
            hipError_t e = hipMemcpyAsync((void *)S.pmt, si.desc.pmt_id, nh * 2, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync((void *)S.t, si.desc.t_ns, nh * 8, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync((void *)S.q, si.desc.charge, nh * 2, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(c, e, "H2D of slice inputs");
        } else {
            S.pmt = si.desc.pmt_id;
            S.t = si.desc.t_ns;
            S.q = si.desc.charge;
        }
        S.n = nh;
        S.chunk_base = si.chunk_base;
        S.n_chunks = si.n_chunks;
        S.tile_base = si.tile_base;
        S.n_tiles = si.n_tiles;
        S.group_base = si.group_base;
        if (si.tune.seg_cap <= (uint32_t)WAVE_CAP) {
            S.seg_cap = si.tune.seg_cap;
            S.seg_target = std::min<uint32_t>(si.tune.seg_target, si.tune.seg_cap * 3 / 4);
        } else {
            S.seg_cap = seg_cap;
            S.seg_target = std::min(si.tune.seg_target, seg_cap / 2);
        }
        S.seg_target = std::max<uint32_t>(S.seg_target, 1);
        S.pos_cap = L.pos_cap;
        S.part = (ChunkPart *)(b + L.part);
        S.ppart = (PlanPart *)(b + L.ppart);
        S.pos = (uint32_t *)(b + L.pos);
        S.o_t = (uint32_t *)(b + L.o_t);
        S.o_pq = (uint32_t *)(b + L.o_pq);
        S.o_idx = (uint32_t *)(b + L.o_idx);
        S.tstat = (TileStat *)(b + L.tstat);
        S.cagg = (TileAgg *)(b + L.cagg);
        S.dmask = (uint64_t *)(b + L.dmask);
        S.fsc = (FireRec *)(b + L.fsc);
        S.fires = (trig_fire *)(b + L.fires);
        S.events = (trig_event *)(b + L.events);
        S.seed_flags = si.want_flags ? (uint8_t *)(b + L.flags) : nullptr;
        S.plan = d_plans + i;
        S.x_fires = si.direct_f ? si.direct_f : x_plans_dev ? (trig_fire *)((char *)x_plans_dev + si.x_off_f) : nullptr;
        S.x_events = si.direct_e ? si.direct_e
                                 : x_plans_dev ? (trig_event *)((char *)x_plans_dev + si.x_off_e) : nullptr;
        S.x_fire_cap = si.x_fcap;
        S.x_event_cap = si.x_ecap;
        S.tagc = (uint32_t *)(b + L.tagc);
        S.tagged = (uint32_t *)(b + L.fsc);   // free once the fires are placed
        S.tag_on = si.want_tag && si.host_status == TRIG_OK ? 1u : 0u;
        S.x_tagged = si.direct_t ? si.direct_t
                     : si.x_tcap && x_plans_dev ? (uint32_t *)((char *)x_plans_dev + si.x_off_t) : nullptr;
        S.x_tag_cap = si.x_tcap;
        S.l0m = (uint64_t *)(b + L.l0m);
        hs[i] = S;
        si.dev = S;
    }
    // the previous round on this job has completed (every entry point synchronises
    // before it returns), so the device copy of an unchanged set is intact
    uint32_t *hbases = (uint32_t *)(hs + n);
    for (uint32_t i = 0; i < n; ++i) {
        hbases[i] = slices[i].chunk_base;
        hbases[n + i] = slices[i].tile_base;
    }
    const size_t up_bytes = desc_upload_bytes(n);
    if (fixed || up_ptr != dmeta.ptr || up_cap != dmeta.cap || up_slices.size() != up_bytes ||
        std::memcmp(up_slices.data(), hs, up_bytes) != 0) {
        up_ptr = nullptr;
        hipError_t e = hipMemcpyAsync(d_slices, hs, up_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(c, e, "H2D of slice descriptors");
        up_slices.assign((const unsigned char *)hs, (const unsigned char *)hs + up_bytes);
        up_ptr = dmeta.ptr;
        up_cap = dmeta.cap;
    }
    batch = {};
    batch.slices = d_slices;
    batch.chunk_bases = (const uint32_t *)(d_slices + n);
    batch.tile_bases = batch.chunk_bases + n;
    batch.plans = d_plans;
    batch.n_slices = n;
    batch.total_chunks = total_chunks;
    batch.total_tiles = total_tiles;
    batch.max_tiles = 1;
    for (const SliceInfo &si : slices) batch.max_tiles = std::max(batch.max_tiles, si.n_tiles);
    batch.tail_state = ST_FAST;
    batch.sort_kernels = sort_kernels;
    batch.block_cap = seg_cap;
    batch.block_target = seg_cap / 2;
    batch.counters = d_counters;
    batch.x_plans = x_plans_dev;
    batch.prm = params;
    batch.tile_group = tile_group;
    batch.window_cap = window_cap;
    {
        uint32_t nb_max = 0;
        for (const SliceInfo &si : slices)
            if (si.host_status == TRIG_OK) nb_max = std::max(nb_max, si.dev.nbk);
        batch.tbnd_lds = nb_max && nb_max <= (uint32_t)TBND_LDS_MAX ? nb_max * nb_max : 0u;
        batch.any_bounds = nb_max ? 1u : 0u;
    }
    batch.total_groups = total_groups;
    batch.group_slice = d_group_slice;
    batch.tile_slice = d_tile_slice;
    batch.chunk_slice = d_chunk_slice;
    return TRIG_OK;
}

// Launch the whole device pipeline on the job's stream.  Every kernel argument
// is in the launch key (the per-slice descriptors are read from device memory),
// so a launch sequence seen twice is captured once into a HIP graph on a private
// stream and replayed on the job's stream from then on.  Timed launches
// (profile) stay eager so the per-kernel events sit between the kernels.
int Job::launch(trig_ctx *c, bool profile) {
    void (*mark)(void *, const char *, int) = profile ? prof_mark : nullptr;
    TrigLaunchCfg cfg = c->cfg;
    cfg.persist_per_cu = (int)std::max<uint32_t>(1, block_wgs);
    auto eager = [&](hipStream_t s) -> int {
        hipError_t e = trig_launch_front(batch, seg_cap, wave_cap, (int)std::max<uint32_t>(1, wave_wgs), cfg, s,
                                         mark, c);
        if (e != hipSuccess) return hip_fail(c, e, "front kernels");
        e = trig_launch_tail(batch, cfg, max_pmt, s, mark, c);
        if (e != hipSuccess) return hip_fail(c, e, "tail kernels");
        if (any_tag) {
            // the slices whose events are final here (no rerun pending) are tagged in
            // the same sequence; a rerun tags again afterwards
            e = trig_launch_tag(batch, s, mark, c);
            if (e != hipSuccess) return hip_fail(c, e, "tagged hits");
        }
        return TRIG_OK;
    };
    if (profile || !graphs_ok || !c->use_graphs || fixed_ws) return eager(stream);
    // every host-side launch choice: kernel arguments, grids, variants, LDS sizes
    const uint32_t extra[5] = {seg_cap, wave_cap, wave_wgs, max_pmt, any_tag ? 1u : 0u};
    std::vector<uint8_t> key(sizeof(BatchDev) + sizeof(TrigLaunchCfg) + sizeof(extra));
    std::memcpy(key.data(), &batch, sizeof(BatchDev));
    std::memcpy(key.data() + sizeof(BatchDev), &cfg, sizeof(TrigLaunchCfg));
    std::memcpy(key.data() + sizeof(BatchDev) + sizeof(TrigLaunchCfg), extra, sizeof(extra));
    if (graph_exec && key == graph_key) {
        hipError_t e = hipGraphLaunch(graph_exec, stream);
        if (e != hipSuccess) return hip_fail(c, e, "graph launch");
        return TRIG_OK;
    }
    if (key != seen_key) {
        seen_key = key;
        return eager(stream);
    }
    if (!capture_stream && hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking) != hipSuccess) {
        graphs_ok = false;
        return eager(stream);
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const int rc = eager(capture_stream);
        hipError_t e2 = hipStreamEndCapture(capture_stream, &g);
        if (rc != TRIG_OK || e2 != hipSuccess) e = e2 != hipSuccess ? e2 : hipErrorUnknown;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        graphs_ok = false;   // this runtime cannot capture the sequence: stay eager
        return eager(stream);
    }
    if (graph_exec) hipGraphExecDestroy(graph_exec);
    graph_exec = ex;
    graph_key = key;
    e = hipGraphLaunch(graph_exec, stream);
    if (e != hipSuccess) return hip_fail(c, e, "graph launch");
    return TRIG_OK;
}

// Seed flags of the slices in `state` to the caller's host buffers (ordered
// after the kernels that wrote them).
int Job::enqueue_flags(trig_ctx *c, const std::vector<uint32_t> *only) {
    const uint32_t cnt = only ? (uint32_t)only->size() : (uint32_t)slices.size();
    for (uint32_t x = 0; x < cnt; ++x) {
        SliceInfo &si = slices[only ? (*only)[x] : x];
        if (!si.want_flags || !si.dev.seed_flags || !si.flags_dst || si.n == 0) continue;
        hipError_t e = hipMemcpyAsync(si.flags_dst, si.dev.seed_flags, si.n, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return hip_fail(c, e, "D2H of seed flags");
    }
    return TRIG_OK;
}

// After the plans arrived on the host: run the general ordering for the slices
// that need it, then their tail.
int Job::generic_pass(trig_ctx *c, bool profile) {
    Plan *hp = host_plans();
    std::vector<uint32_t> todo;
    for (uint32_t i = 0; i < slices.size(); ++i)
        if (slices[i].host_status == TRIG_OK && hp[i].state == ST_NEED_GENERIC) todo.push_back(i);
    if (todo.empty()) return TRIG_OK;
    reran = true;
    void (*mark)(void *, const char *, int) = profile ? prof_mark : nullptr;
    for (uint32_t i : todo) {
        SliceInfo &si = slices[i];
        // the slice's fire and event areas are unused until its trigger stage runs,
        // so the radix scratch lives there when it fits (always but for tiny slices)
        const size_t need = trig_generic_scratch_bytes(si.n);
        const size_t avail = si.L.events + align256(si.n * sizeof(trig_event) + 32) - si.L.fires;
        void *scratch = si.dev.fires;
        if (need > avail && fixed_ws) {
            if (need > FIXED_GEN_BYTES) {
                ctx_set_error(c, "internal: radix scratch of %zu bytes does not fit the fixed region", need);
                return TRIG_ENOMEM;
            }
            scratch = fixed_gen;
        } else if (need > avail) {
            const int rc = gscratch.ensure(c, need, stream);
            if (rc) return rc;
            scratch = gscratch.ptr;
        }
        const uint64_t span = (uint64_t)hp[i].t_max - (uint64_t)hp[i].t_min;
        const uint32_t span_bits = span ? 64u - (uint32_t)__builtin_clzll(span) : 0u;
        const uint32_t key_bits = span_bits + si.dev.pbits;
        hipError_t e = trig_launch_generic_slice(si.dev, hp[i], key_bits, scratch, stream, mark, c);
        if (e != hipSuccess) return hip_fail(c, e, "general ordering");
    }
    // the trigger stage of just those slices, each as a launch of its own
    for (uint32_t i : todo) {
        const BatchDev b1 = one_slice(i, ST_GENERIC_DONE);
        hipError_t e = trig_launch_tail(b1, c->cfg, slices[i].dev.n_pmt, stream, mark, c);
        if (e != hipSuccess) return hip_fail(c, e, "tail kernels (general path)");
    }
    int rc2 = enqueue_flags(c, &todo);
    if (rc2) return rc2;
    rc2 = fetch_plans(c);
    if (rc2) return rc2;
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise (general path)");
    return TRIG_OK;
}

// After the plans arrived on the host: rerun the trigger stage of the slices
// whose windows outran the staged halo, with a precomputed seed mask.
int Job::dense_pass(trig_ctx *c, bool profile) {
    Plan *hp = host_plans();
    std::vector<uint32_t> todo;
    for (uint32_t i = 0; i < slices.size(); ++i)
        if (slices[i].host_status == TRIG_OK && hp[i].status == TRIG_OK && hp[i].dense &&
            (hp[i].state == ST_FAST || hp[i].state == ST_GENERIC_DONE))
            todo.push_back(i);
    if (todo.empty()) return TRIG_OK;
    reran = true;
    void (*mark)(void *, const char *, int) = profile ? prof_mark : nullptr;
    hipError_t e = hipSuccess;
    for (uint32_t i : todo) {
        const BatchDev b1 = one_slice(i, ST_DENSE);
        e = trig_launch_dense(b1, c->cfg, slices[i].dev.n_pmt, stream, mark, c);
        if (e != hipSuccess) return hip_fail(c, e, "trigger stage (dense rerun)");
    }
    int rc = enqueue_flags(c, &todo);
    if (rc) return rc;
    rc = fetch_plans(c);
    if (rc) return rc;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise (dense rerun)");
    return TRIG_OK;
}

// After every pass that can change the events: the tagged-hit lists of the
// slices that asked for them.
int Job::tag_pass(trig_ctx *c, bool profile) {
    // the launch tagged every slice whose events it finished; only a rerun needs more
    if (!any_tag || !reran) return TRIG_OK;
    bool any = false;
    for (const SliceInfo &si : slices) any |= si.want_tag && si.host_status == TRIG_OK && si.n > 0;
    if (!any) return TRIG_OK;
    void (*mark)(void *, const char *, int) = profile ? prof_mark : nullptr;
    hipError_t e = trig_launch_tag(batch, stream, mark, c);
    if (e != hipSuccess) return hip_fail(c, e, "tagged hits");
    const int rc = fetch_plans(c);
    if (rc) return rc;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise (tagged hits)");
    return TRIG_OK;
}

// The batch descriptor narrowed to slice i, for reruns of one slice's trigger
// stage (tiles numbered from 0, its plan exported to its own staging slot).
BatchDev Job::one_slice(uint32_t i, uint32_t state) const {
    BatchDev b1 = batch;
    b1.slices = d_slices + i;
    b1.plans = d_plans + i;
    b1.n_slices = 1;
    b1.total_chunks = slices[i].n_chunks;
    b1.total_tiles = slices[i].n_tiles;
    b1.max_tiles = std::max(1u, slices[i].n_tiles);
    b1.x_plans = x_plans_dev ? x_plans_dev + i : nullptr;
    b1.tail_state = state;
    b1.total_groups = groups_of(slices[i].n_tiles, tile_group);
    return b1;
}

// Copy the results of slice i into the caller's result record.
void Job::host_copy(void *dst, const void *src, size_t bytes) {
    if (defer_copies) host_copies.push_back({dst, src, bytes});
    else std::memcpy(dst, src, bytes);
}

// The collected copies: on the calling thread below 4 MiB, else split by bytes
// over up to four threads (one host thread copies from the pinned staging at a
// fraction of the memory bandwidth; a 256-slice batch hands back about 15 MB).
void Job::run_host_copies() {
    size_t total = 0;
    for (const HostCopy &h : host_copies) total += h.bytes;
    const unsigned hw = std::thread::hardware_concurrency();
    const unsigned nt = total < (4u << 20) ? 1u : std::max(1u, std::min(4u, hw ? hw : 1u));
    if (nt == 1) {
        for (const HostCopy &h : host_copies) std::memcpy(h.dst, h.src, h.bytes);
    } else {
        // part k copies the bytes [k T / nt, (k + 1) T / nt) of the concatenated copies
        auto part = [&](unsigned k) {
            const size_t lo = total * k / nt, hi = total * (k + 1) / nt;
            size_t at = 0;
            for (const HostCopy &h : host_copies) {
                const size_t a = std::max(lo, at), b = std::min(hi, at + h.bytes);
                if (a < b) std::memcpy((char *)h.dst + (a - at), (const char *)h.src + (a - at), b - a);
                at += h.bytes;
                if (at >= hi) break;
            }
        };
        std::vector<std::thread> th;
        for (unsigned k = 1; k < nt; ++k) th.emplace_back(part, k);
        part(0);
        for (std::thread &t : th) t.join();
    }
    host_copies.clear();
}

int Job::deliver(trig_ctx *c, uint32_t i, trig_result *r) {
    const SliceInfo &si = slices[i];
    const Plan &P = host_plans()[i];
    r->tag = si.desc.tag;
    r->n_hits = si.desc.n_hits;
    r->path = (P.generic ? 1u : 0u) | (P.dense ? 2u : 0u);
    r->n_seeds = r->n_fires = r->n_events = r->n_tagged = 0;
    if (si.host_status != TRIG_OK) return r->status = si.host_status;
    if (P.status != TRIG_OK) {
        ctx_set_error(c, "slice %u: input out of range (PMT id, time span or event window)", i);
        return r->status = P.status;
    }
    if (si.n == 0) return r->status = TRIG_OK;
    r->n_seeds = P.n_seeds;
    r->n_fires = P.n_fires;
    r->n_events = P.n_events;
    r->n_tagged = si.want_tag ? P.n_tagged : 0;
    if ((P.n_fires && (!r->fires || r->fire_cap < P.n_fires)) ||
        (P.n_events && (!r->events || r->event_cap < P.n_events)) ||
        (si.want_tag && r->tagged_cap < P.n_tagged)) {
        ctx_set_error(c, "slice %u: result capacity too small (need %u fires, %u events, %u tagged hits)", i,
                      P.n_fires, P.n_events, si.want_tag ? P.n_tagged : 0u);
        return r->status = TRIG_EOVERFLOW;
    }
    // staged lists come from pinned memory; longer ones are copied from the device
    const char *xb = (const char *)h_plans.ptr;
    hipError_t e = hipSuccess;
    if (P.n_fires) {
        if (P.n_fires <= si.x_fcap && si.direct_f)
            ;   // the kernels wrote the list into the caller's pinned buffer
        else if (P.n_fires <= si.x_fcap)
            host_copy(r->fires, xb + si.x_off_f, (size_t)P.n_fires * sizeof(trig_fire));
        else {
            e = hipMemcpyAsync(r->fires, si.dev.fires, (size_t)P.n_fires * sizeof(trig_fire),
                               hipMemcpyDeviceToHost, stream);
            copies_queued = true;
        }
    }
    if (e == hipSuccess && P.n_events) {
        if (P.n_events <= si.x_ecap && si.direct_e)
            ;
        else if (P.n_events <= si.x_ecap)
            host_copy(r->events, xb + si.x_off_e, (size_t)P.n_events * sizeof(trig_event));
        else {
            e = hipMemcpyAsync(r->events, si.dev.events, (size_t)P.n_events * sizeof(trig_event),
                               hipMemcpyDeviceToHost, stream);
            copies_queued = true;
        }
    }
    if (e == hipSuccess && si.want_tag && P.n_tagged) {
        if (P.n_tagged <= si.x_tcap && si.direct_t)
            ;
        else if (P.n_tagged <= si.x_tcap)
            host_copy(r->tagged, xb + si.x_off_t, (size_t)P.n_tagged * sizeof(uint32_t));
        else {
            e = hipMemcpyAsync(r->tagged, si.dev.tagged, (size_t)P.n_tagged * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, stream);
            copies_queued = true;
        }
    }
    if (e != hipSuccess) return r->status = hip_fail(c, e, "D2H of results");
    return r->status = TRIG_OK;
}

Plan *Job::host_plans() const {
    if (fixed_ws) return (Plan *)((char *)fixed_pin + align256(desc_upload_bytes((uint32_t)slices.size())));
    return (Plan *)h_plans.ptr;
}

int Job::fetch_plans(trig_ctx *c) {
    if (!fixed_ws || slices.empty()) return TRIG_OK;
    const hipError_t e = hipMemcpyAsync(host_plans(), d_plans, slices.size() * sizeof(Plan), hipMemcpyDeviceToHost,
                                        stream);
    return e == hipSuccess ? TRIG_OK : hip_fail(c, e, "D2H of the plans");
}

void Job::release(trig_ctx *c) {
    if (graph_exec) hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    if (capture_stream) hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
    ws.release(c);
    dmeta.release(c);
    up_ptr = nullptr;
    up_slices.clear();
    gscratch.release(c);
    h_slices.release();
    h_plans.release();
}

int check_params(trig_ctx *c, const trig_params *p) {
    if (!p) {
        ctx_set_error(c, "null params");
        return TRIG_EINVAL;
    }
    if ((uint64_t)p->half_event_ns > (1ull << 62)) {
        ctx_set_error(c, "half_event_ns too large");
        return TRIG_EINVAL;
    }
    if (p->l0_n > 0 && (p->l0_n > 64 || p->l0_tw_ns == 0 || p->l0_tw_ns > 1000000)) {
        ctx_set_error(c, "level 0 needs 1 <= l0_n <= 64 and 1 <= l0_tw_ns <= 1000000");
        return TRIG_EINVAL;
    }
    if (p->seed_mode > 1) {
        ctx_set_error(c, "seed_mode must be 0 or 1");
        return TRIG_EINVAL;
    }
    return TRIG_OK;
}

int run_sync(trig_ctx *c, Job &J, uint32_t n, const trig_slice_desc *d, const trig_params *prm, trig_result *res,
             hipStream_t s) {
    int rc = check_params(c, prm);
    if (rc) return rc;
    if (n == 0) return TRIG_OK;
    if (!d || !res) {
        ctx_set_error(c, "null slices or results");
        return TRIG_EINVAL;
    }
    std::vector<uint8_t> flags(n), tags(n);
    std::vector<uint64_t> fcap(n), ecap(n), tcap(n);
    for (uint32_t i = 0; i < n; ++i) {
        flags[i] = res[i].seed_flags != nullptr;
        tags[i] = res[i].tagged != nullptr;
        tcap[i] = res[i].tagged ? res[i].tagged_cap : 0;
        fcap[i] = res[i].fires ? res[i].fire_cap : 0;
        ecap[i] = res[i].events ? res[i].event_cap : 0;
    }
    const bool prof = c->prof_on && !J.fixed_ws;
    if (prof) c->prof_stream = s;
    rc = J.prepare(c, n, d, prm, flags.data(), fcap.data(), ecap.data(), s, tags.data(), tcap.data(), res);
    if (rc) return rc;
    for (uint32_t i = 0; i < n; ++i) J.slices[i].flags_dst = res[i].seed_flags;
    rc = J.launch(c, prof);
    if (rc) return rc;
    rc = J.enqueue_flags(c, nullptr);
    if (rc) return rc;
    rc = J.fetch_plans(c);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise");
    rc = J.generic_pass(c, prof);
    if (rc) return rc;
    rc = J.dense_pass(c, prof);
    if (rc) return rc;
    rc = J.tag_pass(c, prof);
    if (rc) return rc;
    int first_bad = TRIG_OK;
    J.copies_queued = false;
    J.defer_copies = true;
    for (uint32_t i = 0; i < n; ++i) {
        const int st = J.deliver(c, i, &res[i]);
        if (st != TRIG_OK && first_bad == TRIG_OK) first_bad = st;
    }
    J.defer_copies = false;
    J.run_host_copies();
    if (J.copies_queued) {
        // lists longer than their staging were queued as copies from the device
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "synchronise results");
    }
    if (prof) prof_collect(c);
    return first_bad;
}

// ------------------------------------------- fixed scratch (no allocation)

// Device memory of trig_slice_noalloc: workspace, descriptors, plans and
// counters of one slice, TRIG_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU
// the library runs on until the process ends.  Host code never uses the name
// itself as an address (on the host it is only a handle of the symbol): the
// device address of each GPU's copy is looked up once per device, with that
// device current, when the first context on it is created.
static __device__ __align__(256) unsigned char scratch[TRIG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
constexpr size_t NA_PIN_BYTES = 4096;
std::mutex na_mu;
char *na_scratch_dev[NA_MAX_DEVICES] = {};
}  // namespace

// The device address of the fixed scratch on `device` (current), or null.
static char *na_scratch_of(int device, hipError_t *err) {
    *err = hipSuccess;
    if (device < 0 || device >= NA_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(na_mu);
    if (!na_scratch_dev[device]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        na_scratch_dev[device] = (char *)ptr;
    }
    return na_scratch_dev[device];
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *trig_version(void) { return "libtrig 0.1 gfx950"; }

int trig_create(trig_ctx **out, int device, uint64_t hbm_budget_bytes) {
    if (!out) return TRIG_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TRIG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TRIG_EHIP;
    trig_ctx *c = new trig_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (64ull << 30);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return TRIG_EHIP;
    }
    c->cfg.n_cu = prop.multiProcessorCount;
    c->cfg.persist_per_cu = 2;
    const char *g = getenv("TRIG_GRAPHS");
    c->use_graphs = !(g && g[0] == '0');
    // wave per segment, 3 workgroups of 4 waves per CU; fold workgroups of two
    // tiles, each wave staging up to 512 window seeds
    const trig_tune tower = {384, (uint32_t)WAVE_CAP, 3, 2, 512, 0};
    const trig_tune block = tower;
    c->tunes.push_back({128u, tower});
    c->tunes.push_back({0xFFFFFFFFu, block});
    // set-up of the allocation-free entry point: this device's fixed scratch and
    // a small pinned block for its descriptor upload and plan read-back
    hipError_t e = hipSuccess;
    c->na_scratch = na_scratch_of(device, &e);
    if (!c->na_scratch || hipHostMalloc(&c->na_pin, NA_PIN_BYTES, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->na_pin = nullptr;
        ctx_set_error(c, "fixed scratch unavailable: %s", hipGetErrorString(e));
    }
    *out = c;
    return TRIG_OK;
}

void trig_destroy(trig_ctx *c) {
    if (!c) return;
    serve_shutdown(c);
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    c->sync_job.release(c);
    c->na_job.release(c);
    if (c->na_pin) hipHostFree(c->na_pin);
    for (auto &g : c->geoms) {
        hipFree(g.floor_id);
        hipFree(g.floor16);
        hipFree(g.thr32);
        hipFree(g.thr16);
        hipFree(g.adj32);
        hipFree(g.afl32);
        hipFree(g.tbnd);
        hipFree(g.rmax);
    }
    for (auto ev : c->ev_pool) hipEventDestroy(ev);
    for (auto &m : c->prof_pending) hipEventDestroy(m.ev);
    delete c;
}

const char *trig_last_error(const trig_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

int trig_geom_load(trig_ctx *c, const trig_geom_desc *g, uint32_t *geom_id) {
    if (!c) return TRIG_EINVAL;
    if (!g || !geom_id || !g->floor_id || !g->thr_ns || g->n_pmt == 0 || g->n_pmt > 65536) {
        ctx_set_error(c, "bad geometry descriptor");
        return TRIG_EINVAL;
    }
    hipSetDevice(c->device);
    const uint64_t P = g->n_pmt;
    const uint64_t nbb = P >= TBND_MIN_PMT ? (P + 31) / 32 : 0;
    const uint64_t bytes = P * 4 + P * 2 + P * P * 4 + P * P * 2 + P * 8 + nbb * nbb * 2 + P * 4;
    if (ctx_reserve(c, bytes) != TRIG_OK) {
        ctx_set_error(c, "device budget exceeded by geometry");
        return TRIG_ENOMEM;
    }
    GeomDev d = {};
    d.n_pmt = g->n_pmt;
    std::vector<uint16_t> t16(P * P);
    for (uint64_t i = 0; i < P * P; ++i) t16[i] = (uint16_t)std::min<uint32_t>(g->thr_ns[i], 65535u);
    // dense floor numbering: equal ids map to equal u16 indices (at most n_pmt floors)
    std::vector<uint16_t> f16(P);
    {
        std::vector<std::pair<int32_t, uint32_t>> byid(P);
        for (uint64_t i = 0; i < P; ++i) byid[i] = {g->floor_id[i], (uint32_t)i};
        std::sort(byid.begin(), byid.end());
        uint32_t k = 0;
        for (uint64_t i = 0; i < P; ++i) {
            if (i && byid[i].first != byid[i - 1].first) ++k;
            f16[byid[i].second] = (uint16_t)k;
        }
    }
    // adjacency groups, densely numbered (each PMT its own group when none given)
    std::vector<uint32_t> adj(P), afl(P);
    {
        std::vector<std::pair<int64_t, uint32_t>> byid(P);
        for (uint64_t i = 0; i < P; ++i) byid[i] = {g->adj_id ? (int64_t)g->adj_id[i] : (int64_t)i, (uint32_t)i};
        std::sort(byid.begin(), byid.end());
        uint32_t k = 0;
        for (uint64_t i = 0; i < P; ++i) {
            if (i && byid[i].first != byid[i - 1].first) ++k;
            adj[byid[i].second] = k;
        }
        // floor ranks: distinct floor ids in order, one apart when the ids differ by 1
        std::vector<std::pair<int64_t, uint32_t>> fl(P);
        for (uint64_t i = 0; i < P; ++i) fl[i] = {(int64_t)g->floor_id[i], (uint32_t)i};
        std::sort(fl.begin(), fl.end());
        uint32_t r = 0;
        for (uint64_t i = 0; i < P; ++i) {
            if (i && fl[i].first != fl[i - 1].first) r += fl[i].first - fl[i - 1].first == 1 ? 1u : 2u;
            afl[fl[i].second] = r;
        }
    }
    // bounds of min(thr, 65535) per pair of 32-PMT blocks, in 16 ns units (the lower
    // bound rounded down, capped at 4080 ns; the upper rounded up, 255 when above
    // 4064 ns: no bound): the fold kernel decides most pairs from them and
    // reads the table only in between
    std::vector<uint16_t> tb;
    if (P >= TBND_MIN_PMT) {
        const uint64_t nb = (P + (1u << TBND_SHIFT) - 1) >> TBND_SHIFT;
        d.nbk = (uint32_t)nb;
        tb.assign(nb * nb, 0);
        for (uint64_t bi = 0; bi < nb; ++bi)
            for (uint64_t bj = 0; bj < nb; ++bj) {
                uint32_t mn = 0xFFFFu, mx = 0u;
                for (uint64_t i = bi << TBND_SHIFT; i < std::min(P, (bi + 1) << TBND_SHIFT); ++i)
                    for (uint64_t j = bj << TBND_SHIFT; j < std::min(P, (bj + 1) << TBND_SHIFT); ++j) {
                        const uint32_t v = t16[i * P + j];
                        mn = std::min(mn, v);
                        mx = std::max(mx, v);
                    }
                const uint32_t lo = std::min(mn, 4080u) / 16u;
                const uint32_t hi = mx <= 4064u ? (mx + 15u) / 16u : 255u;
                tb[bi * nb + bj] = (uint16_t)(lo | (hi << 8));
            }
    }
    // the reach of each PMT's seeds: its row's largest entry
    std::vector<uint32_t> rmax(P, 0u);
    for (uint64_t i = 0; i < P; ++i) {
        for (uint64_t j = 0; j < P; ++j) rmax[i] = std::max(rmax[i], g->thr_ns[i * P + j]);
        d.thr_max = std::max(d.thr_max, rmax[i]);
    }
    hipError_t e = hipMalloc(&d.floor_id, P * 4);
    if (e == hipSuccess) e = hipMalloc(&d.rmax, P * 4);
    if (e == hipSuccess) e = hipMemcpy(d.rmax, rmax.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && d.nbk) e = hipMalloc(&d.tbnd, (tb.size() * 2 + 15) & ~(size_t)15);   // (read in 16-byte pieces)
    if (e == hipSuccess && d.nbk) e = hipMemcpy(d.tbnd, tb.data(), tb.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&d.adj32, P * 4);
    if (e == hipSuccess) e = hipMalloc(&d.afl32, P * 4);
    if (e == hipSuccess) e = hipMemcpy(d.adj32, adj.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.afl32, afl.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&d.floor16, P * 2);
    if (e == hipSuccess) e = hipMalloc(&d.thr32, P * P * 4);
    if (e == hipSuccess) e = hipMalloc(&d.thr16, P * P * 2 + 16);   // read as 32-bit pairs
    if (e == hipSuccess) e = hipMemcpy(d.floor_id, g->floor_id, P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.floor16, f16.data(), P * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.thr32, g->thr_ns, P * P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.thr16, t16.data(), P * P * 2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(d.tbnd);
        hipFree(d.rmax);
        hipFree(d.floor16);
        hipFree(d.floor_id);
        hipFree(d.adj32);
        hipFree(d.afl32);
        hipFree(d.thr32);
        hipFree(d.thr16);
        ctx_release(c, bytes);
        return hip_fail(c, e, "geometry upload");
    }
    std::lock_guard<std::mutex> lk(c->geom_mu);
    c->geoms.push_back(d);
    *geom_id = (uint32_t)(c->geoms.size() - 1);
    return TRIG_OK;
}

int trig_slice(trig_ctx *c, const trig_slice_desc *slice, const trig_params *params, trig_result *result,
               void *hip_stream) {
    if (!c) return TRIG_EINVAL;
    if (!slice || !result) {
        ctx_set_error(c, "null slice or result");
        return TRIG_EINVAL;
    }
    hipSetDevice(c->device);
    int rc = run_sync(c, c->sync_job, 1, slice, params, result, (hipStream_t)hip_stream);
    if (rc != TRIG_OK && result->status == TRIG_OK) result->status = rc;
    return rc;
}

int trig_slice_noalloc(trig_ctx *c, const trig_slice_desc *slice, const trig_params *params, trig_result *result,
                       void *hip_stream) {
    if (!c) return TRIG_EINVAL;
    if (!slice || !result) {
        ctx_set_error(c, "null slice or result");
        return TRIG_EINVAL;
    }
    if (slice->n_hits && slice->mem != TRIG_MEM_DEVICE) {
        ctx_set_error(c, "trig_slice_noalloc takes device inputs only");
        return result->status = TRIG_EINVAL;
    }
    if (!c->na_scratch || !c->na_pin) {
        ctx_set_error(c, "the fixed scratch of device %d is unavailable", c->device);
        return result->status = TRIG_EHIP;
    }
    hipSetDevice(c->device);
    Job &J = c->na_job;
    J.fixed_ws = c->na_scratch;
    J.fixed_cap = TRIG_NOALLOC_SCRATCH_BYTES;
    J.fixed_pin = c->na_pin;
    J.fixed_pin_cap = NA_PIN_BYTES;
    J.graphs_ok = false;
    const int rc = run_sync(c, J, 1, slice, params, result, (hipStream_t)hip_stream);
    if (rc != TRIG_OK && result->status == TRIG_OK) result->status = rc;
    return rc;
}

int trig_batch(trig_ctx *c, uint32_t n, const trig_slice_desc *slices, const trig_params *params,
               trig_result *results, void *hip_stream) {
    if (!c) return TRIG_EINVAL;
    hipSetDevice(c->device);
    return run_sync(c, c->sync_job, n, slices, params, results, (hipStream_t)hip_stream);
}

int trig_tune_get(trig_ctx *c, uint32_t n_pmt, trig_tune *out) {
    if (!c || !out) return TRIG_EINVAL;
    *out = ctx_tune_for(c, n_pmt);
    return TRIG_OK;
}

int trig_tune_set(trig_ctx *c, uint32_t n_pmt_max, const trig_tune *t) {
    if (!c || !t) return TRIG_EINVAL;
    if (!(t->seg_cap == (uint32_t)WAVE_CAP || t->seg_cap == (uint32_t)WAVE_CAP_SMALL || t->seg_cap == 2048 ||
          t->seg_cap == 4096 || t->seg_cap == 8192) ||
        t->seg_target == 0 ||
        t->grid_per_cu == 0 || t->grid_per_cu > 16 ||
        !(t->tile_group == 1 || t->tile_group == 2 || t->tile_group == 4) ||
        !(t->window_cap == 512 || t->window_cap == 2048)) {
        ctx_set_error(c, "bad tuning values");
        return TRIG_EINVAL;
    }
    auto it = std::find_if(c->tunes.begin(), c->tunes.end(),
                           [&](const std::pair<uint32_t, trig_tune> &p) { return p.first == n_pmt_max; });
    if (it != c->tunes.end()) it->second = *t;
    else c->tunes.push_back({n_pmt_max, *t});
    std::sort(c->tunes.begin(), c->tunes.end(),
              [](const std::pair<uint32_t, trig_tune> &a, const std::pair<uint32_t, trig_tune> &b) {
                  return a.first < b.first;
              });
    return TRIG_OK;
}

int trig_profile_enable(trig_ctx *c, int enable) {
    if (!c) return TRIG_EINVAL;
    c->prof_on = enable != 0;
    c->prof.clear();
    return TRIG_OK;
}

int trig_profile_read(trig_ctx *c, trig_kernel_time *out, uint32_t cap, uint32_t *n_out) {
    if (!c || !n_out) return TRIG_EINVAL;
    *n_out = (uint32_t)c->prof.size();
    for (uint32_t i = 0; i < cap && i < c->prof.size(); ++i) out[i] = c->prof[i];
    return TRIG_OK;
}

}  // extern "C"
