// Host-side internals of libtrig shared by api.hip and serve.hip.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "trig_dev.h"

struct trig_ctx;

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    int ensure(trig_ctx *c, size_t want, hipStream_t s);   // grows; contents not kept; budget-accounted
    void release(trig_ctx *c);
};

struct PinBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    int ensure(size_t want);
    void release();
};

struct GeomDev {
    uint32_t n_pmt = 0;
    int32_t *floor_id = nullptr;
    uint16_t *floor16 = nullptr;   // dense renumbering of floor_id (first appearance order)
    uint32_t *thr32 = nullptr;
    uint16_t *thr16 = nullptr;
    uint32_t *adj32 = nullptr;     // dense adjacency group (a PMT of its own when none is given)
    uint32_t *afl32 = nullptr;     // floor rank, consecutive floor ids one apart, others two
    // bounds of the table per pair of 32-PMT blocks (lower | upper << 8, 16 ns
    // units), nbk x nbk; nbk = 0 (no bounds) for small detectors whose table stays in cache
    uint16_t *tbnd = nullptr;
    uint32_t nbk = 0;
    // largest entry of each row of the table (the reach of that PMT's seeds) and of
    // the whole table
    uint32_t *rmax = nullptr;
    uint32_t thr_max = 0;
};

// Byte offsets of one slice's arrays inside a job workspace (SIZE_MAX = absent).
struct SliceLayout {
    size_t in_pmt, in_t, in_q, part, ppart, pos, o_t, o_pq, o_idx, tstat, cagg, dmask, fsc, fires, events, flags, tagc, l0m;
    uint64_t pos_cap;
};

struct SliceInfo {
    trig_slice_desc desc;
    int host_status;
    uint64_t n;
    bool want_flags;
    size_t ws_off;
    SliceLayout L;
    uint32_t chunk_base, n_chunks, tile_base, n_tiles, group_base;
    trig_tune tune;
    trigdev::SliceDev dev;
    size_t x_off_f, x_off_e, x_off_t;   // result staging offsets in the pinned buffer
    uint32_t x_fcap, x_ecap, x_tcap;
    uint8_t *flags_dst;          // caller's host buffer for seed flags (or null)
    bool want_tag;               // the tagged-hit list is asked for
    // device addresses of the caller's result buffers when they are pinned host
    // memory (the kernels write the lists there directly), else null
    trig_fire *direct_f;
    trig_event *direct_e;
    uint32_t *direct_t;
};

// One device round over a set of slices: workspace, descriptors, plans.
struct Job {
    std::vector<SliceInfo> slices;
    trig_params params;
    hipStream_t stream = nullptr;
    uint32_t seg_cap = 4096;          // capacity of the block-per-segment ordering kernel
    uint32_t sort_kernels = 0;        // ordering kernels to launch (bit 0 wave, bit 1 block)
    uint32_t wave_wgs = 0, block_wgs = 0;   // persistent workgroups per CU of each
    uint32_t wave_cap = 0;            // variant of the wave-per-segment kernel (largest tuned capacity)
    uint32_t total_chunks = 0, total_tiles = 0;
    uint32_t tile_group = 1, window_cap = 512, total_groups = 0;   // fold-kernel launch shape
    uint32_t *d_group_slice = nullptr, *d_tile_slice = nullptr, *d_chunk_slice = nullptr;
    uint32_t max_pmt = 0;             // largest PMT count among the slices' geometries
    DevBuf ws, dmeta, gscratch;
    PinBuf h_slices, h_plans;
    trigdev::SliceDev *d_slices = nullptr;
    trigdev::Plan *d_plans = nullptr;
    uint32_t *d_counters = nullptr;
    // the descriptors last uploaded and the device buffer that holds them: an
    // unchanged set is not uploaded again
    std::vector<unsigned char> up_slices;
    const void *up_ptr = nullptr;
    size_t up_cap = 0;
    trigdev::BatchDev batch;
    // per-slice workspace bases supplied by the caller (serving: each ticket's
    // region of the resident arena); empty: one workspace owned by the job
    std::vector<char *> ext_ws;
    // h_plans is the pinned result staging: plans, then each slice's fires and events
    trigdev::Plan *x_plans_dev = nullptr;
    // launch-sequence graph: captured on the second call with the same launch key
    hipStream_t capture_stream = nullptr;
    std::vector<uint8_t> seen_key, graph_key;
    hipGraphExec_t graph_exec = nullptr;
    bool graphs_ok = true;
    // Fixed memory (the allocation-free entry point): when fixed_ws is set, the
    // workspace, descriptors, plans and counters live in the caller-given device
    // region [fixed_ws, fixed_ws + fixed_cap) and the descriptor upload and plan
    // read-back go through the pinned block fixed_pin (allocated beforehand); no
    // result is staged in host-mapped memory and no graph is captured.
    char *fixed_ws = nullptr;
    size_t fixed_cap = 0;
    void *fixed_pin = nullptr;
    size_t fixed_pin_cap = 0;
    char *fixed_gen = nullptr;        // radix scratch of slices too small to hold it in their own lists
    bool copies_queued = false;       // deliver queued a device-to-host copy
    // copies from the host-mapped staging into the callers' buffers, collected by
    // deliver when defer_copies is set and run together (in parallel when large)
    struct HostCopy { void *dst; const void *src; size_t bytes; };
    std::vector<HostCopy> host_copies;
    bool defer_copies = false;
    void host_copy(void *dst, const void *src, size_t bytes);
    void run_host_copies();
    bool any_tag = false;             // some slice asked for its tagged hits (tagged in the launch)
    bool reran = false;               // a general-ordering or dense-window rerun changed events

    // want_flags / fire_caps / event_caps: per slice, may be null (no flags /
    // default staging capacity).
    int prepare(trig_ctx *c, uint32_t n, const trig_slice_desc *d, const trig_params *prm,
                const uint8_t *want_flags, const uint64_t *fire_caps, const uint64_t *event_caps, hipStream_t s,
                const uint8_t *want_tags = nullptr, const uint64_t *tag_caps = nullptr,
                const trig_result *res = nullptr);
    int launch(trig_ctx *c, bool profile);
    int enqueue_flags(trig_ctx *c, const std::vector<uint32_t> *only);   // null: every slice
    int generic_pass(trig_ctx *c, bool profile);
    int dense_pass(trig_ctx *c, bool profile);
    int tag_pass(trig_ctx *c, bool profile);
    int deliver(trig_ctx *c, uint32_t i, trig_result *r);
    trigdev::BatchDev one_slice(uint32_t i, uint32_t state) const;
    // Host copy of the plans: the pinned staging, or (fixed memory) the pinned block.
    trigdev::Plan *host_plans() const;
    // Fixed memory: queue the copy of the device plans to host_plans() (ordered
    // before the next synchronisation); otherwise nothing (the kernels write the
    // host-mapped copy themselves).
    int fetch_plans(trig_ctx *c);
    void release(trig_ctx *c);
};

struct ProfMark {
    std::string name;
    int phase;
    hipEvent_t ev;
};

struct ServeState;   // serve.hip

struct trig_ctx {
    int device = 0;
    uint64_t budget = 0;
    std::string err;
    std::mutex err_mu;
    TrigLaunchCfg cfg = {256, 2};
    std::mutex geom_mu;
    std::vector<GeomDev> geoms;
    std::mutex mem_mu;
    uint64_t bytes_in_use = 0, bytes_peak = 0;
    std::vector<std::pair<uint32_t, trig_tune>> tunes;
    Job sync_job;
    bool use_graphs = true;      // TRIG_GRAPHS=0 in the environment keeps every launch eager
    bool prof_on = false;
    hipStream_t prof_stream = nullptr;
    std::vector<ProfMark> prof_pending;
    std::vector<hipEvent_t> ev_pool;
    std::vector<trig_kernel_time> prof;
    std::mutex serve_mu;     // guards creation of the serving loop
    ServeState *serve = nullptr;
    Job na_job;              // trig_slice_noalloc: runs in the device's fixed scratch
    void *na_pin = nullptr;  // its pinned block (descriptor upload, plan read-back)
    char *na_scratch = nullptr;   // device address of the fixed scratch on this context's device
};

void ctx_set_error(trig_ctx *c, const char *fmt, ...);
int hip_fail(trig_ctx *c, hipError_t e, const char *where);
int ctx_reserve(trig_ctx *c, uint64_t bytes);
void ctx_release(trig_ctx *c, uint64_t bytes);
trig_tune ctx_tune_for(const trig_ctx *c, uint32_t n_pmt);
int run_sync(trig_ctx *c, Job &J, uint32_t n, const trig_slice_desc *d, const trig_params *prm, trig_result *res,
             hipStream_t s);
void serve_shutdown(trig_ctx *c);
// Device bytes one slice of n hits needs in a job workspace (host inputs staged in it or not).
size_t slice_footprint(uint64_t n, bool host_input);
// Device bytes of a job's descriptors, plans, counters and group map for n
// slices of total_tiles trigger tiles.
size_t job_meta_bytes(uint32_t n, uint32_t total_tiles);
int check_params(trig_ctx *c, const trig_params *p);   // TRIG_OK or TRIG_EINVAL (message set)
