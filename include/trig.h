/*
 * trig.h -- C ABI of the MI355X muon-trigger library (libtrig.so).
 *
 * The library runs the data-parallel hot path of the online muon trigger of
 * Bouhadef, Morganti and Terreni, "Parallel Neutrino Triggers using GPUs for
 * an Underwater Telescope" (GPUHEP2014), on one AMD Instinct MI355X:
 *
 *   1. ingest a time slice of PMT hits (Sec. 2: the Hit Managers cut the merged
 *      PMT streams into 200 ms time slices; Sec. 4: each hit reduced to a
 *      fixed record of charge, time and detection-unit id);
 *   2. merge the hits into time order (Sec. 4.2: hits are time-sorted on the
 *      GPU before any trigger; each PMT's stream is already time-ordered);
 *   3. mark L1 seeds: charge over threshold (Sec. 3, Sec. 4.2 QTRIG) or a
 *      coincidence of two PMTs of one floor within a short window (Sec. 4.2 FC);
 *   4. count, for each seed, the other seeds causally correlated with it,
 *      |t_i - t_j| <= min(thr[pmt_i][pmt_j], W) (Sec. 3: Cherenkov hits of one
 *      muon are correlated in space and time within less than 3 us);
 *   5. fire an N-fold trigger on every seed whose count (itself included)
 *      reaches N;
 *   6. emit event windows of +-H around every fire, merging windows that
 *      overlap or touch (Sec. 2: a 6 us window centred on the trigger seed is
 *      sent to the Event Manager; Sec. 4.2: hits within +-3 us are tagged).
 *
 * All arithmetic is integer.  Results are unique (ties in time are ordered by
 * PMT id, then by input position) and independent of launch configuration.
 *
 * Conventions
 *  - Status codes: 0 = OK, >0 informational, <0 error.  No C++ exception
 *    crosses this ABI.  After an error, trig_last_error() describes it.
 *  - Threading: one context per host thread for trig_slice / trig_batch;
 *    trig_stream_submit and trig_stream_poll are thread-safe with respect to
 *    each other on one context.
 *  - hip_stream arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Work is ordered on that stream.
 */
#ifndef TRIG_H
#define TRIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIG_OK         0
#define TRIG_PENDING    1   /* poll: the ticket is not finished yet                     */
#define TRIG_EINVAL    -1   /* null pointer, n_pmt == 0, bad geometry id, bad argument   */
#define TRIG_ERANGE    -2   /* pmt_id >= n_pmt, n_hits >= 2^32, time span >= 2^31 ns,
                               or an event window outside int64                         */
#define TRIG_ENOMEM    -3   /* the request can never fit the HBM budget, or a device
                               allocation failed                                        */
#define TRIG_EAGAIN    -4   /* stream admission: budget or slots currently full; retry */
#define TRIG_EOVERFLOW -5   /* caller capacity too small; n_fires / n_events hold the
                               required counts and no list was written                 */
#define TRIG_EHIP      -6   /* HIP runtime error (message in trig_last_error)           */
#define TRIG_ECANCELED -7   /* poll: the ticket was cancelled                            */

typedef struct trig_ctx trig_ctx;   /* opaque; owns every device buffer it allocates */

/* Create a context on HIP device `device`: the state of one trigger process
 * (Sec. 2: the trigger CPUs receive the time slices of the Hit Managers; Sec. 4:
 * the TCPU keeps its GPU busy with successive slices).  hbm_budget_bytes caps
 * the device memory the context may hold (0 = 64 GiB).  Returns TRIG_OK,
 * TRIG_EINVAL (null out, no such device) or TRIG_EHIP; *out is NULL on
 * failure.  The context owns every device and pinned host buffer it takes. */
int trig_create(trig_ctx **out, int device, uint64_t hbm_budget_bytes);

/* Destroy a context: waits for all submitted stream work to finish (tickets
 * not yet polled are dropped), then frees every device and host buffer. */
void trig_destroy(trig_ctx *ctx);

/* Message of the last error on ctx (empty string if none).  Valid until the
 * next call on ctx. */
const char *trig_last_error(const trig_ctx *ctx);

/* Library version string. */
const char *trig_version(void);

/* Tower geometry (Sec. 2: detection units on floors of a tower).
 *   floor_id[n_pmt]           global floor index of each PMT (floors whose ids
 *                             differ by 1 are consecutive, for the AFC rule)
 *   thr_ns[n_pmt * n_pmt]     row-major causality table in ns; thr_ns[i*n_pmt+j]
 *                             bounds |t_i - t_j| when counting for a seed on PMT i
 *   adj_id[n_pmt]             may be NULL: adjacency group of each PMT for the SC
 *                             rule (Sec. 4.1: two adjacent PMTs); two PMTs of one
 *                             floor with equal adj_id are adjacent (e.g. the PMTs
 *                             at one end of a floor's bar).  NULL: none adjacent.
 * Host pointers; the arrays are copied, the caller keeps ownership.
 * 1 <= n_pmt <= 65536.  On success *geom_id names the copy. */
typedef struct {
    uint32_t        n_pmt;
    const int32_t  *floor_id;
    const uint32_t *thr_ns;
    const int32_t  *adj_id;
} trig_geom_desc;

int trig_geom_load(trig_ctx *ctx, const trig_geom_desc *geom, uint32_t *geom_id);

/* Trigger parameters.
 *   q_seed        charge seed threshold in 0.01 pe (seed if charge >= q_seed;
 *                 > 65535 disables the charge rule)
 *   t_floor_ns    floor-coincidence window (inclusive); < 0 disables the rule
 *   w_ns          cap on the causal window (the table value is min(thr, w_ns))
 *   min_fold      fire when 1 + correlated seeds >= min_fold
 *   half_event_ns half width H of the event window [t - H, t + H]
 *   l0_n, l0_tw_ns, l0_distinct
 *                 level-0 prefilter (paper Sec. 3: N hits in a fixed time window
 *                 TW, N7TW1000; N7TW500 for the 84-PMT tower; Sec. 4.1:
 *                 DN7TW1000 counts hits of distinct PMTs).  l0_n = 0 turns it
 *                 off.  Otherwise a hit passes when a window [t_i, t_i + l0_tw_ns)
 *                 that starts at a hit i and holds it also holds >= l0_n hits
 *                 (>= l0_n distinct PMTs when l0_distinct != 0), and the seed
 *                 rule runs on the hits that pass: a seed and its floor partner
 *                 both pass.  TRIG_EINVAL unless 1 <= l0_n <= 64 and
 *                 1 <= l0_tw_ns <= 1000000 when it is on.
 *   t_adj_ns, t_afloor_ns, seed_mode
 *                 seed menu (Sec. 4.1 trigger list; Sec. 5 candidate selection):
 *                 SC, a hit of an adjacent PMT (same floor, same adj_id) within
 *                 t_adj_ns; FC, a hit of another PMT of the same floor within
 *                 t_floor_ns (the rule above); AFC, a hit on a consecutive floor
 *                 within t_afloor_ns (all inclusive; a negative window turns its
 *                 rule off; partners pass level 0 when it is on).  seed_mode 0:
 *                 a seed meets the charge rule or any enabled partner rule;
 *                 seed_mode 1: the charge rule, or (SC or FC) and AFC, the
 *                 paper's [SC and AFC] or [FC and AFC].  TRIG_EINVAL for another
 *                 seed_mode.  Defaults (-1, -1, 0) give the rule without them. */
typedef struct {
    uint32_t q_seed;
    int32_t  t_floor_ns;
    uint32_t w_ns;
    uint32_t min_fold;
    uint32_t half_event_ns;
    uint32_t l0_n;
    uint32_t l0_tw_ns;
    uint32_t l0_distinct;
    int32_t  t_adj_ns;
    int32_t  t_afloor_ns;
    uint32_t seed_mode;
} trig_params;

enum { TRIG_MEM_HOST = 0, TRIG_MEM_DEVICE = 1 };

/* One time slice, structure of arrays in any order (the fast path is taken
 * when the order is a concatenation of time-ordered runs, as PMT streams
 * are).  mem says whether the three arrays are host or device (HIP) memory.
 * Device arrays are borrowed until the call returns (stream tickets: until
 * the poll that returns the result).  tag is echoed in the result. */
typedef struct {
    uint32_t        geom_id;
    uint32_t        mem;
    uint64_t        n_hits;
    const uint16_t *pmt_id;   /* [n_hits] */
    const int64_t  *t_ns;     /* [n_hits] ns, int64 */
    const uint16_t *charge;   /* [n_hits] 0.01 pe */
    uint64_t        tag;
} trig_slice_desc;

/* A fired seed: its time, input position, fold and PMT. 24 bytes. */
typedef struct {
    int64_t  t_ns;
    uint32_t hit_index;
    uint32_t fold;
    uint16_t pmt_id;
    uint16_t pad[3];
} trig_fire;

/* A merged event window: first fire time, window bounds, number of fires and
 * the largest fold among them. 32 bytes. */
typedef struct {
    int64_t  t_trig, t_begin, t_end;
    uint32_t n_fire, max_fold;
} trig_event;

/* Result of one slice.  The caller sets fires/fire_cap, events/event_cap,
 * seed_flags and tagged/tagged_cap (host buffers; seed_flags may be NULL, else
 * [n_hits] bytes by input position, 1 for a seed; tagged may be NULL, else
 * room for tagged_cap input indices).  The library fills the counts, status
 * and tag.  Fires are ordered by (t_ns, pmt_id, hit_index), events by t_begin.
 * tagged receives the hits inside the event windows (paper Sec. 4.2: the hits
 * within +-3 us of a trigger seed are marked for storage; Sec. 2: the 6 us
 * window of tower data around the trigger is stored): the input index of every
 * hit with t_begin <= t <= t_end for some event, ordered by (t, pmt, input
 * index); it is computed only when tagged is not NULL (trig_slice and
 * trig_batch; the stream entry points leave it NULL and n_tagged 0).
 * On TRIG_EOVERFLOW n_fires / n_events / n_tagged hold the required counts
 * and no list is written.  path reports how the slice was processed: bit 0 set
 * when the general radix sort ordered it (else the run merge), bit 1 set when
 * its trigger stage was rerun with a precomputed seed mask (with the seed menu
 * on, a burst far denser than the slice's mean density; the plain rule reads
 * such windows from device memory in the same pass). */
typedef struct {
    trig_fire  *fires;
    uint64_t    fire_cap, n_fires;
    trig_event *events;
    uint64_t    event_cap, n_events;
    uint8_t    *seed_flags;
    uint64_t    n_hits, n_seeds, tag;
    int32_t     status;
    uint32_t    path;
    uint32_t   *tagged;
    uint64_t    tagged_cap, n_tagged;
} trig_result;

/* Trigger one slice (Sec. 2: the 200 ms time slice is the unit of trigger
 * work; Sec. 4: the TGPU steps of preparing the slice, sending it to the GPU,
 * sorting and triggering there (Sec. 4.2), and bringing the trigger seeds and
 * tagged hits back to be stored).  slice: the hits, host or device memory
 * (borrowed for the call); params: the rule; result: caller-owned host
 * buffers, filled as described above; hip_stream: the work is ordered on it.
 * Synchronous with respect to the caller's buffers: it returns after the
 * results are in host memory.  Returns result->status: TRIG_OK, TRIG_EINVAL,
 * TRIG_ERANGE, TRIG_EOVERFLOW (counts filled, no list written), TRIG_ENOMEM
 * or TRIG_EHIP. */
int trig_slice(trig_ctx *ctx, const trig_slice_desc *slice, const trig_params *params,
               trig_result *result, void *hip_stream);

/* Allocation-free variant of trig_slice, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, semantics and results as
 * trig_slice, except:
 *  - the slice's arrays must be device memory (TRIG_EINVAL otherwise);
 *  - the slice's workspace, descriptors, plans and counters live in a fixed
 *    device scratch of TRIG_NOALLOC_SCRATCH_BYTES per GPU (a static device
 *    array that every GPU the library runs on holds until the process ends;
 *    its device address is looked up once per device when the first context on
 *    it is created), so the call allocates no device or pinned host memory,
 *    captures no graph and records no per-kernel timing;
 *  - a slice whose workspace does not fit the scratch (more than about 2.78
 *    million hits, or 2.75 million with seed flags: 96 bytes per hit) returns
 *    TRIG_ENOMEM, with both sizes in trig_last_error, and runs nothing;
 *  - the result lists are copied from device memory into the caller's buffers.
 * Every call on one GPU shares that GPU's scratch, whichever context makes it,
 * and the scratch keeps the last call's contents (nothing in it needs to start
 * at zero): calls that overlap in time on one GPU (two host threads, two
 * contexts) race and give wrong results, so the caller serialises them. */
#define TRIG_NOALLOC_SCRATCH_BYTES (256ull << 20)
int trig_slice_noalloc(trig_ctx *ctx, const trig_slice_desc *slice, const trig_params *params,
                       trig_result *result, void *hip_stream);

/* Trigger n slices together (Sec. 2: successive slices, possibly of several
 * towers, are handed to trigger processes; Sec. 4: one GPU serves the slices of
 * a trigger CPU; here every stage runs once over all slices, and device work
 * lists spread the uneven slices over the GPU).  slices[n] / results[n]: as for
 * trig_slice, results[i] receives slice i; a bad slice gets its own error
 * status and the others complete.  Returns TRIG_OK if every slice succeeded,
 * else the first failing status. */
int trig_batch(trig_ctx *ctx, uint32_t n, const trig_slice_desc *slices, const trig_params *params,
               trig_result *results, void *hip_stream);

/* Serving: submit a slice for asynchronous triggering (Sec. 2: slices arrive
 * from the Hit Managers every 200 ms and must be triggered within the time the
 * next ones take to arrive; Sec. 4: the host prepares and sends a slice while
 * the GPU works on others).  The inputs are copied (host memory, before the
 * call returns) or borrowed (device memory, until the poll that returns the
 * result) and admitted when the context's device budget allows.  Returns
 * TRIG_OK with *ticket set, TRIG_EAGAIN when the budget or the slots are full
 * right now, TRIG_ENOMEM when the slice can never fit, TRIG_EINVAL /
 * TRIG_ERANGE for bad arguments. */
int trig_stream_submit(trig_ctx *ctx, const trig_slice_desc *slice, const trig_params *params,
                       uint64_t *ticket);

/* Serving: wait up to timeout_us (0 = do not wait, <0 = wait forever) for a
 * ticket (Sec. 4.2: the trigger seeds and tagged data go back to the CPU, to be
 * passed on for storage).  Returns TRIG_PENDING if not done (or while another
 * thread's poll of the same ticket is delivering it), else the slice's status
 * with *result filled as for trig_slice (the caller's buffers in *result are
 * used; TRIG_EOVERFLOW keeps the ticket for a poll with larger buffers).  A
 * ticket is released by the poll that returns its result; polling it again
 * (or one never issued) gives TRIG_EINVAL. */
int trig_stream_poll(trig_ctx *ctx, uint64_t ticket, trig_result *result, int32_t timeout_us);

/* Serving: the next ticket whose slice finished (or was cancelled), in order of
 * completion, each reported once.  Waits up to timeout_us microseconds (0: not
 * at all, negative: until one finishes).  Returns TRIG_OK with *ticket set, or
 * TRIG_PENDING when none finished in time.  The ticket still has to be
 * delivered with trig_stream_poll.  Lets a caller with many tickets in flight
 * wait for whichever finishes first (the paper's trigger processes take slices
 * as they arrive, Sec. 2).  At most 2^20 completions not yet reported are kept;
 * older ones are dropped. */
int trig_stream_next_done(trig_ctx *ctx, uint64_t *ticket, int32_t timeout_us);

/* Serving: hold (paused != 0) or resume (0) the start of new device rounds.
 * Submissions are still admitted against the budget while held; rounds already
 * running finish.  For operators (drain control) and deterministic tests. */
int trig_stream_pause(trig_ctx *ctx, int paused);

/* Serving statistics since trig_create. */
typedef struct {
    uint64_t submitted, completed, rejected_again, in_flight;
    uint64_t device_bytes_in_use, device_bytes_peak;
    uint64_t rounds;        /* device rounds launched by the serving loop */
} trig_stream_stats;

int trig_stream_stats_get(trig_ctx *ctx, trig_stream_stats *out);

/* Tuning knobs of the device pipeline, per PMT-count class.  Chosen by the
 * autotuner; defaults are used until set.  No knob changes a result.
 *   seg_target    expected hits per time segment of the ordering stage
 *   seg_cap       hits one segment may hold: 256 or 512 order each segment
 *                 with one wave (256: fewer registers and LDS per wave, more
 *                 waves in flight), 2048, 4096 or 8192 with one workgroup
 *   grid_per_cu   persistent workgroups per compute unit
 *   tile_group    1024-hit trigger tiles per workgroup of the causal-fold
 *                 stage, a wave per tile (Sec. 4.1 sizes the paper's
 *                 sub-slices per GPU thread): 1, 2 or 4, fewer when the launch
 *                 would otherwise give a compute unit less than two workgroups
 *   window_cap    seeds of a tile's causal window staged in LDS at most, 512 or
 *                 2048 (a larger window is read from device memory)
 * trig_tune_set returns TRIG_EINVAL for other capacities, a zero target, a
 * grid_per_cu outside 1..16 or another tile_group or window_cap.  A batch whose
 * slices fall in several classes takes the largest tile_group and window_cap. */
typedef struct {
    uint32_t seg_target;
    uint32_t seg_cap;
    uint32_t grid_per_cu;
    uint32_t tile_group;
    uint32_t window_cap;
    uint32_t reserved;
} trig_tune;

int trig_tune_get(trig_ctx *ctx, uint32_t n_pmt, trig_tune *out);
int trig_tune_set(trig_ctx *ctx, uint32_t n_pmt_max, const trig_tune *tune);

/* Per-kernel timing with HIP events recorded on the launching stream.
 * enable != 0 starts recording (and clears totals); entries are returned in
 * launch order of first appearance. */
typedef struct {
    char     name[32];
    uint64_t launches;
    double   total_ms;
} trig_kernel_time;

int trig_profile_enable(trig_ctx *ctx, int enable);
int trig_profile_read(trig_ctx *ctx, trig_kernel_time *out, uint32_t cap, uint32_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_H */
