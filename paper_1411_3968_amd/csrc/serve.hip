// Serving loop: trig_stream_submit / trig_stream_poll.
//
// Slices arrive one at a time (the paper's Hit Managers hand successive 200 ms
// time slices to different trigger processes, Sec. 2).  A submitted slice is
// admitted when its device footprint fits the context's HBM budget next to the
// slices already admitted; otherwise submit returns TRIG_EAGAIN (or TRIG_ENOMEM
// if it can never fit).  Host inputs are copied to device memory before submit
// returns, so the hit buffers are resident on the GPU from then on.
//
// Continuous batching: SLOTS worker threads, each with its own HIP stream, take
// every admitted slice that is waiting (up to MAX_PER_ROUND with equal trigger
// parameters) as one device round through the batch-native pipeline.  Slices
// that arrive while rounds are running join the next round of whichever slot
// frees first, so their work overlaps on the device with the rounds in flight.
// Device memory: the loop keeps chunks of device memory for as long as it runs
// (taken from HIP when needed, within the context's budget) and carves each
// admitted slice a region of them (its input copy and its pipeline workspace);
// the region returns to the free list when the slice's results are on the host,
// which admits waiting slices (results longer than the pinned staging stay in the
// region until the poll copies them straight to the caller's buffers).  No HIP
// allocation or free happens per slice.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "api_internal.h"

namespace {

constexpr int SLOTS = 4;
constexpr uint32_t MAX_PER_ROUND = 64;
constexpr size_t DONE_Q_MAX = 1u << 20;

struct Ticket {
    uint64_t id = 0;
    trig_slice_desc desc = {};   // device pointers once admitted
    trig_params params = {};
    char *region = nullptr;      // arena region: input copy (host inputs), then workspace
    uint64_t footprint = 0;      // bytes of the region
    uint64_t in_bytes = 0;       // input copy at the start of the region
    bool done = false;
    int status = TRIG_PENDING;
    uint64_t n_hits = 0, n_seeds = 0, tag = 0;
    uint32_t path = 0;
    std::vector<trig_fire> fires;      // results staged on the host, or
    std::vector<trig_event> events;
    bool on_device = false;            // lists longer than the staging stay in the region
    bool busy = false;                 // a poll is copying the lists out
    const trig_fire *d_fires = nullptr;   // until the poll copies them to the caller
    const trig_event *d_events = nullptr;
    uint64_t n_fires = 0, n_events = 0;
};

bool same_params(const trig_params &a, const trig_params &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

// First-fit allocator over device chunks that live until shutdown.  Chunk bytes
// are accounted in the context budget when a chunk is taken.
struct Arena {
    static constexpr size_t ALIGN = 256;
    static constexpr size_t GROW_MIN = 1ull << 30;
    struct Chunk {
        char *base;
        size_t size;
        std::map<size_t, size_t> free;   // offset -> length
    };
    std::vector<Chunk> chunks;
    size_t total = 0;

    static size_t round_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

    char *take(size_t bytes) {
        for (Chunk &ch : chunks)
            for (auto it = ch.free.begin(); it != ch.free.end(); ++it)
                if (it->second >= bytes) {
                    const size_t off = it->first, len = it->second;
                    ch.free.erase(it);
                    if (len > bytes) ch.free.emplace(off + bytes, len - bytes);
                    return ch.base + off;
                }
        return nullptr;
    }

    // Size of a new chunk: an eighth of the budget, between 64 MiB and 1 GiB.
    static size_t grow_min(const trig_ctx *c) {
        const size_t e = (size_t)(c->budget / 8) & ~(ALIGN - 1);
        return std::min<size_t>(GROW_MIN, std::max<size_t>(e, 64ull << 20));
    }

    // A new chunk that starts with a region of `bytes`; null when the budget
    // does not allow it now.
    char *grow(trig_ctx *c, size_t bytes) {
        uint64_t room;
        {
            std::lock_guard<std::mutex> g(c->mem_mu);
            room = c->budget > c->bytes_in_use ? c->budget - c->bytes_in_use : 0;
        }
        size_t want = std::max(bytes, grow_min(c));
        if (want > room) want = room & ~(ALIGN - 1);
        if (want < bytes || ctx_reserve(c, want) != TRIG_OK) return nullptr;
        char *p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            ctx_release(c, want);
            return nullptr;
        }
        chunks.push_back(Chunk{p, want, {}});
        if (want > bytes) chunks.back().free.emplace(bytes, want - bytes);
        total += want;
        return p;
    }

    // Give every chunk that holds no region back to HIP; true if any was.
    bool shrink(trig_ctx *c) {
        bool any = false;
        for (auto it = chunks.begin(); it != chunks.end();) {
            const bool empty = it->free.size() == 1 && it->free.begin()->first == 0 &&
                               it->free.begin()->second == it->size;
            if (empty) {
                hipFree(it->base);
                ctx_release(c, it->size);
                total -= it->size;
                it = chunks.erase(it);
                any = true;
            } else {
                ++it;
            }
        }
        return any;
    }

    // A region of `bytes`: first fit in the chunks held, else a new chunk; when
    // the budget leaves no room for one, the chunks that hold no region are
    // returned to HIP first (a region never spans chunks, so a slice larger than
    // any chunk held needs the room they occupy).  Null when nothing fits now.
    char *alloc(trig_ctx *c, size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1));
        if (char *p = take(bytes)) return p;
        if (char *p = grow(c, bytes)) return p;
        if (shrink(c)) return grow(c, bytes);
        return nullptr;
    }

    void release(char *p, size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1));
        for (Chunk &ch : chunks) {
            if (p < ch.base || p >= ch.base + ch.size) continue;
            auto it = ch.free.emplace((size_t)(p - ch.base), bytes).first;
            auto nx = std::next(it);
            if (nx != ch.free.end() && it->first + it->second == nx->first) {
                it->second += nx->second;
                ch.free.erase(nx);
            }
            if (it != ch.free.begin()) {
                auto pv = std::prev(it);
                if (pv->first + pv->second == it->first) {
                    pv->second += it->second;
                    ch.free.erase(it);
                }
            }
            return;
        }
    }

    void release_all(trig_ctx *c) {
        for (Chunk &ch : chunks) {
            hipFree(ch.base);
            ctx_release(c, ch.size);
        }
        chunks.clear();
        total = 0;
    }
};

}  // namespace

struct ServeState {
    trig_ctx *c = nullptr;
    std::mutex mu;
    std::condition_variable cv_q, cv_done;
    std::deque<Ticket *> queue;
    std::deque<uint64_t> done_q;   // finished tickets not yet reported by next_done
    std::unordered_map<uint64_t, Ticket *> tickets;
    std::vector<std::thread> threads;
    std::vector<hipStream_t> streams;
    hipStream_t copy_stream = nullptr;
    std::mutex copy_mu;
    bool stop = false;
    bool paused = false;
    uint64_t next_id = 1;
    Arena arena;                 // guarded by mu
    std::vector<std::unique_ptr<Job>> jobs;   // one per slot, descriptors sized for a full round
    trig_stream_stats st = {};
};

static void run_round(ServeState *S, Job &job, hipStream_t stream, std::vector<Ticket *> &round) {
    trig_ctx *c = S->c;
    const uint32_t n = (uint32_t)round.size();
    std::vector<trig_slice_desc> descs(n);
    job.ext_ws.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        descs[i] = round[i]->desc;
        job.ext_ws[i] = round[i]->region + round[i]->in_bytes;
    }
    int rc = job.prepare(c, n, descs.data(), &round[0]->params, nullptr, nullptr, nullptr, stream);
    if (rc == TRIG_OK) rc = job.launch(c, false);
    if (rc == TRIG_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "serving round");
    }
    if (rc == TRIG_OK) rc = job.generic_pass(c, false);
    if (rc == TRIG_OK) rc = job.dense_pass(c, false);
    if (rc == TRIG_OK) {
        const trigdev::Plan *hp = job.host_plans();
        for (uint32_t i = 0; i < n; ++i) {
            Ticket *t = round[i];
            const SliceInfo &si = job.slices[i];
            trig_result r = {};
            const trigdev::Plan &P = hp[i];
            const bool ok = si.host_status == TRIG_OK && P.status == TRIG_OK && si.n > 0;
            t->on_device = ok && (P.n_fires > si.x_fcap || P.n_events > si.x_ecap);
            if (t->on_device) {
                // the counts only; the lists stay in the ticket's region
                r.n_hits = si.desc.n_hits;
                r.n_seeds = P.n_seeds;
                r.tag = si.desc.tag;
                r.path = (P.generic ? 1u : 0u) | (P.dense ? 2u : 0u);
                t->status = TRIG_OK;
                t->d_fires = si.dev.fires;
                t->d_events = si.dev.events;
                t->n_fires = P.n_fires;
                t->n_events = P.n_events;
            } else {
                t->fires.resize(ok ? P.n_fires : 0);
                t->events.resize(ok ? P.n_events : 0);
                r.fires = t->fires.data();
                r.fire_cap = t->fires.size();
                r.events = t->events.data();
                r.event_cap = t->events.size();
                t->status = job.deliver(c, i, &r);
                t->n_fires = t->fires.size();
                t->n_events = t->events.size();
            }
            t->n_hits = r.n_hits;
            t->n_seeds = r.n_seeds;
            t->tag = r.tag;
            t->path = r.path;
        }
    }
    if (rc != TRIG_OK)
        for (Ticket *t : round) {
            t->status = rc;
            t->fires.clear();
            t->events.clear();
            t->on_device = false;
            t->n_fires = t->n_events = 0;
        }
    job.ext_ws.clear();
}

static void slot_main(ServeState *S, int slot) {
    hipSetDevice(S->c->device);
    hipStream_t stream = S->streams[slot];
    Job &job = *S->jobs[slot];
    for (;;) {
        std::vector<Ticket *> round;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_q.wait(lk, [&] { return S->stop || (!S->paused && !S->queue.empty()); });
            if (S->queue.empty()) break;   // stop requested and nothing queued
            const trig_params p0 = S->queue.front()->params;
            for (auto it = S->queue.begin(); it != S->queue.end() && round.size() < MAX_PER_ROUND;) {
                if (same_params((*it)->params, p0)) { round.push_back(*it); it = S->queue.erase(it); }
                else ++it;
            }
            S->st.rounds += 1;
        }
        run_round(S, job, stream, round);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Ticket *t : round) {
                t->done = true;
                S->done_q.push_back(t->id);
                if (S->done_q.size() > DONE_Q_MAX) S->done_q.pop_front();
                if (!t->on_device) {
                    S->arena.release(t->region, t->footprint);
                    t->region = nullptr;
                }
                S->st.completed += 1;
            }
        }
        S->cv_done.notify_all();
    }
    job.release(S->c);
}

static ServeState *serve_get(trig_ctx *c) {
    std::lock_guard<std::mutex> once(c->serve_mu);   // first submits may race from several threads
    if (c->serve) return c->serve;
    ServeState *S = new ServeState();
    S->c = c;
    hipSetDevice(c->device);
    hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    S->streams.resize(SLOTS);
    for (int i = 0; i < SLOTS; ++i) hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
    // descriptor buffers of every slot are taken before any slice is admitted, so
    // a budget filled by admitted slices never starves a round of them
    for (int i = 0; i < SLOTS; ++i) {
        S->jobs.emplace_back(new Job());
        (void)S->jobs.back()->dmeta.ensure(c, job_meta_bytes(MAX_PER_ROUND, MAX_PER_ROUND * 4096u), S->streams[i]);
    }
    for (int i = 0; i < SLOTS; ++i) S->threads.emplace_back(slot_main, S, i);
    c->serve = S;
    return S;
}

// Stop the loop: slices not yet started are cancelled, running rounds finish.
void serve_shutdown(trig_ctx *c) {
    ServeState *S = c->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Ticket *t : S->queue) {
            t->done = true;
            S->done_q.push_back(t->id);
            t->status = TRIG_ECANCELED;
            S->arena.release(t->region, t->footprint);
            t->region = nullptr;
        }
        S->queue.clear();
    }
    S->cv_q.notify_all();
    for (auto &th : S->threads) th.join();
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &kv : S->tickets) delete kv.second;
    S->arena.release_all(c);
    for (auto s : S->streams) hipStreamDestroy(s);
    hipStreamDestroy(S->copy_stream);
    delete S;
    c->serve = nullptr;
}

extern "C" {

int trig_stream_submit(trig_ctx *c, const trig_slice_desc *d, const trig_params *prm, uint64_t *ticket) {
    if (!c) return TRIG_EINVAL;
    if (!d || !prm || !ticket) {
        ctx_set_error(c, "null argument to trig_stream_submit");
        return TRIG_EINVAL;
    }
    if (d->geom_id >= c->geoms.size()) {
        ctx_set_error(c, "unknown geom_id %u", d->geom_id);
        return TRIG_EINVAL;
    }
    if (d->n_hits >= (1ull << 32)) {
        ctx_set_error(c, "n_hits >= 2^32");
        return TRIG_ERANGE;
    }
    if (d->n_hits && (!d->pmt_id || !d->t_ns || !d->charge)) {
        ctx_set_error(c, "null input array");
        return TRIG_EINVAL;
    }
    if (d->mem != TRIG_MEM_HOST && d->mem != TRIG_MEM_DEVICE) {
        ctx_set_error(c, "bad mem kind");
        return TRIG_EINVAL;
    }
    const int prc = check_params(c, prm);
    if (prc != TRIG_OK) return prc;
    ServeState *S = serve_get(c);
    const uint64_t n = d->n_hits;
    const bool host = d->mem == TRIG_MEM_HOST && n > 0;
    const uint64_t in_bytes = host ? ((n * 2 + 255) & ~255ull) * 2 + ((n * 8 + 255) & ~255ull) : 0;
    const uint64_t foot = slice_footprint(n, false) + in_bytes;
    Ticket *t = new Ticket();
    t->params = *prm;
    t->desc = *d;
    t->footprint = foot;
    t->in_bytes = in_bytes;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete t;
            return TRIG_ECANCELED;
        }
        uint64_t other;   // device bytes held outside the arena (geometry, synchronous jobs)
        {
            std::lock_guard<std::mutex> g(c->mem_mu);
            other = c->bytes_in_use - S->arena.total;
        }
        if (foot + other > c->budget) {
            ctx_set_error(c, "slice of %llu hits can never fit the device budget", (unsigned long long)n);
            delete t;
            return TRIG_ENOMEM;
        }
        hipSetDevice(c->device);
        t->region = S->arena.alloc(c, foot);
        if (!t->region) {
            S->st.rejected_again += 1;
            delete t;
            return TRIG_EAGAIN;
        }
    }
    if (host) {
        std::lock_guard<std::mutex> g(S->copy_mu);
        hipSetDevice(c->device);
        char *b = t->region;
        const uint64_t o_t = (n * 2 + 255) & ~255ull, o_q = o_t + ((n * 8 + 255) & ~255ull);
        hipError_t e = hipMemcpyAsync(b, d->pmt_id, n * 2, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b + o_t, d->t_ns, n * 8, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b + o_q, d->charge, n * 2, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(S->copy_stream);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(t->region, t->footprint);
            delete t;
            return hip_fail(c, e, "copying slice inputs to the device");
        }
        t->desc.mem = TRIG_MEM_DEVICE;
        t->desc.pmt_id = (const uint16_t *)b;
        t->desc.t_ns = (const int64_t *)(b + o_t);
        t->desc.charge = (const uint16_t *)(b + o_q);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        t->id = S->next_id++;
        S->tickets[t->id] = t;
        S->queue.push_back(t);
        S->st.submitted += 1;
        *ticket = t->id;
    }
    S->cv_q.notify_one();
    return TRIG_OK;
}

int trig_stream_poll(trig_ctx *c, uint64_t ticket, trig_result *r, int32_t timeout_us) {
    if (!c) return TRIG_EINVAL;
    if (!r) {
        ctx_set_error(c, "null result");
        return TRIG_EINVAL;
    }
    ServeState *S;
    {
        std::lock_guard<std::mutex> once(c->serve_mu);
        S = c->serve;
    }
    if (!S) {
        ctx_set_error(c, "unknown ticket %llu", (unsigned long long)ticket);
        return TRIG_EINVAL;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    // The ticket is looked up again after every wait: another thread's poll may
    // have delivered (and deleted) it meanwhile.  Only the poll that marks the
    // ticket busy may erase it.
    auto lookup = [&]() -> Ticket * {
        auto f = S->tickets.find(ticket);
        return f == S->tickets.end() ? nullptr : f->second;
    };
    Ticket *t = lookup();
    if (!t) {
        ctx_set_error(c, "unknown ticket %llu", (unsigned long long)ticket);
        return TRIG_EINVAL;
    }
    if (t->busy) return TRIG_PENDING;   // another poll of this ticket is delivering it
    if (!t->done) {
        if (timeout_us == 0) return TRIG_PENDING;
        auto ready = [&] {
            Ticket *x = lookup();
            return !x || x->done;
        };
        if (timeout_us < 0) S->cv_done.wait(lk, ready);
        else S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
        t = lookup();
        if (!t) {
            ctx_set_error(c, "ticket %llu was delivered by another poll", (unsigned long long)ticket);
            return TRIG_EINVAL;
        }
        if (!t->done || t->busy) return TRIG_PENDING;
    }
    auto it = S->tickets.find(ticket);
    r->n_hits = t->n_hits ? t->n_hits : t->desc.n_hits;
    r->n_seeds = t->n_seeds;
    r->n_fires = t->n_fires;
    r->n_events = t->n_events;
    r->tag = t->desc.tag;
    r->path = t->path;
    r->status = t->status;
    r->n_tagged = 0;   // the stream path computes no tagged-hit list
    if (t->status == TRIG_OK) {
        if ((r->n_fires && (!r->fires || r->fire_cap < r->n_fires)) ||
            (r->n_events && (!r->events || r->event_cap < r->n_events))) {
            ctx_set_error(c, "result capacity too small; poll again with larger buffers");
            r->status = TRIG_EOVERFLOW;
            return TRIG_EOVERFLOW;   // the ticket stays until a poll delivers it
        }
        if (t->on_device) {
            // one copy from the ticket's region to the caller's buffers, then the
            // region goes back to the arena
            t->busy = true;
            lk.unlock();
            hipError_t e = hipSuccess;
            {
                std::lock_guard<std::mutex> g(S->copy_mu);
                hipSetDevice(c->device);
                if (r->n_fires)
                    e = hipMemcpyAsync(r->fires, t->d_fires, r->n_fires * sizeof(trig_fire), hipMemcpyDeviceToHost,
                                       S->copy_stream);
                if (e == hipSuccess && r->n_events)
                    e = hipMemcpyAsync(r->events, t->d_events, r->n_events * sizeof(trig_event),
                                       hipMemcpyDeviceToHost, S->copy_stream);
                if (e == hipSuccess) e = hipStreamSynchronize(S->copy_stream);
            }
            lk.lock();
            t->busy = false;
            it = S->tickets.find(ticket);   // submits may have rehashed the map meanwhile
            if (e != hipSuccess) {
                r->status = hip_fail(c, e, "copying results to the caller");
                return r->status;   // the ticket stays; a later poll may succeed
            }
            S->arena.release(t->region, t->footprint);
            t->region = nullptr;
        } else {
            // the copy out of the ticket's host lists runs without the loop's lock
            // (the ticket is done and marked busy, so no worker or other poll
            // touches it), so the workers finishing rounds are not held up
            t->busy = true;
            lk.unlock();
            if (r->n_fires) std::memcpy(r->fires, t->fires.data(), r->n_fires * sizeof(trig_fire));
            if (r->n_events) std::memcpy(r->events, t->events.data(), r->n_events * sizeof(trig_event));
            lk.lock();
            t->busy = false;
            it = S->tickets.find(ticket);   // submits may have rehashed the map meanwhile
        }
    }
    const int st = t->status;
    S->tickets.erase(it);
    delete t;
    lk.unlock();
    S->cv_done.notify_all();   // other polls waiting on this ticket see it gone
    return st;
}

int trig_stream_next_done(trig_ctx *c, uint64_t *ticket, int32_t timeout_us) {
    if (!c) return TRIG_EINVAL;
    if (!ticket) {
        ctx_set_error(c, "null ticket");
        return TRIG_EINVAL;
    }
    ServeState *S;
    {
        std::lock_guard<std::mutex> once(c->serve_mu);
        S = c->serve;
    }
    if (!S) return TRIG_PENDING;   // nothing was ever submitted
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] {
        // drop ids already delivered and forgotten
        while (!S->done_q.empty() && !S->tickets.count(S->done_q.front())) S->done_q.pop_front();
        return !S->done_q.empty();
    };
    if (!ready()) {
        if (timeout_us == 0) return TRIG_PENDING;
        if (timeout_us < 0)
            S->cv_done.wait(lk, ready);
        else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return TRIG_PENDING;
    }
    *ticket = S->done_q.front();
    S->done_q.pop_front();
    return TRIG_OK;
}

int trig_stream_pause(trig_ctx *c, int paused) {
    if (!c) return TRIG_EINVAL;
    ServeState *S = serve_get(c);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->paused = paused != 0;
    }
    S->cv_q.notify_all();
    return TRIG_OK;
}

int trig_stream_stats_get(trig_ctx *c, trig_stream_stats *out) {
    if (!c || !out) return TRIG_EINVAL;
    *out = trig_stream_stats{};
    ServeState *S = c->serve;
    if (S) {
        std::lock_guard<std::mutex> lk(S->mu);
        *out = S->st;
        out->in_flight = S->st.submitted - S->st.completed;
    }
    std::lock_guard<std::mutex> g(c->mem_mu);
    out->device_bytes_in_use = c->bytes_in_use;
    out->device_bytes_peak = c->bytes_peak;
    return TRIG_OK;
}

}  // extern "C"
