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
// Device memory of a round comes from the stream-ordered pool and returns to it
// when the round's results are on the host, which admits waiting slices.
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "api_internal.h"

namespace {

constexpr int SLOTS = 4;
constexpr uint32_t MAX_PER_ROUND = 64;

struct Ticket {
    uint64_t id = 0;
    trig_slice_desc desc = {};   // device pointers once admitted
    trig_params params = {};
    void *dev_input = nullptr;   // owned device copy of host inputs
    uint64_t footprint = 0;
    bool done = false;
    int status = TRIG_PENDING;
    uint64_t n_hits = 0, n_seeds = 0, tag = 0;
    uint32_t path = 0;
    std::vector<trig_fire> fires;
    std::vector<trig_event> events;
};

bool same_params(const trig_params &a, const trig_params &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

}  // namespace

struct ServeState {
    trig_ctx *c = nullptr;
    std::mutex mu;
    std::condition_variable cv_q, cv_done;
    std::deque<Ticket *> queue;
    std::unordered_map<uint64_t, Ticket *> tickets;
    std::vector<std::thread> threads;
    std::vector<hipStream_t> streams;
    hipStream_t copy_stream = nullptr;
    std::mutex copy_mu;
    bool stop = false;
    bool paused = false;
    uint64_t next_id = 1;
    uint64_t reserved = 0;       // bytes of admitted, unfinished tickets
    trig_stream_stats st = {};
};

static void run_round(ServeState *S, Job &job, hipStream_t stream, std::vector<Ticket *> &round) {
    trig_ctx *c = S->c;
    const uint32_t n = (uint32_t)round.size();
    std::vector<trig_slice_desc> descs(n);
    for (uint32_t i = 0; i < n; ++i) descs[i] = round[i]->desc;
    int rc = job.prepare(c, n, descs.data(), &round[0]->params, nullptr, nullptr, nullptr, stream);
    if (rc == TRIG_OK) rc = job.launch(c, false);
    if (rc == TRIG_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "serving round");
    }
    if (rc == TRIG_OK) rc = job.generic_pass(c, false);
    if (rc == TRIG_OK) {
        const trigdev::Plan *hp = (const trigdev::Plan *)job.h_plans.ptr;
        for (uint32_t i = 0; i < n; ++i) {
            Ticket *t = round[i];
            trig_result r = {};
            const trigdev::Plan &P = hp[i];
            const bool ok = job.slices[i].host_status == TRIG_OK && P.status == TRIG_OK && job.slices[i].n > 0;
            t->fires.resize(ok ? P.n_fires : 0);
            t->events.resize(ok ? P.n_events : 0);
            r.fires = t->fires.data();
            r.fire_cap = t->fires.size();
            r.events = t->events.data();
            r.event_cap = t->events.size();
            t->status = job.deliver(c, i, &r);
            t->n_hits = r.n_hits;
            t->n_seeds = r.n_seeds;
            t->tag = r.tag;
            t->path = r.path;
        }
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "serving results");
    }
    if (rc != TRIG_OK)
        for (Ticket *t : round) { t->status = rc; t->fires.clear(); t->events.clear(); }
    job.ws.release_async(stream);
    job.dmeta.release_async(stream);
    job.gscratch.release_async(stream);
    for (Ticket *t : round)
        if (t->dev_input) { hipFreeAsync(t->dev_input, stream); t->dev_input = nullptr; }
    hipStreamSynchronize(stream);
    if (job.async_extra) { ctx_release(c, job.async_extra); job.async_extra = 0; }
}

static void slot_main(ServeState *S, int slot) {
    hipSetDevice(S->c->device);
    hipStream_t stream = S->streams[slot];
    Job job;
    job.async_mem = true;
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
                S->reserved -= t->footprint;
                ctx_release(S->c, t->footprint);
                S->st.completed += 1;
            }
        }
        S->cv_done.notify_all();
    }
    job.h_slices.release();
    job.h_plans.release();
}

static ServeState *serve_get(trig_ctx *c) {
    std::lock_guard<std::mutex> once(c->serve_mu);   // first submits may race from several threads
    if (c->serve) return c->serve;
    ServeState *S = new ServeState();
    S->c = c;
    hipSetDevice(c->device);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    S->streams.resize(SLOTS);
    for (int i = 0; i < SLOTS; ++i) hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
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
            t->status = TRIG_ECANCELED;
            S->reserved -= t->footprint;
            ctx_release(c, t->footprint);
        }
        S->queue.clear();
    }
    S->cv_q.notify_all();
    for (auto &th : S->threads) th.join();
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &kv : S->tickets) {
        if (kv.second->dev_input) hipFree(kv.second->dev_input);
        delete kv.second;
    }
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
    ServeState *S = serve_get(c);
    const uint64_t n = d->n_hits;
    const bool host = d->mem == TRIG_MEM_HOST && n > 0;
    const uint64_t in_bytes = host ? ((n * 2 + 255) & ~255ull) * 2 + ((n * 8 + 255) & ~255ull) : 0;
    const uint64_t foot = slice_footprint(n, false) + in_bytes;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return TRIG_ECANCELED;
        uint64_t other;
        {
            std::lock_guard<std::mutex> g(c->mem_mu);
            other = c->bytes_in_use - S->reserved;
        }
        if (foot + other > c->budget) {
            ctx_set_error(c, "slice of %llu hits can never fit the device budget", (unsigned long long)n);
            return TRIG_ENOMEM;
        }
        if (ctx_reserve(c, foot) != TRIG_OK) {
            S->st.rejected_again += 1;
            return TRIG_EAGAIN;
        }
        S->reserved += foot;
    }
    Ticket *t = new Ticket();
    t->params = *prm;
    t->desc = *d;
    t->footprint = foot;
    if (host) {
        std::lock_guard<std::mutex> g(S->copy_mu);
        hipSetDevice(c->device);
        hipError_t e = hipMallocAsync(&t->dev_input, in_bytes, S->copy_stream);
        char *b = (char *)t->dev_input;
        const uint64_t o_t = (n * 2 + 255) & ~255ull, o_q = o_t + ((n * 8 + 255) & ~255ull);
        if (e == hipSuccess) e = hipMemcpyAsync(b, d->pmt_id, n * 2, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b + o_t, d->t_ns, n * 8, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b + o_q, d->charge, n * 2, hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(S->copy_stream);
        if (e != hipSuccess) {
            if (t->dev_input) hipFree(t->dev_input);
            std::lock_guard<std::mutex> lk(S->mu);
            S->reserved -= foot;
            ctx_release(c, foot);
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
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) {
        ctx_set_error(c, "unknown ticket %llu", (unsigned long long)ticket);
        return TRIG_EINVAL;
    }
    Ticket *t = it->second;
    if (!t->done) {
        if (timeout_us == 0) return TRIG_PENDING;
        if (timeout_us < 0) {
            S->cv_done.wait(lk, [&] { return t->done; });
        } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return t->done; })) {
            return TRIG_PENDING;
        }
    }
    r->n_hits = t->n_hits ? t->n_hits : t->desc.n_hits;
    r->n_seeds = t->n_seeds;
    r->n_fires = t->fires.size();
    r->n_events = t->events.size();
    r->tag = t->desc.tag;
    r->path = t->path;
    r->status = t->status;
    if (t->status == TRIG_OK) {
        if ((r->n_fires && (!r->fires || r->fire_cap < r->n_fires)) ||
            (r->n_events && (!r->events || r->event_cap < r->n_events))) {
            ctx_set_error(c, "result capacity too small; poll again with larger buffers");
            r->status = TRIG_EOVERFLOW;
            return TRIG_EOVERFLOW;   // the ticket stays until a poll delivers it
        }
        if (r->n_fires) std::memcpy(r->fires, t->fires.data(), r->n_fires * sizeof(trig_fire));
        if (r->n_events) std::memcpy(r->events, t->events.data(), r->n_events * sizeof(trig_event));
    }
    const int st = t->status;
    S->tickets.erase(it);
    delete t;
    return st;
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
