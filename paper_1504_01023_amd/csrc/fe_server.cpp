// fe_server.cpp -- continuous-batching integration server.
//
// Requests (one mesh each: a kind, an element count, host or device inputs)
// arrive at any time. A scheduler thread:
//   1. admits queued requests in arrival order while a slot is free and the
//      request's device bytes (inputs + outputs) fit in the HBM budget
//      (one arena allocated at creation; first-fit sub-allocation);
//   2. copies admitted inputs to the device on a copy stream;
//   3. every tick, cuts the ready requests into chunks and launches them
//      together through one persistent batched launch (fe_batch), so work of
//      requests that arrived while others ran is fused into the next launch;
//   4. marks a request complete when all its chunks' ticks have finished;
//      outputs stay resident in the arena until the consumer releases them
//      (the output is "stored in memory available to subsequent solution
//      steps", Sec. 3.1).
// Two ticks may be in flight, so filling the next table overlaps the device.
// Latency = completion - submission; the timestamps of admission and input
// readiness split it into queue, transfer and device parts (the transfer
// share is the host-device traffic Sec. 4.6 warns dominates when integration
// stands alone).
//
// The FAKE backend replaces every device action by a timing model on the
// host (no GPU needed), so admission, ordering, failure isolation and the
// latency bookkeeping are testable on any machine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fe.h"
#include "fe_api_internal.h"

using namespace fe;

namespace {

// A roctx range over a scope (visible in rocprofv3 --marker-trace; a no-op
// when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
};


double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ------------------------------------------------------------------ arena
class Arena {
public:
    explicit Arena(int64_t cap) : cap_(cap) { free_[0] = cap; }
    static int64_t round(int64_t n) { return (n + 255) & ~int64_t(255); }
    int64_t alloc(int64_t n)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, rem = it->second - n;
                free_.erase(it);
                if (rem > 0)
                    free_[off + n] = rem;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        n = round(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t capacity() const { return cap_; }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }

private:
    int64_t cap_, used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;
};

enum State { QUEUED, ADMITTED, READY, DONE };

struct KindInfo {
    int nv = 4;              // vertices
    int64_t nk = 0, nf = 0;  // K and F rows
    int64_t nc = 0;          // coefficient rows
    size_t tsize = 8;
};

struct Req {
    uint64_t id = 0, tag = 0;
    int kind = 0;
    int64_t n = 0;
    bool dev_inputs = false;
    const double *h_coords = nullptr;  // host inputs, leading dimension ld_host
    const void *h_coeffs = nullptr;
    int64_t ld_host = 0;
    const double *coords = nullptr;    // device inputs used by the kernels
    const void *coeffs = nullptr;
    int64_t ld_in = 0;
    void *out_K = nullptr, *out_F = nullptr;
    int64_t ld_out = 0;
    int64_t off[4] = {-1, -1, -1, -1};  // arena offsets: coords, coeffs, K, F
    int64_t sz[4] = {0, 0, 0, 0};
    State state = QUEUED;
    int status = FE_OK;
    int64_t next_elem = 0;       // first element not yet dispatched
    int64_t chunks_total = 0, chunks_done = 0;
    int64_t chunks_inflight = 0; // dispatched in ticks that have not finished
    bool released = false;       // the consumer released it while chunks ran
    hipEvent_t ev_in = nullptr;  // GPU: inputs copied
    double fake_ready = 0;       // FAKE: time the inputs are ready
    double t_submit = 0, t_admit = 0, t_ready = 0, t_done = 0;
};

struct Tick {
    std::vector<std::pair<uint64_t, int64_t>> parts;  // (request id, chunks)
    int64_t elems = 0;
    hipEvent_t ev = nullptr;
    double fake_done = 0;
};

}  // namespace

struct fe_server {
    fe_server_config cfg{};
    std::vector<fe_batch_kind> kinds;
    std::vector<std::vector<double>> rule_xi, rule_w;
    std::vector<KindInfo> kinfo;
    bool fake = false;

    // device resources
    void *arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    fe_batch *batch = nullptr;
    hipStream_t copy = nullptr, compute = nullptr;
    std::vector<hipEvent_t> event_pool;
    int device = 0;
    double fake_copy_free = 0, fake_dev_free = 0;

    // Scheduler-owned state: only the scheduler thread touches these.
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<uint64_t> active;  // admitted, not done, in admission order
    std::deque<Tick> ticks;
    int slots_used = 0;
    std::vector<fe_completion> finished;  // completions of this iteration

    // Hand-over between callers and the scheduler (io_mu, held briefly).
    std::mutex io_mu;
    std::condition_variable cv_work, cv_done;
    std::vector<std::unique_ptr<Req>> inbox;
    std::vector<uint64_t> release_q;
    std::deque<fe_completion> done_q;
    std::unordered_set<uint64_t> completed;  // done, not yet released
    uint64_t next_id = 1;
    uint64_t release_posted = 0, release_done = 0;  // release calls queued / applied
    bool stop = false;
    std::thread thread;

    // Statistics (stats_mu).
    std::mutex stats_mu;
    int64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_failed = 0, n_ticks = 0;
    int64_t elements_done = 0, bytes_in_use = 0, bytes_peak = 0, n_queue = 0, n_active = 0;
    std::vector<double> lat, q_t, h2d_t, dev_t;
};

namespace {

hipEvent_t take_event(fe_server *s)
{
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    return e;
}

void give_event(fe_server *s, hipEvent_t e)
{
    if (e)
        s->event_pool.push_back(e);
}

void free_request_memory(fe_server *s, Req &r)
{
    for (int i = 0; i < 4; ++i)
        if (r.off[i] >= 0) {
            s->arena->release(r.off[i], r.sz[i]);
            r.off[i] = -1;
        }
}

void complete(fe_server *s, Req &r, int status, double t)
{
    r.state = DONE;
    r.status = status;
    r.t_done = t;
    s->slots_used -= (r.t_admit > 0) ? 1 : 0;
    if (r.ev_in) {
        give_event(s, r.ev_in);
        r.ev_in = nullptr;
    }
    fe_completion c;
    std::memset(&c, 0, sizeof(c));
    c.id = r.id;
    c.tag = r.tag;
    c.status = status;
    c.kind = r.kind;
    c.n_elem = r.n;
    c.out_K = status == FE_OK ? r.out_K : nullptr;
    c.out_F = status == FE_OK ? r.out_F : nullptr;
    c.ld_out = r.ld_out;
    c.t_submit = r.t_submit;
    c.t_admit = r.t_admit;
    c.t_ready = r.t_ready;
    c.t_done = r.t_done;
    // A failed request's memory is reused only once no launched chunk of it
    // can still write there.
    if (status != FE_OK && r.chunks_inflight == 0)
        free_request_memory(s, r);
    s->active.erase(std::remove(s->active.begin(), s->active.end(), r.id), s->active.end());
    s->finished.push_back(c);
}

// Device bytes a request needs and its layout.
void layout(const fe_server *s, Req &r)
{
    const KindInfo &ki = s->kinfo[r.kind];
    // rows padded to 64 elements: with the arena's 256-byte alignment every
    // row starts on a cache line, so the kernels' wavefront segments cover
    // whole lines (partial-line writes cut the HBM write rate markedly)
    const int64_t ld = (r.n + 63) / 64 * 64;
    r.ld_out = ld;
    if (!r.dev_inputs) {
        r.ld_in = ld;
        r.sz[0] = 8 * 3 * ki.nv * ld;
        r.sz[1] = (int64_t)ki.tsize * ki.nc * ld;
    }
    r.sz[2] = (int64_t)ki.tsize * ki.nk * ld;
    r.sz[3] = (int64_t)ki.tsize * ki.nf * ld;
}

int64_t need_bytes(const Req &r)
{
    int64_t t = 0;
    for (int i = 0; i < 4; ++i)
        t += r.sz[i] > 0 ? Arena::round(r.sz[i]) : 0;
    return t;
}

// Try to admit the head of the queue; returns false when it must wait.
bool admit_one(fe_server *s)
{
    if (s->queue.empty() || s->slots_used >= s->cfg.max_slots)
        return false;
    Req &r = *s->reqs[s->queue.front()];
    layout(s, r);
    const double t = now_s();
    if (need_bytes(r) > s->arena->capacity()) {
        s->queue.pop_front();
        complete(s, r, FE_ERR_CAPACITY, t);
        return true;
    }
    int64_t offs[4] = {-1, -1, -1, -1};
    for (int i = 0; i < 4; ++i) {
        if (r.sz[i] <= 0)
            continue;
        offs[i] = s->arena->alloc(r.sz[i]);
        if (offs[i] < 0) {
            for (int j = 0; j < i; ++j)
                if (offs[j] >= 0)
                    s->arena->release(offs[j], r.sz[j]);
            return false;  // wait for memory
        }
    }
    s->queue.pop_front();
    for (int i = 0; i < 4; ++i)
        r.off[i] = offs[i];
    char *base = static_cast<char *>(s->arena_base);
    r.out_K = base + r.off[2];
    r.out_F = base + r.off[3];
    r.state = ADMITTED;
    r.t_admit = t;
    ++s->slots_used;
    {
        std::lock_guard<std::mutex> lk(s->stats_mu);
        ++s->n_admitted;
    }
    s->active.push_back(r.id);
    const KindInfo &ki = s->kinfo[r.kind];
    if (r.dev_inputs) {
        r.state = READY;
        r.t_ready = t;
        return true;
    }
    r.coords = reinterpret_cast<const double *>(base + r.off[0]);
    r.coeffs = r.off[1] >= 0 ? base + r.off[1] : nullptr;
    const int64_t in_bytes = r.sz[0] + r.sz[1];
    if (s->fake) {
        s->fake_copy_free = std::max(s->fake_copy_free, t) + in_bytes / s->cfg.fake_h2d_bytes_per_s;
        r.fake_ready = s->fake_copy_free;
        return true;
    }
    const TraceRange trace("fe_server admit: H2D");
    hipError_t err = hipMemcpy2DAsync(const_cast<double *>(r.coords), 8 * r.ld_in, r.h_coords,
                                      8 * r.ld_host, 8 * r.n, 3 * ki.nv, hipMemcpyHostToDevice,
                                      s->copy);
    if (err == hipSuccess && ki.nc > 0 && r.h_coeffs)
        err = hipMemcpy2DAsync(const_cast<void *>(r.coeffs), ki.tsize * r.ld_in, r.h_coeffs,
                               ki.tsize * r.ld_host, ki.tsize * r.n, ki.nc, hipMemcpyHostToDevice,
                               s->copy);
    if (err == hipSuccess) {
        r.ev_in = take_event(s);
        err = r.ev_in ? hipEventRecord(r.ev_in, s->copy) : hipErrorOutOfMemory;
    }
    if (err != hipSuccess) {
        // a copy may already be in flight into this request's memory
        (void)hipStreamSynchronize(s->copy);
        complete(s, r, FE_ERR_HIP, t);
    }
    return true;
}

bool inputs_ready(fe_server *s, Req &r, double t)
{
    if (s->fake)
        return t >= r.fake_ready;
    return hipEventQuery(r.ev_in) == hipSuccess;
}

// Build and launch one tick from the ready requests. Chunks are shared
// fairly: every ready request gets an equal share of the tick (at least one
// chunk), and capacity a request cannot use goes to the others in admission
// order, so a large request never holds back requests that arrive while it
// runs.

void launch_tick(fe_server *s)
{
    const int64_t ce = s->cfg.chunk_elems;
    std::vector<Req *> ready;
    for (uint64_t id : s->active) {
        Req &r = *s->reqs[id];
        if (r.state == READY && r.next_elem < r.n)
            ready.push_back(&r);
    }
    if (ready.empty())
        return;
    const TraceRange trace("fe_server tick");
    std::vector<int64_t> want(ready.size()), give(ready.size(), 0);
    int64_t cap = s->cfg.max_chunks;
    for (size_t i = 0; i < ready.size(); ++i)
        want[i] = (ready[i]->n - ready[i]->next_elem + ce - 1) / ce;
    const int64_t share = std::max<int64_t>(1, cap / (int64_t)ready.size());
    for (size_t i = 0; i < ready.size() && cap > 0; ++i) {
        give[i] = std::min({want[i], share, cap});
        cap -= give[i];
    }
    for (size_t i = 0; i < ready.size() && cap > 0; ++i) {
        const int64_t more = std::min(want[i] - give[i], cap);
        give[i] += more;
        cap -= more;
    }
    Tick tk;
    for (size_t i = 0; i < ready.size(); ++i) {
        if (give[i] == 0)
            continue;
        Req &r = *ready[i];
        const int64_t take = std::min(r.n - r.next_elem, give[i] * ce);
        const int64_t e0 = r.next_elem;
        const KindInfo &ki = s->kinfo[r.kind];
        int st = FE_OK;
        if (!s->fake) {
            const double *c = r.coords + e0;
            const void *cf = r.coeffs ? static_cast<const char *>(r.coeffs) + ki.tsize * e0 : nullptr;
            void *K = static_cast<char *>(r.out_K) + ki.tsize * e0;
            void *F = static_cast<char *>(r.out_F) + ki.tsize * e0;
            st = fe_batch_add(s->batch, r.kind, take, c, cf, r.ld_in, K, F, r.ld_out);
        }
        if (st != FE_OK) {
            // this request cannot run (e.g. unsuitable device inputs): fail it alone
            complete(s, r, st, now_s());
            continue;
        }
        if (r.chunks_total == 0)
            r.chunks_total = (r.n + ce - 1) / ce;
        r.next_elem += take;
        tk.parts.emplace_back(r.id, give[i]);
        tk.elems += take;
    }
    if (tk.parts.empty())
        return;
    const double t = now_s();
    if (s->fake) {
        s->fake_dev_free = std::max(s->fake_dev_free, t) + s->cfg.fake_tick_overhead_s +
                           tk.elems * s->cfg.fake_ns_per_elem * 1e-9;
        tk.fake_done = s->fake_dev_free;
    } else {
        int st = fe_batch_launch(s->batch, s->compute);
        if (st == FE_OK) {
            tk.ev = take_event(s);
            if (!tk.ev || hipEventRecord(tk.ev, s->compute) != hipSuccess)
                st = FE_ERR_HIP;
        }
        if (st != FE_OK) {
            for (auto &pr : tk.parts)
                complete(s, *s->reqs[pr.first], FE_ERR_HIP, t);
            return;
        }
    }
    for (auto &pr : tk.parts)
        s->reqs[pr.first]->chunks_inflight += pr.second;
    {
        std::lock_guard<std::mutex> lk(s->stats_mu);
        ++s->n_ticks;
    }
    s->ticks.push_back(std::move(tk));
}

bool tick_done(fe_server *s, Tick &tk, double t)
{
    if (s->fake)
        return t >= tk.fake_done;
    return hipEventQuery(tk.ev) == hipSuccess;
}

// Hand completions to the callers and update the statistics.
void publish(fe_server *s)
{
    {
        std::lock_guard<std::mutex> lk(s->stats_mu);
        for (const fe_completion &c : s->finished) {
            if (c.status == FE_OK) {
                ++s->n_completed;
                s->elements_done += c.n_elem;
                s->lat.push_back(c.t_done - c.t_submit);
                s->q_t.push_back(c.t_admit - c.t_submit);
                s->h2d_t.push_back(c.t_ready - c.t_admit);
                s->dev_t.push_back(c.t_done - c.t_ready);
            } else {
                ++s->n_failed;
            }
        }
        s->bytes_in_use = s->arena->used();
        s->bytes_peak = s->arena->peak();
        s->n_queue = (int64_t)s->queue.size();
        s->n_active = (int64_t)s->active.size();
    }
    if (!s->finished.empty()) {
        {
            std::lock_guard<std::mutex> lk(s->io_mu);
            for (const fe_completion &c : s->finished) {
                s->done_q.push_back(c);
                s->completed.insert(c.id);
            }
        }
        s->cv_done.notify_all();
        s->finished.clear();
    }
}

void loop(fe_server *s)
{
    if (!s->fake)
        (void)hipSetDevice(s->device);
    std::vector<std::unique_ptr<Req>> arrived;
    std::vector<uint64_t> released;
    for (;;) {
        uint64_t release_seq = 0;
        {
            std::lock_guard<std::mutex> lk(s->io_mu);
            if (s->stop)
                break;
            arrived.swap(s->inbox);
            released.swap(s->release_q);
            release_seq = s->release_posted;
        }
        const bool had_releases = !released.empty();
        bool progress = !arrived.empty() || !released.empty();
        for (auto &r : arrived) {
            const uint64_t id = r->id;
            s->queue.push_back(id);
            s->reqs[id] = std::move(r);
        }
        arrived.clear();
        for (uint64_t id : released) {
            auto it = s->reqs.find(id);
            if (it == s->reqs.end())
                continue;
            if (it->second->chunks_inflight > 0) {
                it->second->released = true;  // freed when its last tick ends
                continue;
            }
            free_request_memory(s, *it->second);
            s->reqs.erase(it);
        }
        released.clear();
        while (admit_one(s))
            progress = true;
        double t = now_s();
        for (uint64_t id : std::vector<uint64_t>(s->active)) {
            Req &r = *s->reqs[id];
            if (r.state == ADMITTED && inputs_ready(s, r, t)) {
                r.state = READY;
                r.t_ready = t;
                if (r.ev_in) {
                    give_event(s, r.ev_in);
                    r.ev_in = nullptr;
                }
                progress = true;
            }
        }
        while (!s->ticks.empty() && tick_done(s, s->ticks.front(), t = now_s())) {
            Tick tk = std::move(s->ticks.front());
            s->ticks.pop_front();
            give_event(s, tk.ev);
            for (auto &pr : tk.parts) {
                auto it = s->reqs.find(pr.first);
                Req &r = *it->second;
                r.chunks_inflight -= pr.second;
                if (r.state == DONE) {
                    // failed while this tick ran: its memory is free to go now
                    if (r.chunks_inflight == 0) {
                        free_request_memory(s, r);
                        if (r.released)
                            s->reqs.erase(it);
                    }
                    continue;
                }
                r.chunks_done += pr.second;
                if (r.chunks_done >= r.chunks_total && r.next_elem >= r.n)
                    complete(s, r, FE_OK, t);
            }
            progress = true;
        }
        if (s->ticks.size() < 2) {
            const size_t before = s->ticks.size();
            launch_tick(s);
            progress = progress || s->ticks.size() != before;
        }
        publish(s);
        if (had_releases) {
            {
                std::lock_guard<std::mutex> lk(s->io_mu);
                s->release_done = release_seq;
            }
            s->cv_done.notify_all();
        }
        if (!progress) {
            // Poll quickly while work is in flight; sleep until woken otherwise.
            const bool busy = !s->ticks.empty() || !s->active.empty();
            std::unique_lock<std::mutex> lk(s->io_mu);
            s->cv_work.wait_for(lk, busy ? std::chrono::microseconds(20) : std::chrono::milliseconds(5),
                                [&] { return s->stop || !s->inbox.empty() || !s->release_q.empty(); });
        }
    }
}

void destroy_server(fe_server *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->io_mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->thread.joinable())
        s->thread.join();
    if (!s->fake) {
        if (s->compute)
            (void)hipStreamSynchronize(s->compute);
        if (s->copy)
            (void)hipStreamSynchronize(s->copy);
        for (auto &kv : s->reqs)
            if (kv.second->ev_in)
                (void)hipEventDestroy(kv.second->ev_in);
        for (auto &tk : s->ticks)
            if (tk.ev)
                (void)hipEventDestroy(tk.ev);
        for (hipEvent_t e : s->event_pool)
            (void)hipEventDestroy(e);
        if (s->batch)
            fe_batch_destroy(s->batch);
        if (s->arena_base)
            (void)hipFree(s->arena_base);
        if (s->copy)
            (void)hipStreamDestroy(s->copy);
        if (s->compute)
            (void)hipStreamDestroy(s->compute);
    } else {
        std::free(s->arena_base);
    }
    delete s;
}

double percentile(std::vector<double> v, double p)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = p * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

double mean(const std::vector<double> &v)
{
    double t = 0;
    for (double x : v)
        t += x;
    return v.empty() ? 0.0 : t / v.size();
}

}  // namespace

extern "C" {

double fe_server_now(void) { return now_s(); }

int fe_server_create(const fe_server_config *cfg, fe_server **out)
{
    if (!out)
        return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !cfg->kinds || cfg->n_kinds < 1 || cfg->n_kinds > FE_MAX_BATCH_KINDS)
        return fail(FE_ERR_INVALID_ARG, "need 1..%d kinds", FE_MAX_BATCH_KINDS);
    if (cfg->max_slots < 1 || cfg->hbm_budget_bytes < 4096 || cfg->max_chunks < 1 ||
        cfg->chunk_elems < 4 || cfg->chunk_elems % 4)
        return fail(FE_ERR_INVALID_ARG, "bad server limits");
    if (cfg->backend != FE_SERVER_GPU && cfg->backend != FE_SERVER_FAKE)
        return fail(FE_ERR_INVALID_ARG, "bad backend %d", cfg->backend);
    if (cfg->backend == FE_SERVER_FAKE &&
        (cfg->fake_ns_per_elem < 0 || cfg->fake_h2d_bytes_per_s <= 0 || cfg->fake_tick_overhead_s < 0))
        return fail(FE_ERR_INVALID_ARG, "bad fake backend timing model");
    fe_server *s = new (std::nothrow) fe_server();
    if (!s)
        return fail(FE_ERR_CAPACITY, "out of host memory");
    s->cfg = *cfg;
    s->fake = cfg->backend == FE_SERVER_FAKE;
    s->kinds.assign(cfg->kinds, cfg->kinds + cfg->n_kinds);
    for (int k = 0; k < cfg->n_kinds; ++k) {
        fe_batch_kind &bk = s->kinds[k];
        if (bk.n_q < 1 || bk.n_q > FE_MAX_QP || !bk.xi || !bk.w) {
            destroy_server(s);
            return fail(FE_ERR_INVALID_ARG, "kind %d has a bad rule", k);
        }
        s->rule_xi.emplace_back(bk.xi, bk.xi + 3 * bk.n_q);
        s->rule_w.emplace_back(bk.w, bk.w + bk.n_q);
        bk.xi = s->rule_xi.back().data();
        bk.w = s->rule_w.back().data();
        KindInfo ki;
        ki.nv = bk.elem_type == FE_TET4 ? 4 : 6;
        ki.nk = fe_k_entries(&bk.problem, (fe_elem_type)bk.elem_type);
        ki.nf = fe_f_entries(&bk.problem, (fe_elem_type)bk.elem_type);
        ki.nc = fe_coeff_entries(&bk.problem, (fe_elem_type)bk.elem_type, bk.n_q);
        ki.tsize = bk.problem.precision == FE_FP64 ? 8 : 4;
        if (ki.nk < 0 || ki.nf < 0 || ki.nc < 0) {
            destroy_server(s);
            return fail(FE_ERR_INVALID_ARG, "kind %d has an invalid problem", k);
        }
        s->kinfo.push_back(ki);
    }
    s->arena.reset(new Arena(cfg->hbm_budget_bytes));
    if (s->fake) {
        s->arena_base = std::malloc(4096);  // addresses are never dereferenced
        if (!s->arena_base) {
            destroy_server(s);
            return fail(FE_ERR_CAPACITY, "out of host memory");
        }
    } else {
        int st = FE_OK;
        hipError_t err = hipGetDevice(&s->device);
        if (err == hipSuccess)
            err = hipMalloc(&s->arena_base, (size_t)cfg->hbm_budget_bytes);
        if (err == hipSuccess)
            err = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
        if (err == hipSuccess)
            err = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
        if (err != hipSuccess) {
            destroy_server(s);
            return fail(FE_ERR_HIP, "server device setup failed: %s", hipGetErrorString(err));
        }
        st = fe_batch_create(s->kinds.data(), cfg->n_kinds, cfg->max_chunks, cfg->chunk_elems,
                             cfg->blocks_per_kind, &s->batch);
        if (st != FE_OK) {
            destroy_server(s);
            return st;
        }
    }
    s->thread = std::thread(loop, s);
    *out = s;
    return FE_OK;
}

int fe_server_submit(fe_server *s, const fe_request *req, uint64_t *id)
{
    if (!s || !req)
        return fail(FE_ERR_INVALID_ARG, "server or request is NULL");
    if (req->kind < 0 || req->kind >= s->cfg.n_kinds)
        return fail(FE_ERR_INVALID_ARG, "kind %d out of range", req->kind);
    if (req->n_elem < 1)
        return fail(FE_ERR_INVALID_ARG, "a request needs at least one element");
    const KindInfo &ki = s->kinfo[req->kind];
    if (!req->coords || (ki.nc > 0 && !req->coeffs))
        return fail(FE_ERR_INVALID_ARG, "request inputs are NULL");
    if (req->ld_in < req->n_elem)
        return fail(FE_ERR_INVALID_ARG, "ld_in must be >= n_elem");
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r)
        return fail(FE_ERR_CAPACITY, "out of host memory");
    r->kind = req->kind;
    r->n = req->n_elem;
    r->tag = req->tag;
    r->dev_inputs = req->inputs_on_device != 0;
    if (r->dev_inputs) {
        r->coords = req->coords;
        r->coeffs = req->coeffs;
        r->ld_in = req->ld_in;
    } else {
        r->h_coords = req->coords;
        r->h_coeffs = req->coeffs;
        r->ld_host = req->ld_in;
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->stats_mu);
        ++s->n_submitted;
    }
    {
        std::lock_guard<std::mutex> lk(s->io_mu);
        r->id = s->next_id++;
        if (id)
            *id = r->id;
        s->inbox.push_back(std::move(r));
    }
    s->cv_work.notify_all();
    return FE_OK;
}

int fe_server_poll(fe_server *s, fe_completion *out, int max, double timeout_s)
{
    if (!s || !out || max < 1)
        return -FE_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->io_mu);
    if (s->done_q.empty() && timeout_s > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                            [&] { return !s->done_q.empty(); });
    int n = 0;
    while (n < max && !s->done_q.empty()) {
        out[n++] = s->done_q.front();
        s->done_q.pop_front();
    }
    return n;
}

int fe_server_release(fe_server *s, uint64_t id)
{
    if (!s)
        return fail(FE_ERR_INVALID_ARG, "server is NULL");
    uint64_t seq = 0;
    {
        std::lock_guard<std::mutex> lk(s->io_mu);
        auto it = s->completed.find(id);
        if (it == s->completed.end()) {
            if (id >= 1 && id < s->next_id)
                return fail(FE_ERR_INVALID_ARG, "request %llu has not completed or was released",
                            (unsigned long long)id);
            return fail(FE_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
        }
        s->completed.erase(it);
        s->release_q.push_back(id);
        seq = ++s->release_posted;
    }
    s->cv_work.notify_all();
    // Return once the scheduler has put the memory back into the budget.
    std::unique_lock<std::mutex> lk(s->io_mu);
    s->cv_done.wait(lk, [&] { return s->release_done >= seq || s->stop; });
    return FE_OK;
}

int fe_server_stats_get(fe_server *s, fe_server_stats *out)
{
    if (!s || !out)
        return fail(FE_ERR_INVALID_ARG, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->stats_mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->n_submitted;
    out->admitted = s->n_admitted;
    out->completed = s->n_completed;
    out->failed = s->n_failed;
    out->in_queue = s->n_queue;
    out->in_flight = s->n_active;
    out->bytes_in_use = s->bytes_in_use;
    out->bytes_peak = s->bytes_peak;
    out->elements_done = s->elements_done;
    out->ticks = s->n_ticks;
    out->p50_s = percentile(s->lat, 0.50);
    out->p99_s = percentile(s->lat, 0.99);
    out->mean_s = mean(s->lat);
    out->mean_queue_s = mean(s->q_t);
    out->mean_h2d_s = mean(s->h2d_t);
    out->mean_device_s = mean(s->dev_t);
    return FE_OK;
}

int fe_server_reset_stats(fe_server *s)
{
    if (!s)
        return fail(FE_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->stats_mu);
    s->n_submitted = s->n_admitted = s->n_completed = s->n_failed = s->n_ticks = 0;
    s->elements_done = 0;
    s->lat.clear();
    s->q_t.clear();
    s->h2d_t.clear();
    s->dev_t.clear();
    return FE_OK;
}

int fe_server_destroy(fe_server *s)
{
    destroy_server(s);
    return FE_OK;
}

}  // extern "C"
