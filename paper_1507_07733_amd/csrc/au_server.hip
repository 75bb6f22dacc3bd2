// au_server.hip -- continuous-batching unfolding server (au_server_* in
// include/aeraunfold.h).
//
// The paper found its GPU port dominated by blocking host<->device copies
// around isolated calls and names keeping traces resident on the device as
// the way forward (arXiv:1507.07733, section 5).  This server keeps the
// pattern table and every admitted event's traces, work space and results
// in one device arena, and overlaps the work of events that arrive while
// others are running:
//
//   client threads  au_submit: validate, copy traces into pinned staging,
//                   append to the FIFO queue (timestamped)
//   scheduler       admit the queue head while the arena has room and a
//   thread          slot is free; gather admitted events into a micro-batch
//                   (launched when the batch is full or its oldest event has
//                   waited tick_s); enqueue copies + the three kernels on the
//                   next of n_streams streams; poll batch completion events
//   client threads  au_poll (result + timestamps once complete), au_copy_result,
//                   au_release (returns the event's arena space)
//
// The hot path allocates nothing: the arena (device) and the staging area
// (pinned host) are allocated once at au_server_create and carved up by a
// first-fit allocator on the host.
#include "au_arena.h"
#include "au_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace au;

namespace {

enum State { QUEUED, ADMITTED, INFLIGHT, DONE, FAILED };

struct Ticket {
    uint64_t id = 0;
    int S = 0, N = 0, D = 0, k_lo = 0, nb = 0;
    size_t stage_off = 0, stage_bytes = 0;  // pinned: traces then directions
    size_t volt_bytes = 0, dir_bytes = 0;
    size_t dev_off = 0, dev_bytes = 0;      // arena: traces, output, spectra, coefs, directions
    size_t o_volt = 0, o_efield = 0, o_x = 0, o_m = 0, o_dirs = 0;
    double t_arrival = 0, t_submit = 0, t_admit = 0, t_launch = 0, t_complete = 0;
    State state = QUEUED;
    bool has_dev = false;  // owns [dev_off, dev_off + dev_bytes) of the arena
    bool release_pending = false;
    int batch_events = 0;
};

struct Batch {
    hipEvent_t done = nullptr;
    int stream = 0;
    std::vector<uint64_t> ids;
    size_t desc_dev_off = 0, desc_dev_bytes = 0;
    size_t desc_stage_off = 0, desc_stage_bytes = 0;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct au_server {
    const au_table* tb = nullptr;
    au_server_cfg cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    unsigned char* d_arena = nullptr;
    unsigned char* h_stage = nullptr;
    uint64_t* d_counts = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> event_pool;

    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    au_status dead = AU_OK;
    std::string dead_msg;

    au::Arena arena, stage;
    uint64_t next_id = 1;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> queue;  // submitted, not admitted (FIFO)
    std::deque<uint64_t> ready;  // admitted, not launched
    std::deque<Batch> inflight;
    int admitted_unreleased = 0;
    int next_stream = 0;
    uint64_t n_submitted = 0, n_completed = 0, n_batches = 0, n_rejected = 0;
};

// ---------------------------------------------------------------------------
// sizes of one event's arena region
// ---------------------------------------------------------------------------

static void layout_ticket(const au_server* sv, Ticket& t)
{
    const bool f64 = sv->cfg.prec == AU_PREC_FP64;
    const size_t tin = sv->cfg.trace_dtype == AU_F64 ? 8 : 4;
    const size_t tout = f64 ? 8 : 4;
    const size_t xb = f64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = f64 ? sizeof(MBin<double>) : sizeof(MBin<float>);
    t.volt_bytes = (size_t)t.S * 2 * t.N * tin;
    t.dir_bytes = (size_t)t.D * 2 * sizeof(double);
    size_t o = 0;
    t.o_volt = o;
    o += align256(t.volt_bytes);
    t.o_efield = o;
    o += align256((size_t)t.D * t.S * 2 * t.N * tout);
    t.o_x = o;
    o += align256((size_t)t.S * t.nb * xb + 1);
    t.o_m = o;
    o += align256((size_t)t.D * t.nb * mb + 1);
    t.o_dirs = o;
    o += align256(t.dir_bytes);
    t.dev_bytes = o;
}

// ---------------------------------------------------------------------------
// scheduler (runs with sv->mu held)
// ---------------------------------------------------------------------------

static void fail_server(au_server* sv, au_status s, const std::string& msg)
{
    sv->dead = s;
    sv->dead_msg = msg;
    for (auto& kv : sv->tickets)
        if (kv.second.state != DONE) kv.second.state = FAILED;
}

static void free_ticket_space(au_server* sv, Ticket& t)
{
    if (t.stage_bytes) {
        sv->stage.release(t.stage_off, t.stage_bytes);
        t.stage_bytes = 0;
    }
    if (t.has_dev) {
        sv->arena.release(t.dev_off, t.dev_bytes);
        t.has_dev = false;
        --sv->admitted_unreleased;
    }
}

static void poll_completions(au_server* sv)
{
    while (!sv->inflight.empty()) {
        // batches complete in launch order per stream; check them all
        bool progressed = false;
        for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
            const hipError_t q = hipEventQuery(it->done);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            if (q != hipSuccess) {
                fail_server(sv, AU_EDEVICE, std::string("batch failed: ") + hipGetErrorString(q));
                return;
            }
            const double tc = now_s(sv->t0);
            for (uint64_t id : it->ids) {
                auto f = sv->tickets.find(id);
                if (f == sv->tickets.end()) continue;
                Ticket& t = f->second;
                t.state = DONE;
                t.t_complete = tc;
                sv->stage.release(t.stage_off, t.stage_bytes);
                t.stage_bytes = 0;
                ++sv->n_completed;
                if (t.release_pending) {
                    free_ticket_space(sv, t);
                    sv->tickets.erase(f);
                }
            }
            sv->arena.release(it->desc_dev_off, it->desc_dev_bytes);
            sv->stage.release(it->desc_stage_off, it->desc_stage_bytes);
            sv->event_pool.push_back(it->done);
            it = sv->inflight.erase(it);
            progressed = true;
        }
        if (!progressed) break;
    }
}

static void admit(au_server* sv)
{
    const double ta = now_s(sv->t0);
    while (!sv->queue.empty() && sv->admitted_unreleased < sv->cfg.max_inflight) {
        Ticket& t = sv->tickets[sv->queue.front()];
        size_t off = 0;
        if (!sv->arena.alloc(t.dev_bytes, &off)) break;  // FIFO: wait for memory
        t.dev_off = off;
        t.has_dev = true;
        t.state = ADMITTED;
        t.t_admit = ta;
        ++sv->admitted_unreleased;
        sv->ready.push_back(t.id);
        sv->queue.pop_front();
    }
}

template <typename T>
static size_t xbin_size() { return sizeof(XBin<T>); }

static void launch_batch(au_server* sv)
{
    const int max_ev = std::max(1, sv->cfg.max_batch_events);
    std::vector<uint64_t> ids;
    while (!sv->ready.empty() && (int)ids.size() < max_ev) {
        ids.push_back(sv->ready.front());
        sv->ready.pop_front();
    }
    if (ids.empty()) return;
    const bool f64 = sv->cfg.prec == AU_PREC_FP64;
    const size_t tin = sv->cfg.trace_dtype == AU_F64 ? 8 : 4;
    const size_t tout = f64 ? 8 : 4;
    const size_t xb = f64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = f64 ? sizeof(MBin<double>) : sizeof(MBin<float>);

    // descriptors per trace-length class
    struct HostClass {
        int N;
        std::vector<EvDesc> evs;
        std::vector<int2> su, cu;
        std::vector<int4> uu;
    };
    std::vector<HostClass> hc;
    for (uint64_t id : ids) {
        Ticket& t = sv->tickets[id];
        HostClass* c = nullptr;
        for (auto& h : hc)
            if (h.N == t.N) c = &h;
        if (!c) {
            hc.push_back(HostClass{t.N, {}, {}, {}, {}});
            c = &hc.back();
        }
        const int ci = (int)c->evs.size();
        EvDesc d{};
        const size_t base = t.dev_off;
        d.volt_off = (int64_t)((base + t.o_volt) / tin);
        d.efield_off = (int64_t)((base + t.o_efield) / tout);
        d.x_off = (int64_t)((base + t.o_x) / xb);
        d.m_off = (int64_t)((base + t.o_m) / mb);
        d.dir_off = (int64_t)((base + t.o_dirs) / (2 * sizeof(double)));
        d.S = t.S;
        d.N = t.N;
        d.D = t.D;
        d.k_lo = t.k_lo;
        d.nb = t.nb;
        c->evs.push_back(d);
        for (int s = 0; s < t.S; ++s) c->su.push_back(int2{ci, s});
        for (int dd = 0; dd < t.D; ++dd) {
            c->cu.push_back(int2{ci, dd});
            for (int s0 = 0; s0 < t.S; s0 += kStationsPerUnit)
                c->uu.push_back(int4{ci, dd, s0, std::min(t.S, s0 + kStationsPerUnit)});
        }
    }
    size_t desc_bytes = 0;
    std::vector<size_t> co;
    for (auto& h : hc) {
        co.push_back(desc_bytes);
        desc_bytes += align256(h.evs.size() * sizeof(EvDesc)) + align256(h.su.size() * sizeof(int2)) +
                      align256(h.cu.size() * sizeof(int2)) + align256(h.uu.size() * sizeof(int4));
    }
    Batch b;
    b.desc_dev_bytes = b.desc_stage_bytes = desc_bytes;
    if (!sv->arena.alloc(desc_bytes, &b.desc_dev_off)) {
        for (auto it = ids.rbegin(); it != ids.rend(); ++it) sv->ready.push_front(*it);
        return;  // retry once batches complete and release space
    }
    if (!sv->stage.alloc(desc_bytes, &b.desc_stage_off)) {
        sv->arena.release(b.desc_dev_off, desc_bytes);
        for (auto it = ids.rbegin(); it != ids.rend(); ++it) sv->ready.push_front(*it);
        return;
    }
    unsigned char* hs = sv->h_stage + b.desc_stage_off;
    unsigned char* ds = sv->d_arena + b.desc_dev_off;
    std::vector<ClassLaunch> cl;
    for (size_t i = 0; i < hc.size(); ++i) {
        size_t o = co[i];
        auto put = [&](const void* src, size_t bytes) {
            std::memcpy(hs + o, src, bytes);
            const size_t at = o;
            o += align256(bytes);
            return ds + at;
        };
        ClassLaunch c;
        c.N = hc[i].N;
        c.variant = current_variant(sv->cfg.prec, c.N);
        c.d_evs = (const EvDesc*)put(hc[i].evs.data(), hc[i].evs.size() * sizeof(EvDesc));
        c.d_sunits = (const int2*)put(hc[i].su.data(), hc[i].su.size() * sizeof(int2));
        c.n_sunits = (int)hc[i].su.size();
        c.d_cunits = (const int2*)put(hc[i].cu.data(), hc[i].cu.size() * sizeof(int2));
        c.n_cunits = (int)hc[i].cu.size();
        c.d_uunits = (const int4*)put(hc[i].uu.data(), hc[i].uu.size() * sizeof(int4));
        c.n_uunits = (int)hc[i].uu.size();
        c.max_nb = 0;
        for (const EvDesc& d : hc[i].evs) c.max_nb = std::max(c.max_nb, d.nb);
        cl.push_back(c);
    }
    const int si = sv->next_stream;
    sv->next_stream = (sv->next_stream + 1) % (int)sv->streams.size();
    hipStream_t st = sv->streams[si];
    auto hip_fail = [&](hipError_t e, const char* what) {
        fail_server(sv, AU_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipMemcpyAsync(ds, hs, desc_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor copy");
    const double tl = now_s(sv->t0);
    for (uint64_t id : ids) {
        Ticket& t = sv->tickets[id];
        e = hipMemcpyAsync(sv->d_arena + t.dev_off + t.o_volt, sv->h_stage + t.stage_off, t.volt_bytes,
                           hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sv->d_arena + t.dev_off + t.o_dirs, sv->h_stage + t.stage_off + align256(t.volt_bytes),
                               t.dir_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "trace copy");
        t.state = INFLIGHT;
        t.t_launch = tl;
        t.batch_events = (int)ids.size();
    }
    for (const ClassLaunch& c : cl) {
        au_status s = enqueue_class(sv->tb, sv->cfg.prec, sv->cfg.trace_dtype, sv->cfg.fs_hz, sv->cfg.fallback_rel,
                                    sv->cfg.singular_rel, c, sv->d_arena, sv->d_arena, sv->d_arena, sv->d_arena,
                                    (const double*)sv->d_arena, st, sv->d_counts, nullptr);
        if (s != AU_OK) return fail_server(sv, s, error_string());
    }
    if (sv->event_pool.empty()) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "event create");
        sv->event_pool.push_back(ev);
    }
    b.done = sv->event_pool.back();
    sv->event_pool.pop_back();
    e = hipEventRecord(b.done, st);
    if (e != hipSuccess) return hip_fail(e, "event record");
    b.stream = si;
    b.ids = std::move(ids);
    sv->inflight.push_back(std::move(b));
    ++sv->n_batches;
}

static void scheduler(au_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        if (sv->dead == AU_OK) {
            poll_completions(sv);
            admit(sv);
            if (!sv->ready.empty()) {
                const Ticket& head = sv->tickets[sv->ready.front()];
                const bool full = (int)sv->ready.size() >= std::max(1, sv->cfg.max_batch_events);
                if (full || now_s(sv->t0) - head.t_admit >= sv->cfg.tick_s) launch_batch(sv);
            }
        }
        const bool busy = !sv->inflight.empty() || !sv->ready.empty();
        if (busy) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            sv->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" au_status au_server_create(const au_table* tb, const au_server_cfg* cfg, au_server** out)
{
    if (!tb || !cfg || !out) return set_error(AU_EINVAL, "null argument");
    au_status s = check_common(tb, cfg->fs_hz, cfg->band_lo_hz, cfg->band_hi_hz, cfg->prec, cfg->trace_dtype,
                               cfg->fallback_rel, cfg->singular_rel);
    if (s != AU_OK) return s;
    if (cfg->hbm_budget_bytes < 4096 || cfg->staging_bytes < 4096 || cfg->max_inflight < 1 ||
        cfg->n_streams < 1 || cfg->n_streams > 16 || cfg->max_batch_events < 1 || !(cfg->tick_s >= 0.0))
        return set_error(AU_EINVAL, "server configuration out of range");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(AU_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != tb->device) return set_error(AU_EINVAL, "table lives on another device");
    au_server* sv = new au_server();
    sv->tb = tb;
    sv->cfg = *cfg;
    sv->device = dev;
    sv->t0 = std::chrono::steady_clock::now();
    auto undo = [&](au_status st, const std::string& msg) {
        for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
        if (sv->d_arena) (void)hipFree(sv->d_arena);
        if (sv->d_counts) (void)hipFree(sv->d_counts);
        if (sv->h_stage) (void)hipHostFree(sv->h_stage);
        delete sv;
        return set_error(st, msg);
    };
    e = hipMalloc((void**)&sv->d_arena, cfg->hbm_budget_bytes);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("arena: ") + hipGetErrorString(e));
    e = hipHostMalloc((void**)&sv->h_stage, cfg->staging_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("staging: ") + hipGetErrorString(e));
    e = hipMalloc((void**)&sv->d_counts, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(sv->d_counts, 0, 2 * sizeof(uint64_t));
    if (e != hipSuccess) return undo(AU_EDEVICE, std::string("counters: ") + hipGetErrorString(e));
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t x;
        e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return undo(AU_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
        sv->streams.push_back(x);
    }
    sv->arena.init(cfg->hbm_budget_bytes);
    sv->stage.init(cfg->staging_bytes);
    sv->worker = std::thread(scheduler, sv);
    *out = sv;
    return AU_OK;
}

extern "C" au_status au_server_destroy(au_server* sv)
{
    if (!sv) return AU_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (hipStream_t x : sv->streams) (void)hipStreamSynchronize(x);
    for (auto& b : sv->inflight) (void)hipEventDestroy(b.done);
    for (hipEvent_t ev : sv->event_pool) (void)hipEventDestroy(ev);
    for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
    (void)hipFree(sv->d_arena);
    (void)hipFree(sv->d_counts);
    (void)hipHostFree(sv->h_stage);
    delete sv;
    return AU_OK;
}

extern "C" au_status au_server_now(const au_server* sv, double* t)
{
    if (!sv || !t) return set_error(AU_EINVAL, "null argument");
    *t = now_s(sv->t0);
    return AU_OK;
}

extern "C" au_status au_submit(au_server* sv, const au_request* rq, uint64_t* ticket)
{
    if (!sv || !rq || !ticket || !rq->h_volt || !rq->h_dirs) return set_error(AU_EINVAL, "null argument");
    const double t_sub = now_s(sv->t0);
    EvParams p;
    au_status s = check_n(sv->tb, rq->n_stations, rq->n_samples, sv->cfg.fs_hz, sv->cfg.band_lo_hz,
                          sv->cfg.band_hi_hz, &p);
    if (s != AU_OK) return s;
    if (rq->n_dirs < 1) return set_error(AU_EINVAL, "n_dirs must be >= 1");
    if (!dirs_finite(rq->h_dirs, rq->n_dirs)) return set_error(AU_EINVAL, "directions must be finite");
    Ticket t;
    t.S = p.S;
    t.N = p.N;
    t.D = rq->n_dirs;
    t.k_lo = p.k_lo;
    t.nb = p.nb;
    layout_ticket(sv, t);
    if (t.dev_bytes + 1024 * 1024 > sv->arena.size())
        return set_error(AU_ENOMEM, "event needs more device memory than the server's whole budget");
    t.stage_bytes = align256(t.volt_bytes) + align256(t.dir_bytes);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->dead != AU_OK) return set_error(sv->dead, "server failed: " + sv->dead_msg);
        if (!sv->stage.alloc(t.stage_bytes, &t.stage_off)) {
            ++sv->n_rejected;
            return set_error(AU_EAGAIN, "staging area full; retry after earlier requests complete");
        }
        t.id = sv->next_id++;
    }
    // the staging region is private to this request until it is queued
    std::memcpy(sv->h_stage + t.stage_off, rq->h_volt, t.volt_bytes);
    std::memcpy(sv->h_stage + t.stage_off + align256(t.volt_bytes), rq->h_dirs, t.dir_bytes);
    t.t_submit = t_sub;
    t.t_arrival = rq->t_arrival > 0.0 ? rq->t_arrival : t_sub;
    t.state = QUEUED;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->tickets[t.id] = t;
        sv->queue.push_back(t.id);
        ++sv->n_submitted;
    }
    sv->cv.notify_all();
    *ticket = t.id;
    return AU_OK;
}

extern "C" au_status au_poll(au_server* sv, uint64_t ticket, au_result* res)
{
    if (!sv) return set_error(AU_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto f = sv->tickets.find(ticket);
    if (f == sv->tickets.end() || f->second.release_pending) return set_error(AU_ENOTFOUND, "unknown ticket");
    const Ticket& t = f->second;
    if (t.state == FAILED) return set_error(AU_EDEVICE, "server failed: " + sv->dead_msg);
    if (t.state != DONE) return AU_EAGAIN;
    if (res) {
        res->d_efield = sv->d_arena + t.dev_off + t.o_efield;
        res->efield_bytes = (uint64_t)t.D * t.S * 2 * t.N * (sv->cfg.prec == AU_PREC_FP64 ? 8 : 4);
        res->n_stations = t.S;
        res->n_samples = t.N;
        res->n_dirs = t.D;
        res->batch_events = t.batch_events;
        res->t_arrival = t.t_arrival;
        res->t_submit = t.t_submit;
        res->t_admit = t.t_admit;
        res->t_launch = t.t_launch;
        res->t_complete = t.t_complete;
    }
    return AU_OK;
}

extern "C" au_status au_copy_result(au_server* sv, uint64_t ticket, void* dst, uint64_t dst_bytes)
{
    if (!dst) return set_error(AU_EINVAL, "null destination");
    au_result r;
    au_status s = au_poll(sv, ticket, &r);
    if (s != AU_OK) return s == AU_EAGAIN ? set_error(AU_EAGAIN, "result not ready") : s;
    if (dst_bytes < r.efield_bytes) return set_error(AU_EINVAL, "destination too small");
    const hipError_t e = hipMemcpy(dst, r.d_efield, r.efield_bytes, hipMemcpyDefault);
    if (e != hipSuccess) return set_error(AU_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    return AU_OK;
}

extern "C" au_status au_release(au_server* sv, uint64_t ticket)
{
    if (!sv) return set_error(AU_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto f = sv->tickets.find(ticket);
        if (f == sv->tickets.end() || f->second.release_pending) return set_error(AU_ENOTFOUND, "unknown ticket");
        Ticket& t = f->second;
        if (t.state == INFLIGHT) {
            t.release_pending = true;  // freed when its batch completes
        } else {
            if (t.state == QUEUED) sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), ticket));
            if (t.state == ADMITTED) sv->ready.erase(std::find(sv->ready.begin(), sv->ready.end(), ticket));
            free_ticket_space(sv, t);
            sv->tickets.erase(f);
        }
    }
    sv->cv.notify_all();
    return AU_OK;
}

extern "C" au_status au_server_stats(au_server* sv, au_server_counters* st)
{
    if (!sv || !st) return set_error(AU_EINVAL, "null argument");
    uint64_t counts[2] = {0, 0};
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        st->submitted = sv->n_submitted;
        st->completed = sv->n_completed;
        st->rejected = sv->n_rejected;
        st->batches = sv->n_batches;
        st->queued = sv->queue.size();
        st->in_flight = (uint64_t)sv->admitted_unreleased;
        st->arena_bytes = sv->arena.size();
        st->arena_in_use = sv->arena.in_use();
        st->arena_peak = sv->arena.peak();
        if (sv->dead != AU_OK) return set_error(sv->dead, "server failed: " + sv->dead_msg);
    }
    const hipError_t e = hipMemcpy(counts, sv->d_counts, sizeof(counts), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(AU_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    st->fallback_bins = counts[0];
    st->singular_bins = counts[1];
    return AU_OK;
}
