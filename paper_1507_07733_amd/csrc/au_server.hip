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
//   au_submit     validate; if nothing waits ahead of the event and the arena
//   (caller)      has room, admit it at once: copy its traces and directions
//                 straight into its arena region (a copy stream; the call
//                 returns once the copy is done) and, with tick_s = 0, launch
//                 it (with whatever else is ready) in the same call; else
//                 copy the traces into pinned staging and queue it (FIFO)
//   scheduler     admits queued events as arena space and slots free up,
//   thread        launches micro-batches (when max_batch_events are ready or
//                 the oldest has waited tick_s); sleeps on a condition
//                 variable otherwise (no polling)
//   reaper        waits on the oldest in-flight batch's completion event,
//   thread        then collects every batch that has completed, stamps its
//                 events and wakes waiters (au_wait) and the scheduler
//   au_poll / au_wait / au_copy_result / au_release (callers)
//
// A batch of one event launches the single-event path with the event passed
// by value (no descriptors).  A batch of several takes one of 2 * n_streams
// descriptor slots (device + pinned host, allocated at creation, never part
// of the arena); with no slot free the batch shrinks to one event.  So a
// launch never needs arena or staging space beyond what its events already
// hold, and an arena filled exactly by admitted events still launches.
//
// Nothing here allocates device or pinned memory after au_server_create.
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

// Descriptor space of one multi-event batch.
constexpr size_t kSlotBytes = 2u << 20;

struct Ticket {
    uint64_t id = 0;
    int S = 0, N = 0, D = 0, k_lo = 0, nb = 0;
    size_t stage_off = 0, stage_bytes = 0;  // pinned staging (queued events): directions then traces
    size_t volt_bytes = 0, dir_bytes = 0;
    size_t dev_off = 0, dev_bytes = 0;      // arena: output, spectra, coefficients, directions, traces
    size_t o_efield = 0, o_x = 0, o_m = 0, o_dirs = 0, o_volt = 0;
    double t_arrival = 0, t_submit = 0, t_admit = 0, t_launch = 0, t_complete = 0;
    State state = QUEUED;
    bool has_dev = false;      // owns [dev_off, dev_off + dev_bytes) of the arena
    bool on_device = false;    // traces and directions are in the arena (else in staging)
    hipEvent_t copy_ev = nullptr;  // set while the direct copy may still run
    bool release_pending = false;
    int batch_events = 0;
    uint64_t batch_id = 0;
};

struct Batch {
    uint64_t id = 0;
    hipEvent_t done = nullptr;
    int stream = 0;
    int slot = -1;
    std::vector<uint64_t> ids;
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct au_server {
    const au_table* tb = nullptr;
    au_server_cfg cfg{};
    au_event ev{};  // the configuration's event fields (sizes per request)
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    unsigned char* d_arena = nullptr;
    unsigned char* h_stage = nullptr;
    unsigned char* d_slots = nullptr;
    unsigned char* h_slots = nullptr;
    uint64_t* d_counts = nullptr;
    std::vector<hipStream_t> streams;
    hipStream_t copy_stream = nullptr;
    std::vector<hipEvent_t> event_pool;

    std::mutex mu;
    std::condition_variable cv_sched;  // scheduler: queued / ready work, space freed, stop
    std::condition_variable cv_reap;   // reaper: a batch launched, stop
    std::condition_variable cv_done;   // au_wait callers: an event completed or the server failed
    std::thread scheduler, reaper;
    bool stop = false;
    au_status dead = AU_OK;
    std::string dead_msg;

    au::Arena arena, stage;
    std::vector<bool> slot_busy;
    uint64_t next_id = 1, next_batch = 1;
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

// Arena region of one event: output, then the single-event workspace
// (spectra, coefficients, directions: the layout enqueue_event expects),
// then the traces; directions and traces adjacent, as in staging.
static void layout_ticket(const au_server* sv, Ticket& t)
{
    const bool f64 = sv->cfg.prec == AU_PREC_FP64;
    const size_t tin = sv->cfg.trace_dtype == AU_F64 ? 8 : 4;
    const size_t tout = f64 ? 8 : 4;
    t.volt_bytes = (size_t)t.S * 2 * t.N * tin;
    t.dir_bytes = (size_t)t.D * 2 * sizeof(double);
    const EvParams p{t.S, t.N, t.k_lo, t.nb};
    size_t wx, wm, wd;
    workspace_layout(p, sv->cfg.prec, t.D, &wx, &wm, &wd);
    size_t o = 0;
    t.o_efield = o;
    o += align256((size_t)t.D * t.S * 2 * t.N * tout);
    t.o_x = o;
    o += wx;
    t.o_m = o;
    o += wm;
    t.o_dirs = o;
    o += wd;
    t.o_volt = o;
    o += align256(t.volt_bytes);
    t.dev_bytes = o;
    t.stage_bytes = wd + align256(t.volt_bytes);
}

static void wake_all(au_server* sv)
{
    sv->cv_sched.notify_all();
    sv->cv_reap.notify_all();
    sv->cv_done.notify_all();
}

// ---------------------------------------------------------------------------
// scheduling (every function below runs with sv->mu held)
// ---------------------------------------------------------------------------

static void fail_server(au_server* sv, au_status s, const std::string& msg)
{
    if (sv->dead == AU_OK) {
        sv->dead = s;
        sv->dead_msg = msg;
    }
    for (auto& kv : sv->tickets)
        if (kv.second.state != DONE) kv.second.state = FAILED;
    wake_all(sv);
}

static hipEvent_t take_event(au_server* sv)
{
    if (sv->event_pool.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
        return ev;
    }
    hipEvent_t ev = sv->event_pool.back();
    sv->event_pool.pop_back();
    return ev;
}

static void free_ticket_space(au_server* sv, Ticket& t)
{
    if (t.stage_bytes && !t.on_device) {
        sv->stage.release(t.stage_off, t.stage_bytes);
    }
    t.stage_bytes = 0;
    if (t.has_dev) {
        sv->arena.release(t.dev_off, t.dev_bytes);
        t.has_dev = false;
        --sv->admitted_unreleased;
    }
}

// Marks every event of a completed batch done and returns its resources.
static void finish_batch(au_server* sv, Batch& b, double tc)
{
    for (uint64_t id : b.ids) {
        auto f = sv->tickets.find(id);
        if (f == sv->tickets.end()) continue;
        Ticket& t = f->second;
        t.state = DONE;
        t.t_complete = tc;
        if (t.stage_bytes && !t.on_device) sv->stage.release(t.stage_off, t.stage_bytes);
        t.stage_bytes = 0;
        ++sv->n_completed;
        if (t.release_pending) {
            free_ticket_space(sv, t);
            sv->tickets.erase(f);
        }
    }
    if (b.slot >= 0) sv->slot_busy[b.slot] = false;
    sv->event_pool.push_back(b.done);
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

static int free_slot(const au_server* sv)
{
    for (size_t i = 0; i < sv->slot_busy.size(); ++i)
        if (!sv->slot_busy[i]) return (int)i;
    return -1;
}

// Launches one micro-batch from the head of the ready list.
static void launch_batch(au_server* sv)
{
    if (sv->ready.empty() || sv->dead != AU_OK) return;
    const bool f64 = sv->cfg.prec == AU_PREC_FP64;
    const size_t tin = sv->cfg.trace_dtype == AU_F64 ? 8 : 4;
    const size_t tout = f64 ? 8 : 4;
    const size_t xb = f64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = f64 ? sizeof(MBin<double>) : sizeof(MBin<float>);
    const int max_ev = std::max(1, sv->cfg.max_batch_events);
    const int slot = (int)sv->ready.size() > 1 && max_ev > 1 ? free_slot(sv) : -1;

    // events per trace-length class, with their descriptors (several-event batches)
    struct HostClass {
        int N;
        std::vector<EvDesc> evs;
        std::vector<int2> su, cu;
        std::vector<int4> uu;
    };
    auto class_bytes = [](const HostClass& h) {
        return align256(h.evs.size() * sizeof(EvDesc)) + align256(h.su.size() * sizeof(int2)) +
               align256(h.cu.size() * sizeof(int2)) + align256(h.uu.size() * sizeof(int4));
    };
    std::vector<HostClass> hc;
    std::vector<uint64_t> ids;
    ids.push_back(sv->ready.front());
    if (slot >= 0) {
        for (size_t qi = 0; qi < sv->ready.size() && (int)ids.size() <= max_ev; ++qi) {
            const Ticket& t = sv->tickets[sv->ready[qi]];
            std::vector<HostClass> trial = hc;
            HostClass* c = nullptr;
            for (auto& h : trial)
                if (h.N == t.N) c = &h;
            if (!c) {
                trial.push_back(HostClass{t.N, {}, {}, {}, {}});
                c = &trial.back();
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
            size_t tot = 0;
            for (auto& h : trial) tot += class_bytes(h);
            if (tot > kSlotBytes) break;  // the event waits for the next batch
            hc.swap(trial);
            if (qi > 0) ids.push_back(sv->ready[qi]);
            if ((int)ids.size() == max_ev) break;
        }
        if (ids.size() < 2) hc.clear();
    }
    const bool multi = ids.size() > 1;
    for (size_t i = 0; i < ids.size(); ++i) sv->ready.pop_front();

    const int si = sv->next_stream;
    sv->next_stream = (sv->next_stream + 1) % (int)sv->streams.size();
    hipStream_t st = sv->streams[si];
    auto hip_fail = [&](hipError_t e, const char* what) {
        fail_server(sv, AU_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipSuccess;
    // traces and directions: from staging on this stream, or after the direct copy
    for (uint64_t id : ids) {
        Ticket& t = sv->tickets[id];
        if (!t.on_device) {
            e = hipMemcpyAsync(sv->d_arena + t.dev_off + t.o_dirs, sv->h_stage + t.stage_off, t.stage_bytes,
                               hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "trace copy");
        } else if (t.copy_ev != nullptr) {
            e = hipStreamWaitEvent(st, t.copy_ev, 0);
            if (e != hipSuccess) return hip_fail(e, "copy wait");
        }
    }
    const double tl = now_s(sv->t0);
    const uint64_t bid = sv->next_batch++;
    for (uint64_t id : ids) {
        Ticket& t = sv->tickets[id];
        t.state = INFLIGHT;
        t.t_launch = tl;
        t.batch_events = (int)ids.size();
        t.batch_id = bid;
    }
    if (multi) {
        unsigned char* hs = sv->h_slots + (size_t)slot * kSlotBytes;
        unsigned char* ds = sv->d_slots + (size_t)slot * kSlotBytes;
        size_t o = 0;
        std::vector<ClassLaunch> cl;
        for (auto& h : hc) {
            auto put = [&](const void* src, size_t bytes) {
                std::memcpy(hs + o, src, bytes);
                const size_t at = o;
                o += align256(bytes);
                return ds + at;
            };
            ClassLaunch c;
            c.N = h.N;
            c.variant = current_variant(sv->cfg.prec, c.N);
            c.d_evs = (const EvDesc*)put(h.evs.data(), h.evs.size() * sizeof(EvDesc));
            c.d_sunits = (const int2*)put(h.su.data(), h.su.size() * sizeof(int2));
            c.n_sunits = (int)h.su.size();
            c.d_cunits = (const int2*)put(h.cu.data(), h.cu.size() * sizeof(int2));
            c.n_cunits = (int)h.cu.size();
            c.d_uunits = (const int4*)put(h.uu.data(), h.uu.size() * sizeof(int4));
            c.n_uunits = (int)h.uu.size();
            c.max_nb = 0;
            for (const EvDesc& d : h.evs) c.max_nb = std::max(c.max_nb, d.nb);
            cl.push_back(c);
        }
        e = hipMemcpyAsync(ds, hs, o, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "descriptor copy");
        sv->slot_busy[slot] = true;
        for (const ClassLaunch& c : cl) {
            au_status s = enqueue_class(sv->tb, sv->cfg.prec, sv->cfg.trace_dtype, sv->cfg.fs_hz,
                                        sv->cfg.fallback_rel, sv->cfg.singular_rel, c, sv->d_arena, sv->d_arena,
                                        sv->d_arena, sv->d_arena, (const double*)sv->d_arena, st, sv->d_counts,
                                        nullptr);
            if (s != AU_OK) return fail_server(sv, s, error_string());
        }
    } else {
        const Ticket& t = sv->tickets[ids[0]];
        au_event ev = sv->ev;
        ev.n_stations = t.S;
        ev.n_samples = t.N;
        const EvParams p{t.S, t.N, t.k_lo, t.nb};
        unsigned char* base = sv->d_arena + t.dev_off;
        au_status s = enqueue_event(sv->tb, &ev, p, base + t.o_volt, t.D, base + t.o_efield, base + t.o_x, st,
                                    sv->d_counts);
        if (s != AU_OK) return fail_server(sv, s, error_string());
    }
    Batch b;
    b.id = bid;
    b.done = take_event(sv);
    if (!b.done) return hip_fail(hipErrorOutOfMemory, "event create");
    e = hipEventRecord(b.done, st);
    if (e != hipSuccess) return hip_fail(e, "event record");
    b.stream = si;
    b.slot = multi ? slot : -1;
    b.ids = std::move(ids);
    sv->inflight.push_back(std::move(b));
    ++sv->n_batches;
    sv->cv_reap.notify_one();
}

// Launches batches while the head of the ready list is due.
static void launch_due(au_server* sv)
{
    while (!sv->ready.empty() && sv->dead == AU_OK) {
        const Ticket& head = sv->tickets[sv->ready.front()];
        const bool full = (int)sv->ready.size() >= std::max(1, sv->cfg.max_batch_events);
        if (!(full || now_s(sv->t0) - head.t_admit >= sv->cfg.tick_s)) break;
        launch_batch(sv);
    }
}

static void scheduler_loop(au_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        if (sv->dead == AU_OK) {
            admit(sv);
            launch_due(sv);
        }
        if (sv->stop) break;
        if (sv->dead == AU_OK && !sv->ready.empty()) {
            const double due = sv->tickets[sv->ready.front()].t_admit + sv->cfg.tick_s;
            const auto when = sv->t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                           std::chrono::duration<double>(due));
            sv->cv_sched.wait_until(lk, when);
        } else {
            sv->cv_sched.wait(lk);
        }
    }
}

static void reaper_loop(au_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        while (!sv->stop && (sv->inflight.empty() || sv->dead != AU_OK)) sv->cv_reap.wait(lk);
        if (sv->inflight.empty() || sv->dead != AU_OK) break;  // stopping with nothing left to collect
        const hipEvent_t oldest = sv->inflight.front().done;
        lk.unlock();
        const hipError_t w = hipEventSynchronize(oldest);  // the wait: no lock held
        lk.lock();
        if (w != hipSuccess) {
            fail_server(sv, AU_EDEVICE, std::string("batch failed: ") + hipGetErrorString(w));
            continue;
        }
        // collect every batch that has completed by now (batches on other streams may finish first)
        const double tc = now_s(sv->t0);
        bool any = false;
        for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
            const hipError_t q = it->done == oldest ? hipSuccess : hipEventQuery(it->done);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            if (q != hipSuccess) {
                fail_server(sv, AU_EDEVICE, std::string("batch failed: ") + hipGetErrorString(q));
                break;
            }
            finish_batch(sv, *it, tc);
            it = sv->inflight.erase(it);
            any = true;
        }
        if (any) {
            sv->cv_done.notify_all();
            sv->cv_sched.notify_one();
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
        cfg->n_streams < 1 || cfg->n_streams > 16 || cfg->max_batch_events < 1 || !(cfg->tick_s >= 0.0) ||
        !(cfg->tick_s <= 10.0))
        return set_error(AU_EINVAL, "server configuration out of range");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(AU_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != tb->device) return set_error(AU_EINVAL, "table lives on another device");
    au_server* sv = new au_server();
    sv->tb = tb;
    sv->cfg = *cfg;
    sv->ev = au_event{0, 0, cfg->fs_hz, cfg->band_lo_hz, cfg->band_hi_hz, cfg->trace_dtype, cfg->prec,
                      cfg->fallback_rel, cfg->singular_rel};
    sv->device = dev;
    sv->t0 = std::chrono::steady_clock::now();
    const int n_slots = 2 * cfg->n_streams;
    auto undo = [&](au_status st, const std::string& msg) {
        for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
        if (sv->copy_stream) (void)hipStreamDestroy(sv->copy_stream);
        if (sv->d_arena) (void)hipFree(sv->d_arena);
        if (sv->d_slots) (void)hipFree(sv->d_slots);
        if (sv->d_counts) (void)hipFree(sv->d_counts);
        if (sv->h_stage) (void)hipHostFree(sv->h_stage);
        if (sv->h_slots) (void)hipHostFree(sv->h_slots);
        delete sv;
        return set_error(st, msg);
    };
    e = hipMalloc((void**)&sv->d_arena, cfg->hbm_budget_bytes);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("arena: ") + hipGetErrorString(e));
    e = hipMalloc((void**)&sv->d_slots, (size_t)n_slots * kSlotBytes);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("descriptor slots: ") + hipGetErrorString(e));
    e = hipHostMalloc((void**)&sv->h_stage, cfg->staging_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("staging: ") + hipGetErrorString(e));
    e = hipHostMalloc((void**)&sv->h_slots, (size_t)n_slots * kSlotBytes, hipHostMallocDefault);
    if (e != hipSuccess) return undo(AU_ENOMEM, std::string("descriptor staging: ") + hipGetErrorString(e));
    e = hipMalloc((void**)&sv->d_counts, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(sv->d_counts, 0, 2 * sizeof(uint64_t));
    if (e != hipSuccess) return undo(AU_EDEVICE, std::string("counters: ") + hipGetErrorString(e));
    for (int i = 0; i <= cfg->n_streams; ++i) {
        hipStream_t x;
        e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return undo(AU_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
        if (i < cfg->n_streams)
            sv->streams.push_back(x);
        else
            sv->copy_stream = x;
    }
    sv->slot_busy.assign(n_slots, false);
    sv->arena.init(cfg->hbm_budget_bytes);
    sv->stage.init(cfg->staging_bytes);
    sv->scheduler = std::thread(scheduler_loop, sv);
    sv->reaper = std::thread(reaper_loop, sv);
    *out = sv;
    return AU_OK;
}

extern "C" au_status au_server_destroy(au_server* sv)
{
    if (!sv) return AU_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        wake_all(sv);
    }
    if (sv->scheduler.joinable()) sv->scheduler.join();
    if (sv->reaper.joinable()) sv->reaper.join();  // returns once every launched batch has completed
    for (hipStream_t x : sv->streams) (void)hipStreamSynchronize(x);
    (void)hipStreamSynchronize(sv->copy_stream);
    for (auto& b : sv->inflight) (void)hipEventDestroy(b.done);
    for (hipEvent_t ev : sv->event_pool) (void)hipEventDestroy(ev);
    for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
    (void)hipStreamDestroy(sv->copy_stream);
    (void)hipFree(sv->d_arena);
    (void)hipFree(sv->d_slots);
    (void)hipFree(sv->d_counts);
    (void)hipHostFree(sv->h_stage);
    (void)hipHostFree(sv->h_slots);
    delete sv;
    return AU_OK;
}

extern "C" au_status au_server_now(const au_server* sv, double* t)
{
    if (!sv || !t) return set_error(AU_EINVAL, "null argument");
    *t = now_s(sv->t0);
    return AU_OK;
}

extern "C" au_status au_server_request_bytes(const au_server* sv, int32_t n_stations, int32_t n_samples,
                                             int32_t n_dirs, uint64_t* dev_bytes)
{
    if (!sv || !dev_bytes) return set_error(AU_EINVAL, "null argument");
    EvParams p;
    au_status s = check_n(sv->tb, n_stations, n_samples, sv->cfg.fs_hz, sv->cfg.band_lo_hz, sv->cfg.band_hi_hz, &p);
    if (s != AU_OK) return s;
    if (n_dirs < 1) return set_error(AU_EINVAL, "n_dirs must be >= 1");
    Ticket t;
    t.S = p.S;
    t.N = p.N;
    t.D = n_dirs;
    t.k_lo = p.k_lo;
    t.nb = p.nb;
    layout_ticket(sv, t);
    *dev_bytes = t.dev_bytes;
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
    if (t.dev_bytes > sv->arena.size())
        return set_error(AU_ENOMEM, "event needs more device memory than the server's whole budget");
    t.t_submit = t_sub;
    t.t_arrival = rq->t_arrival > 0.0 ? rq->t_arrival : t_sub;
    bool direct = false;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->dead != AU_OK) return set_error(sv->dead, "server failed: " + sv->dead_msg);
        // nothing queued ahead and room now: admit at once and copy straight into the arena
        if (sv->queue.empty() && sv->admitted_unreleased < sv->cfg.max_inflight &&
            sv->arena.alloc(t.dev_bytes, &t.dev_off)) {
            direct = true;
            t.has_dev = true;
            t.on_device = true;
            t.state = ADMITTED;
            ++sv->admitted_unreleased;
            t.copy_ev = take_event(sv);
            if (!t.copy_ev) {
                sv->arena.release(t.dev_off, t.dev_bytes);
                --sv->admitted_unreleased;
                return set_error(AU_EDEVICE, "event create failed");
            }
        } else if (!sv->stage.alloc(t.stage_bytes, &t.stage_off)) {
            ++sv->n_rejected;
            return set_error(AU_EAGAIN, "staging area full; retry after earlier requests complete");
        }
        t.id = sv->next_id++;
    }
    if (direct) {
        unsigned char* base = sv->d_arena + t.dev_off;
        hipError_t e = hipMemcpyAsync(base + t.o_dirs, rq->h_dirs, t.dir_bytes, hipMemcpyHostToDevice,
                                      sv->copy_stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(base + t.o_volt, rq->h_volt, t.volt_bytes, hipMemcpyHostToDevice, sv->copy_stream);
        if (e == hipSuccess) e = hipEventRecord(t.copy_ev, sv->copy_stream);
        const hipEvent_t cev = t.copy_ev;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (e != hipSuccess) {
                fail_server(sv, AU_EDEVICE, std::string("trace copy: ") + hipGetErrorString(e));
                return set_error(AU_EDEVICE, "server failed: " + sv->dead_msg);
            }
            t.t_admit = now_s(sv->t0);
            sv->tickets[t.id] = t;
            sv->ready.push_back(t.id);
            ++sv->n_submitted;
            if (sv->cfg.tick_s <= 0.0 || (int)sv->ready.size() >= std::max(1, sv->cfg.max_batch_events))
                launch_due(sv);  // launch in this call: no hand-over to the scheduler thread
            else
                sv->cv_sched.notify_one();
        }
        // the caller may reuse its buffers once the copy has run
        e = hipEventSynchronize(cev);
        std::lock_guard<std::mutex> lk(sv->mu);
        auto f = sv->tickets.find(t.id);
        if (f != sv->tickets.end() && f->second.copy_ev == cev) f->second.copy_ev = nullptr;
        sv->event_pool.push_back(cev);
        if (e != hipSuccess) {
            fail_server(sv, AU_EDEVICE, std::string("trace copy: ") + hipGetErrorString(e));
            return set_error(AU_EDEVICE, "server failed: " + sv->dead_msg);
        }
        *ticket = t.id;
        return AU_OK;
    }
    // the staging region is private to this request until it is queued
    std::memcpy(sv->h_stage + t.stage_off, rq->h_dirs, t.dir_bytes);
    std::memcpy(sv->h_stage + t.stage_off + (t.o_volt - t.o_dirs), rq->h_volt, t.volt_bytes);
    t.state = QUEUED;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->tickets[t.id] = t;
        sv->queue.push_back(t.id);
        ++sv->n_submitted;
        sv->cv_sched.notify_one();
    }
    *ticket = t.id;
    return AU_OK;
}

static void fill_result(const au_server* sv, const Ticket& t, au_result* res)
{
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
    res->batch_id = t.batch_id;
}

extern "C" au_status au_wait(au_server* sv, uint64_t ticket, double timeout_s, au_result* res)
{
    if (!sv) return set_error(AU_EINVAL, "null server");
    if (!(timeout_s >= 0.0)) return set_error(AU_EINVAL, "timeout must be >= 0");
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                           std::chrono::duration<double>(std::min(timeout_s, 1e6)));
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        auto f = sv->tickets.find(ticket);
        if (f == sv->tickets.end() || f->second.release_pending)
            return set_error(AU_ENOTFOUND, "unknown ticket");
        const Ticket& t = f->second;
        if (t.state == FAILED) return set_error(AU_EDEVICE, "server failed: " + sv->dead_msg);
        if (t.state == DONE) {
            if (res) fill_result(sv, t, res);
            return AU_OK;
        }
        if (sv->cv_done.wait_until(lk, until) == std::cv_status::timeout) {
            auto g = sv->tickets.find(ticket);
            if (g != sv->tickets.end() && g->second.state == DONE) continue;
            return AU_EAGAIN;
        }
    }
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
    if (res) fill_result(sv, t, res);
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
        sv->cv_sched.notify_one();
    }
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
