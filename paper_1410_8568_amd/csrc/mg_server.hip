// Continuous-batching solve server with batched execution per grid size.
//
// Requests arrive through mg_batch_submit from any thread.  A scheduler thread
// admits them in arrival order as soon as (a) fewer than max_slots problems are
// resident and (b) their workspace fits in the free part of the caller's HBM
// arena (first fit).  Each admitted problem belongs to the size class of its
// grid.  On the class's stream it waits for the caller's producer work, builds
// its hierarchy in place (resident until it finishes), copies its initial guess
// into its workspace and forms its initial residual; then it joins the class.
//
// A class advances all of its resident problems together: one replay of the
// class's graph is one outer iteration (a V-cycle, or m FP32 V-cycles with the
// FP64 refinement step) of every problem in it, each kernel launch covering all
// of them (the grid repeated once per slot, every pointer an offset into a
// problem's workspace, made an address through a device table of per-slot
// address shifts; see mgk::Bt).  One graph is built per (class, capacity), the
// capacity being the power of two that covers the occupied slots; empty slots
// cost one early-exiting workgroup per launch block.  After a replay the
// scheduler reads every member's residual, finishes the converged ones (final
// projection, copy of p back to the caller) and frees their slots, which
// waiting problems take at the next replay.  Classes run on different streams
// and overlap on the device.  The same request gives the same result alone
// (mg_solve) and in any mix: the batched kernels compute exactly what the
// single-problem launches compute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mg_arena.h"
#include "mg_core.h"

using namespace mgrt;

namespace {

// Stand-in workspace base of a class's template handle: the template's arrays
// sit at this base plus their offsets, and a batched launch turns them into a
// problem's addresses by adding (its workspace - this base).  Non-zero, so no
// array of a problem is at a null offset pointer.
constexpr uintptr_t kStandInBase = (uintptr_t)1 << 20;

enum JobState { QUEUED, STARTING, RUNNING, ENDING, DONE };

struct Class;

struct Job {
    uint64_t ticket = 0;
    mg_request req;
    size_t bytes = 0, off = 0;
    mg_handle* h = nullptr;        // the problem's own handle (its workspace, real addresses)
    SolveState S;
    hipEvent_t ready = nullptr;    // recorded on the caller's stream at submit
    int res = -1;                  // resident slot: its pinned scalar block and event
    hipEvent_t ev = nullptr;       // end of the problem's own start or end work (the slot's event)
    Class* cls = nullptr;
    int slot = -1;                 // batch slot while it iterates
    JobState state = QUEUED;
    mg_result result;
};

struct GraphEntry {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    std::shared_ptr<Recording> rec;
};

struct Class {
    mg_grid g{};
    hipStream_t stream = nullptr;
    mg_handle* tmpl = nullptr;     // template handle at the stand-in base (offset pointers)
    SolveState tS;                 // its solve state (p: the offset of the workspace copy of p)
    std::vector<Job*> slots;       // max_slots entries, nullptr = free
    uintptr_t* base_dev = nullptr; // [max_slots] address shift of each slot's workspace (0: empty)
    uintptr_t* base_host = nullptr;
    double* res_dev = nullptr;     // [2 max_slots] sum r^2 and sum p of each slot after a replay
    double* res_host = nullptr;
    std::map<int, GraphEntry> graphs;   // per capacity
    hipEvent_t ev = nullptr;       // end of the replay in flight
    bool in_flight = false;
    bool table_dirty = true;       // the device table differs from base_host
    int table_cap = 0;
    std::vector<std::pair<int, Job*>> members;   // the slots of the replay in flight
    std::vector<Job*> joining;     // started problems waiting for the next replay
};

}  // namespace

struct mg_server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    mg_server_options o;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, Job*> jobs;
    int resident = 0;                        // admitted and not yet complete
    // per resident slot, allocated once (pinned allocations and their frees would
    // synchronise the device on every request): a pinned block for the problem's
    // scalars and an event
    double* host_blocks = nullptr;           // [max_slots][16]
    std::vector<hipEvent_t> res_events;
    std::vector<int> res_free;               // free resident slot indices
    std::vector<Job*> starting, ending;      // scheduler thread only
    std::map<std::array<int, 3>, Class*> classes;
    std::vector<hipStream_t> streams;        // class c runs on streams[c % streams.size()]
    bool own_streams = false;
    mgrt::Arena alloc;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    mg_server_info info{};                   // counters (under mu)
    std::chrono::steady_clock::time_point t0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void destroy_class(Class* c) {
    for (auto& kv : c->graphs) {
        if (kv.second.x) (void)hipGraphExecDestroy(kv.second.x);
        if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
    if (c->base_dev) (void)hipFree(c->base_dev);
    if (c->res_dev) (void)hipFree(c->res_dev);
    if (c->base_host) (void)hipHostFree(c->base_host);
    if (c->res_host) (void)hipHostFree(c->res_host);
    if (c->ev) (void)hipEventDestroy(c->ev);
    delete c->tmpl;
    delete c;
}

Class* class_for(mg_server* sv, const mg_grid& g) {
    const std::array<int, 3> key{g.nx, g.ny, g.nz};
    auto it = sv->classes.find(key);
    if (it != sv->classes.end()) return it->second;
    Class* c = new Class();
    c->g = g;
    c->stream = sv->streams[sv->classes.size() % sv->streams.size()];
    const size_t ns = (size_t)sv->o.max_slots;
    c->slots.assign(ns, nullptr);
    if (hipMalloc((void**)&c->base_dev, ns * sizeof(uintptr_t)) != hipSuccess ||
        hipMalloc((void**)&c->res_dev, 2 * ns * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&c->base_host, ns * sizeof(uintptr_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->res_host, 2 * ns * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        set_error("could not allocate the tables of a size class");
        destroy_class(c);
        return nullptr;
    }
    std::memset(c->base_host, 0, ns * sizeof(uintptr_t));
    sv->classes[key] = c;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->info.classes = (int)sv->classes.size();
    return c;
}

// Final bookkeeping of a request: status and time, its handle and memory freed.
// sync: wait for work still queued for it on its class stream first (failure
// paths), so that its memory is not handed out while a kernel may still use it.
void complete(mg_server* sv, Job* j, int status, bool sync) {
    if (sync && j->cls) (void)hipStreamSynchronize(j->cls->stream);
    solve_release(j->S);
    j->ev = nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    j->result.status = status;
    j->result.finish_ms = sv->now_ms();
    j->state = DONE;
    if (j->h) {
        j->h->host = nullptr;   // the slot's pinned block stays with the server
        mg_destroy(j->h);
        j->h = nullptr;
    }
    sv->alloc.release(j->off, j->bytes);
    sv->res_free.push_back(j->res);
    j->res = -1;
    sv->resident--;
    sv->info.completed++;
}

// Enqueue a problem's start on its class stream: wait for the caller's producer
// work, build the hierarchy, copy the initial guess into the workspace, the
// initial residual; record the job's event.
bool start_job(mg_server* sv, Job* j) {
    j->result.start_ms = sv->now_ms();
    Class* c = class_for(sv, j->req.grid);
    if (!c) {
        complete(sv, j, MG_E_HIP, false);
        return false;
    }
    j->cls = c;
    mg_handle* h = new mg_handle();
    h->g = j->req.grid;
    h->o = sv->o.solver;
    h->o.profile = 0;
    h->o.graph = 0;   // the problem iterates in its class's graph, never in one of its own
    plan(&h->g, &h->o, &h->L, true);
    h->ws = sv->arena + j->off;
    h->stream = c->stream;
    h->host = sv->host_blocks + 16 * (size_t)j->res;
    j->h = h;
    j->ev = sv->res_events[j->res];
    if (hipStreamWaitEvent(c->stream, j->ready, 0) != hipSuccess) {
        complete(sv, j, MG_E_HIP, false);
        return false;
    }
    mg_status r = setup_launch(h, j->req.bx, j->req.by, j->req.bz);
    if (r == MG_OK && hipMemcpyAsync(h->pw, j->req.p, h->L.d[0].ncell() * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream) != hipSuccess)
        r = MG_E_HIP;
    if (r == MG_OK) {
        j->S = SolveState();
        j->S.h = h;
        j->S.rhs = j->req.rhs;
        j->S.p = h->pw;
        j->S.tol = j->req.tol;
        r = solve_begin_launch(j->S);
    }
    if (r == MG_OK && hipEventRecord(j->ev, c->stream) != hipSuccess) r = MG_E_HIP;
    if (r != MG_OK) {
        complete(sv, j, r, true);
        return false;
    }
    j->state = STARTING;
    sv->starting.push_back(j);
    return true;
}

// Enqueue a problem's end: the final mean-zero projection of its copy of p and
// the copy back to the caller's p.
void end_job(mg_server* sv, Job* j) {
    Class* c = j->cls;
    solve_end_launch(j->S);
    if (hipMemcpyAsync(j->req.p, j->h->pw, j->h->L.d[0].ncell() * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess ||
        hipEventRecord(j->ev, c->stream) != hipSuccess) {
        complete(sv, j, MG_E_HIP, true);
        return;
    }
    j->state = ENDING;
    sv->ending.push_back(j);
}

// The class's template handle, from the first problem whose start completed:
// the same plan and smoother choices (per grid size), arrays at the stand-in base.
void init_template(Class* c, const mg_handle* h) {
    if (c->tmpl) return;
    mg_handle* t = new mg_handle(*h);
    t->ws = (char*)kStandInBase;
    t->host = nullptr;
    t->ev.clear();
    t->recs.clear();
    bind(t);
    t->stream = c->stream;
    t->bt_base = c->base_dev;
    t->bt_slots = 1;
    t->rec = nullptr;
    c->tmpl = t;
    c->tS = SolveState();
    c->tS.h = t;
    c->tS.p = t->pw;
}

// The graph of one outer iteration of `cap` slots: the iteration's launches
// recorded on the template handle, then the gather of every slot's residual
// sums into the class's result table.
GraphEntry* graph_for(Class* c, int cap) {
    auto it = c->graphs.find(cap);
    if (it != c->graphs.end()) return &it->second;
    GraphEntry ge;
    ge.rec = std::make_shared<Recording>();
    mg_handle* t = c->tmpl;
    t->bt_slots = cap;
    t->rec = ge.rec.get();
    mg_status r = launch_iteration_kernels(c->tS);
    if (r == MG_OK) launch_gather(t, c->res_dev);
    t->rec = nullptr;
    t->bt_slots = 1;
    if (r != MG_OK || build_graph(*ge.rec, &ge.g, &ge.x) != hipSuccess) {
        (void)hipGetLastError();
        set_error("could not build the graph of a size class");
        return nullptr;
    }
    return &(c->graphs[cap] = ge);
}

// Every problem of the class fails (graph or runtime failure of its replay).
void fail_class(mg_server* sv, Class* c) {
    for (Job*& j : c->slots)
        if (j) {
            Job* x = j;
            j = nullptr;
            x->slot = -1;
            complete(sv, x, MG_E_HIP, true);
        }
    for (Job* j : c->joining) complete(sv, j, MG_E_HIP, true);
    c->joining.clear();
    c->members.clear();
    c->in_flight = false;
    c->table_dirty = true;
}

// One scheduler step of a class: collect the finished replay (residuals, ends),
// let waiting problems join, launch the next replay.  Returns true on progress.
bool advance_class(mg_server* sv, Class* c) {
    bool progressed = false;
    if (c->in_flight) {
        const hipError_t e = hipEventQuery(c->ev);
        if (e == hipErrorNotReady) return false;
        progressed = true;
        c->in_flight = false;
        if (e != hipSuccess) {
            fail_class(sv, c);
            return true;
        }
        for (auto& m : c->members) {
            Job* j = m.second;
            j->h->host[0] = c->res_host[2 * m.first];
            j->h->host[1] = c->res_host[2 * m.first + 1];
            solve_after_sync(j->S);
            if (!solve_running(j->S)) {
                c->slots[m.first] = nullptr;
                c->table_dirty = true;
                j->slot = -1;
                end_job(sv, j);
            }
        }
        c->members.clear();
    }
    for (Job* j : c->joining) {
        for (size_t s = 0; s < c->slots.size(); s++)
            if (!c->slots[s]) {
                c->slots[s] = j;
                j->slot = (int)s;
                c->table_dirty = true;
                break;
            }
        progressed = true;
    }
    c->joining.clear();
    int hi = 0;
    for (size_t s = 0; s < c->slots.size(); s++)
        if (c->slots[s]) hi = (int)s + 1;
    if (hi == 0) return progressed;
    int cap = 1;
    while (cap < hi) cap *= 2;
    cap = std::min(cap, sv->o.max_slots);
    if (c->table_dirty || cap != c->table_cap) {
        for (int s = 0; s < cap; s++)
            c->base_host[s] = c->slots[s] ? (uintptr_t)c->slots[s]->h->ws - kStandInBase : 0;
        if (hipMemcpyAsync(c->base_dev, c->base_host, cap * sizeof(uintptr_t), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess) {
            fail_class(sv, c);
            return true;
        }
        c->table_dirty = false;
        c->table_cap = cap;
    }
    const size_t ngraphs = c->graphs.size();
    GraphEntry* ge = graph_for(c, cap);
    if (!ge || hipGraphLaunch(ge->x, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->res_host, c->res_dev, 2 * cap * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipEventRecord(c->ev, c->stream) != hipSuccess) {
        fail_class(sv, c);
        return true;
    }
    for (int s = 0; s < cap; s++)
        if (c->slots[s]) c->members.emplace_back(s, c->slots[s]);
    c->in_flight = true;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->info.graphs += (int)(c->graphs.size() - ngraphs);
        sv->info.replays++;
        sv->info.problem_iterations += (long long)c->members.size();
        sv->info.max_batch = std::max(sv->info.max_batch, (int)c->members.size());
    }
    return true;
}

bool idle(const mg_server* sv) {
    if (!sv->starting.empty() || !sv->ending.empty()) return false;
    for (auto& kv : sv->classes)
        if (kv.second->in_flight || !kv.second->joining.empty()) return false;
    return true;
}

void scheduler(mg_server* sv) {
    for (;;) {
        // ---- admission, in arrival order
        std::vector<Job*> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->queue.empty() && idle(sv)) {
                if (sv->stop) return;
                sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
                if (sv->stop && sv->queue.empty() && idle(sv)) return;
            }
            while (!sv->queue.empty() && !sv->res_free.empty()) {
                Job* j = sv->queue.front();
                size_t off;
                if (!sv->alloc.alloc(j->bytes, &off)) break;
                sv->queue.pop_front();
                sv->resident++;
                j->res = sv->res_free.back();
                sv->res_free.pop_back();
                j->off = off;
                j->state = STARTING;
                admitted.push_back(j);
            }
        }
        bool progressed = !admitted.empty();
        for (Job* j : admitted) start_job(sv, j);
        // ---- problems whose start completed join their class
        for (size_t q = 0; q < sv->starting.size();) {
            Job* j = sv->starting[q];
            const hipError_t e = hipEventQuery(j->ev);
            if (e == hipErrorNotReady) {
                q++;
                continue;
            }
            progressed = true;
            sv->starting.erase(sv->starting.begin() + q);
            if (e != hipSuccess) {
                complete(sv, j, MG_E_HIP, true);
                continue;
            }
            mg_status r = setup_finish(j->h);
            if (r == MG_OK) r = solve_begin_finish(j->S);
            if (r != MG_OK) {
                complete(sv, j, r, true);
            } else if (!solve_running(j->S)) {
                end_job(sv, j);
            } else {
                init_template(j->cls, j->h);
                j->state = RUNNING;
                j->cls->joining.push_back(j);
            }
        }
        // ---- one step of every class
        for (auto& kv : sv->classes) progressed = advance_class(sv, kv.second) || progressed;
        // ---- problems whose end completed
        for (size_t q = 0; q < sv->ending.size();) {
            Job* j = sv->ending[q];
            const hipError_t e = hipEventQuery(j->ev);
            if (e == hipErrorNotReady) {
                q++;
                continue;
            }
            progressed = true;
            sv->ending.erase(sv->ending.begin() + q);
            if (e != hipSuccess) {
                complete(sv, j, MG_E_HIP, true);
                continue;
            }
            solve_end_finish(j->S, &j->result.stats);
            complete(sv, j, j->S.status, false);
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

mg_status mg_server_request_bytes(const mg_grid* g, const mg_options* o, size_t* bytes) {
    if (!bytes) {
        set_error("null argument");
        return MG_E_INVALID;
    }
    Layout L;
    const mg_status r = plan(g, o, &L, true);
    if (r != MG_OK) return r;
    *bytes = (L.total + 255) & ~(size_t)255;
    return MG_OK;
}

mg_status mg_server_stats(mg_server* sv, mg_server_info* out) {
    if (!sv || !out) {
        set_error("null server or output");
        return MG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->info;
    out->resident = sv->resident;
    return MG_OK;
}

mg_status mg_server_create(void* arena, size_t arena_bytes, const mg_server_options* o, mg_server** out) {
    try {
        if (!arena || !o || !out || ((uintptr_t)arena & 255) || arena_bytes == 0 || o->max_slots < 1 ||
            o->max_slots > 256 || o->nstreams < 0 || o->nstreams > 256 || (o->nstreams > 0 && !o->streams)) {
            set_error("null/misaligned arena, null options/out, max_slots outside 1..256, or a bad stream list");
            return MG_E_INVALID;
        }
        for (int s = 0; s < o->nstreams; s++)
            if (!o->streams[s]) {
                set_error("null stream in the server's stream list");
                return MG_E_INVALID;
            }
        mg_grid probe{8, 8, 8};
        Layout L;
        mg_status r = plan(&probe, &o->solver, &L, true);
        if (r != MG_OK) return r;
        mg_server* sv = new mg_server();
        sv->arena = (char*)arena;
        sv->arena_bytes = arena_bytes;
        sv->o = *o;
        sv->o.streams = nullptr;   // the list is copied below; the caller's array need not outlive the call
        sv->alloc.reset(arena_bytes & ~(size_t)255);
        sv->t0 = std::chrono::steady_clock::now();
        if (o->nstreams > 0) {
            for (int s = 0; s < o->nstreams; s++) sv->streams.push_back((hipStream_t)o->streams[s]);
        } else {
            sv->own_streams = true;
            for (int s = 0; s < o->max_slots; s++) {
                hipStream_t st;
                if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                    set_error("stream creation failed");
                    for (auto x : sv->streams) (void)hipStreamDestroy(x);
                    delete sv;
                    return MG_E_HIP;
                }
                sv->streams.push_back(st);
            }
        }
        if (hipHostMalloc((void**)&sv->host_blocks, (size_t)o->max_slots * 16 * sizeof(double),
                          hipHostMallocDefault) != hipSuccess) {
            sv->host_blocks = nullptr;
            set_error("pinned host allocation failed");
            mg_server_destroy(sv);
            return MG_E_HIP;
        }
        for (int q = 0; q < o->max_slots; q++) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                set_error("event creation failed");
                mg_server_destroy(sv);
                return MG_E_HIP;
            }
            sv->res_events.push_back(ev);
            sv->res_free.push_back(o->max_slots - 1 - q);
        }
        sv->th = std::thread(scheduler, sv);
        *out = sv;
        return MG_OK;
    } catch (...) {
        set_error("host exception in mg_server_create");
        return MG_E_HIP;
    }
}

mg_status mg_batch_submit(mg_server* sv, const mg_request* r, uint64_t* ticket) {
    try {
        if (!sv || !r || !ticket || !r->bx || !r->by || !r->bz || !r->rhs || !r->p || !(r->tol >= 0)) {
            set_error("null server/request/array or bad tolerance");
            return MG_E_INVALID;
        }
        if (check_solve_arrays(r->rhs, r->p) != MG_OK) return MG_E_INVALID;
        Layout L;
        mg_status st = plan(&r->grid, &sv->o.solver, &L, true);
        if (st != MG_OK) return st;
        size_t bytes = (L.total + 255) & ~(size_t)255;
        if (bytes > (sv->arena_bytes & ~(size_t)255)) {
            set_error("request workspace " + std::to_string(bytes) + " B exceeds the arena");
            return MG_E_BUDGET;
        }
        Job* j = new Job();
        j->req = *r;
        j->bytes = bytes;
        memset(&j->result, 0, sizeof j->result);
        if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(j->ready, (hipStream_t)r->stream) != hipSuccess) {
            if (j->ready) (void)hipEventDestroy(j->ready);
            delete j;
            set_error("could not record the request's ready event on its stream");
            return MG_E_HIP;
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->stop) {
                (void)hipEventDestroy(j->ready);
                delete j;
                set_error("server is shutting down");
                return MG_E_INVALID;
            }
            j->ticket = sv->next_ticket++;
            j->result.submit_ms = sv->now_ms();
            sv->jobs[j->ticket] = j;
            sv->queue.push_back(j);
        }
        sv->cv.notify_one();
        *ticket = j->ticket;
        return MG_OK;
    } catch (...) {
        set_error("host exception in mg_batch_submit");
        return MG_E_HIP;
    }
}

mg_status mg_poll(mg_server* sv, uint64_t ticket, mg_result* out) {
    if (!sv) {
        set_error("null server");
        return MG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) {
        set_error("unknown ticket");
        return MG_E_NOT_FOUND;
    }
    Job* j = it->second;
    if (j->state != DONE) return MG_PENDING;
    if (out) *out = j->result;
    mg_status s = (mg_status)j->result.status;
    sv->jobs.erase(it);
    if (j->ready) (void)hipEventDestroy(j->ready);
    delete j;
    return s;
}

void mg_server_destroy(mg_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->th.joinable()) sv->th.join();
    for (auto& kv : sv->jobs) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    for (auto& kv : sv->classes) destroy_class(kv.second);
    for (auto e : sv->res_events) (void)hipEventDestroy(e);
    if (sv->host_blocks) (void)hipHostFree(sv->host_blocks);
    if (sv->own_streams)
        for (auto x : sv->streams) (void)hipStreamDestroy(x);
    delete sv;
}

}  // extern "C"
