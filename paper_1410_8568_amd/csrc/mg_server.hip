// Continuous-batching solve server.
//
// Requests arrive through mg_batch_submit from any thread.  A scheduler thread
// admits them in arrival order as soon as (a) a slot is free and (b) their
// workspace fits in the free part of the caller's HBM arena (first-fit),
// enqueues the build of their hierarchy in place (it stays resident until the
// request finishes) and the initial residual, and then advances every resident
// problem one outer iteration at a time.  The scheduler never blocks on a
// problem's stream (only smoother tuning, on the first problem of a new grid
// size, synchronises).  Each
// slot has its own HIP stream, so iterations of different problems overlap on
// the device; a problem whose iteration has completed is tested for
// convergence and relaunched immediately, without waiting for the others, and
// a finished problem frees its slot and memory for the next waiting request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mg_arena.h"
#include "mg_core.h"

using namespace mgrt;

namespace {

enum JobState { QUEUED, RUNNING, DONE };

struct Job {
    uint64_t ticket = 0;
    mg_request req;
    size_t bytes = 0, off = 0;
    int slot = -1;
    mg_handle* h = nullptr;
    SolveState S;
    hipEvent_t ev = nullptr;
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit
    bool begin_pending = false;   // setup and the initial residual are in flight
    JobState state = QUEUED;
    mg_result result;
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
    std::vector<Job*> active;
    std::vector<hipStream_t> streams;   // slot s runs on streams[s % streams.size()]
    bool own_streams = false;
    std::vector<int> slot_free;
    std::vector<hipEvent_t> events;
    mgrt::Arena alloc;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::chrono::steady_clock::time_point t0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

hipStream_t slot_stream(const mg_server* sv, int slot) { return sv->streams[(size_t)slot % sv->streams.size()]; }

void complete(mg_server* sv, Job* j, int status) {
    // work already queued for this job (setup, tuning, a partly launched
    // iteration on a failure path) must end before its memory is handed out again
    if (j->slot >= 0) (void)hipStreamSynchronize(slot_stream(sv, j->slot));
    solve_release(j->S);
    std::lock_guard<std::mutex> lk(sv->mu);
    j->result.status = status;
    j->result.finish_ms = sv->now_ms();
    j->state = DONE;
    if (j->h) {
        mg_destroy(j->h);
        j->h = nullptr;
    }
    if (j->slot >= 0) {
        sv->slot_free[j->slot] = 1;
        j->slot = -1;
    }
    sv->alloc.release(j->off, j->bytes);
}

// Enqueue the hierarchy build and the initial residual of an admitted job
// (scheduler thread) and record the slot's event after them; the scheduler
// finishes the start once the event has completed.  Returns true if the job is
// in flight.
bool start_job(mg_server* sv, Job* j) {
    j->result.start_ms = sv->now_ms();
    mg_handle* h = new mg_handle();
    h->g = j->req.grid;
    h->o = sv->o.solver;
    h->o.profile = 0;
    h->o.graph = 1;
    plan(&h->g, &h->o, &h->L);
    h->ws = sv->arena + j->off;
    h->stream = slot_stream(sv, j->slot);
    // nothing of this request is read before the caller's producer work
    if (hipStreamWaitEvent(h->stream, j->ready, 0) != hipSuccess) {
        delete h;
        complete(sv, j, MG_E_HIP);
        return false;
    }
    if (hipHostMalloc((void**)&h->host, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        h->host = nullptr;
        delete h;
        complete(sv, j, MG_E_HIP);
        return false;
    }
    j->h = h;
    mg_status r = setup_launch(h, j->req.bx, j->req.by, j->req.bz);
    if (r != MG_OK) {
        complete(sv, j, r);
        return false;
    }
    j->S = SolveState();
    j->S.h = h;
    j->S.rhs = j->req.rhs;
    j->S.p = j->req.p;
    j->S.tol = j->req.tol;
    r = solve_begin_launch(j->S);
    j->ev = sv->events[j->slot];
    if (r != MG_OK || hipEventRecord(j->ev, h->stream) != hipSuccess) {
        complete(sv, j, r != MG_OK ? r : MG_E_HIP);
        return false;
    }
    j->begin_pending = true;
    return true;
}

bool launch(mg_server* sv, Job* j) {
    if (solve_launch_iteration(j->S) != MG_OK) return false;
    j->ev = sv->events[j->slot];
    return hipEventRecord(j->ev, j->h->stream) == hipSuccess;
}

void scheduler(mg_server* sv) {
    for (;;) {
        // ---- admission, in arrival order
        std::vector<Job*> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty() && sv->queue.empty()) {
                if (sv->stop) return;
                sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
                if (sv->stop && sv->queue.empty()) return;
            }
            while (!sv->queue.empty()) {
                Job* j = sv->queue.front();
                int slot = -1;
                for (size_t s = 0; s < sv->slot_free.size(); s++)
                    if (sv->slot_free[s]) {
                        slot = (int)s;
                        break;
                    }
                if (slot < 0) break;
                size_t off;
                if (!sv->alloc.alloc(j->bytes, &off)) break;
                sv->queue.pop_front();
                sv->slot_free[slot] = 0;
                j->slot = slot;
                j->off = off;
                j->state = RUNNING;
                admitted.push_back(j);
            }
        }
        for (Job* j : admitted)
            if (start_job(sv, j)) sv->active.push_back(j);
        // ---- advance every resident problem whose iteration has finished
        bool progressed = !admitted.empty();
        for (size_t q = 0; q < sv->active.size();) {
            Job* j = sv->active[q];
            hipError_t e = hipEventQuery(j->ev);
            if (e == hipErrorNotReady) {
                q++;
                continue;
            }
            progressed = true;
            if (e != hipSuccess) {
                complete(sv, j, MG_E_HIP);
                sv->active.erase(sv->active.begin() + q);
                continue;
            }
            if (j->begin_pending) {
                j->begin_pending = false;
                mg_status r = setup_finish(j->h);
                if (r == MG_OK) r = solve_begin_finish(j->S);
                if (r != MG_OK) {
                    complete(sv, j, r);
                    sv->active.erase(sv->active.begin() + q);
                } else if (!solve_running(j->S)) {
                    solve_end(j->S, &j->result.stats);
                    complete(sv, j, j->S.status);
                    sv->active.erase(sv->active.begin() + q);
                } else if (!launch(sv, j)) {
                    complete(sv, j, MG_E_HIP);
                    sv->active.erase(sv->active.begin() + q);
                } else {
                    q++;
                }
                continue;
            }
            solve_after_sync(j->S);
            if (solve_running(j->S)) {
                if (!launch(sv, j)) {
                    complete(sv, j, MG_E_HIP);
                    sv->active.erase(sv->active.begin() + q);
                    continue;
                }
                q++;
            } else {
                solve_end(j->S, &j->result.stats);
                complete(sv, j, j->S.status);
                sv->active.erase(sv->active.begin() + q);
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

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
        mg_status r = plan(&probe, &o->solver, &L);
        if (r != MG_OK) return r;
        mg_server* sv = new mg_server();
        sv->arena = (char*)arena;
        sv->arena_bytes = arena_bytes;
        sv->o = *o;
        sv->alloc.reset(arena_bytes & ~(size_t)255);
        sv->t0 = std::chrono::steady_clock::now();
        auto fail = [&](const char* msg) {
            set_error(msg);
            if (sv->own_streams)
                for (auto x : sv->streams) (void)hipStreamDestroy(x);
            for (auto x : sv->events) (void)hipEventDestroy(x);
            delete sv;
            return MG_E_HIP;
        };
        if (o->nstreams > 0) {
            for (int s = 0; s < o->nstreams; s++) sv->streams.push_back((hipStream_t)o->streams[s]);
        } else {
            sv->own_streams = true;
            for (int s = 0; s < o->max_slots; s++) {
                hipStream_t st;
                if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                    return fail("stream creation failed");
                sv->streams.push_back(st);
            }
        }
        for (int s = 0; s < o->max_slots; s++) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail("event creation failed");
            sv->events.push_back(ev);
            sv->slot_free.push_back(1);
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
        mg_status st = plan(&r->grid, &sv->o.solver, &L);
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
    if (sv->own_streams)
        for (auto x : sv->streams) (void)hipStreamDestroy(x);
    for (auto x : sv->events) (void)hipEventDestroy(x);
    delete sv;
}

}  // extern "C"
