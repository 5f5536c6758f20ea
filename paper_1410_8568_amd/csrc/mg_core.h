// Host-side runtime of the multigrid solver: workspace planning, hierarchy
// setup, V-cycle driver, FP64 iterative refinement.  Shared by the C ABI
// (mg_core.hip) and the solve server (mg_server.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mg.h"
#include "mg_launch.h"


namespace mgrt {

void set_error(const std::string& msg);

struct LevelDims {
    int nx, ny, nz;
    size_t ncell() const { return (size_t)nx * ny * nz; }
    size_t nfx() const { return (size_t)(nx + 1) * ny * nz; }
    size_t nfy() const { return (size_t)nx * (ny + 1) * nz; }
    size_t nfz() const { return (size_t)nx * ny * (nz + 1); }
    size_t nfaces() const { return nfx() + nfy() + nfz(); }
};

// Offsets (bytes from the workspace base) of every device array.
struct Layout {
    int nlev = 0;
    LevelDims d[MG_MAX_LEVELS];
    size_t bx[MG_MAX_LEVELS], by[MG_MAX_LEVELS], bz[MG_MAX_LEVELS], a[MG_MAX_LEVELS];
    size_t e[MG_MAX_LEVELS], rhs[MG_MAX_LEVELS];                  // FP64 levels >= 1 (FP64 mode)
    size_t tmp[MG_MAX_LEVELS], ftmp[MG_MAX_LEVELS];               // ping-pong buffers of the fused sweep
    size_t fbx[MG_MAX_LEVELS], fby[MG_MAX_LEVELS], fbz[MG_MAX_LEVELS], fa[MG_MAX_LEVELS];
    size_t fe[MG_MAX_LEVELS], frhs[MG_MAX_LEVELS];                // FP32 levels (refined mode)
    size_t bbar = 0, binv = 0, scal = 0, part = 0, flag = 0;
    size_t kr = 0, kz = 0, ks = 0, kq = 0;                         // Krylov vectors (level 0, FP64)
    size_t pw = 0;                                                 // the server's copy of p (0: none)
    int ncoarse = 0;
    int max_blocks = 0;
    size_t total = 0;
};

// Validates the grid/options and fills the layout.  with_p: also room for a copy
// of p (the solve server iterates on it, so that every array of a problem lies
// in its workspace).  Returns MG_OK or MG_E_INVALID.
mg_status plan(const mg_grid* g, const mg_options* o, Layout* L, bool with_p = false);

dim3 col_grid(int nx, int ny, int nz);

}  // namespace mgrt

struct mg_handle {
    mg_grid g;
    mg_options o;
    mgrt::Layout L;
    char* ws = nullptr;
    // typed device pointers
    double *bx[MG_MAX_LEVELS], *by[MG_MAX_LEVELS], *bz[MG_MAX_LEVELS], *a[MG_MAX_LEVELS];
    double *e[MG_MAX_LEVELS], *rhs[MG_MAX_LEVELS];
    float *fbx[MG_MAX_LEVELS], *fby[MG_MAX_LEVELS], *fbz[MG_MAX_LEVELS], *fa[MG_MAX_LEVELS];
    float *fe[MG_MAX_LEVELS], *frhs[MG_MAX_LEVELS];
    double* tmp[MG_MAX_LEVELS];
    float* ftmp[MG_MAX_LEVELS];
    double* bbar = nullptr;
    double* binv = nullptr;
    double* scal = nullptr;
    double* part = nullptr;
    int* flag = nullptr;
    double *kr = nullptr, *kz = nullptr, *ks = nullptr, *kq = nullptr;   // Krylov: r, z, s, q
    double* pw = nullptr;   // the workspace copy of p (server), if planned
    hipStream_t stream = nullptr;
    // batch context of the cycle launches (one problem: base == nullptr, nslots == 1)
    // and, while a graph is being built, the recording that receives them
    const uintptr_t* bt_base = nullptr;
    int bt_slots = 1;
    mgrt::Recording* rec = nullptr;
    int launch_failed = 0;   // set by a launch the batch geometry does not allow
    // no allocation anywhere (static workspace): smoother variants come from the
    // tuning cache or a fixed default instead of timed trials
    bool no_alloc = false;
    double* host = nullptr;  // pinned host copy of device scalars
    int tile[MG_MAX_LEVELS];   // smoother variant per level
    int rtile[MG_MAX_LEVELS];  // variant of the fused pre-smoothing + restriction pass (0: none)
    // profiling
    struct Rec {
        int cls;
        double bytes;
    };
    std::vector<hipEvent_t> ev;
    std::vector<Rec> recs;
    double kernel_ms[MG_K_COUNT];
    long long kernel_launches[MG_K_COUNT];
    double kernel_bytes[MG_K_COUNT];
};

namespace mgrt {
// The launcher of a handle's cycle kernels: its stream, batch context and recording.
inline Launcher launcher(mg_handle* h) {
    Launcher l;
    l.stream = h->stream;
    l.base = h->bt_base;
    l.nslots = h->bt_slots;
    l.rec = h->rec;
    l.failed = &h->launch_failed;
    return l;
}

// Bracket a kernel launch with profiling events when enabled.
struct Prof {
    mg_handle* h;
    int cls;
    double bytes;
    size_t idx;
    Prof(mg_handle* h_, int cls_, double bytes_);
    ~Prof();
};

// Setup in two halves: setup_launch enqueues the hierarchy build (and tunes
// the smoother, which synchronises, for grid sizes not tuned before) and the
// copy of the validation flags to the pinned host block; setup_finish checks
// them once h->stream has been synchronised.
mg_status setup_launch(mg_handle* h, const double* bx, const double* by, const double* bz);
mg_status setup_finish(mg_handle* h);
inline int* setup_flags(mg_handle* h) { return reinterpret_cast<int*>(h->host + 14); }
mg_status solve_impl(mg_handle* h, const double* rhs, double* p, double tol, mg_stats* st);
// The solve's level-0 passes read and write p and b with 16-byte vector accesses:
// MG_E_INVALID (with a message) unless both are 16-byte aligned.
mg_status check_solve_arrays(const double* rhs, const double* p);

// Solve as a state machine, so that a scheduler can interleave many problems.
struct SolveState {
    mg_handle* h = nullptr;
    const double* rhs = nullptr;
    double* p = nullptr;
    double tol = 0;
    mg_stats st;
    double norm_b = 0, rho0 = 0, rho = 0, scale = 1;
    int it = 0;
    int status = MG_OK;
    bool project = false;  // p still needs its final mean-zero projection
    hipGraph_t graph = nullptr;          // one iteration's launches as a graph (options.graph)
    hipGraphExec_t gexec = nullptr;
    std::shared_ptr<Recording> rec;      // the launches the graph was built from (kept with it)
    bool graph_failed = false;
    std::chrono::steady_clock::time_point t0;
};
mg_status solve_begin_launch(SolveState& S);      // asynchronous: projection + initial residual
mg_status solve_begin_finish(SolveState& S);      // after h->stream is synchronised
mg_status solve_launch_iteration(SolveState& S);  // asynchronous: one (outer) iteration
// The launches of one (outer) iteration, on the handle's launcher (direct or recorded).
mg_status launch_iteration_kernels(SolveState& S);
void solve_after_sync(SolveState& S);             // after h->stream is synchronised
bool solve_running(const SolveState& S);
void solve_end(SolveState& S, mg_stats* st);        // solve_end_launch, synchronise, solve_end_finish
void solve_end_launch(SolveState& S);                // asynchronous: the final mean-zero projection of p
void solve_end_finish(SolveState& S, mg_stats* st);  // after the stream has passed solve_end_launch
// The residual sums of the last iteration (sum r^2, sum p) of every problem of
// the handle's launcher into out[2 s], out[2 s + 1] (s: the batch slot; 0 for one
// problem); out is a device address.
void launch_gather(mg_handle* h, double* out);
// Handle arrays bound to the workspace base h->ws (which may be a stand-in base
// for a batch's offset pointers).
void bind(mg_handle* h);
void solve_release(SolveState& S);                // frees the captured graph (error paths)
}  // namespace mgrt
