// Setup and solve of one problem with no allocation: the workspace is a
// file-scope device array of fixed size (one per GPU, held until the process
// ends), for callers that cannot allocate device memory.  It runs the same
// kernels as mg_setup + mg_solve, launched directly (no graph), with the host
// copies of the solve's scalars in a stack buffer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "mg_core.h"

using namespace mgrt;

namespace {

// The static workspace.  In host code this name is a stand-in, not a device
// address: only the address that hipGetSymbolAddress returns for the current
// device is ever passed to kernels or runtime calls.
__device__ __align__(256) unsigned char scratch[MG_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch`, looked up once per device
// with that device current.
mg_status scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return MG_E_HIP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return MG_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_solve_static(const mg_grid* g, const mg_options* o, const double* bx, const double* by,
                          const double* bz, mg_bc bc, const double* rhs, double* p, double tol, mg_stats* st,
                          void* stream) {
    try {
        if (!g || !o || !bx || !by || !bz || !rhs || !p || !(tol >= 0) || !std::isfinite(tol)) {
            set_error("null argument or invalid tolerance");
            return MG_E_INVALID;
        }
        if (bc != MG_BC_NEUMANN) {
            set_error("only MG_BC_NEUMANN is supported");
            return MG_E_INVALID;
        }
        if (check_solve_arrays(rhs, p) != MG_OK) return MG_E_INVALID;
        mg_handle h;   // on the stack: nothing of it outlives the call
        h.g = *g;
        h.o = *o;
        h.o.profile = 0;   // profiling creates events
        h.o.graph = 0;     // a graph is an allocation
        mg_status r = plan(g, &h.o, &h.L);
        if (r != MG_OK) return r;
        if (h.L.total > (size_t)MG_STATIC_WORKSPACE_BYTES) {
            set_error("grid needs " + std::to_string(h.L.total) + " bytes of workspace, more than the " +
                      std::to_string((size_t)MG_STATIC_WORKSPACE_BYTES) + " of the static workspace");
            return MG_E_WORKSPACE;
        }
        void* ws = nullptr;
        r = scratch_ptr(&ws);
        if (r != MG_OK) return r;
        double host[16];
        std::memset(host, 0, sizeof host);
        h.ws = (char*)ws;
        h.stream = (hipStream_t)stream;
        h.host = host;
        h.no_alloc = true;
        r = setup_launch(&h, bx, by, bz);
        if (r == MG_OK && hipStreamSynchronize(h.stream) != hipSuccess) {
            set_error("hipStreamSynchronize failed during the setup");
            r = MG_E_HIP;
        }
        if (r == MG_OK) r = setup_finish(&h);
        if (r == MG_OK) r = solve_impl(&h, rhs, p, tol, st);
        h.host = nullptr;
        return r;
    } catch (...) {
        set_error("host exception in mg_solve_static");
        return MG_E_HIP;
    }
}

}  // extern "C"
