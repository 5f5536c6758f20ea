// Launching the cycle kernels: directly on a stream, or recorded as the nodes
// of an explicitly built HIP graph (no stream capture, so a graph can be built
// while other threads synchronise the device), for one problem or for a batch
// of same-size problems (the grid repeated once per slot, pointers made
// per-problem through a device table of address shifts; see mgk::Bt).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <tuple>
#include <utility>
#include <vector>

#include "mg_device.h"

namespace mgrt {

// One recorded launch: the kernel, its geometry and a copy of its arguments.
struct KNode {
    const void* func;
    dim3 grid, block;
    std::shared_ptr<void> args;   // the argument tuple
    std::vector<void*> ptrs;      // addresses of the tuple's elements
};

struct Recording {
    std::vector<KNode> nodes;
};

namespace detail {
template <class Tup, size_t... I>
void fill_ptrs(Tup& t, void** out, std::index_sequence<I...>) {
    ((out[I] = (void*)&std::get<I>(t)), ...);
}
}  // namespace detail

// Every kernel launched through a Launcher takes an mgk::Bt as its last
// parameter, which the launcher supplies.  A failed launch leaves its error in
// the thread's last-error state (checked with hipGetLastError by the callers).
struct Launcher {
    hipStream_t stream = nullptr;
    const uintptr_t* base = nullptr;   // device table of per-slot address shifts (batch), else nullptr
    int nslots = 1;                    // problems per launch (batch capacity)
    Recording* rec = nullptr;          // record instead of launching

    // 1-D grid of nblk workgroups per problem (the slot is the x block index / nblk).
    template <class... P, class... A>
    void x(void (*k)(P...), unsigned nblk, unsigned nthr, A&&... a) const {
        go(k, dim3(nblk * (unsigned)nslots), dim3(nthr), nblk, std::forward<A>(a)...);
    }
    // Column grid g of blocks b per problem (the slot is the z block index / g.z).
    // A batch whose z extent would pass kMaxGridZ is neither launched nor recorded:
    // *failed is set instead (the caller turns it into an error).
    static constexpr unsigned long long kMaxGridZ = 65535;
    int* failed = nullptr;
    template <class... P, class... A>
    void z(void (*k)(P...), dim3 g, dim3 b, A&&... a) const {
        const unsigned per = g.z;
        if ((unsigned long long)per * (unsigned long long)nslots > kMaxGridZ) {
            if (failed) *failed = 1;
            return;
        }
        g.z *= (unsigned)nslots;
        go(k, g, b, per, std::forward<A>(a)...);
    }

   private:
    template <class... P, class... A>
    void go(void (*k)(P...), dim3 g, dim3 b, unsigned per, A&&... a) const {
        using Tup = std::tuple<std::decay_t<P>...>;
        const mgk::Bt bt{base, (int)per};
        if (rec) {
            auto t = std::make_shared<Tup>(std::forward<A>(a)..., bt);
            KNode n{(const void*)k, g, b, t, std::vector<void*>(sizeof...(P))};
            detail::fill_ptrs(*t, n.ptrs.data(), std::index_sequence_for<P...>{});
            rec->nodes.push_back(std::move(n));
            return;
        }
        Tup t(std::forward<A>(a)..., bt);   // no heap use on the direct path
        void* ptrs[sizeof...(P)];
        detail::fill_ptrs(t, ptrs, std::index_sequence_for<P...>{});
        (void)hipLaunchKernel((const void*)k, g, b, ptrs, 0, stream);
    }
};

// A linear chain of the recorded kernels as an instantiated graph.  On failure
// nothing is left allocated.
inline hipError_t build_graph(const Recording& r, hipGraph_t* graph, hipGraphExec_t* exec) {
    *graph = nullptr;
    *exec = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    for (const KNode& n : r.nodes) {
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(n.func);
        p.gridDim = n.grid;
        p.blockDim = n.block;
        p.sharedMemBytes = 0;
        p.kernelParams = const_cast<void**>(n.ptrs.data());
        p.extra = nullptr;
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return e;
        }
        prev = node;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    *graph = g;
    *exec = x;
    return hipSuccess;
}

}  // namespace mgrt
