// Device helpers shared by the kernel files of the library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mgk {

// Map the dispatch order of workgroups onto tiles so that each XCD works on a
// contiguous range of tiles: workgroup w is dispatched to XCD w % 8, and XCD x
// receives logical tiles [start_x, start_x + count_x).  Neighbouring tiles then
// share one L2, where their halo re-reads hit.
__device__ __forceinline__ int xcd_tile(int w, int nwg) {
    const int q = nwg >> 3, r = nwg & 7, x = w & 7, m = w >> 3;
    return x * q + min(x, r) + m;
}

// Launch context of the cycle kernels.  One problem: base == nullptr, every
// pointer argument is a device address and the grid is the problem's own.  A
// batch of problems of one grid size (same workspace layout): the grid is the
// problem's grid repeated once per slot along x (or along z for the column-grid
// kernels), slot s = block index / per, and every pointer argument is an offset
// that becomes an address by adding base[s]; base[s] == 0 marks an empty slot,
// whose blocks return at once.  The shift is applied to non-null pointers only,
// so no array of a batched problem may sit at the zero offset.
struct Bt {
    const uintptr_t* base;
    int per;
};

// The shift is applied as byte-pointer arithmetic (not through an integer), so
// the result keeps the parameter's provenance and no-alias information.
template <class P>
__device__ __forceinline__ P* rb(P* p, uintptr_t off) {
    using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return p ? reinterpret_cast<P*>(reinterpret_cast<C*>(p) + off) : p;
}

// Block index and count within the problem along the slot dimension (x of a
// 1-D grid, z of a column grid) and the problem's address shift; false for an
// empty slot (the whole block returns, before any barrier).
__device__ __forceinline__ bool bt_enter(const Bt& bt, unsigned blk, unsigned nblk, int& bid, int& nb,
                                         uintptr_t& off) {
    if (!bt.base) {
        bid = (int)blk;
        nb = (int)nblk;
        off = 0;
        return true;
    }
    const int slot = (int)blk / bt.per;
    bid = (int)blk - slot * bt.per;
    nb = bt.per;
    off = bt.base[slot];
    return off != 0;
}

}  // namespace mgk
