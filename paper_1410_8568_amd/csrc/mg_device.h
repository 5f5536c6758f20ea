// Device helpers shared by the kernel files of the library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace mgk {

// Map the dispatch order of workgroups onto tiles so that each XCD works on a
// contiguous range of tiles: workgroup w is dispatched to XCD w % 8, and XCD x
// receives logical tiles [start_x, start_x + count_x).  Neighbouring tiles then
// share one L2, where their halo re-reads hit.
__device__ __forceinline__ int xcd_tile(int w, int nwg) {
    const int q = nwg >> 3, r = nwg & 7, x = w & 7, m = w >> 3;
    return x * q + min(x, r) + m;
}

}  // namespace mgk
