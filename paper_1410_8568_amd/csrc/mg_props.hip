// Material properties from a level set, on the device (Sec. 2.2, eq. 8).
//
// The flow solver's indicator I goes from 0 to 1 across the interface over
// three to four cells; from a level set phi (positive in the liquid) it is the
// smoothed Heaviside of half-width eps:
//     I = 0 (phi <= -eps),  1 (phi >= eps),  (1/2)(1 + x + sin(pi x)/pi), x = phi/eps,
// the density is mixed linearly, rho = rho_g + (rho_l - rho_g) I (eq. 8), and the
// pressure equation's coefficient alpha = 1/rho is averaged onto each interior
// face: arithmetic mean, or the harmonic mean of eqs. (11)-(12).  Wall faces
// are 0.  This builds the solver's input from the interface description
// without a host round trip (the serving path hands the device phi in and
// gets device faces back).
//
// Streaming pass: 8 bytes of phi in and 24 bytes of faces out per cell.  Each
// thread owns two neighbouring cells of a row, evaluates alpha for them and for
// the cells below them in x, y and z, and writes the three lower faces of both
// (and the upper wall faces at the end of a row, column or the top plane).
// Arithmetic in a fixed order without fused multiply-adds:
//     x = phi/eps, I = 0.5 * ((1 + x) + sin(pi * x) / pi),
//     alpha = 1 / (rho_g + (rho_l - rho_g) * I),
//     arithmetic 0.5 * (a + b), harmonic (2 * a * b) / (a + b).
// Outside the band alpha is the value of that formula at I = 0 or 1, which each
// thread computes once (most cells then need no division).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "mg_core.h"

using mgrt::set_error;

namespace {

constexpr int PT = 512;   // threads per workgroup

struct Props {
    double rho_l, rho_g, eps;
    int harmonic;
};

__device__ __forceinline__ double alpha_of(double ind, const Props& q) {
#pragma clang fp contract(off)
    return 1.0 / (q.rho_g + (q.rho_l - q.rho_g) * ind);
}

// ag, al: alpha_of(0) and alpha_of(1), computed once per thread, so only the
// cells inside the band pay for a division.
__device__ __forceinline__ double cell_alpha(double phi, const Props& q, double ag, double al) {
#pragma clang fp contract(off)
    if (phi <= -q.eps) return ag;
    if (phi >= q.eps) return al;
    const double x = phi / q.eps;
    return alpha_of(0.5 * ((1.0 + x) + sin(M_PI * x) / M_PI), q);
}

__device__ __forceinline__ double face_mean(double a, double b, int harmonic) {
#pragma clang fp contract(off)
    return harmonic ? (2.0 * a * b) / (a + b) : 0.5 * (a + b);
}

template <int NC>
__global__ void __launch_bounds__(PT)
    k_faces_from_levelset(const double* __restrict__ phi, Props q, double* __restrict__ bx, double* __restrict__ by,
                          double* __restrict__ bz, int nx, int ny, int nz, uint32_t units) {
#pragma clang fp contract(off)
    const uint32_t t = blockIdx.x * PT + threadIdx.x;
    if (t >= units) return;
    const uint32_t ux = (uint32_t)nx / NC;
    const uint32_t r = t / ux;
    const int i = (int)(t - r * ux) * NC, j = (int)(r % (uint32_t)ny), k = (int)(r / (uint32_t)ny);
    const size_t plane = (size_t)nx * ny, c = (size_t)r * nx + i;
    const double ag = alpha_of(0.0, q), al = alpha_of(1.0, q);
    auto cell_alpha = [&](double v) { return ::cell_alpha(v, q, ag, al); };
    double a[NC];
#pragma unroll
    for (int e = 0; e < NC; e++) a[e] = cell_alpha(phi[c + e]);
    // x-faces: i .. i + NC - 1 (the first is a wall at i = 0), and the upper wall
    const size_t fx = ((size_t)k * ny + j) * (nx + 1) + i;
    bx[fx] = i > 0 ? face_mean(cell_alpha(phi[c - 1]), a[0], q.harmonic) : 0.0;
#pragma unroll
    for (int e = 1; e < NC; e++) bx[fx + e] = face_mean(a[e - 1], a[e], q.harmonic);
    if (i + NC == nx) bx[fx + NC] = 0.0;
    // y-faces of the cells (row j; walls at j = 0 and j = ny)
    const size_t fy = ((size_t)k * (ny + 1) + j) * nx + i;
    double o[NC];
#pragma unroll
    for (int e = 0; e < NC; e++) o[e] = j > 0 ? face_mean(cell_alpha(phi[c - nx + e]), a[e], q.harmonic) : 0.0;
    if constexpr (NC == 2) {
        *reinterpret_cast<double2*>(by + fy) = make_double2(o[0], o[1]);
        if (j == ny - 1) *reinterpret_cast<double2*>(by + fy + nx) = make_double2(0.0, 0.0);
    } else {
        by[fy] = o[0];
        if (j == ny - 1) by[fy + nx] = 0.0;
    }
    // z-faces (plane k; walls at k = 0 and k = nz)
#pragma unroll
    for (int e = 0; e < NC; e++)
        o[e] = k > 0 ? face_mean(cell_alpha(phi[c - plane + e]), a[e], q.harmonic) : 0.0;
    if constexpr (NC == 2) {
        *reinterpret_cast<double2*>(bz + c) = make_double2(o[0], o[1]);
        if (k == nz - 1) *reinterpret_cast<double2*>(bz + c + plane) = make_double2(0.0, 0.0);
    } else {
        bz[c] = o[0];
        if (k == nz - 1) bz[c + plane] = 0.0;
    }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

mg_status mg_faces_from_levelset(const mg_grid* g, const double* phi, double rho_l, double rho_g, double eps,
                                 int harmonic, double* bx, double* by, double* bz, void* stream) {
    try {
        if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || !phi || !bx || !by || !bz) {
            set_error("null grid/array or a dimension < 1");
            return MG_E_INVALID;
        }
        if (!(rho_l > 0) || !(rho_g > 0) || !(eps > 0) || !std::isfinite(rho_l) || !std::isfinite(rho_g) ||
            !std::isfinite(eps) || (harmonic != 0 && harmonic != 1)) {
            set_error("densities and eps must be finite and > 0, harmonic 0 or 1");
            return MG_E_INVALID;
        }
        const bool pair = (g->nx % 2) == 0 && aligned16(phi) && aligned16(by) && aligned16(bz);
        const int nc = pair ? 2 : 1;
        const size_t n = (size_t)g->nx * g->ny * g->nz / nc;
        if (n > (size_t)UINT32_MAX - PT) {
            set_error("grid too large for one launch");
            return MG_E_INVALID;
        }
        const unsigned blocks = (unsigned)((n + PT - 1) / PT);
        const Props q{rho_l, rho_g, eps, harmonic};
        hipStream_t s = (hipStream_t)stream;
        if (pair)
            k_faces_from_levelset<2><<<blocks, PT, 0, s>>>(phi, q, bx, by, bz, g->nx, g->ny, g->nz, (uint32_t)n);
        else
            k_faces_from_levelset<1><<<blocks, PT, 0, s>>>(phi, q, bx, by, bz, g->nx, g->ny, g->nz, (uint32_t)n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error(std::string("k_faces_from_levelset launch: ") + hipGetErrorString(e));
            return MG_E_HIP;
        }
        return MG_OK;
    } catch (...) {
        set_error("host exception in mg_faces_from_levelset");
        return MG_E_HIP;
    }
}

}  // extern "C"
