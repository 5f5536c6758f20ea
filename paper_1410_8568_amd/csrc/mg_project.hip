// Projection step around the pressure solve (Sec. 2.2): the flow solver's
// Chorin projection on the staggered MAC mesh.  Velocity components live on the
// faces normal to them and the pressure in the cells; derivatives are
// second-order centred differences.  With the h^2 of eq. (10) folded into the
// right-hand side, the source S = div(u*) / dt of eq. (9) becomes
//     b_c = (h / dt) * sum_d (u_d(upper face of c) - u_d(lower face of c)),
// and the projected velocity on every interior face f between cells c- and c+ is
//     u_f = u*_f - (dt / h) * beta_f * (p(c+) - p(c-)),
// beta_f being the face coefficient of eq. (10), so that the discrete divergence
// of the result is (dt / h^2) (b - L p).  Wall faces keep their values.
//
// Both kernels are pure streaming passes (about 32 and 80 bytes of HBM traffic
// per cell, a handful of flops), bound by HBM bandwidth.  Each thread owns two
// neighbouring cells of a row (16-byte loads and stores of every array whose
// rows are aligned: cells, y- and z-faces; the x-face rows have nx + 1 entries
// and are read as scalars), 512 threads per workgroup, workgroups in plain
// dispatch order: for these passes, which re-read only a neighbouring row or
// plane, that measured faster than column marching and than an XCD-grouped
// order.  Odd nx or arrays that are not 16-byte aligned use one cell per thread.
// Arithmetic is evaluated in a fixed order without fused multiply-adds:
//     b = scale * ((du + dv) + dw),   u_f = u_f - (scale * beta_f) * (p(c+) - p(c-)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "mg_core.h"

using mgrt::set_error;

namespace {

constexpr int PT = 512;   // threads per workgroup

// First cell (i, j, k), index c, of this thread's unit of NC cells of a row.
struct Unit {
    uint32_t i, j, k;
    size_t c;
};

template <int NC>
__device__ __forceinline__ bool unit_of(int nx, int ny, uint32_t units, Unit& q) {
    const uint32_t t = blockIdx.x * PT + threadIdx.x;
    if (t >= units) return false;
    const uint32_t ux = (uint32_t)nx / NC;
    const uint32_t r = t / ux;
    q.i = (t - r * ux) * NC;
    q.j = r % (uint32_t)ny;
    q.k = r / (uint32_t)ny;
    q.c = (size_t)r * nx + q.i;
    return true;
}

__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ void st2(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }

// b = scale * ((u(i+1) - u(i)) + (v(j+1) - v(j)) + (w(k+1) - w(k))) per cell.
template <int NC>
__global__ void __launch_bounds__(PT)
    k_divergence(const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
                 double scale, double* __restrict__ b, int nx, int ny, uint32_t units) {
#pragma clang fp contract(off)
    Unit q;
    if (!unit_of<NC>(nx, ny, units, q)) return;
    const size_t plane = (size_t)nx * ny;
    const size_t uo = ((size_t)q.k * ny + q.j) * (nx + 1) + q.i;   // x-face i of the row
    const size_t vo = ((size_t)q.k * (ny + 1) + q.j) * nx + q.i;   // y-face j of the column
    if constexpr (NC == 2) {
        const double ua = u[uo], ub = u[uo + 1], uc = u[uo + 2];
        const double2 v0 = ld2(v + vo), v1 = ld2(v + vo + nx), w0 = ld2(w + q.c), w1 = ld2(w + q.c + plane);
        double2 o;
        o.x = scale * (((ub - ua) + (v1.x - v0.x)) + (w1.x - w0.x));
        o.y = scale * (((uc - ub) + (v1.y - v0.y)) + (w1.y - w0.y));
        st2(b + q.c, o);
    } else {
        const double du = u[uo + 1] - u[uo], dv = v[vo + nx] - v[vo], dw = w[q.c + plane] - w[q.c];
        b[q.c] = scale * ((du + dv) + dw);
    }
}

// Every cell corrects its three lower faces when they are interior: x-face i
// (i > 0), y-face j (j > 0), z-face k (k > 0).  fx, fy, fz: the solver's level-0
// faces, lower face of each cell ([nz][ny][nx]).  Each interior face has exactly
// one owner, so there are no write conflicts.
template <int NC>
__global__ void __launch_bounds__(PT)
    k_correct(const double* __restrict__ fx, const double* __restrict__ fy, const double* __restrict__ fz,
              const double* __restrict__ p, double scale, double* __restrict__ u, double* __restrict__ v,
              double* __restrict__ w, int nx, int ny, uint32_t units) {
#pragma clang fp contract(off)
    Unit q;
    if (!unit_of<NC>(nx, ny, units, q)) return;
    const size_t plane = (size_t)nx * ny, c = q.c;
    const size_t fu = ((size_t)q.k * ny + q.j) * (nx + 1) + q.i;
    const size_t fv = ((size_t)q.k * (ny + 1) + q.j) * nx + q.i;
    if constexpr (NC == 2) {
        const double2 pc = ld2(p + c), bx = ld2(fx + c);
        const double pw = p[q.i > 0 ? c - 1 : c];
        const double u0 = u[fu], u1 = u[fu + 1];
        if (q.i > 0) u[fu] = u0 - (scale * bx.x) * (pc.x - pw);
        u[fu + 1] = u1 - (scale * bx.y) * (pc.y - pc.x);   // face i + 1 is always interior
        if (q.j > 0) {
            const double2 ps = ld2(p + c - nx), by = ld2(fy + c), vv = ld2(v + fv);
            double2 o;
            o.x = vv.x - (scale * by.x) * (pc.x - ps.x);
            o.y = vv.y - (scale * by.y) * (pc.y - ps.y);
            st2(v + fv, o);
        }
        if (q.k > 0) {
            const double2 pb = ld2(p + c - plane), bz = ld2(fz + c), ww = ld2(w + c);
            double2 o;
            o.x = ww.x - (scale * bz.x) * (pc.x - pb.x);
            o.y = ww.y - (scale * bz.y) * (pc.y - pb.y);
            st2(w + c, o);
        }
    } else {
        const double pc = p[c];
        if (q.i > 0) u[fu] = u[fu] - (scale * fx[c]) * (pc - p[c - 1]);
        if (q.j > 0) v[fv] = v[fv] - (scale * fy[c]) * (pc - p[c - nx]);
        if (q.k > 0) w[c] = w[c] - (scale * fz[c]) * (pc - p[c - plane]);
    }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Units of work and workgroups for a grid; false if the grid is too large for
// the 32-bit unit index (about 4e9 cells, far beyond one GPU's memory).
bool launch_shape(const mg_grid& g, int nc, uint32_t* units, unsigned* blocks) {
    const size_t n = (size_t)g.nx * g.ny * g.nz / nc;
    if (n > (size_t)UINT32_MAX - PT) {
        set_error("grid too large for one launch");
        return false;
    }
    *units = (uint32_t)n;
    *blocks = (unsigned)((n + PT - 1) / PT);
    return true;
}

mg_status launch_divergence(const mg_grid& g, const double* u, const double* v, const double* w, double scale,
                            double* b, hipStream_t s) {
    const bool pair = (g.nx % 2) == 0 && aligned16(v) && aligned16(w) && aligned16(b);
    uint32_t units;
    unsigned blocks;
    if (!launch_shape(g, pair ? 2 : 1, &units, &blocks)) return MG_E_INVALID;
    if (pair)
        k_divergence<2><<<blocks, PT, 0, s>>>(u, v, w, scale, b, g.nx, g.ny, units);
    else
        k_divergence<1><<<blocks, PT, 0, s>>>(u, v, w, scale, b, g.nx, g.ny, units);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("k_divergence launch: ") + hipGetErrorString(e));
        return MG_E_HIP;
    }
    return MG_OK;
}

mg_status launch_correct(const mg_handle* h, const double* p, double scale, double* u, double* v, double* w,
                         hipStream_t s) {
    const mg_grid& g = h->g;
    const bool pair = (g.nx % 2) == 0 && aligned16(p) && aligned16(v) && aligned16(w);   // faces: 256-aligned
    uint32_t units;
    unsigned blocks;
    if (!launch_shape(g, pair ? 2 : 1, &units, &blocks)) return MG_E_INVALID;
    if (pair)
        k_correct<2><<<blocks, PT, 0, s>>>(h->bx[0], h->by[0], h->bz[0], p, scale, u, v, w, g.nx, g.ny, units);
    else
        k_correct<1><<<blocks, PT, 0, s>>>(h->bx[0], h->by[0], h->bz[0], p, scale, u, v, w, g.nx, g.ny, units);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("k_correct launch: ") + hipGetErrorString(e));
        return MG_E_HIP;
    }
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_divergence(const mg_grid* g, const double* u, const double* v, const double* w, double scale,
                        double* b, void* stream) {
    try {
        if (!g || g->nx < 0 || g->ny < 0 || g->nz < 0 || !std::isfinite(scale)) {
            set_error("null grid, negative dimension or non-finite scale");
            return MG_E_INVALID;
        }
        if ((size_t)g->nx * (size_t)g->ny * (size_t)g->nz == 0) return MG_OK;
        if (!u || !v || !w || !b) {
            set_error("null array");
            return MG_E_INVALID;
        }
        return launch_divergence(*g, u, v, w, scale, b, (hipStream_t)stream);
    } catch (...) {
        set_error("host exception in mg_divergence");
        return MG_E_HIP;
    }
}

mg_status mg_correct_velocity(const mg_handle* h, const double* p, double scale, double* u, double* v, double* w,
                              void* stream) {
    try {
        if (!h || !p || !u || !v || !w || !std::isfinite(scale)) {
            set_error("null handle/array or non-finite scale");
            return MG_E_INVALID;
        }
        return launch_correct(h, p, scale, u, v, w, (hipStream_t)stream);
    } catch (...) {
        set_error("host exception in mg_correct_velocity");
        return MG_E_HIP;
    }
}

mg_status mg_project(mg_handle* h, double* u, double* v, double* w, double dt, double hcell, double* b, double* p,
                     double tol, mg_stats* st, void* stream) {
    try {
        if (!h || !u || !v || !w || !b || !p || !(dt > 0) || !std::isfinite(dt) || !(hcell > 0) ||
            !std::isfinite(hcell) || !(tol >= 0) || !std::isfinite(tol) || !std::isfinite(hcell / dt) ||
            !std::isfinite(dt / hcell)) {
            set_error("null handle/array, dt or h not finite and > 0, or invalid tolerance");
            return MG_E_INVALID;
        }
        if (mgrt::check_solve_arrays(b, p) != MG_OK) return MG_E_INVALID;
        hipStream_t s = (hipStream_t)stream;
        mg_status r = launch_divergence(h->g, u, v, w, hcell / dt, b, s);
        if (r != MG_OK) return r;
        h->stream = s;
        r = mgrt::solve_impl(h, b, p, tol, st);
        if (r != MG_OK) return r;
        r = launch_correct(h, p, dt / hcell, u, v, w, s);
        if (r != MG_OK) return r;
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
            return MG_E_HIP;
        }
        return MG_OK;
    } catch (...) {
        set_error("host exception in mg_project");
        return MG_E_HIP;
    }
}

}  // extern "C"
