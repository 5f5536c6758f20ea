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
// per cell, a handful of flops), bound by HBM bandwidth.  A workgroup owns a
// 64 x 4 tile of columns and marches up a chunk of planes; each thread keeps the
// values it shares with the next plane (the z-face velocity below the cell, the
// pressure below it) in registers and loads the next plane's operands one step
// ahead.  Arithmetic is evaluated in a fixed order without fused multiply-adds:
//     b = scale * ((du + dv) + dw),   u_f = u_f - (scale * beta_f) * (p(c+) - p(c-)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "mg_core.h"
#include "mg_device.h"

using mgrt::set_error;

namespace {

constexpr int PBX = 64, PBY = 4;   // columns per workgroup: one wavefront per row
constexpr int P_TARGET_BLOCKS = 4096;

struct PGrid {
    int tiles_x, tiles_y, kc;
    long nblocks;
};

// Tiles of columns and chunks of planes: about P_TARGET_BLOCKS workgroups, XCD
// mapped by xcd_tile.
PGrid pgrid(int nx, int ny, int nz) {
    PGrid G;
    G.tiles_x = (nx + PBX - 1) / PBX;
    G.tiles_y = (ny + PBY - 1) / PBY;
    const long tiles = (long)G.tiles_x * G.tiles_y;
    long chunks = std::max(1L, std::min<long>(nz, (P_TARGET_BLOCKS + tiles - 1) / tiles));
    G.kc = (int)((nz + chunks - 1) / chunks);
    chunks = (nz + G.kc - 1) / G.kc;
    G.nblocks = tiles * chunks;
    return G;
}

struct Col {
    int i, j, k0, k1;
};

__device__ __forceinline__ Col column(const PGrid& G, int nx, int ny, int nz) {
    const int tile = mgk::xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    Col c;
    c.i = tx * PBX + (int)(threadIdx.x % PBX);
    c.j = ty * PBY + (int)(threadIdx.x / PBX);
    c.k0 = chunk * G.kc;
    c.k1 = min(nz, c.k0 + G.kc);
    return c;
}

// b = scale * ((u(i+1) - u(i)) + (v(j+1) - v(j)) + (w(k+1) - w(k))) per cell.
__global__ void __launch_bounds__(PBX* PBY)
    k_divergence(const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
                 double scale, double* __restrict__ b, int nx, int ny, int nz, PGrid G) {
#pragma clang fp contract(off)
    const Col q = column(G, nx, ny, nz);
    if (q.i >= nx || q.j >= ny || q.k0 >= q.k1) return;
    const size_t plane = (size_t)nx * ny, uplane = (size_t)(nx + 1) * ny, vplane = (size_t)nx * (ny + 1);
    const double* up = u + (size_t)q.k0 * uplane + (size_t)q.j * (nx + 1) + q.i;
    const double* vp = v + (size_t)q.k0 * vplane + (size_t)q.j * nx + q.i;
    const double* wp = w + (size_t)q.k0 * plane + (size_t)q.j * nx + q.i;
    double* bp = b + (size_t)q.k0 * plane + (size_t)q.j * nx + q.i;
    double wlo = wp[0];
    double u0 = up[0], u1 = up[1], v0 = vp[0], v1 = vp[nx], whi = wp[plane];
    for (int k = q.k0; k < q.k1; k++) {
        double nu0 = 0, nu1 = 0, nv0 = 0, nv1 = 0, nwhi = 0;
        if (k + 1 < q.k1) {   // the next plane's loads stay in flight during this plane
            up += uplane;
            vp += vplane;
            wp += plane;
            nu0 = up[0];
            nu1 = up[1];
            nv0 = vp[0];
            nv1 = vp[nx];
            nwhi = wp[plane];
        }
        const double du = u1 - u0, dv = v1 - v0, dw = whi - wlo;
        *bp = scale * ((du + dv) + dw);
        bp += plane;
        wlo = whi;
        u0 = nu0;
        u1 = nu1;
        v0 = nv0;
        v1 = nv1;
        whi = nwhi;
    }
}

// Every cell corrects its three lower faces when they are interior:
// x-face i (i > 0), y-face j (j > 0), z-face k (k > 0).  fx, fy, fz: the
// solver's level-0 faces, lower face of each cell ([nz][ny][nx]).  Each interior
// face has exactly one owner, so there are no write conflicts.
__global__ void __launch_bounds__(PBX* PBY)
    k_correct(const double* __restrict__ fx, const double* __restrict__ fy, const double* __restrict__ fz,
              const double* __restrict__ p, double scale, double* __restrict__ u, double* __restrict__ v,
              double* __restrict__ w, int nx, int ny, int nz, PGrid G) {
#pragma clang fp contract(off)
    const Col q = column(G, nx, ny, nz);
    if (q.i >= nx || q.j >= ny || q.k0 >= q.k1) return;
    const size_t plane = (size_t)nx * ny, uplane = (size_t)(nx + 1) * ny, vplane = (size_t)nx * (ny + 1);
    const bool xin = q.i > 0, yin = q.j > 0;
    // neighbour offsets clamped to the cell itself on the lower walls (no store there)
    const size_t xm = xin ? 1 : 0, ym = yin ? (size_t)nx : 0;
    size_t c = (size_t)q.k0 * plane + (size_t)q.j * nx + q.i;
    size_t fu = (size_t)q.k0 * uplane + (size_t)q.j * (nx + 1) + q.i;
    size_t fv = (size_t)q.k0 * vplane + (size_t)q.j * nx + q.i;
    double pbelow = q.k0 > 0 ? p[c - plane] : 0.0;
    double pc = p[c], pw = p[c - xm], ps = p[c - ym];
    double bxc = fx[c], byc = fy[c], bzc = fz[c];
    double uc = u[fu], vc = v[fv], wc = w[c];
    for (int k = q.k0; k < q.k1; k++) {
        const size_t cn = c + plane, fun = fu + uplane, fvn = fv + vplane;
        double npc = 0, npw = 0, nps = 0, nbx = 0, nby = 0, nbz = 0, nu = 0, nv = 0, nw = 0;
        if (k + 1 < q.k1) {   // the next plane's loads stay in flight during this plane
            npc = p[cn];
            npw = p[cn - xm];
            nps = p[cn - ym];
            nbx = fx[cn];
            nby = fy[cn];
            nbz = fz[cn];
            nu = u[fun];
            nv = v[fvn];
            nw = w[cn];
        }
        if (xin) u[fu] = uc - (scale * bxc) * (pc - pw);
        if (yin) v[fv] = vc - (scale * byc) * (pc - ps);
        if (k > 0) w[c] = wc - (scale * bzc) * (pc - pbelow);
        pbelow = pc;
        c = cn;
        fu = fun;
        fv = fvn;
        pc = npc;
        pw = npw;
        ps = nps;
        bxc = nbx;
        byc = nby;
        bzc = nbz;
        uc = nu;
        vc = nv;
        wc = nw;
    }
}

bool grid_fits(const PGrid& G) { return G.nblocks > 0 && G.nblocks <= INT_MAX; }

mg_status launch_divergence(const mg_grid& g, const double* u, const double* v, const double* w, double scale,
                            double* b, hipStream_t s) {
    const PGrid G = pgrid(g.nx, g.ny, g.nz);
    if (!grid_fits(G)) {
        set_error("grid too large for one launch");
        return MG_E_INVALID;
    }
    k_divergence<<<dim3((unsigned)G.nblocks), PBX * PBY, 0, s>>>(u, v, w, scale, b, g.nx, g.ny, g.nz, G);
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
    const PGrid G = pgrid(g.nx, g.ny, g.nz);
    if (!grid_fits(G)) {
        set_error("grid too large for one launch");
        return MG_E_INVALID;
    }
    k_correct<<<dim3((unsigned)G.nblocks), PBX * PBY, 0, s>>>(h->bx[0], h->by[0], h->bz[0], p, scale, u, v, w, g.nx,
                                                               g.ny, g.nz, G);
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
