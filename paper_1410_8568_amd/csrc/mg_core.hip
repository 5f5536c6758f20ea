// Host runtime and C ABI of the multigrid pressure solver (gfx950).
//
// Setup (per coefficient field): copy faces with zero walls, coarsen faces
// level by level, cell weights for the flux-weighted prolongation, dense inverse
// of the coarsest operator, FP32 copies in refined mode.
// Solve: project b onto the range of L, then V-cycles (FP64 mode) or FP32
// V-cycles inside FP64 iterative refinement, with the relative residual, gamma
// (eq. 15) and the mean-zero projection of p after every cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "mg_core.h"
#include "mg_kernels.h"

using namespace mgk;

namespace mgrt {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                     \
            return MG_E_HIP;                                                                  \
        }                                                                                     \
    } while (0)

#define HIPCHK_VOID(expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) set_error(std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

dim3 col_grid(int nx, int ny, int nz) {
    int gx = (nx + BX - 1) / BX, gy = (ny + BY - 1) / BY;
    int gz = std::max(1, std::min(nz, 4096 / std::max(1, gx * gy)));
    return dim3(gx, gy, gz);
}

static int col_blocks(int nx, int ny, int nz) {
    dim3 g = col_grid(nx, ny, nz);
    return (int)(g.x * g.y * g.z);
}

// Tiles and z-chunks of the z-marching column kernels: about `target` (default
// 2048) workgroups, chunks of >= 4 planes (an even count when `even`); short
// chunks keep small levels from marching many planes in few workgroups.
static ColGrid zgrid(int cols_x, int cols_y, int nz, bool even, int* nblocks, int target = 2048) {
    ColGrid G;
    G.tiles_x = (cols_x + CBX - 1) / CBX;
    G.tiles_y = (cols_y + CBY - 1) / CBY;
    const int tiles = G.tiles_x * G.tiles_y;
    int chunks = std::max(1, std::min(std::max(1, nz / 4), (target + tiles - 1) / tiles));
    int kc = (nz + chunks - 1) / chunks;
    if (even && (kc & 1)) kc++;
    G.kc = kc;
    chunks = (nz + kc - 1) / kc;
    *nblocks = tiles * chunks;
    return G;
}

// The flat finest-level residual re-reads the neighbouring planes from the
// caches: it beats the column kernel while a plane holds at most 512 x 512 cells
// (11% at 512^3) and loses beyond (42% slower at 1024^3, 8 MB planes).
static bool resid_flat_fits(const LevelDims& d) {
    return (d.nx & 1) == 0 && (size_t)d.nx * d.ny <= (size_t)512 * 512;
}

mg_status plan(const mg_grid* g, const mg_options* o, Layout* L, bool with_p) {
    if (!g || !o || !L) {
        set_error("null argument");
        return MG_E_INVALID;
    }
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) {
        set_error("every grid dimension must be >= 2");
        return MG_E_INVALID;
    }
    if ((double)g->nx * g->ny * g->nz > 4.0e9) {
        set_error("grid too large");
        return MG_E_INVALID;
    }
    if (o->precision != MG_FP64 && o->precision != MG_FP32_REFINED) {
        set_error("unknown precision");
        return MG_E_INVALID;
    }
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 16 || o->nu2 > 16 || o->n_coarsest < 1 || o->inner_m < 1 ||
        o->inner_m > 16 || o->max_cycles < 1 || o->max_cycles > MG_MAX_HISTORY - 1 || o->tile < -1 ||
        o->tile > MG_NUM_TILES || (o->krylov != MG_KRYLOV_NONE && o->krylov != MG_KRYLOV_FCG)) {
        set_error("option out of range");
        return MG_E_INVALID;
    }
    if (!(o->omega > 0.0 && o->omega < 2.0) || (o->restrict64 != 0 && o->restrict64 != 1) ||
        o->coarse_gmres < 0 || o->coarse_gmres > MG_GMRES_MAX_M ||
        (o->coarse_gmres > 0 && (!(o->coarse_gmres_tol > 0.0) || o->coarse_gmres_maxit < 1 ||
                                 o->coarse_gmres_maxit > 1000000))) {
        set_error("cycle variant option out of range");
        return MG_E_INVALID;
    }
    if (o->krylov == MG_KRYLOV_FCG && o->precision != MG_FP64) {
        set_error("the Krylov solve runs in FP64 precision only");
        return MG_E_INVALID;
    }
    *L = Layout();
    int d[3] = {g->nx, g->ny, g->nz};
    for (;;) {
        LevelDims& ld = L->d[L->nlev];
        ld.nx = d[0];
        ld.ny = d[1];
        ld.nz = d[2];
        L->nlev++;
        if (L->nlev == MG_MAX_LEVELS) break;
        int mx = std::max(d[0], std::max(d[1], d[2]));
        if ((d[0] & 1) || (d[1] & 1) || (d[2] & 1) || mx <= o->n_coarsest) break;
        d[0] /= 2;
        d[1] /= 2;
        d[2] /= 2;
    }
    const LevelDims& c = L->d[L->nlev - 1];
    if (c.ncell() > MG_MAX_COARSE_CELLS) {
        char buf[160];
        snprintf(buf, sizeof buf, "coarsest grid %dx%dx%d has more than %d cells", c.nx, c.ny, c.nz,
                 MG_MAX_COARSE_CELLS);
        set_error(buf);
        return MG_E_INVALID;
    }
    L->ncoarse = (int)c.ncell();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t r = off;
        off += align256(bytes);
        return r;
    };
    const bool f32 = o->precision == MG_FP32_REFINED;
    for (int l = 0; l < L->nlev; l++) {
        const LevelDims& ld = L->d[l];
        L->bx[l] = take(ld.ncell() * 8);
        L->by[l] = take(ld.ncell() * 8);
        L->bz[l] = take(ld.ncell() * 8);
        L->a[l] = take(ld.ncell() * 8);
        if (l > 0 && !f32) {
            L->e[l] = take(ld.ncell() * 8);
            L->rhs[l] = take(ld.ncell() * 8);
        }
        if (!f32 && l < L->nlev - 1) L->tmp[l] = take(ld.ncell() * 8);
        if (f32) {
            L->fbx[l] = take(ld.ncell() * 4);
            L->fby[l] = take(ld.ncell() * 4);
            L->fbz[l] = take(ld.ncell() * 4);
            L->fa[l] = take(ld.ncell() * 4);
            L->fe[l] = take(ld.ncell() * 4);
            L->frhs[l] = take(ld.ncell() * 4);
            if (l < L->nlev - 1) L->ftmp[l] = take(ld.ncell() * 4);
        }
    }
    L->bbar = take(L->d[0].ncell() * 8);
    if (o->krylov == MG_KRYLOV_FCG) {
        L->kr = take(L->d[0].ncell() * 8);
        L->kz = take(L->d[0].ncell() * 8);
        L->ks = take(L->d[0].ncell() * 8);
        L->kq = take(L->d[0].ncell() * 8);
    }
    if (with_p) L->pw = take(L->d[0].ncell() * 8);
    L->binv = take((size_t)L->ncoarse * L->ncoarse * 8);
    L->scal = take(64 * 8);
    int mb = 0;
    for (int l = 0; l < L->nlev; l++) {
        int zb = 0;
        zgrid(L->d[l].nx, L->d[l].ny, L->d[l].nz, false, &zb);
        mb = std::max(mb, std::max(zb, col_blocks(L->d[l].nx, L->d[l].ny, L->d[l].nz)));
        zgrid((L->d[l].nx + 1) / 2, L->d[l].ny, L->d[l].nz, false, &zb);   // cell-pair kernels
        mb = std::max(mb, zb);
    }
    // the flat finest-level residual: one workgroup per RES_FLAT_THREADS cell pairs
    if (resid_flat_fits(L->d[0]))
        mb = std::max(mb, (int)(((size_t)L->d[0].ncell() / 2 + RES_FLAT_THREADS - 1) / RES_FLAT_THREADS));
    L->max_blocks = mb;
    L->part = take((size_t)2 * (mb + FIN_PARTS) * 8);   // partial pairs, then the first stage's
    L->flag = take(64);
    L->total = off;
    return MG_OK;
}

static dim3 lin_grid(size_t n) {
    size_t b = (n + 255) / 256;
    return dim3((unsigned)std::max<size_t>(1, std::min<size_t>(b, 16384)));
}

// ------------------------------------------------------------------ profiling

Prof::Prof(mg_handle* h_, int cls_, double bytes_) : h(h_), cls(cls_), bytes(bytes_), idx(0) {
    if (!h->o.profile) return;
    idx = h->recs.size();
    while (h->ev.size() < 2 * (idx + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        h->ev.push_back(e);
    }
    h->recs.push_back({cls, bytes});
    (void)hipEventRecord(h->ev[2 * idx], h->stream);
}

Prof::~Prof() {
    if (!h->o.profile || h->ev.size() < 2 * (idx + 1)) return;
    (void)hipEventRecord(h->ev[2 * idx + 1], h->stream);
}

static void prof_reset(mg_handle* h) {
    h->recs.clear();
    for (int c = 0; c < MG_K_COUNT; c++) {
        h->kernel_ms[c] = 0;
        h->kernel_launches[c] = 0;
        h->kernel_bytes[c] = 0;
    }
}

static void prof_collect(mg_handle* h) {
    if (!h->o.profile) return;
    for (size_t i = 0; i < h->recs.size(); i++) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) != hipSuccess) continue;
        int c = h->recs[i].cls;
        h->kernel_ms[c] += ms;
        h->kernel_launches[c] += 1;
        h->kernel_bytes[c] += h->recs[i].bytes;
    }
    h->recs.clear();
}

// ------------------------------------------------------------------ setup

template <class T>
static mg_status tune_level(mg_handle* h, const Lvl<T>& L, T* pin, T* pout, T* b, T* rc, int* choice,
                            int* rchoice);
template <class T>
static bool has_restrict_variant(int v);

void bind(mg_handle* h) {
    const Layout& L = h->L;
    char* w = h->ws;
    const bool f32 = h->o.precision == MG_FP32_REFINED;
    for (int l = 0; l < L.nlev; l++) {
        h->bx[l] = (double*)(w + L.bx[l]);
        h->by[l] = (double*)(w + L.by[l]);
        h->bz[l] = (double*)(w + L.bz[l]);
        h->a[l] = (double*)(w + L.a[l]);
        h->e[l] = (l > 0 && !f32) ? (double*)(w + L.e[l]) : nullptr;
        h->rhs[l] = (l > 0 && !f32) ? (double*)(w + L.rhs[l]) : nullptr;
        h->tmp[l] = (!f32 && l < L.nlev - 1) ? (double*)(w + L.tmp[l]) : nullptr;
        h->ftmp[l] = (f32 && l < L.nlev - 1) ? (float*)(w + L.ftmp[l]) : nullptr;
        if (f32) {
            h->fbx[l] = (float*)(w + L.fbx[l]);
            h->fby[l] = (float*)(w + L.fby[l]);
            h->fbz[l] = (float*)(w + L.fbz[l]);
            h->fa[l] = (float*)(w + L.fa[l]);
            h->fe[l] = (float*)(w + L.fe[l]);
            h->frhs[l] = (float*)(w + L.frhs[l]);
        } else {
            h->fbx[l] = h->fby[l] = h->fbz[l] = h->fa[l] = h->fe[l] = h->frhs[l] = nullptr;
        }
    }
    h->bbar = (double*)(w + L.bbar);
    h->binv = (double*)(w + L.binv);
    h->scal = (double*)(w + L.scal);
    h->part = (double*)(w + L.part);
    h->flag = (int*)(w + L.flag);
    const bool kry = h->o.krylov == MG_KRYLOV_FCG;
    h->kr = kry ? (double*)(w + L.kr) : nullptr;
    h->kz = kry ? (double*)(w + L.kz) : nullptr;
    h->ks = kry ? (double*)(w + L.ks) : nullptr;
    h->kq = kry ? (double*)(w + L.kq) : nullptr;
    h->pw = L.pw ? (double*)(w + L.pw) : nullptr;
}

mg_status setup_launch(mg_handle* h, const double* bx, const double* by, const double* bz) {
    bind(h);
    const Layout& L = h->L;
    hipStream_t s = h->stream;
    HIPCHK(hipMemsetAsync(h->flag, 0, 64, s));
    const LevelDims& d0 = L.d[0];
    k_faces_from_api<<<lin_grid(d0.ncell()), 256, 0, s>>>(bx, by, bz, h->bx[0], h->by[0], h->bz[0], d0.nx, d0.ny,
                                                          d0.nz, h->flag);
    HIPCHK(hipGetLastError());
    for (int l = 0; l < L.nlev; l++) {
        const LevelDims& d = L.d[l];
        if (l > 0) {
            const LevelDims& f = L.d[l - 1];
            k_coarsen<<<lin_grid(d.ncell()), 256, 0, s>>>(h->bx[l - 1], h->by[l - 1], h->bz[l - 1], h->bx[l], h->by[l],
                                                          h->bz[l], f.nx, f.ny, d.nx, d.ny, d.nz);
        }
        k_cell_weights<<<lin_grid(d.ncell()), 256, 0, s>>>(Lvl<double>{d.nx, d.ny, d.nz, h->bx[l], h->by[l], h->bz[l]},
                                                           h->a[l]);
    }
    HIPCHK(hipGetLastError());
    const LevelDims& c = L.d[L.nlev - 1];
    const int lc = L.nlev - 1;
    k_coarse_invert<<<1, FIN_THREADS, 0, s>>>(Lvl<double>{c.nx, c.ny, c.nz, h->bx[lc], h->by[lc], h->bz[lc]}, h->binv,
                                              h->flag + 1);
    HIPCHK(hipGetLastError());
    if (h->o.precision == MG_FP32_REFINED) {
        for (int l = 0; l < L.nlev; l++) {
            const LevelDims& d = L.d[l];
            k_cast_d2f<<<lin_grid(d.ncell()), 256, 0, s>>>(h->bx[l], h->fbx[l], d.ncell());
            k_cast_d2f<<<lin_grid(d.ncell()), 256, 0, s>>>(h->by[l], h->fby[l], d.ncell());
            k_cast_d2f<<<lin_grid(d.ncell()), 256, 0, s>>>(h->bz[l], h->fbz[l], d.ncell());
            k_cast_d2f<<<lin_grid(d.ncell()), 256, 0, s>>>(h->a[l], h->fa[l], d.ncell());
        }
        HIPCHK(hipGetLastError());
    }
    // smoother variant (and fused pre-smoothing + restriction variant) per level
    const bool f32 = h->o.precision == MG_FP32_REFINED;
    for (int l = 0; l < MG_MAX_LEVELS; l++) h->tile[l] = h->rtile[l] = 0;
    for (int l = 0; l + 1 < L.nlev; l++) {
        if (h->o.tile != 0) {
            h->tile[l] = h->o.tile;
            h->rtile[l] = (h->o.nu1 == 2 && (f32 ? has_restrict_variant<float>(h->o.tile)
                                                 : has_restrict_variant<double>(h->o.tile)))
                              ? h->o.tile
                              : 0;
            continue;
        }
        const LevelDims& d = L.d[l];
        mg_status r;
        if (f32) {
            Lvl<float> lv{d.nx, d.ny, d.nz, h->fbx[l], h->fby[l], h->fbz[l]};
            r = tune_level<float>(h, lv, h->fe[l], h->ftmp[l], h->frhs[l], h->frhs[l + 1], &h->tile[l],
                                  &h->rtile[l]);
        } else {
            Lvl<double> lv{d.nx, d.ny, d.nz, h->bx[l], h->by[l], h->bz[l]};
            double* pin = l == 0 ? h->bbar : h->e[l];
            double* b = l == 0 ? h->bbar : h->rhs[l];
            r = tune_level<double>(h, lv, pin, h->tmp[l], b, h->rhs[l + 1], &h->tile[l], &h->rtile[l]);
        }
        if (r != MG_OK) return r;
    }
    // the fused pre-smoothing passes restrict with the 8-child mean only
    if (h->o.restrict64)
        for (int l = 0; l < MG_MAX_LEVELS; l++) h->rtile[l] = 0;
    // validation flags land in the pinned host block; setup_finish reads them
    HIPCHK(hipMemcpyAsync(setup_flags(h), h->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    return MG_OK;
}

mg_status setup_finish(mg_handle* h) {
    const int* flags = setup_flags(h);
    if (flags[0]) {
        set_error(std::to_string(flags[0]) + " interior face coefficient(s) not finite and > 0");
        return MG_E_INVALID;
    }
    if (flags[1]) {
        set_error("coarsest operator not positive definite (disconnected grid?)");
        return MG_E_INVALID;
    }
    return MG_OK;
}

// ------------------------------------------------------------------ solve

template <class T>
struct Hier {
    int nlev;
    const LevelDims* d;
    Lvl<T> L[MG_MAX_LEVELS];
    T* e[MG_MAX_LEVELS];
    T* rhs[MG_MAX_LEVELS];
    T* tmp[MG_MAX_LEVELS];
    const T* a[MG_MAX_LEVELS];
};

// The FP64 refinement update p <- (p - sum / N) + s * e, fused into the FP32
// pass that writes the correction e of level 0 in final form.
struct RefineUpd {
    double* p;
    const double* s;     // scale of the FP32 right-hand side
    const double* sum;   // sum of p (its mean is taken out on the way)
};

template <class T, int TX, int TY, int NSW, bool RES = false, bool SKIP = false, bool UPD = false>
static void launch_sweep(const Launcher& ln, const Lvl<T>& L, const T* pin, T* pout, const T* b, int c0, int target,
                         const double* shift_sum, int zero_in, T* rc, double omega, const RefineUpd& u = {}) {
    const int gx = (L.nx + TX - 1) / TX, gy = (L.ny + TY - 1) / TY;
    const int tiles = gx * gy;
    // chunks of >= 8 planes, so the redundant planes at chunk ends stay a small fraction
    int chunks = std::max(1, std::min(std::max(1, L.nz / 8), (target + tiles - 1) / tiles));
    int kc = (L.nz + chunks - 1) / chunks;
    if (RES && (kc & 1)) kc++;   // the restriction pairs planes 2K, 2K+1 within a chunk
    chunks = (L.nz + kc - 1) / kc;
    constexpr int NT = (TX / 2 + 2 * NSW) * (TY + 4 * NSW - 2 + (RES ? 2 : 0));
    const double N = (double)L.nx * L.ny * L.nz;
    if constexpr (UPD)   // FP32 Gauss-Seidel only: the caller checked omega == 1
        ln.x(k_rb_sweep<T, TX, TY, NSW, false, false, false, true>, tiles * chunks, NT, L, pin, pout, b, c0, kc, gx,
             gy, shift_sum, N, zero_in, rc, T(1), u.p, u.s, u.sum);
    else if constexpr (SKIP)   // Gauss-Seidel only: the caller checked omega == 1
        ln.x(k_rb_sweep<T, TX, TY, NSW, RES, false, true>, tiles * chunks, NT, L, pin, pout, b, c0, kc, gx, gy,
             shift_sum, N, zero_in, rc, T(1), nullptr, nullptr, nullptr);
    else if (omega != 1.0)   // successive over-relaxation (a separate instantiation)
        ln.x(k_rb_sweep<T, TX, TY, NSW, RES, true>, tiles * chunks, NT, L, pin, pout, b, c0, kc, gx, gy, shift_sum, N,
             zero_in, rc, (T)omega, nullptr, nullptr, nullptr);
    else
        ln.x(k_rb_sweep<T, TX, TY, NSW, RES, false>, tiles * chunks, NT, L, pin, pout, b, c0, kc, gx, gy, shift_sum, N,
             zero_in, rc, T(1), nullptr, nullptr, nullptr);
}

// Fused variant v (1..MG_NUM_TILES): tile (v - 1) / 3 of the list (four one-sweep
// tiles, then four two-sweep ones), about 256, 1024 or 4096 workgroups for
// (v - 1) mod 3 = 0, 1, 2.  256 is one workgroup per CU with a whole column per
// workgroup (no redundant planes at chunk ends); the larger targets cut the
// columns into z-chunks for levels with few tiles.
static int variant_target(int v) { return (v - 1) % 3 == 0 ? 256 : ((v - 1) % 3 == 1 ? 1024 : 4096); }

// Sweeps done by one pass of fused variant v.
static int sweeps_per_pass(int v) { return v > 12 ? 2 : 1; }

// Variants 19..24 (two sweeps, 128x8 and 64x16 tiles) need more than 64 KiB of
// LDS in FP64; there they fall back to the 64x8 two-sweep tile.
template <class T>
static bool variant_native(int v) {
    return sizeof(T) == 4 || v <= 18;
}

// True when a pass of variant v can apply the refinement update (FP32 two-sweep
// Gauss-Seidel passes).
template <class T>
static bool has_update_variant(int v, double omega) {
    return sizeof(T) == 4 && v > 12 && omega == 1.0;
}

// Fused sweep variant v in 1..MG_NUM_TILES: one pass doing sweeps_per_pass(v) sweeps
// (with u non-null, also the refinement update; has_update_variant(v) must hold).
template <class T>
static void fused_sweep(const Launcher& s, int v, const Lvl<T>& L, const T* pin, T* pout, const T* b, int c0,
                        const double* shift_sum = nullptr, int zero_in = 0, double omega = 1.0,
                        const RefineUpd* u = nullptr) {
    const int target = variant_target(v);
    if constexpr (sizeof(T) == 4) {
        if (u) {
            switch ((v - 1) / 3) {
                case 4: launch_sweep<T, 64, 4, 2, false, false, true>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, 1.0, *u); return;
                case 5: launch_sweep<T, 64, 8, 2, false, false, true>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, 1.0, *u); return;
                case 6: launch_sweep<T, 128, 8, 2, false, false, true>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, 1.0, *u); return;
                default: launch_sweep<T, 64, 16, 2, false, false, true>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, 1.0, *u); return;
            }
        }
    }
    switch ((v - 1) / 3) {
        case 0: launch_sweep<T, 64, 8, 1>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 1: launch_sweep<T, 128, 4, 1>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 2: launch_sweep<T, 128, 8, 1>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 3: launch_sweep<T, 64, 16, 1>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 4: launch_sweep<T, 64, 4, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 5: launch_sweep<T, 64, 8, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega); break;
        case 6:
            if constexpr (sizeof(T) == 4)
                launch_sweep<T, 128, 8, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega);
            else
                launch_sweep<T, 64, 8, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega);
            break;
        default:
            if constexpr (sizeof(T) == 4)
                launch_sweep<T, 64, 16, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega);
            else
                launch_sweep<T, 64, 8, 2>(s, L, pin, pout, b, c0, target, shift_sum, zero_in, nullptr, omega);
            break;
    }
}

// Variants whose two-sweep pass can also form the residual and restrict it:
// tiles 64x4 and 64x8, and 64x16 in FP32 (128x8 would need more than 1024
// threads; an FP64 64x16 pass would not fit its registers).
template <class T>
static bool has_restrict_variant(int v) {
    const int t = (v - 1) / 3;
    return v > 0 && (t == 4 || t == 5 || (sizeof(T) == 4 && t == 7));
}

// Two-sweep pass of variant v that also forms the residual of its result and
// restricts it into rc (the next level's right-hand side); returns false
// (nothing launched) when v has no such pass.
//
// skip_red: the iterate's red cells already hold what the pass's first (red)
// stage would compute (the previous cycle's post-smoothing ended with red, and
// omega == 1), so that stage is left out (bit-identical results; FP32 only).
template <class T>
static bool fused_sweep_restrict(const Launcher& s, int v, const Lvl<T>& L, const T* pin, T* pout, const T* b,
                                 const double* shift_sum, int zero_in, T* rc, double omega = 1.0,
                                 bool skip_red = false) {
    const int target = variant_target(v);
    if constexpr (sizeof(T) == 4) {
        if (skip_red) {
            switch ((v - 1) / 3) {
                case 4: launch_sweep<T, 64, 4, 2, true, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, 1.0); return true;
                case 5: launch_sweep<T, 64, 8, 2, true, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, 1.0); return true;
                case 7: launch_sweep<T, 64, 16, 2, true, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, 1.0); return true;
                default: return false;
            }
        }
    }
    switch ((v - 1) / 3) {
        case 4: launch_sweep<T, 64, 4, 2, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, omega); return true;
        case 5: launch_sweep<T, 64, 8, 2, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, omega); return true;
        case 7:
            if constexpr (sizeof(T) == 4) {
                launch_sweep<T, 64, 16, 2, true>(s, L, pin, pout, b, 0, target, shift_sum, zero_in, rc, omega);
                return true;
            }
            return false;
        default: return false;
    }
}

template <class T>
static void ref_sweep(const Launcher& ln, const Lvl<T>& L, T* p, const T* b, int c0, double omega = 1.0) {
    const dim3 g = col_grid(L.nx, L.ny, L.nz), blk(BX, BY);
    ln.z(k_rb_half<T>, g, blk, L, p, b, c0, (T)omega);
    ln.z(k_rb_half<T>, g, blk, L, p, b, 1 - c0, (T)omega);
}

// Residual of level L restricted into rc (the next level's right-hand side),
// as a separate pass: 4 cells per thread in FP32 when nx allows, else 2.
template <class T>
static void launch_restrict(const Launcher& ln, const Lvl<T>& L, const T* p, const T* b, T* rc) {
    int nb = 0;
    if constexpr (sizeof(T) == 4) {
        if (L.nx % 4 == 0) {
            const ColGrid G = zgrid(L.nx / 4, L.ny, L.nz, true, &nb);
            ln.x(k_resid_restrict_cells<T, 4>, nb, CBX * CBY, L, p, b, G, rc);
            return;
        }
    }
    const ColGrid G = zgrid(L.nx / 2, L.ny, L.nz, true, &nb);
    ln.x(k_resid_restrict_cells<T, 2>, nb, CBX * CBY, L, p, b, G, rc);
}

// ------------------------------------------------------------------ smoother tuning
//
// For every smoothed level the variant with the shortest measured sweep is
// chosen at setup (each variant: one warm-up and three timed passes on the
// level's own scratch buffers, zero-filled).  Where nu1 = 2 and the level has
// fused pre-smoothing + restriction variants, each is timed against two sweeps
// of the chosen variant plus the separate restriction, and the fastest way is
// kept.  Choices are remembered per (precision, grid size) for the life of the
// process and, when MG_TUNE_CACHE names a file, across processes (one JSON
// object per line).

namespace {
std::mutex g_tune_mu;
std::map<std::array<int, 4>, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("MG_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        int pr, x, y, z, v, rv;
        int nt = 0;   // entries written for another variant list are skipped
        if (sscanf(line,
                   "{\"bytes\": %d, \"nx\": %d, \"ny\": %d, \"nz\": %d, \"variant\": %d, \"restrict\": %d, "
                   "\"variants\": %d}",
                   &pr, &x, &y, &z, &v, &rv, &nt) == 7 &&
            nt == MG_NUM_TILES && v >= -1 && v <= MG_NUM_TILES && v != 0 && rv >= 0 && rv <= MG_NUM_TILES)
            g_tune[{pr, x, y, z}] = {v, rv};
    }
    fclose(f);
}

void tune_store_locked(const std::array<int, 4>& k, int v, int rv) {
    g_tune[k] = {v, rv};
    const char* path = getenv("MG_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"bytes\": %d, \"nx\": %d, \"ny\": %d, \"nz\": %d, \"variant\": %d, \"restrict\": %d, \"variants\": %d}\n",
            k[0], k[1], k[2], k[3], v, rv, MG_NUM_TILES);
    fclose(f);
}
}  // namespace

// Variant used without timing (no-allocation setups on grid sizes not tuned
// before): the two-sweep 64x8 tile with about 256 workgroups, which has a fused
// pre-smoothing + restriction pass in both precisions.  Every variant gives
// bit-identical results; only the speed differs.
constexpr int UNTUNED_VARIANT = 16;

template <class T>
static mg_status tune_level(mg_handle* h, const Lvl<T>& L, T* pin, T* pout, T* b, T* rc, int* choice,
                            int* rchoice) {
    // the cached fused-restriction choice assumes nu1 = 2; other nu1 never fuse
    const std::array<int, 4> key{(int)sizeof(T), L.nx, L.ny, L.nz};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *choice = it->second.first;
            *rchoice = h->o.nu1 == 2 ? it->second.second : 0;
            return MG_OK;
        }
    }
    if (h->no_alloc) {   // timing needs events and scratch fills: use the fixed variant
        *choice = UNTUNED_VARIANT;
        *rchoice = h->o.nu1 == 2 && has_restrict_variant<T>(UNTUNED_VARIANT) ? UNTUNED_VARIANT : 0;
        return MG_OK;
    }
    hipStream_t s = h->stream;
    Launcher ls;
    ls.stream = s;
    const size_t n = (size_t)L.nx * L.ny * L.nz;
    HIPCHK(hipMemsetAsync(pin, 0, n * sizeof(T), s));
    if (b != pin) HIPCHK(hipMemsetAsync(b, 0, n * sizeof(T), s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_ms = [&](auto&& run) {
        run();
        float tmin = 1e30f;
        for (int rep = 0; rep < 3; rep++) {
            (void)hipEventRecord(e0, s);
            run();
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        return tmin;
    };
    float best = 1e30f;
    int bestv = -1;
    for (int v = -1; v <= MG_NUM_TILES; v++) {
        if (v == 0 || (v > 0 && !variant_native<T>(v))) continue;
        float t = time_ms([&]() {
            if (v < 0)
                ref_sweep<T>(ls, L, pin, b, 0);
            else
                fused_sweep<T>(ls, v, L, pin, pout, b, 0);
        });
        if (v > 0) t /= sweeps_per_pass(v);
        if (t < best) {
            best = t;
            bestv = v;
        }
    }
    // fused pre-smoothing + restriction against two sweeps plus the separate pass
    int bestr = 0;
    bool any = false;
    for (int v = 1; v <= MG_NUM_TILES; v++) any = any || has_restrict_variant<T>(v);
    if (any) {
        float rbest = 2.0f * best + time_ms([&]() { launch_restrict<T>(ls, L, pin, b, rc); });
        for (int v = 1; v <= MG_NUM_TILES; v++) {
            if (!has_restrict_variant<T>(v)) continue;
            const float t = time_ms([&]() { fused_sweep_restrict<T>(ls, v, L, pin, pout, b, nullptr, 0, rc); });
            if (t < rbest) {
                rbest = t;
                bestr = v;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    *choice = bestv;
    *rchoice = h->o.nu1 == 2 ? bestr : 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store_locked(key, bestv, bestr);
    return MG_OK;
}

// nsweep red-black sweeps on level l, first colour c0 (0: red first): passes of
// the level's fused variant (each pass does sweeps_per_pass sweeps, out of
// place: cur -> alt, then the two pointers swap), then in-place sweeps of the
// reference kernels for what is left (or for everything, on levels that use
// them).  shift_sum (optional): the first fused pass subtracts shift_sum[0]/N
// from the iterate as it reads it; returns false if there was no fused pass.
// upd (optional): when the last pass is a fused one that can apply the
// refinement update, it does, and *upd_done is set.
template <class T>
static bool smooth(mg_handle* h, Hier<T>& H, int l, int nsweep, int c0, T*& cur, T*& alt,
                   const double* shift_sum = nullptr, bool zero_in = false, const RefineUpd* upd = nullptr,
                   bool* upd_done = nullptr) {
    const Launcher s = launcher(h);
    const LevelDims& d = H.d[l];
    const int tile = alt ? h->tile[l] : -1;
    const bool fused = tile > 0 && nsweep >= sweeps_per_pass(tile);
    if (zero_in && !fused) {
        Prof pf(h, MG_K_OTHER, (double)d.ncell() * sizeof(T));
        s.x(k_fill<T>, lin_grid(d.ncell()).x, 256, cur, d.ncell(), T(0));
        zero_in = false;
    }
    if (nsweep <= 0) return shift_sum == nullptr;
    const int cls = l == 0 ? MG_K_SMOOTH_FINE : MG_K_SMOOTH;
    const double full = (3.0 * d.ncell() + d.nfaces()) * sizeof(T);
    bool shifted = shift_sum == nullptr;
    int rem = nsweep;
    if (tile > 0) {
        const int spp = sweeps_per_pass(tile);
        const bool with_upd = upd && rem % spp == 0 && has_update_variant<T>(tile, h->o.omega);
        for (; rem >= spp; rem -= spp) {
            // algorithmic bytes: one sweep's worth per sweep done (less the
            // iterate's read when it starts from zero; plus the FP64 iterate's
            // read and write when the pass also applies the update)
            const bool u = with_upd && rem == spp;
            Prof pf(h, cls, spp * full - (zero_in ? (double)d.ncell() * sizeof(T) : 0.0) + (u ? 16.0 * d.ncell() : 0.0));
            fused_sweep<T>(s, tile, H.L[l], cur, alt, H.rhs[l], c0, shifted ? nullptr : shift_sum, zero_in ? 1 : 0,
                           h->o.omega, u ? upd : nullptr);
            if (u) *upd_done = true;
            shifted = true;
            zero_in = false;
            std::swap(cur, alt);
        }
    }
    for (; rem > 0; rem--) {
        Prof pf(h, cls, full);
        ref_sweep<T>(s, H.L[l], cur, H.rhs[l], c0, h->o.omega);
    }
    return shifted;
}

// True when the first pre-smoothing pass on level 0 can absorb the mean shift.
static bool fused_first_sweep(const mg_handle* h) {
    return h->L.nlev > 1 && h->tile[0] > 0 && h->o.nu1 >= sweeps_per_pass(h->tile[0]);
}

// red_done: the level's iterate was last updated by a red half-sweep (the
// previous cycle's post-smoothing on this level), so a fused pre-smoothing pass
// may leave out its first (red) stage.
//
// upd (level 0 only, optional): the refinement update, applied by the last
// post-smoothing pass where it can be (*upd_done set), else left to the caller.
template <class T>
static void vcycle(mg_handle* h, Hier<T>& H, int l, const double* shift_sum = nullptr, bool zero_init = false,
                   bool red_done = false, const RefineUpd* upd = nullptr, bool* upd_done = nullptr) {
    const Launcher s = launcher(h);
    const LevelDims& d = H.d[l];
    if (l == H.nlev - 1) {
        if (h->o.coarse_gmres > 0) {
            Prof pf(h, MG_K_COARSE, (2.0 * d.ncell() + 3.0 * d.ncell()) * 8.0);
            s.x(k_coarse_gmres<T>, 1, 512, Lvl<double>{d.nx, d.ny, d.nz, h->bx[l], h->by[l], h->bz[l]}, H.rhs[l],
                H.e[l], h->o.coarse_gmres, h->o.coarse_gmres_tol, h->o.coarse_gmres_maxit);
            return;
        }
        Prof pf(h, MG_K_COARSE, (double)h->L.ncoarse * h->L.ncoarse * 8 + 2.0 * d.ncell() * sizeof(T));
        s.x(k_coarse_solve<T>, (h->L.ncoarse + 7) / 8, 512, (const double*)h->binv, h->L.ncoarse, (const T*)H.rhs[l],
            H.e[l]);
        return;
    }
    // the current iterate moves between e and tmp as fused passes run
    T* cur = H.e[l];
    T* alt = H.tmp[l];
    const LevelDims& c = H.d[l + 1];
    const double restrict_bytes = ((2.0 * d.ncell() + d.nfaces()) + c.ncell()) * sizeof(T);
    // pre-smoothing; where the level's tuning chose the fused pass (one two-sweep
    // pass is all of it), that pass also forms the residual and its restriction
    const int rtile = alt ? h->rtile[l] : 0;
    if (rtile > 0) {
        // a pass that leaves out its red stage is credited with the three
        // half-sweeps it does (1.5 sweeps' algorithmic bytes)
        const bool skip = sizeof(T) == 4 && red_done && !zero_init && h->o.omega == 1.0;
        const double sweep_bytes = (skip ? 1.5 : 2.0) * (3.0 * d.ncell() + d.nfaces()) * sizeof(T) -
                                   (zero_init ? (double)d.ncell() * sizeof(T) : 0.0);
        Prof pf(h, l == 0 ? MG_K_SMOOTH_FINE : MG_K_SMOOTH, sweep_bytes + restrict_bytes);
        fused_sweep_restrict<T>(s, rtile, H.L[l], cur, alt, H.rhs[l], shift_sum, zero_init ? 1 : 0, H.rhs[l + 1],
                                h->o.omega, skip);
        std::swap(cur, alt);
    } else if (h->o.restrict64) {
        // residual stored in whichever of the level's two iterate buffers the
        // smoothing left free, then the 64-point restriction
        smooth(h, H, l, h->o.nu1, 0, cur, alt, shift_sum, zero_init);
        T* res = cur == H.e[l] ? H.tmp[l] : H.e[l];
        Prof pf(h, MG_K_RESTRICT, restrict_bytes + 2.0 * d.ncell() * sizeof(T));
        int nbr = 0;
        const ColGrid G = zgrid(d.nx / 2, d.ny, d.nz, false, &nbr);
        s.x(k_resid_cells<T, 2, 2>, nbr, CBX * CBY, H.L[l], cur, H.rhs[l], G, nullptr, nullptr, h->part, res);
        s.x(k_restrict64<T>, lin_grid(c.ncell()).x, 256, (const T*)res, d.nx, d.ny, d.nz, H.rhs[l + 1]);
    } else {
        smooth(h, H, l, h->o.nu1, 0, cur, alt, shift_sum, zero_init);
        Prof pf(h, MG_K_RESTRICT, restrict_bytes);
        launch_restrict<T>(s, H.L[l], cur, H.rhs[l], H.rhs[l + 1]);
    }
    vcycle(h, H, l + 1, nullptr, true);   // the coarse correction starts from zero
    {
        Prof pf(h, MG_K_PROLONG, (2.0 * d.ncell() + 2.0 * c.ncell()) * sizeof(T));
        int nbp = 0;
        // columns: coarse x by fine y; chunks of coarse planes (FP32: about 16384 workgroups,
        // chunks of 8 coarse planes at 512^3; 8192 measured 11% faster than 2048 there and
        // 16384 a little faster again; FP64 is faster with 2048)
        const ColGrid G = zgrid(c.nx, d.ny, c.nz, false, &nbp, sizeof(T) == 4 ? 16384 : 2048);
        s.x(k_prolong_col<T>, nbp, CBX * CBY, H.e[l + 1], H.a[l + 1], c.nx, c.ny, c.nz, G, cur);
    }
    smooth(h, H, l, h->o.nu2, 1, cur, alt, nullptr, false, upd, upd_done);
    if (cur != H.e[l]) {
        Prof pf(h, MG_K_OTHER, 2.0 * d.ncell() * sizeof(T));
        s.x(k_copy<T>, lin_grid(d.ncell()).x, 256, H.e[l], cur, d.ncell());
    }
}

// Run partial-sum kernel output through k_finish2 into scal[slot], scal[slot+1]:
// in one workgroup for a few thousand pairs, else in two stages (the finest-level
// residual of a 512^3 grid leaves 131072 pairs, 55 us for one workgroup).
static void finish(mg_handle* h, int nblk, int slot) {
    Prof pf(h, MG_K_OTHER, 16.0 * nblk);
    const Launcher s = launcher(h);
    if (nblk > 4 * FIN_THREADS) {
        const int per = (nblk + FIN_PARTS - 1) / FIN_PARTS, g = (nblk + per - 1) / per;
        double* p2 = h->part + (size_t)2 * h->L.max_blocks;
        s.x(k_finish2_part, g, FIN_THREADS, (const double*)h->part, nblk, per, p2);
        s.x(k_finish2, 1, FIN_THREADS, (const double*)p2, g, h->scal + slot);
    } else {
        s.x(k_finish2, 1, FIN_THREADS, (const double*)h->part, nblk, h->scal + slot);
    }
}

static void build_hier(mg_handle* h, double* p, Hier<double>& H64, Hier<float>& H32) {
    const Layout& L = h->L;
    H64.nlev = H32.nlev = L.nlev;
    H64.d = H32.d = L.d;
    for (int l = 0; l < L.nlev; l++) {
        const LevelDims& d = L.d[l];
        H64.L[l] = Lvl<double>{d.nx, d.ny, d.nz, h->bx[l], h->by[l], h->bz[l]};
        H64.e[l] = l == 0 ? p : h->e[l];
        H64.rhs[l] = l == 0 ? h->bbar : h->rhs[l];
        H64.tmp[l] = h->tmp[l];
        H64.a[l] = h->a[l];
        if (h->o.precision == MG_FP32_REFINED) {
            H32.L[l] = Lvl<float>{d.nx, d.ny, d.nz, h->fbx[l], h->fby[l], h->fbz[l]};
            H32.e[l] = h->fe[l];
            H32.rhs[l] = h->frhs[l];
            H32.tmp[l] = h->ftmp[l];
            H32.a[l] = h->fa[l];
        }
    }
}

// Residual pass over level 0 (FP64; MODE as k_resid_col): the cell-pair
// kernel when nx is even.  Returns the number of partial-sum blocks.  The flat
// kernel serves the modes that write the residual where it fits; the norm alone
// (MODE 0) is faster marching columns (512^3: 0.91 against 0.99 ms).
template <int MODE>
static int launch_resid(const Launcher& s, const Lvl<double>& L, const double* p, const double* b,
                        const double* inv_s, float* r32, double* part, double* r64 = nullptr) {
    int nb = 0;
    if (MODE != 0 && resid_flat_fits(LevelDims{L.nx, L.ny, L.nz}) && ((uintptr_t)p & 15) == 0 &&
        ((uintptr_t)b & 15) == 0) {
        const uint32_t units = (uint32_t)((size_t)L.nx * L.ny * L.nz / 2);
        nb = (int)((units + RES_FLAT_THREADS - 1) / RES_FLAT_THREADS);
        s.x(k_resid_flat<MODE>, nb, RES_FLAT_THREADS, L, p, b, units, inv_s, r32, part, r64);
    } else if ((L.nx & 1) == 0 && ((uintptr_t)p & 15) == 0) {
        const ColGrid G = zgrid(L.nx / 2, L.ny, L.nz, false, &nb);
        s.x(k_resid_cells<double, 2, MODE>, nb, CBX * CBY, L, p, b, G, inv_s, r32, part, r64);
    } else {
        const ColGrid G = zgrid(L.nx, L.ny, L.nz, false, &nb);
        s.x(k_resid_col<double, MODE>, nb, CBX * CBY, L, p, b, G, inv_s, r32, part, r64);
    }
    return nb;
}

// Step 1a (asynchronous): project b, initial residual, and the copy of the
// scalars (sum b, sum b^2, sum b_bar, sum b_bar^2, sum r^2, sum p) to h->host.
mg_status solve_begin_launch(SolveState& S) {
    mg_handle* h = S.h;
    S.t0 = std::chrono::steady_clock::now();
    prof_reset(h);
    memset(&S.st, 0, sizeof S.st);
    S.st.levels = h->L.nlev;
    S.it = 0;
    const LevelDims& d0 = h->L.d[0];
    const double N = (double)d0.ncell();
    const Launcher s = launcher(h);
    const dim3 g0 = col_grid(d0.nx, d0.ny, d0.nz), blk(BX, BY);
    const int nb0 = (int)(g0.x * g0.y * g0.z);
    const bool f32 = h->o.precision == MG_FP32_REFINED;
    Lvl<double> L64{d0.nx, d0.ny, d0.nz, h->bx[0], h->by[0], h->bz[0]};
    {
        Prof pf(h, MG_K_OTHER, 8.0 * N);
        s.z(k_sum_sq<double>, g0, blk, S.rhs, d0.nx, d0.ny, d0.nz, h->part);
    }
    finish(h, nb0, 0);
    {
        Prof pf(h, MG_K_OTHER, 16.0 * N);
        s.z(k_project, g0, blk, S.rhs, h->bbar, (const double*)h->scal, d0.nx, d0.ny, d0.nz, h->part);
    }
    finish(h, nb0, 2);
    const double resid_bytes = (2.0 * N + d0.nfaces()) * 8.0;
    int nbz = 0;
    if (f32) {
        // first FP32 right-hand side scaled by a power of two near the RMS of b_bar
        s.x(k_refine_scale, 1, 64, (const double*)(h->scal + 3), N, h->scal + 8);
        Prof pf(h, MG_K_REFINE, resid_bytes + 4.0 * N);
        nbz = launch_resid<1>(s, L64, S.p, h->bbar, h->scal + 9, h->frhs[0], h->part);
    } else if (h->o.krylov == MG_KRYLOV_FCG) {
        {
            Prof pf(h, MG_K_KRYLOV, resid_bytes + 8.0 * N);
            nbz = launch_resid<2>(s, L64, S.p, h->bbar, nullptr, nullptr, h->part, h->kr);
        }
        // no previous direction: s = q = 0 and s.q = 0 (so the first beta is 0)
        Prof pf(h, MG_K_KRYLOV, 16.0 * N);
        s.x(k_fill<double>, lin_grid(d0.ncell()).x, 256, h->ks, d0.ncell(), 0.0);
        s.x(k_fill<double>, lin_grid(d0.ncell()).x, 256, h->kq, d0.ncell(), 0.0);
        s.x(k_fill<double>, 1, 64, h->scal + 12, (size_t)1, 0.0);
    } else {
        Prof pf(h, MG_K_NORM, resid_bytes);
        nbz = launch_resid<0>(s, L64, S.p, h->bbar, nullptr, nullptr, h->part);
    }
    finish(h, nbz, 4);
    S.project = true;  // scal[5] now holds sum(p); p is made mean-zero lazily
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->host, h->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return MG_OK;
}

// Step 1b (after h->stream is synchronised): history[0], status.  A zero
// right-hand side gives p = 0 (one blocking fill).
mg_status solve_begin_finish(SolveState& S) {
    mg_handle* h = S.h;
    const LevelDims& d0 = h->L.d[0];
    const double N = (double)d0.ncell();
    S.st.mean_b = h->host[0] / N;
    S.norm_b = std::sqrt(h->host[3]);
    S.st.norm_b = S.norm_b;
    if (S.norm_b == 0.0) {
        launcher(h).x(k_fill<double>, lin_grid(d0.ncell()).x, 256, S.p, d0.ncell(), 0.0);
        HIPCHK(hipStreamSynchronize(h->stream));
        S.project = false;
        S.st.nhist = 1;
        S.st.history[0] = 0.0;
        S.rho0 = S.rho = 0.0;
        S.status = MG_OK;
        return MG_OK;
    }
    S.rho0 = S.rho = std::sqrt(h->host[4]) / S.norm_b;
    S.st.history[0] = S.rho0;
    S.st.nhist = 1;
    S.status = S.rho0 <= S.tol ? MG_OK : MG_E_NOT_CONVERGED;
    return MG_OK;
}

// Step 2 (asynchronous): one V-cycle (FP64) or one outer refinement iteration,
// the new residual norm and sum(p), and the copy of both to h->host.  The
// mean-zero projection of p after each iteration is folded into the next pass
// that rewrites p (the first fused pre-smoothing sweep, or the refinement
// update) and, after the last iteration, done by solve_end.  The caller
// synchronises h->stream before solve_after_sync.
mg_status launch_iteration_kernels(SolveState& S) {
    mg_handle* h = S.h;
    const LevelDims& d0 = h->L.d[0];
    const double N = (double)d0.ncell();
    const Launcher s = launcher(h);
    const dim3 g0 = col_grid(d0.nx, d0.ny, d0.nz), blk(BX, BY);
    const bool f32 = h->o.precision == MG_FP32_REFINED;
    const double resid_bytes = (2.0 * N + d0.nfaces()) * 8.0;
    Lvl<double> L64{d0.nx, d0.ny, d0.nz, h->bx[0], h->by[0], h->bz[0]};
    Hier<double> H64;
    Hier<float> H32;
    build_hier(h, S.p, H64, H32);
    int nbz = 0;
    if (h->o.krylov == MG_KRYLOV_FCG) {
        // z = V(r) from zero, then the direction, the update and the new residual
        Hier<double> HK = H64;
        HK.e[0] = h->kz;
        HK.rhs[0] = h->kr;
        vcycle(h, HK, 0, nullptr, true);
        {
            Prof pf(h, MG_K_KRYLOV, 24.0 * N);
            s.z(k_fcg_dots, g0, blk, (const double*)h->kz, (const double*)h->kq, (const double*)h->kr, d0.nx, d0.ny,
                d0.nz, h->part);
        }
        finish(h, (int)(g0.x * g0.y * g0.z), 10);
        s.x(k_fcg_beta, 1, 64, h->scal);
        {
            Prof pf(h, MG_K_KRYLOV, (3.0 * N + d0.nfaces()) * 8.0);
            int nbd = 0;
            if ((d0.nx & 1) == 0) {
                const ColGrid G = zgrid(d0.nx / 2, d0.ny, d0.nz, false, &nbd);
                s.x(k_fcg_direction<2>, nbd, CBX * CBY, L64, (const double*)h->kz, (const double*)h->ks,
                    (const double*)h->scal, G, h->kq, h->part);
            } else {
                const ColGrid G = zgrid(d0.nx, d0.ny, d0.nz, false, &nbd);
                s.x(k_fcg_direction<1>, nbd, CBX * CBY, L64, (const double*)h->kz, (const double*)h->ks,
                    (const double*)h->scal, G, h->kq, h->part);
            }
            finish(h, nbd, 12);
        }
        {
            Prof pf(h, MG_K_KRYLOV, 40.0 * N);
            s.x(k_fcg_update, lin_grid(d0.ncell()).x, 256, (const double*)h->kz, h->ks, S.p, (const double*)h->scal,
                d0.ncell());
        }
        Prof pf(h, MG_K_KRYLOV, resid_bytes + 8.0 * N);
        nbz = launch_resid<2>(s, L64, S.p, h->bbar, nullptr, nullptr, h->part, h->kr);
    } else if (!f32) {
        const double* shift = h->scal + 5;
        if (!fused_first_sweep(h)) {
            Prof pf(h, MG_K_OTHER, 16.0 * N);
            s.z(k_sub_mean<double>, g0, blk, S.p, (const double*)(h->scal + 5), d0.nx, d0.ny, d0.nz);
            shift = nullptr;
        }
        vcycle(h, H64, 0, shift);
        Prof pf(h, MG_K_NORM, resid_bytes);
        nbz = launch_resid<0>(s, L64, S.p, h->bbar, nullptr, nullptr, h->part);
    } else {
        // e starts from zero; from the second inner cycle on, the previous cycle's
        // post-smoothing (nu2 >= 1 sweeps, black then red) has left the red cells
        // of level 0 exactly where the next pre-smoothing's red half-sweep would put them
        // the last cycle's final level-0 pass applies the update p <- (p - mean) + s e
        // where its variant allows
        const RefineUpd upd{S.p, h->scal + 8, h->scal + 5};
        bool upd_done = false;
        for (int m = 0; m < h->o.inner_m; m++)
            vcycle(h, H32, 0, nullptr, m == 0, m > 0 && h->o.nu2 >= 1, m + 1 == h->o.inner_m ? &upd : nullptr,
                   &upd_done);
        if (!upd_done) {
            Prof pf(h, MG_K_REFINE, 20.0 * N);
            if ((d0.ncell() & 1) == 0 && ((uintptr_t)S.p & 15) == 0)
                s.x(k_refine_update2, (unsigned)((d0.ncell() / 2 + 511) / 512), 512, S.p, (const float*)h->fe[0],
                    (const double*)(h->scal + 8), d0.ncell(), (const double*)(h->scal + 5));
            else
                s.x(k_refine_update, lin_grid(d0.ncell()).x, 256, S.p, (const float*)h->fe[0],
                    (const double*)(h->scal + 8), d0.ncell(), (const double*)(h->scal + 5));
        }
        // r32 of the next step is scaled by a power of two near the RMS of the
        // residual just used (any power of two leaves the FP32 arithmetic unchanged)
        s.x(k_refine_scale, 1, 64, (const double*)(h->scal + 4), N, h->scal + 8);
        Prof pf(h, MG_K_REFINE, resid_bytes + 4.0 * N);
        nbz = launch_resid<1>(s, L64, S.p, h->bbar, h->scal + 9, h->frhs[0], h->part);
    }
    finish(h, nbz, 4);
    HIPCHK(hipGetLastError());
    if (h->launch_failed) {
        h->launch_failed = 0;
        set_error("a column-grid launch of this batch would exceed the grid's z limit");
        return MG_E_HIP;
    }
    return MG_OK;
}

void launch_gather(mg_handle* h, double* out) {
    launcher(h).x(k_gather2, 1, 64, (const double*)(h->scal + 4), out);
}

mg_status solve_launch_iteration(SolveState& S) {
    mg_handle* h = S.h;
    hipStream_t s = h->stream;
    if (h->o.graph && !h->o.profile && !S.graph_failed) {
        if (!S.gexec) {
            // record this iteration's launches once and build the graph from them (no
            // stream capture); on any failure fall back to direct launches
            S.rec = std::make_shared<Recording>();
            h->rec = S.rec.get();
            const mg_status r = launch_iteration_kernels(S);
            h->rec = nullptr;
            if (r != MG_OK || build_graph(*S.rec, &S.graph, &S.gexec) != hipSuccess) {
                (void)hipGetLastError();
                S.graph_failed = true;
                S.graph = nullptr;
                S.gexec = nullptr;
                S.rec.reset();
            }
        }
        if (S.gexec) {
            HIPCHK(hipGraphLaunch(S.gexec, s));
            HIPCHK(hipMemcpyAsync(h->host, h->scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            return MG_OK;
        }
    }
    const mg_status r = launch_iteration_kernels(S);
    if (r != MG_OK) return r;
    HIPCHK(hipMemcpyAsync(h->host, h->scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    return MG_OK;
}

// Step 3 (after the stream is synchronised): record the residual, test convergence.
void solve_after_sync(SolveState& S) {
    S.it++;
    S.st.cycles += S.h->o.precision == MG_FP32_REFINED ? S.h->o.inner_m : 1;
    S.rho = std::sqrt(S.h->host[0]) / S.norm_b;
    if (S.st.nhist < MG_MAX_HISTORY) S.st.history[S.st.nhist++] = S.rho;
    if (!(S.rho == S.rho) || S.rho > 1e6 * S.rho0)
        S.status = MG_E_DIVERGED;
    else if (S.rho <= S.tol)
        S.status = MG_OK;
    else
        S.status = MG_E_NOT_CONVERGED;
}

bool solve_running(const SolveState& S) {
    return S.status == MG_E_NOT_CONVERGED && S.it < S.h->o.max_cycles;
}

// Release the captured iteration graph, if any.
void solve_release(SolveState& S) {
    if (S.gexec) (void)hipGraphExecDestroy(S.gexec);
    if (S.graph) (void)hipGraphDestroy(S.graph);
    S.gexec = nullptr;
    S.graph = nullptr;
    S.rec.reset();
}

// Step 4: final mean-zero projection of p (sum(p) from the last residual pass),
// enqueued (solve_end_launch); then statistics (solve_end_finish, once the stream
// has passed it).  solve_end does both, blocking.
void solve_end_launch(SolveState& S) {
    mg_handle* h = S.h;
    if (S.project) {
        const LevelDims& d0 = h->L.d[0];
        Prof pf(h, MG_K_OTHER, 16.0 * d0.ncell());
        if ((d0.ncell() & 1) == 0 && ((uintptr_t)S.p & 15) == 0)
            launcher(h).x(k_sub_mean2, (unsigned)((d0.ncell() / 2 + 511) / 512), 512, S.p,
                          (const double*)(h->scal + 5), d0.ncell());
        else
            launcher(h).z(k_sub_mean<double>, col_grid(d0.nx, d0.ny, d0.nz), dim3(BX, BY), S.p,
                          (const double*)(h->scal + 5), d0.nx, d0.ny, d0.nz);
        S.project = false;
    }
}

void solve_end_finish(SolveState& S, mg_stats* st) {
    mg_handle* h = S.h;
    solve_release(S);
    S.st.outer = S.it;
    if (h->o.precision == MG_FP64) S.st.cycles = S.it;
    S.st.rel_residual = S.rho;
    S.st.gamma = S.it > 0 && S.rho0 > 0 ? std::pow(S.rho / S.rho0, 1.0 / S.it) : 0.0;
    S.st.status = S.status;
    prof_collect(h);
    for (int c = 0; c < MG_K_COUNT; c++) {
        S.st.kernel_ms[c] = h->kernel_ms[c];
        S.st.kernel_launches[c] = h->kernel_launches[c];
        S.st.kernel_bytes[c] = h->kernel_bytes[c];
    }
    S.st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - S.t0).count();
    if (st) *st = S.st;
}

void solve_end(SolveState& S, mg_stats* st) {
    solve_end_launch(S);
    (void)hipStreamSynchronize(S.h->stream);
    solve_end_finish(S, st);
}

mg_status solve_impl(mg_handle* h, const double* rhs, double* p, double tol, mg_stats* st) {
    SolveState S;
    S.h = h;
    S.rhs = rhs;
    S.p = p;
    S.tol = tol;
    mg_status r = solve_begin_launch(S);
    if (r == MG_OK) r = hipStreamSynchronize(h->stream) == hipSuccess ? MG_OK : MG_E_HIP;
    if (r == MG_OK) r = solve_begin_finish(S);
    if (r != MG_OK) return r;
    while (solve_running(S)) {
        r = solve_launch_iteration(S);
        if (r == MG_OK && hipStreamSynchronize(h->stream) != hipSuccess) {
            set_error("hipStreamSynchronize failed during the solve");
            r = MG_E_HIP;
        }
        if (r != MG_OK) {
            solve_release(S);
            return r;
        }
        solve_after_sync(S);
    }
    solve_end(S, st);
    if (S.status == MG_E_NOT_CONVERGED) set_error("max_cycles reached before the tolerance");
    if (S.status == MG_E_DIVERGED) set_error("residual diverged");
    return (mg_status)S.status;
}

mg_status check_solve_arrays(const double* rhs, const double* p) {
    if (((uintptr_t)rhs & 15) || ((uintptr_t)p & 15)) {
        set_error("rhs and p must be 16-byte aligned");
        return MG_E_INVALID;
    }
    return MG_OK;
}

const char* last_error() { return g_err.c_str(); }

}  // namespace mgrt

// ====================================================================== C ABI

using namespace mgrt;

extern "C" {

mg_status mg_default_options(mg_options* o) {
    if (!o) return MG_E_INVALID;
    o->precision = MG_FP64;
    o->nu1 = 2;
    o->nu2 = 2;
    o->n_coarsest = 4;
    o->inner_m = 3;
    o->max_cycles = 100;
    o->profile = 0;
    o->tile = 0;
    o->graph = 0;
    o->krylov = MG_KRYLOV_NONE;
    o->omega = 1.0;
    o->restrict64 = 0;
    o->coarse_gmres = 0;
    o->coarse_gmres_maxit = 200;
    o->coarse_gmres_tol = 1e-3;
    return MG_OK;
}

mg_status mg_workspace_bytes(const mg_grid* g, const mg_options* o, size_t* bytes) {
    if (!bytes) {
        set_error("null argument");
        return MG_E_INVALID;
    }
    Layout L;
    mg_status r = plan(g, o, &L);
    if (r != MG_OK) return r;
    *bytes = L.total;
    return MG_OK;
}

mg_status mg_setup(const mg_grid* g, const mg_options* o, const double* bx, const double* by, const double* bz,
                   mg_bc bc, void* ws, size_t ws_bytes, void* stream, mg_handle** out) {
    try {
        if (!out || !bx || !by || !bz) {
            set_error("null argument");
            return MG_E_INVALID;
        }
        *out = nullptr;
        if (bc != MG_BC_NEUMANN) {
            set_error("only MG_BC_NEUMANN is supported");
            return MG_E_INVALID;
        }
        mg_handle* h = new mg_handle();
        h->g = *g;
        h->o = *o;
        mg_status r = plan(g, o, &h->L);
        if (r != MG_OK) {
            delete h;
            return r;
        }
        if (!ws || ((uintptr_t)ws & 255) || ws_bytes < h->L.total) {
            set_error("workspace missing, not 256-byte aligned, or smaller than mg_workspace_bytes");
            delete h;
            return MG_E_WORKSPACE;
        }
        h->ws = (char*)ws;
        h->stream = (hipStream_t)stream;
        if (hipHostMalloc((void**)&h->host, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            h->host = nullptr;
            set_error("hipHostMalloc failed");
            mg_destroy(h);
            return MG_E_HIP;
        }
        r = setup_launch(h, bx, by, bz);
        if (r == MG_OK) r = hipStreamSynchronize(h->stream) == hipSuccess ? MG_OK : MG_E_HIP;
        if (r == MG_OK) r = setup_finish(h);
        if (r != MG_OK) {
            mg_destroy(h);
            return r;
        }
        *out = h;
        return MG_OK;
    } catch (...) {
        set_error("host exception in mg_setup");
        return MG_E_HIP;
    }
}

mg_status mg_solve(mg_handle* h, const double* rhs, double* p, double tol, mg_stats* st, void* stream) {
    try {
        if (!h || !rhs || !p || !(tol >= 0) || !std::isfinite(tol)) {
            set_error("null handle/array or invalid tolerance");
            return MG_E_INVALID;
        }
        if (check_solve_arrays(rhs, p) != MG_OK) return MG_E_INVALID;
        h->stream = (hipStream_t)stream;
        return solve_impl(h, rhs, p, tol, st);
    } catch (...) {
        set_error("host exception in mg_solve");
        return MG_E_HIP;
    }
}

void mg_destroy(mg_handle* h) {
    if (!h) return;
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->host) (void)hipHostFree(h->host);
    delete h;
}

mg_status mg_level_dims(const mg_handle* h, int l, int* nx, int* ny, int* nz) {
    if (!h || l < 0 || l >= h->L.nlev || !nx || !ny || !nz) {
        set_error("bad handle or level");
        return MG_E_INVALID;
    }
    *nx = h->L.d[l].nx;
    *ny = h->L.d[l].ny;
    *nz = h->L.d[l].nz;
    return MG_OK;
}

mg_status mg_level_tile(const mg_handle* h, int l, int* tile) {
    if (!h || l < 0 || l >= h->L.nlev || !tile) {
        set_error("bad handle or level");
        return MG_E_INVALID;
    }
    *tile = h->tile[l];
    return MG_OK;
}

mg_status mg_copy_level(const mg_handle* h, int l, double* bx, double* by, double* bz, double* a, void* stream) {
    if (!h || l < 0 || l >= h->L.nlev) {
        set_error("bad handle or level");
        return MG_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const LevelDims& d = h->L.d[l];
    if (bx || by || bz) {
        k_faces_to_api<<<lin_grid(d.nfx() + d.nfy() + d.nfz()), 256, 0, s>>>(h->bx[l], h->by[l], h->bz[l], bx, by, bz,
                                                                             d.nx, d.ny, d.nz);
        HIPCHK(hipGetLastError());
    }
    if (a) HIPCHK(hipMemcpyAsync(a, h->a[l], d.ncell() * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return MG_OK;
}

const char* mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "MG_OK";
        case MG_PENDING: return "MG_PENDING";
        case MG_E_INVALID: return "MG_E_INVALID: invalid argument";
        case MG_E_WORKSPACE: return "MG_E_WORKSPACE: workspace missing, misaligned or too small";
        case MG_E_HIP: return "MG_E_HIP: HIP runtime error";
        case MG_E_NOT_CONVERGED: return "MG_E_NOT_CONVERGED: tolerance not reached within max_cycles";
        case MG_E_DIVERGED: return "MG_E_DIVERGED: residual diverged";
        case MG_E_BUDGET: return "MG_E_BUDGET: request larger than the server arena";
        case MG_E_NOT_FOUND: return "MG_E_NOT_FOUND: unknown ticket";
    }
    return "unknown status";
}

const char* mg_last_error(void) { return mgrt::last_error(); }

}  // extern "C"
