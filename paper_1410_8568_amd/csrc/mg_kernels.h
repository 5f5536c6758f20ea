// Device kernels of the multigrid pressure solve (gfx950).
//
// Every kernel here is bandwidth-bound stencil or transfer work; none is a dense
// contraction, so none uses MFMA.  Every device array of a level is [k][j][i]
// with i fastest and n_x n_y n_z entries, so all arrays share one index c and
// every row starts on the same alignment.  The face coefficients are stored as
// "lower face of each cell": fx[c] is the x-face between cells i-1 and i, fy[c]
// the y-face between rows j-1 and j, fz[c] the z-face between planes k-1 and k;
// the lower wall faces hold 0 and the upper wall faces are not stored (reads of
// them are guarded and give 0).  Out-of-grid neighbour values read as 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mg_device.h"

namespace mgk {

constexpr int BX = 64;   // threads along i (one wavefront)
constexpr int BY = 4;    // rows per block
constexpr int RED_THREADS = 256;
constexpr int FIN_THREADS = 1024;
constexpr int FIN_PARTS = 256;   // first-stage workgroups of a two-stage final sum

__device__ __forceinline__ size_t cidx(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * nx + i;
}
template <class T>
struct Lvl {
    int nx, ny, nz;
    const T* fx;  // lower x-face of each cell
    const T* fy;  // lower y-face
    const T* fz;  // lower z-face
    __device__ __forceinline__ Lvl rebased(uintptr_t off) const { return {nx, ny, nz, rb(fx, off), rb(fy, off), rb(fz, off)}; }
};

// The six face coefficients of cell (i,j,k) at index c, in the order x-, x+,
// y-, y+, z-, z+ (upper wall faces are 0).
template <class T>
__device__ __forceinline__ void faces6(const Lvl<T>& L, int i, int j, int k, size_t c, T& w0, T& w1, T& w2, T& w3,
                                       T& w4, T& w5) {
    w0 = L.fx[c];
    w1 = i < L.nx - 1 ? L.fx[c + 1] : T(0);
    w2 = L.fy[c];
    w3 = j < L.ny - 1 ? L.fy[c + L.nx] : T(0);
    w4 = L.fz[c];
    w5 = k < L.nz - 1 ? L.fz[c + (size_t)L.nx * L.ny] : T(0);
}

// Gauss-Seidel update value and the neighbour sum of eq. (10) from the six face
// coefficients and neighbour values, faces in the order x-, x+, y-, y+, z-, z+.
// Explicit fma order, so every kernel that evaluates the stencil (fused or not)
// produces bit-identical results.
template <class T>
__device__ __forceinline__ T stencil_sum(T w0, T w1, T w2, T w3, T w4, T w5, T p0, T p1, T p2, T p3, T p4,
                                         T p5) {
    T acc = w0 * p0;
    acc = fma(w1, p1, acc);
    acc = fma(w2, p2, acc);
    acc = fma(w3, p3, acc);
    acc = fma(w4, p4, acc);
    acc = fma(w5, p5, acc);
    return acc;
}

template <class T>
__device__ __forceinline__ T stencil_diag(T w0, T w1, T w2, T w3, T w4, T w5) {
    return ((((w0 + w1) + w2) + w3) + w4) + w5;
}

// Quotient num / d of the cycle kernels.  FP32: the hardware reciprocal (within
// 1 ulp) and one Newton correction of the quotient from its exact fma residual,
// which is within about half an ulp (and almost always equal to the correctly
// rounded quotient) at a fraction of the cost of the full IEEE division
// sequence.  FP64 divides exactly.
__device__ __forceinline__ float quot(float num, float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = num * r;
    return fmaf(fmaf(-d, q, num), r, q);
}
__device__ __forceinline__ double quot(double num, double d) { return num / d; }

// ---------------------------------------------------------------- prolongation corner values
//
// Flux-conserving prolongation (eqs. 13-14, extended to the octant corners of a
// 3-D cell): the fine child of coarse cell C on x side sx (C - 1 or C + 1), y
// side sy and z side sz gets (1/8) * sum over the 8 corners T of its octant of
// V_T = sum(a e) / sum(a) over the 2^|T| coarse cells that share corner T (T =
// {} is C itself, V = e_C), a being the coarse cell weight.  A corner's cells
// are summed with C first, then its x neighbour, y neighbour, x-y neighbour,
// lower plane before upper; the corners in the order {}, x, y, xy, z, xz, yz,
// xyz.  The products a e are formed with contraction off, so every kernel that
// applies the prolongation through these helpers gets the same bits, whatever
// its launch shape (a contracted product would be rounded differently in a
// kernel's prologue and in its loop).

// One coarse plane as seen from one fine x-pair: a and w = a e at columns
// (I, I - 1, I + 1) of row J and of the y-side row Jy (walls: clamped), and e_C.
template <class T>
struct ProPlane {
    T a0, am, ap, ay0, aym, ayp;
    T w0, wm, wp, wy0, wym, wyp;
    T e0;
};
template <class T>
__device__ __forceinline__ ProPlane<T> pro_plane(T a0, T am, T ap, T ay0, T aym, T ayp, T e0, T em, T ep, T ey0,
                                                 T eym, T eyp) {
#pragma clang fp contract(off)
    ProPlane<T> c;
    c.a0 = a0; c.am = am; c.ap = ap; c.ay0 = ay0; c.aym = aym; c.ayp = ayp;
    c.e0 = e0;
    c.w0 = a0 * e0; c.wm = am * em; c.wp = ap * ep;
    c.wy0 = ay0 * ey0; c.wym = aym * eym; c.wyp = ayp * eyp;
    return c;
}

// Corners on the face between coarse planes lo (below) and up: z, yz and, per
// child (0: x side I - 1, 1: I + 1), xz and xyz.
template <class T>
struct ProFace {
    T z, yz, xz[2], xyz[2];
};
template <class T>
__device__ __forceinline__ ProFace<T> pro_face(const ProPlane<T>& lo, const ProPlane<T>& up) {
#pragma clang fp contract(off)
    ProFace<T> f;
    f.z = quot(lo.w0 + up.w0, lo.a0 + up.a0);
    f.yz = quot(((lo.w0 + lo.wy0) + up.w0) + up.wy0, ((lo.a0 + lo.ay0) + up.a0) + up.ay0);
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const T lax = e ? lo.ap : lo.am, lwx = e ? lo.wp : lo.wm;
        const T lay = e ? lo.ayp : lo.aym, lwy = e ? lo.wyp : lo.wym;
        const T uax = e ? up.ap : up.am, uwx = e ? up.wp : up.wm;
        const T uay = e ? up.ayp : up.aym, uwy = e ? up.wyp : up.wym;
        f.xz[e] = quot(((lo.w0 + lwx) + up.w0) + uwx, ((lo.a0 + lax) + up.a0) + uax);
        f.xyz[e] = quot(((((((lo.w0 + lwx) + lo.wy0) + lwy) + up.w0) + uwx) + up.wy0) + uwy,
                        ((((((lo.a0 + lax) + lo.ay0) + lay) + up.a0) + uax) + up.ay0) + uay);
    }
    return f;
}

// Sum over the octant corners of child e of coarse plane c0 whose z corners are
// those of face f (unscaled: the correction is 1/8 of it).
template <class T>
__device__ __forceinline__ T pro_child(const ProPlane<T>& c0, const ProFace<T>& f, int e) {
#pragma clang fp contract(off)
    const T vy = quot(c0.w0 + c0.wy0, c0.a0 + c0.ay0);
    const T ax = e ? c0.ap : c0.am, wx = e ? c0.wp : c0.wm;
    const T axy = e ? c0.ayp : c0.aym, wxy = e ? c0.wyp : c0.wym;
    T t = c0.e0;
    t += quot(c0.w0 + wx, c0.a0 + ax);
    t += vy;
    t += quot(((c0.w0 + wx) + c0.wy0) + wxy, ((c0.a0 + ax) + c0.ay0) + axy);
    return (((t + f.z) + f.xz[e]) + f.yz) + f.xyz[e];
}

// Successive over-relaxation of a Gauss-Seidel value g (feature 5): the cell
// moves omega times the Gauss-Seidel step from its current value c[oc].  The
// reference kernel forms the same expression, so both agree bit for bit.
// Without SOR (omega = 1) this is g itself, compiled without the extra read.
template <bool SOR, class T>
__device__ __forceinline__ T sor(T g, const T* c, int oc, T omega) {
    if constexpr (SOR)
        return fma(omega, g - c[oc], c[oc]);
    else
        return g;
}

// Residual b - (s - d p) of one cell from its neighbour sum s and diagonal d,
// with the product taken in a fused multiply-add in every kernel that forms it
// (so all of them agree bit for bit).
template <class T>
__device__ __forceinline__ T resid_val(T b, T s, T d, T p) {
    return b - fma(-d, p, s);
}

// Neighbour sum s = sum_f beta_f p_nb and diagonal d = sum_f beta_f for cell
// (i,j,k); out-of-grid neighbours read as 0 (their face coefficient is 0).
template <class T>
__device__ __forceinline__ void nbsum(const Lvl<T>& L, const T* __restrict__ p, int i, int j, int k,
                                      T& s, T& d) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const size_t c = cidx(i, j, k, nx, ny);
    T w0, w1, w2, w3, w4, w5;
    faces6(L, i, j, k, c, w0, w1, w2, w3, w4, w5);
    T p0 = i > 0 ? p[c - 1] : T(0);
    T p1 = i < nx - 1 ? p[c + 1] : T(0);
    T p2 = j > 0 ? p[c - nx] : T(0);
    T p3 = j < ny - 1 ? p[c + nx] : T(0);
    T p4 = k > 0 ? p[c - (size_t)nx * ny] : T(0);
    T p5 = k < nz - 1 ? p[c + (size_t)nx * ny] : T(0);
    s = stencil_sum(w0, w1, w2, w3, w4, w5, p0, p1, p2, p3, p4, p5);
    d = stencil_diag(w0, w1, w2, w3, w4, w5);
}

// ---------------------------------------------------------------- reductions

// Deterministic block sum of two values; result valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
    __shared__ double sa[NT / 64], sb[NT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    if (lane == 0) { sa[wid] = a; sb[wid] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < NT / 64; w++) { ta += sa[w]; tb += sb[w]; }
        a = ta;
        b = tb;
    }
}

__device__ __forceinline__ int flat_tid() { return threadIdx.y * blockDim.x + threadIdx.x; }
// Flat index within its problem of a column-grid block whose z index within the
// problem is kz.
__device__ __forceinline__ int flat_bid(int kz) { return (kz * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x; }

// 2-D block (BX x BY) variant writing two partial sums per block; bid is the
// block's index within its problem.
__device__ __forceinline__ void block_partials2(double a, double b, double* __restrict__ part, int bid) {
    __shared__ double sa[BX * BY / 64], sb[BX * BY / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int t = flat_tid();
    if (t % 64 == 0) { sa[t / 64] = a; sb[t / 64] = b; }
    __syncthreads();
    if (t == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < BX * BY / 64; w++) { ta += sa[w]; tb += sb[w]; }
        part[2 * bid] = ta;
        part[2 * bid + 1] = tb;
    }
}

// out[q] = sum over blocks of part[2*blk+q] (q = 0,1), fixed order.  One block.
// First stage of the final sum of many partial pairs: workgroup g adds pairs
// [g per, min((g + 1) per, nblk)) in a fixed order into out[2g], out[2g + 1]
// (k_finish2 then adds the workgroups' results), so a large sum is spread over
// the chip instead of one CU.
__global__ void __launch_bounds__(FIN_THREADS) k_finish2_part(const double* __restrict__ part, int nblk, int per,
                                                              double* __restrict__ out, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    part = rb(part, off_);
    out = rb(out, off_);
    const int lo = bid_ * per, hi = min(nblk, lo + per);
    double a = 0, b = 0;
    for (int t = lo + (int)threadIdx.x; t < hi; t += FIN_THREADS) {
        a += part[2 * t];
        b += part[2 * t + 1];
    }
    block_sum2<FIN_THREADS>(a, b);
    if (threadIdx.x == 0) {
        out[2 * bid_] = a;
        out[2 * bid_ + 1] = b;
    }
}

__global__ void __launch_bounds__(FIN_THREADS) k_finish2(const double* __restrict__ part, int nblk,
                                                         double* __restrict__ out, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    part = rb(part, off_);
    out = rb(out, off_);
    double a = 0, b = 0;
    for (int t = threadIdx.x; t < nblk; t += FIN_THREADS) {
        a += part[2 * t];
        b += part[2 * t + 1];
    }
    block_sum2<FIN_THREADS>(a, b);
    if (threadIdx.x == 0) { out[0] = a; out[1] = b; }
}

// Partial sums of x and x^2 over the cells (column grid, k strided by gridDim.z).
template <class T>
__global__ void __launch_bounds__(BX* BY) k_sum_sq(const T* __restrict__ x, int nx, int ny, int nz,
                                                  double* __restrict__ part, Bt bt) {
    int kz_, nkz_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.z, gridDim.z, kz_, nkz_, off_)) return;
    x = rb(x, off_);
    part = rb(part, off_);
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, b = 0;
    if (i < nx && j < ny)
        for (int k = kz_; k < nz; k += nkz_) {
            double v = (double)x[cidx(i, j, k, nx, ny)];
            a += v;
            b += v * v;
        }
    block_partials2(a, b, part, flat_bid(kz_));
}

// y = x - sum/n (sum read from device memory); partial sums of y and y^2.
__global__ void __launch_bounds__(BX* BY) k_project(const double* __restrict__ x, double* __restrict__ y,
                                                   const double* __restrict__ sum, int nx, int ny, int nz,
                                                   double* __restrict__ part, Bt bt) {
    int kz_, nkz_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.z, gridDim.z, kz_, nkz_, off_)) return;
    x = rb(x, off_);
    y = rb(y, off_);
    sum = rb(sum, off_);
    part = rb(part, off_);
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    const double mean = sum[0] / ((double)nx * ny * nz);
    double a = 0, b = 0;
    if (i < nx && j < ny)
        for (int k = kz_; k < nz; k += nkz_) {
            size_t c = cidx(i, j, k, nx, ny);
            double v = x[c] - mean;
            y[c] = v;
            a += v;
            b += v * v;
        }
    block_partials2(a, b, part, flat_bid(kz_));
}

// x -= sum/n (sum from device memory).
template <class T>
__global__ void __launch_bounds__(BX* BY) k_sub_mean(T* __restrict__ x, const double* __restrict__ sum,
                                                    int nx, int ny, int nz, Bt bt) {
    int kz_, nkz_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.z, gridDim.z, kz_, nkz_, off_)) return;
    x = rb(x, off_);
    sum = rb(sum, off_);
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const double mean = sum[0] / ((double)nx * ny * nz);
    for (int k = kz_; k < nz; k += nkz_) {
        size_t c = cidx(i, j, k, nx, ny);
        x[c] = (T)((double)x[c] - mean);
    }
}

template <class T>
__global__ void k_fill(T* __restrict__ x, size_t n, T v, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    x = rb(x, off_);
    size_t t = (size_t)bid_ * blockDim.x + threadIdx.x;
    for (; t < n; t += (size_t)nb_ * blockDim.x) x[t] = v;
}

__global__ void k_cast_d2f(const double* __restrict__ x, float* __restrict__ y, size_t n) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t < n; t += (size_t)gridDim.x * blockDim.x) y[t] = (float)x[t];
}

// Scale of the FP32 right-hand side of the next refinement step: the power of
// two at or below the RMS of the residual whose sum of squares is sumsq[0]
// (1 for a zero residual); out[0] = s, out[1] = 1/s (both exact).  Any power of
// two gives the same FP32 arithmetic up to that scale.
__global__ void k_refine_scale(const double* __restrict__ sumsq, double n, double* __restrict__ out, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    sumsq = rb(sumsq, off_);
    out = rb(out, off_);
    if (threadIdx.x == 0 && bid_ == 0) {
        const double rms = sqrt(sumsq[0] / n);
        double s = 1.0;
        if (rms > 0.0 && rms < 1e300) s = ldexp(1.0, ilogb(rms));
        out[0] = s;
        out[1] = 1.0 / s;
    }
}

// ---------------------------------------------------------------- setup

// Caller faces (x: [nz][ny][nx+1], y: [nz][ny+1][nx], z: [nz+1][ny][nx]) to
// the lower-face layout, lower wall faces forced to 0; counts non-finite or
// non-positive interior coefficients into *bad.
__global__ void k_faces_from_api(const double* __restrict__ sx, const double* __restrict__ sy,
                                 const double* __restrict__ sz, double* __restrict__ fx, double* __restrict__ fy,
                                 double* __restrict__ fz, int nx, int ny, int nz, int* __restrict__ bad) {
    const size_t total = (size_t)nx * ny * nz;
    int nbad = 0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % nx);
        const size_t r = t / nx;
        const int j = (int)(r % ny), k = (int)(r / ny);
        double vx = 0.0, vy = 0.0, vz = 0.0;
        if (i > 0) {
            vx = sx[((size_t)k * ny + j) * (nx + 1) + i];
            if (!(vx > 0.0) || !(vx < 1e300)) nbad++;
        }
        if (j > 0) {
            vy = sy[((size_t)k * (ny + 1) + j) * nx + i];
            if (!(vy > 0.0) || !(vy < 1e300)) nbad++;
        }
        if (k > 0) {
            vz = sz[((size_t)k * ny + j) * nx + i];
            if (!(vz > 0.0) || !(vz < 1e300)) nbad++;
        }
        fx[t] = vx;
        fy[t] = vy;
        fz[t] = vz;
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Lower-face layout back to the caller layout (walls 0), for inspection.
__global__ void k_faces_to_api(const double* __restrict__ fx, const double* __restrict__ fy,
                               const double* __restrict__ fz, double* __restrict__ sx, double* __restrict__ sy,
                               double* __restrict__ sz, int nx, int ny, int nz) {
    const size_t tx = (size_t)(nx + 1) * ny * nz, ty = (size_t)nx * (ny + 1) * nz, tz = (size_t)nx * ny * (nz + 1);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tx + ty + tz;
         t += (size_t)gridDim.x * blockDim.x) {
        if (t < tx) {
            const int i = (int)(t % (nx + 1));
            const size_t r = t / (nx + 1);
            if (sx) sx[t] = i < nx ? fx[r * nx + i] : 0.0;
        } else if (t < tx + ty) {
            const size_t u = t - tx;
            const int i = (int)(u % nx);
            const size_t r = u / nx;
            const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
            if (sy) sy[u] = j < ny ? fy[((size_t)k * ny + j) * nx + i] : 0.0;
        } else {
            const size_t u = t - tx - ty;
            const size_t plane = (size_t)nx * ny;
            const size_t k = u / plane;
            if (sz) sz[u] = k < (size_t)nz ? fz[u] : 0.0;
        }
    }
}

// Coarse faces = mean of the 2 x 2 fine faces of the same orientation that the
// coarse face covers, ((f00 + f10) + (f01 + f11)) / 4, the first index along the
// first tangential axis.  One thread per coarse cell computes its three lower
// faces (the lower wall faces come out 0 from the fine wall faces).
__global__ void k_coarsen(const double* __restrict__ fx, const double* __restrict__ fy,
                          const double* __restrict__ fz, double* __restrict__ cx, double* __restrict__ cy,
                          double* __restrict__ cz, int fnx, int fny, int cnx, int cny, int cnz) {
    const size_t total = (size_t)cnx * cny * cnz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int I = (int)(t % cnx);
        const size_t r = t / cnx;
        const int J = (int)(r % cny), K = (int)(r / cny);
        const size_t f000 = cidx(2 * I, 2 * J, 2 * K, fnx, fny);
        const size_t dy = fnx, dz = (size_t)fnx * fny;
        cx[t] = 0.25 * ((fx[f000] + fx[f000 + dy]) + (fx[f000 + dz] + fx[f000 + dz + dy]));
        cy[t] = 0.25 * ((fy[f000] + fy[f000 + 1]) + (fy[f000 + dz] + fy[f000 + dz + 1]));
        cz[t] = 0.25 * ((fz[f000] + fz[f000 + 1]) + (fz[f000 + dy] + fz[f000 + dy + 1]));
    }
}

// Cell weight = mean of beta over the cell's interior faces (x-, x+, y-, y+, z-, z+).
__global__ void k_cell_weights(Lvl<double> L, double* __restrict__ a) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const size_t total = (size_t)nx * ny * nz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % nx);
        const size_t r = t / nx;
        const int j = (int)(r % ny), k = (int)(r / ny);
        double w0, w1, w2, w3, w4, w5;
        faces6(L, i, j, k, t, w0, w1, w2, w3, w4, w5);
        double s = 0;
        int cnt = 0;
        if (i > 0) { s += w0; cnt++; }
        if (i < nx - 1) { s += w1; cnt++; }
        if (j > 0) { s += w2; cnt++; }
        if (j < ny - 1) { s += w3; cnt++; }
        if (k > 0) { s += w4; cnt++; }
        if (k < nz - 1) { s += w5; cnt++; }
        a[t] = cnt ? s / cnt : 1.0;
    }
}

// Dense inverse of B = -L + (sigma/n) 1 1^T on the coarsest grid (one block,
// B in global memory, n <= 512): assemble, then in-place Gauss-Jordan without
// pivoting (B is symmetric positive definite, every pivot is positive).
// *bad is incremented if a pivot is not positive.
__global__ void __launch_bounds__(FIN_THREADS) k_coarse_invert(Lvl<double> L, double* __restrict__ B,
                                                               int* __restrict__ bad) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    __shared__ double rowk[512];
    __shared__ double colk[512];
    __shared__ double red[FIN_THREADS / 64];
    const int n = nx * ny * nz;
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += FIN_THREADS) B[t] = 0.0;
    __syncthreads();
    double dsum = 0;
    for (int c = tid; c < n; c += FIN_THREADS) {
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        double w0, w1, w2, w3, w4, w5;
        faces6(L, i, j, k, (size_t)c, w0, w1, w2, w3, w4, w5);
        double dg = 0;
        if (i > 0) { dg += w0; B[(size_t)c * n + c - 1] = -w0; }
        if (i < nx - 1) { dg += w1; B[(size_t)c * n + c + 1] = -w1; }
        if (j > 0) { dg += w2; B[(size_t)c * n + c - nx] = -w2; }
        if (j < ny - 1) { dg += w3; B[(size_t)c * n + c + nx] = -w3; }
        if (k > 0) { dg += w4; B[(size_t)c * n + c - nx * ny] = -w4; }
        if (k < nz - 1) { dg += w5; B[(size_t)c * n + c + nx * ny] = -w5; }
        B[(size_t)c * n + c] = dg;
        dsum += dg;
    }
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_down(dsum, off, 64);
    if (tid % 64 == 0) red[tid / 64] = dsum;
    __syncthreads();
    double sig = 0;
    for (int w = 0; w < FIN_THREADS / 64; w++) sig += red[w];
    const double shift = (sig / n) / n;
    __syncthreads();
    for (int t = tid; t < n * n; t += FIN_THREADS) B[t] += shift;
    __syncthreads();
    for (int k = 0; k < n; k++) {
        const double piv = B[(size_t)k * n + k];
        if (!(piv > 0.0)) {
            if (tid == 0) atomicAdd(bad, 1);
            return;
        }
        const double ip = 1.0 / piv;
        for (int j = tid; j < n; j += FIN_THREADS) {
            rowk[j] = (j == k) ? ip : B[(size_t)k * n + j] * ip;
            colk[j] = B[(size_t)j * n + k];
        }
        __syncthreads();
        for (int t = tid; t < n * n; t += FIN_THREADS) {
            int i = t / n, j = t % n;
            double v;
            if (i == k)
                v = rowk[j];
            else if (j == k)
                v = -colk[i] * ip;
            else
                v = B[t] - colk[i] * rowk[j];
            B[t] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- cycle kernels

// One red-black Gauss-Seidel half-sweep of one colour ((i+j+k) & 1 == colour),
// p_c = (s - b_c) / d.  Column grid, k strided by gridDim.z.
template <class T>
__global__ void __launch_bounds__(BX* BY) k_rb_half(Lvl<T> L, T* __restrict__ p, const T* __restrict__ b,
                                                   int colour, T omega, Bt bt) {
    int kz_, nkz_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.z, gridDim.z, kz_, nkz_, off_)) return;
    L = L.rebased(off_);
    p = rb(p, off_);
    b = rb(b, off_);
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= L.nx || j >= L.ny) return;
    for (int k = kz_; k < L.nz; k += nkz_) {
        if (((i + j + k) & 1) != colour) continue;
        T s, d;
        nbsum(L, p, i, j, k, s, d);
        size_t c = cidx(i, j, k, L.nx, L.ny);
        const T g = quot(s - b[c], d);
        // successive over-relaxation by omega (feature 5); omega = 1 is Gauss-Seidel
        p[c] = omega == T(1) ? g : fma(omega, g - p[c], p[c]);
    }
}

// 64-point restriction: rc(I,J,K) = 4 * sum over the fine cells 2I-1..2I+2 (and
// likewise in y, z) of w_a w_b w_c r, w = (1, 3, 3, 1) / 8, a fine index
// outside the grid replaced by its wall mirror (clamped): the transpose of
// trilinear interpolation.  One thread per coarse cell; r is the level's
// residual (stored by the residual kernel).
template <class T>
__global__ void k_restrict64(const T* __restrict__ r, int nx, int ny, int nz, T* __restrict__ rc, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    r = rb(r, off_);
    rc = rb(rc, off_);
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const size_t nc = (size_t)cx * cy * cz;
    const double w[4] = {0.125, 0.375, 0.375, 0.125};
    for (size_t t = (size_t)bid_ * blockDim.x + threadIdx.x; t < nc; t += (size_t)nb_ * blockDim.x) {
        const int I = (int)(t % cx);
        const size_t q = t / cx;
        const int J = (int)(q % cy), K = (int)(q / cy);
        T s = 0;
        for (int c = 0; c < 4; c++) {
            const int kk = min(max(2 * K - 1 + c, 0), nz - 1);
            for (int b = 0; b < 4; b++) {
                const int jj = min(max(2 * J - 1 + b, 0), ny - 1);
                const T* row = r + ((size_t)kk * ny + jj) * nx;
                for (int a = 0; a < 4; a++) {
                    const int ii = min(max(2 * I - 1 + a, 0), nx - 1);
                    s = fma((T)(w[a] * w[b] * w[c]), row[ii], s);
                }
            }
        }
        rc[t] = T(4) * s;
    }
}

// Restarted GMRES(m) on the coarsest grid (feature 6), FP64 arithmetic,
// n <= 512 cells, one workgroup of 512 threads (thread t owns cell t): solve
// L e = r - mean(r) from e = 0 with Arnoldi (modified Gram-Schmidt, the basis
// in LDS, where the operator reads neighbours), the least-squares problem kept
// triangular by Givens rotations, restart every m iterations, stop when the
// residual is <= tol of the mean-free right-hand side or after maxit
// iterations; e is returned mean-zero.  Every loop test reads values all
// threads share, so the barriers are uniform.
constexpr int GMRES_MAX_M = 16;
template <class T>
__global__ void __launch_bounds__(512) k_coarse_gmres(Lvl<double> L, const T* __restrict__ rin, T* __restrict__ eout,
                                                     int m, double tol, int maxit, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    rin = rb(rin, off_);
    eout = rb(eout, off_);
    __shared__ double V[GMRES_MAX_M + 1][512];
    __shared__ double H[(GMRES_MAX_M + 1) * GMRES_MAX_M];
    __shared__ double cs[GMRES_MAX_M], sn[GMRES_MAX_M], g[GMRES_MAX_M + 1], y[GMRES_MAX_M];
    __shared__ double red[8];
    const int t = threadIdx.x;
    const int nx = L.nx, ny = L.ny, n = nx * ny * L.nz;
    const bool act = t < n;
    auto bsum = [&](double v) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (t % 64 == 0) red[t / 64] = v;
        __syncthreads();
        double s = 0;
        for (int w = 0; w < 8; w++) s += red[w];
        __syncthreads();
        return s;
    };
    // this cell's faces and neighbour indices (a neighbour across a wall is the
    // cell itself, multiplied by a zero face)
    double w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
    int nw = t, ne = t, ns = t, nn = t, nd = t, nu = t;
    if (act) {
        const int i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
        faces6(L, i, j, k, (size_t)t, w0, w1, w2, w3, w4, w5);
        if (i > 0) nw = t - 1;
        if (i < nx - 1) ne = t + 1;
        if (j > 0) ns = t - nx;
        if (j < ny - 1) nn = t + nx;
        if (k > 0) nd = t - nx * ny;
        if (k < L.nz - 1) nu = t + nx * ny;
    }
    const double diag = stencil_diag(w0, w1, w2, w3, w4, w5);
    auto apply = [&](const double* x) {   // (L x)_t; x in LDS, synchronised
        if (!act) return 0.0;
        const double s = stencil_sum(w0, w1, w2, w3, w4, w5, x[nw], x[ne], x[ns], x[nn], x[nd], x[nu]);
        return fma(-diag, x[t], s);
    };
    const double rt = act ? (double)rin[t] : 0.0;
    const double mb = bsum(rt) / n;
    const double bb = act ? rt - mb : 0.0;
    const double nb = sqrt(bsum(bb * bb));
    double x = 0.0, r = bb, beta = nb;
    int it = 0;
    while (nb > 0.0 && beta > tol * nb && it < maxit) {
        V[0][t] = r / beta;
        if (t == 0) {
            for (int i = 0; i <= m; i++) g[i] = 0.0;
            g[0] = beta;
        }
        __syncthreads();
        int jj = 0;
        for (int j = 0; j < m && it < maxit; j++) {
            double w = apply(V[j]);
            it++;
            for (int i = 0; i <= j; i++) {
                const double h = bsum(w * V[i][t]);
                w -= h * V[i][t];
                if (t == 0) H[i * m + j] = h;
            }
            const double hn = sqrt(bsum(w * w));
            V[j + 1][t] = hn > 0.0 ? w / hn : 0.0;
            if (t == 0) {
                H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; i++) {   // earlier rotations on the new column
                    const double a = H[i * m + j], b = H[(i + 1) * m + j];
                    H[i * m + j] = cs[i] * a + sn[i] * b;
                    H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
                }
                const double a = H[j * m + j], b = hn, den = sqrt(a * a + b * b);
                cs[j] = den > 0.0 ? a / den : 1.0;
                sn[j] = den > 0.0 ? b / den : 0.0;
                H[j * m + j] = den;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            __syncthreads();
            jj = j + 1;
            if (fabs(g[j + 1]) <= tol * nb || hn == 0.0) break;
        }
        if (t == 0)
            for (int i = jj - 1; i >= 0; i--) {   // back substitution
                double s = g[i];
                for (int q = i + 1; q < jj; q++) s -= H[i * m + q] * y[q];
                y[i] = H[i * m + i] != 0.0 ? s / H[i * m + i] : 0.0;
            }
        __syncthreads();
        for (int i = 0; i < jj; i++) x += y[i] * V[i][t];
        __syncthreads();
        V[0][t] = x;   // the true residual of the new iterate
        __syncthreads();
        r = act ? bb - apply(V[0]) : 0.0;
        beta = sqrt(bsum(r * r));
    }
    const double me = bsum(act ? x : 0.0) / n;
    if (act) eout[t] = (T)(x - me);
}

// Exact coarsest solve e = -B^{-1} (r - mean r), FP64 arithmetic, n <= 512.
// Wavefront w of workgroup g computes row 8g + w: each lane sums every 64th
// column of the row (consecutive lanes, consecutive addresses, all loads
// independent), then the wavefront adds the 64 partial sums in a fixed tree.
// Every workgroup forms the mean of r itself.
template <class T>
__global__ void __launch_bounds__(512) k_coarse_solve(const double* __restrict__ Binv, int n,
                                                     const T* __restrict__ r, T* __restrict__ e, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    Binv = rb(Binv, off_);
    r = rb(r, off_);
    e = rb(e, off_);
    __shared__ double rs[512];
    __shared__ double red[8];
    const int t = threadIdx.x;
    double v = t < n ? (double)r[t] : 0.0;
    double s = v;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (t % 64 == 0) red[t / 64] = s;
    __syncthreads();
    double tot = 0;
    for (int w = 0; w < 8; w++) tot += red[w];
    const double mean = tot / n;
    if (t < n) rs[t] = v - mean;
    __syncthreads();
    const int lane = t % 64, row = bid_ * 8 + t / 64;
    if (row >= n) return;   // whole wavefronts
    double acc = 0;
    for (int c = lane; c < n; c += 64) acc += Binv[(size_t)row * n + c] * rs[c];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) e[row] = (T)(-acc);
}

// Workgroup barrier that only orders LDS traffic: waits for this wave's
// outstanding LDS operations, not for its global loads, so loads issued for the
// next plane stay in flight across it.  (Global results are only consumed by
// the issuing thread, after the compiler's own wait.)
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Raw buffer access: a resource (base address, range, format word) in scalar
// registers plus a per-lane 32-bit byte offset, so a load costs no per-lane
// address arithmetic and no 64-bit address registers.  The format word is the
// gfx9-family one for untyped 32-bit elements; the range is the maximum unless
// stated (every access here is in bounds by construction).  The resource is
// built with the compiler's own resource builtin, whose result it keeps in
// scalar registers: a resource assembled as a plain integer vector could be
// placed in vector registers, and every access through it then becomes a loop
// over the distinct values of the wavefront.
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// range: bytes addressable from p; loads at or past it return 0 without
// touching memory (used with range 0 to read an all-zero operand).  p and range
// must be the same in every lane of the wavefront: the resource takes lane 0's.
__device__ __forceinline__ Rsrc buf_rsrc(const void* p, int range = -1) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0,
                                             __builtin_amdgcn_readfirstlane(range), 0x00020000);
}
__device__ __forceinline__ float2 buf_ld2(Rsrc r, uint32_t off, const float*) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ double2 buf_ld2(Rsrc r, uint32_t off, const double*) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ float buf_ld1(Rsrc r, uint32_t off, const float*) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld1(Rsrc r, uint32_t off, const double*) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st2(float2 v, Rsrc r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st2(double2 v, Rsrc r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
}

// Compile-time loop: f(std::integral_constant<int, i>) for i = B .. E-1, so that
// arrays indexed by i are only ever indexed by constants (and stay in registers).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// NSW full red-black Gauss-Seidel sweeps (each colour c0 first, then 1 - c0)
// in a single pass over HBM, out of place (pin -> pout, so tiles never race).
//
// A workgroup owns a TX x TY column of cells and marches upward through a chunk
// of kc planes.  The sweeps are R = 2*NSW colour stages; stage h (h = 1 .. R)
// updates colour c0 (h odd) or 1 - c0 (h even) on plane t - h + 1 at step t, on
// the tile plus a ring of R - h cells.  Planes of pin are staged in LDS with an
// R-cell ring and updated in place stage by stage; a ring value is the same one
// the neighbouring tile computes, bit for bit, so after stage R the tile's plane
// t - R + 1 is final and written out.  Planes below k0 and above k1 - 1 are
// recomputed redundantly, so chunks are independent.
//
// Thread (q, lj) owns the aligned cell pair i = i0-R+2q, i0-R+1+2q of row
// j = j0-R+1+lj, so every global access is a 2-element vector; at step t all
// R stages fall on the same cell of the pair (the colour of a column flips
// from plane to plane).  In LDS each row of a plane is kept as two half rows.
// FP32 passes split a row by colour class, so a stage (which updates one class
// and reads the other) has every lane of a wave in the same class, and the
// half-row stride is chosen for the thread-row width so that the rows a wave
// spans fall on consecutive banks; FP64 passes (whose registers are full) split
// it by column parity, which needs fewer index operations.  The face
// coefficients and right-hand side of the pair stay in registers while their
// plane is in flight (the upper z-face of a cell is the lower z-face of the
// plane above).  Planes of pin and the z-faces are
// loaded two steps ahead, the other faces and b one step ahead, before the
// compute of the current step.  Requires even nx (every smoothed level has one).
//
// SKIP (two-sweep passes, Gauss-Seidel only): the first colour stage is left
// out.  Valid when every cell of that colour already holds the value the stage
// would compute, i.e. the iterate was last updated by a half-sweep of that
// colour (a cycle's post-smoothing ends with the colour the next cycle's
// pre-smoothing starts with): Gauss-Seidel on one colour given the other is
// exact, so repeating it reproduces the stored values bit for bit.
//
// UPD (FP32 plain passes of the refined solve): as each plane of the iterate is
// written in final form, the FP64 refinement update of the same cells is done
// too, p64 = (p64 - upd_sum[0] / n_cells) + upd_s[0] * (double)e, the expression
// of k_refine_update2 (so the update pass of the outer iteration is left out).
//
// With shift_sum non-null, every value of pin is first reduced by
// shift_sum[0] / n_cells (the mean-zero projection of the previous iterate, done
// on the fly instead of as a separate pass; same arithmetic as k_sub_mean).
// With zero_in set, the iterate entering the pass is zero and pin is not read:
// its loads go through a buffer resource of range 0, which returns 0 (a
// coarse-grid correction's first smoothing pass; no separate fill).
template <class T, int TX, int TY, int NSW, bool RES = false, bool SOR = false, bool SKIP = false,
          bool UPD = false>
__global__ void __launch_bounds__((TX / 2 + 2 * NSW) * (TY + 4 * NSW - 2 + (RES ? 2 : 0)))
    k_rb_sweep(Lvl<T> L, const T* __restrict__ pin, T* __restrict__ pout, const T* __restrict__ b, int c0, int kc,
               int tiles_x, int tiles_y, const double* __restrict__ shift_sum, double n_cells, int zero_in,
               T* __restrict__ rc, T omega, double* __restrict__ p64, const double* __restrict__ upd_s,
               const double* __restrict__ upd_sum, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    pin = rb(pin, off_);
    pout = rb(pout, off_);
    b = rb(b, off_);
    shift_sum = rb(shift_sum, off_);
    rc = rb(rc, off_);
    p64 = rb(p64, off_);
    upd_s = rb(upd_s, off_);
    upd_sum = rb(upd_sum, off_);
    static_assert(!UPD || (sizeof(T) == 4 && !RES), "the fused refinement update is for FP32 plain passes");
    using V = typename Vec2<T>::type;
    constexpr int R = 2 * NSW;                  // number of colour stages
    static_assert(!SKIP || (NSW == 2 && !SOR), "the first stage may be skipped in Gauss-Seidel two-sweep passes");
    constexpr int E = RES ? 1 : 0;              // extra ring for the residual's neighbours
    constexpr int RXs = R + 2 * E, RYs = R + E; // staged ring (x: whole pairs)
    constexpr int W = TX + 2 * RXs, H = TY + 2 * RYs, W2 = W / 2;
    constexpr int PW = TX / 2 + R, PH = TY + 2 * (R - 1 + E), NT = PW * PH;
    // Half rows by colour class (CL, FP32) with stride HS, the smallest
    // PW/2 + 32k >= W2, so two thread rows of PW lanes, 2 HS apart, cover
    // consecutive banks (64 banks of 4 bytes); else by column parity, stride W2.
    constexpr bool CL = sizeof(T) == 4;
    constexpr int HS = CL ? PW / 2 + 32 * ((2 * W2 - PW + 63) / 64) : W2;
    static_assert(PW % 2 == 0 && HS >= W2, "half-row stride");
    // plane slots: R + 2 (+1) live, one being refilled; FP32 rounds up to 8 so
    // that a slot index is a mask, not a division (one more plane of LDS)
    constexpr int NS = sizeof(T) == 4 ? 8 : R + 3 + E;
    static_assert(NS >= R + 3 + E, "too few plane slots");
    static_assert(!RES || (TX % 2 == 0 && TY % 2 == 0), "restriction needs even tiles");
    constexpr int PL = H * 2 * HS;              // elements of a staged plane
    constexpr int NV = H * W2;                  // pairs in a staged plane
    constexpr int NP = (NV + NT - 1) / NT;      // staged pairs per thread
    __shared__ __align__(16) T sp[NS * PL];
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, chunk = tile / (tiles_x * tiles_y);
    const int i0 = tx * TX, j0 = ty * TY;
    const int k0 = chunk * kc, k1 = min(nz, k0 + kc);
    const int tid = threadIdx.x;
    const int q = tid % PW, lj = tid / PW;
    const int ia = i0 - R + 2 * q, gj = j0 - (R - 1 + E) + lj;   // first cell of the pair, row
    const int row = lj + 1;                                   // LDS row of this thread
    const int qq = q + E;                                     // LDS half-row index of its pair
    const bool inpair = ia >= 0 && ia < nx && gj >= 0 && gj < ny;   // nx even: both cells in or both out
    const size_t plane = (size_t)nx * ny;
    const T shift = shift_sum ? (T)(shift_sum[0] / n_cells) : T(0);
    const int tfirst = k0 - R + 1 - E, tlast = k1 + R - 2 + E;

    // LDS position of (row r, column c) within a plane: (2r + ((r + c) & 1)) * HS + c / 2
    // with CL, else (2r + (c & 1)) * HS + c / 2 (staged coordinates: r, c from the
    // tile's corner minus the ring).
    // Global loads are unconditional (clamped to a valid address) so the compiler
    // can leave them in flight until first use; out-of-grid values are zeroed
    // where they are written to LDS or consumed.  Addresses are a per-plane base
    // (uniform) plus a fixed 32-bit byte offset per thread.
    uint32_t roff[NP];   // byte offset of staged pair u within a plane, clamped
    int rpos[NP];        // LDS position 2 r HS + c / 2 of its row (-1: no pair u for this thread)
    bool rodd[NP];       // odd row: the even cell is in the second half row
    bool rin[NP];        // inside the grid
#pragma unroll
    for (int u = 0; u < NP; u++) {
        const int v = tid + u * NT;
        const int vi = v % W2, vj = v / W2;
        const int ii = i0 - RXs + 2 * vi, jj = j0 - RYs + vj;
        rpos[u] = v < NV ? 2 * vj * HS + vi : -1;
        rodd[u] = CL && (vj & 1);
        rin[u] = v < NV && ii >= 0 && ii < nx && jj >= 0 && jj < ny;
        roff[u] = rin[u] ? (uint32_t)(jj * nx + ii) * (uint32_t)sizeof(T) : 0u;
    }
    constexpr const T* tag = nullptr;
    auto kclamp = [&](int k) { return k < 0 ? 0 : (k >= nz ? nz - 1 : k); };
    const int pin_range = zero_in ? 0 : -1;   // zero_in: every load of pin returns 0
    auto fetch_ring = [&](int k, V* v) {
        const Rsrc r = buf_rsrc(pin + (size_t)kclamp(k) * plane, pin_range);
#pragma unroll
        for (int u = 0; u < NP; u++) v[u] = buf_ld2(r, roff[u], tag);
    };
    auto store_ring = [&](int sl, int k, const V* v) {
        T* dst = sp + sl * PL;
        const bool kin = k >= 0 && k < nz;
#pragma unroll
        for (int u = 0; u < NP; u++)
            if (rpos[u] >= 0) {
                const bool ok = kin && rin[u];
                const T ev = ok ? v[u].x - shift : T(0), od = ok ? v[u].y - shift : T(0);
                dst[rpos[u]] = rodd[u] ? od : ev;
                dst[rpos[u] + HS] = rodd[u] ? ev : od;
            }
    };
    // x- and y-face coefficients and right-hand side of the pair on one plane (the
    // z-faces are kept apart: a plane's lower z-faces are also the upper z-faces
    // of the plane below and are loaded one step earlier)
    struct FB {
        V fx, fy, fyu, bb;
        T fxu;   // upper x-face of the second cell
    };
    const bool xu = ia + 2 < nx, yu = gj + 1 < ny;
    const uint32_t cb = inpair ? (uint32_t)(gj * nx + ia) * (uint32_t)sizeof(T) : 0u;
    const uint32_t cb64 = inpair ? (uint32_t)(gj * nx + ia) * 8u : 0u;   // the pair in an FP64 plane
    const double upd_c = UPD ? upd_sum[0] / n_cells : 0.0, upd_scale = UPD ? upd_s[0] : 0.0;
    // Offsets of the upper faces (those of the pair itself at a wall, where the
    // value is masked).  They pass through an empty asm so the compiler cannot
    // see that they may equal another load's address and fold the loads into a
    // copy (a copy would have to wait for the load right away).
    uint32_t cbx = cb + (xu ? 2u : 0u) * (uint32_t)sizeof(T), cby = cb + (yu ? (uint32_t)nx * sizeof(T) : 0u);
    asm volatile("" : "+v"(cbx), "+v"(cby));
    auto fetch_fb = [&](int k, FB& f) {
        const size_t pk = (size_t)kclamp(k) * plane;
        const Rsrc rx = buf_rsrc(L.fx + pk), ry = buf_rsrc(L.fy + pk);
        f.fx = buf_ld2(rx, cb, tag);
        f.fxu = buf_ld1(rx, cbx, tag);
        f.fy = buf_ld2(ry, cb, tag);
        f.fyu = buf_ld2(ry, cby, tag);
        f.bb = buf_ld2(buf_rsrc(b + pk), cb, tag);
    };
    auto fetch_fz = [&](int k) { return buf_ld2(buf_rsrc(L.fz + (size_t)kclamp(k) * plane), cb, tag); };
    // Zero the faces that lie on an upper wall (once per plane, one step after
    // its loads were issued).
    auto mask_fb = [&](FB& f) {
        if (!xu) f.fxu = T(0);
        if (!yu) f.fyu.x = f.fyu.y = T(0);
    };
    auto mask_fz = [&](int k, V& f) {
        if (k >= nz) f.x = f.y = T(0);
    };
    // Ring distance of each cell of the pair (c: LDS column): stage h updates the
    // cell when it is within R - h (+1 with RES) of the tile (large when the pair
    // is outside the grid).
    auto ring_dist = [&](int c) {
        const int dx = max(RXs - c, c - (RXs + TX - 1)), dy = max(RYs - row, row - (RYs + TY - 1));
        return inpair ? max(max(dx, dy), 0) : 4 * R;
    };
    const int dist0 = ring_dist(2 * qq), dist1 = ring_dist(2 * qq + 1);

    V ring[NP];
    if constexpr (sizeof(T) == 4 || NSW == 1 || RES) {
        // The register queues shift with the planes.  U steps per iteration:
        // step j of an iteration reads its queues at offset A = U - 1 - j and the
        // queues shift by U at the end, so every entry moves once per U steps.
        // U = 2 in FP32 two-sweep passes without the residual (one more queue
        // entry fits their registers without costing waves), else 1.
        constexpr int U = (sizeof(T) == 4 && NSW == 2 && !RES) ? 2 : 1;
        constexpr int NQ = R + 1 + 2 * E;   // RES keeps two more planes for the residual
        constexpr int NZ = R + 2 + 2 * E;
        FB fq[NQ + U - 1];   // fq[h + A]: x/y faces and b of plane t - h + 1 during step t (fq[A] in flight)
        V fzq[NZ + U - 1];   // fzq[h + A]: z-faces of plane t - h + 2 during step t (fzq[A] in flight)
        auto lslot = [&](int k) { return (int)((unsigned)(k - tfirst + NS) % (unsigned)NS); };   // k >= tfirst - 1
        fetch_ring(tfirst - 1, ring);
        store_ring(lslot(tfirst - 1), tfirst - 1, ring);
        fetch_ring(tfirst, ring);
        store_ring(lslot(tfirst), tfirst, ring);
        fetch_ring(tfirst + 1, ring);
        fetch_fb(tfirst, fq[U]);
        fzq[U] = fetch_fz(tfirst + 1);
        fzq[U + 1] = fetch_fz(tfirst);
        static_for<U + 1, NQ + U - 1>([&](auto sc) { fq[decltype(sc)::value] = fq[U]; });
        static_for<U + 2, NZ + U - 1>([&](auto sc) { fzq[decltype(sc)::value] = fzq[U + 1]; });
        // RES: residual r = b - (s - d p) of the tile's cells on plane t - R - 1 (whose
        // neighbours are final), summed over the x pair, then over the plane pair;
        // the row pair is added through LDS one step later.
        __shared__ T red[RES ? PH : 1][RES ? PW : 1];
        const bool tpair = RES && dist0 == 0 && dist1 == 0;   // a pair of the tile
        T racc = T(0);
        auto epilogue = [&](int zr, auto ac) {
            if constexpr (RES) {
                constexpr int A = decltype(ac)::value;
                if (zr - 1 >= k0 && ((zr - 1) & 1) && tpair && !(gj & 1))
                    rc[cidx(ia >> 1, gj >> 1, (zr - 1) >> 1, nx >> 1, ny >> 1)] = T(0.5) * (racc + red[lj + 1][q]);
                if (zr >= k0 && zr < k1 && tpair) {
                    const FB& f = fq[R + 2 + A];
                    const V wz0 = fzq[R + 3 + A], wz1 = fzq[R + 2 + A];
                    const T* c = sp + lslot(zr) * PL;
                    const T* cd = sp + lslot(zr - 1) * PL;
                    const T* cu = sp + lslot(zr + 1) * PL;
                    // even and odd cell; with CL a cell's y-neighbours are in the other
                    // class's half rows
                    const int ro = CL ? (row & 1) : 0;
                    const int o0 = (2 * row + ro) * HS + qq, o1 = (2 * row + 1 - ro) * HS + qq;
                    const int y0 = CL ? o1 : o0, y1 = CL ? o0 : o1;
                    const T s0 = stencil_sum(f.fx.x, f.fx.y, f.fy.x, f.fyu.x, wz0.x, wz1.x, c[o1 - 1], c[o1],
                                             c[y0 - 2 * HS], c[y0 + 2 * HS], cd[o0], cu[o0]);
                    const T d0 = stencil_diag(f.fx.x, f.fx.y, f.fy.x, f.fyu.x, wz0.x, wz1.x);
                    const T s1 = stencil_sum(f.fx.y, f.fxu, f.fy.y, f.fyu.y, wz0.y, wz1.y, c[o0], c[o0 + 1],
                                             c[y1 - 2 * HS], c[y1 + 2 * HS], cd[o1], cu[o1]);
                    const T d1 = stencil_diag(f.fx.y, f.fxu, f.fy.y, f.fyu.y, wz0.y, wz1.y);
                    const T sum = resid_val(f.bb.x, s0, d0, c[o0]) + resid_val(f.bb.y, s1, d1, c[o1]);
                    if (zr & 1) {
                        racc += sum;
                        red[lj][q] = racc;
                    } else {
                        racc = sum;
                    }
                }
            }
        };
        auto step = [&](int t, auto ac) {
            constexpr int A = decltype(ac)::value;
            store_ring(lslot(t + 1), t + 1, ring);
            mask_fb(fq[1 + A]);
            mask_fz(t + 1, fzq[1 + A]);
            lds_barrier();
            fetch_ring(t + 2, ring);                  // in flight during this step
            fetch_fb(t + 1, fq[A]);
            fzq[A] = fetch_fz(t + 2);
            // UPD: the FP64 values of the pair on this step's output plane (tile pairs
            // only; the ring's lanes write no output)
            double2 pold{};
            if constexpr (UPD) {
                if (dist0 == 0 && dist1 == 0)
                    pold = buf_ld2(buf_rsrc(p64 + (size_t)kclamp(t - R + 1) * plane), cb64, (const double*)nullptr);
            }
            epilogue(t - R - 1, ac);
            const int e = (c0 + i0 + gj + t) & 1;
            const int dist = e ? dist1 : dist0;
            const int hc = CL ? (e + row) & 1 : e;                    // the cell's half row
            const int oc = (2 * row + hc) * HS + qq;                  // the cell
            const int opart = (2 * row + 1 - hc) * HS + qq;           // its pair partner
            const int ol = e ? opart : opart - 1, orr = e ? opart + 1 : opart;   // x-neighbours
            const int oy = CL ? opart : oc;
            const int os = oy - 2 * HS, on = oy + 2 * HS;             // y-neighbours
            static_for<1 + (SKIP ? 1 : 0), R + 1>([&](auto hc) {
                constexpr int h = decltype(hc)::value;
                constexpr int rg = R - h + E;                           // this stage's ring width
                const int z = t - h + 1;
                const int sz = lslot(z), sd = lslot(z - 1), su = lslot(z + 1);
                const bool in_z = z >= 0 && z < nz && z >= k0 - rg && z < k1 + rg;
                const FB& f = fq[h + A];
                const T w0 = e ? f.fx.y : f.fx.x;
                const T w1 = e ? f.fxu : f.fx.y;
                const T w2 = e ? f.fy.y : f.fy.x;
                const T w3 = e ? f.fyu.y : f.fyu.x;
                const T w4 = e ? fzq[h + 1 + A].y : fzq[h + 1 + A].x;
                const T w5 = e ? fzq[h + A].y : fzq[h + A].x;
                const T bb = e ? f.bb.y : f.bb.x;
                const T* c = sp + sz * PL;
                const T s = stencil_sum(w0, w1, w2, w3, w4, w5, c[ol], c[orr], c[os], c[on],
                                        sp[sd * PL + oc], sp[su * PL + oc]);
                const T vnew = sor<SOR>(quot(s - bb, stencil_diag(w0, w1, w2, w3, w4, w5)), c, oc, omega);
                if constexpr (h < R) {
                    if (in_z && dist <= rg) sp[sz * PL + oc] = vnew;
                    lds_barrier();
                } else {
                    // the tile's plane z is final: this cell from stage R, its pair
                    // partner from stage R-1 of the previous step
                    if (RES && in_z && dist <= rg) sp[sz * PL + oc] = vnew;
                    if (in_z && dist == 0 && z >= k0 && z < k1) {
                        const T vold = c[opart];
                        V out;
                        out.x = e ? vold : vnew;
                        out.y = e ? vnew : vold;
                        buf_st2(out, buf_rsrc(pout + (size_t)z * plane), cb);
                        if constexpr (UPD) {
                            double2 q;
                            q.x = (pold.x - upd_c) + upd_scale * (double)out.x;
                            q.y = (pold.y - upd_c) + upd_scale * (double)out.y;
                            buf_st2(q, buf_rsrc(p64 + (size_t)z * plane), cb64);
                        }
                    }
                }
            });
        };
        const int tend = tlast + E;
        for (int t = tfirst; t <= tend; t += U) {
            step(t, std::integral_constant<int, U - 1>{});
            if constexpr (U == 2) {
                if (t + 1 <= tend) step(t + 1, std::integral_constant<int, 0>{});
            }
            static_for<0, NQ - 1>([&](auto hc) {   // shift by U
                constexpr int h = NQ + U - 2 - decltype(hc)::value;
                fq[h] = fq[h - U];
            });
            static_for<0, NZ - 1>([&](auto hc) {
                constexpr int h = NZ + U - 2 - decltype(hc)::value;
                fzq[h] = fzq[h - U];
            });
        }
        if constexpr (RES) {
            // the row pairs of the last (odd) plane of the chunk
            lds_barrier();
            epilogue(tlast + E - R, std::integral_constant<int, 0>{});
        }
    } else {
        // FP64, several sweeps: the loop is unrolled by NS steps, so every queue
        // slot and LDS slot is a compile-time index (no register shifts,
        // immediate LDS offsets); measured faster here despite more registers.
        // Plane z is held in LDS slot, face slot and z-face slot (z - tfirst) mod NS.
        // Loads in flight at step t: pin of plane t+2, x/y faces and b of plane t+1,
        // z-faces of plane t+2.
        FB fq[NS];
        V fzq[NS];
        fetch_ring(tfirst - 1, ring);
        store_ring(NS - 1, tfirst - 1, ring);
        fetch_ring(tfirst, ring);
        store_ring(0, tfirst, ring);
        fetch_ring(tfirst + 1, ring);
        fetch_fb(tfirst, fq[0]);
        fzq[0] = fetch_fz(tfirst);
        fzq[1] = fetch_fz(tfirst + 1);
        static_for<1, NS>([&](auto sc) { fq[decltype(sc)::value] = fq[0]; });
        static_for<2, NS>([&](auto sc) { fzq[decltype(sc)::value] = fzq[0]; });
        for (int tg = tfirst; tg <= tlast; tg += NS) {
            static_for<0, NS>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                constexpr int s0 = u % NS, s1 = (u + 1) % NS, s2 = (u + 2) % NS;
                const int t = tg + u;
                if (t > tlast) return;
                store_ring(s1, t + 1, ring);
                mask_fb(fq[s0]);
                mask_fz(t + 1, fzq[s1]);
                lds_barrier();
                fetch_ring(t + 2, ring);                  // in flight during this step
                fetch_fb(t + 1, fq[s1]);
                fzq[s2] = fetch_fz(t + 2);
                // the cell of the pair that stage 1 updates on plane t; every stage of
                // this step updates the same cell (on its own plane)
                const int e = (c0 + i0 + gj + t) & 1;
                const int dist = e ? dist1 : dist0;
                const int hc = CL ? (e + row) & 1 : e;                    // the cell's half row
                const int oc = (2 * row + hc) * HS + q;                   // the cell
                const int opart = (2 * row + 1 - hc) * HS + q;            // its pair partner
                const int ol = e ? opart : opart - 1, orr = e ? opart + 1 : opart;   // x-neighbours
                const int oy = CL ? opart : oc;
                const int os = oy - 2 * HS, on = oy + 2 * HS;             // y-neighbours
                static_for<1, R + 1>([&](auto hc) {
                    constexpr int h = decltype(hc)::value;
                    constexpr int sz = (u - h + 1 + 2 * NS) % NS;         // slot of this stage's plane
                    constexpr int sd = (sz + NS - 1) % NS, su = (sz + 1) % NS;
                    constexpr int rg = R - h;                               // this stage's ring width
                    const int z = t - h + 1;
                    const bool in_z = z >= 0 && z < nz && z >= k0 - rg && z < k1 + rg;
                    const FB& f = fq[sz];
                    const T w0 = e ? f.fx.y : f.fx.x;
                    const T w1 = e ? f.fxu : f.fx.y;
                    const T w2 = e ? f.fy.y : f.fy.x;
                    const T w3 = e ? f.fyu.y : f.fyu.x;
                    const T w4 = e ? fzq[sz].y : fzq[sz].x;
                    const T w5 = e ? fzq[su].y : fzq[su].x;
                    const T bb = e ? f.bb.y : f.bb.x;
                    const T* c = sp + sz * PL;
                    const T s = stencil_sum(w0, w1, w2, w3, w4, w5, c[ol], c[orr], c[os], c[on],
                                            sp[sd * PL + oc], sp[su * PL + oc]);
                    const T vnew = sor<SOR>(quot(s - bb, stencil_diag(w0, w1, w2, w3, w4, w5)), c, oc, omega);
                    if constexpr (h < R) {
                        if (in_z && dist <= rg) sp[sz * PL + oc] = vnew;
                        lds_barrier();
                    } else if (in_z && dist <= rg) {
                        // the tile's plane z is final: this cell from stage R, its pair
                        // partner from stage R-1 of the previous step
                        const T vold = c[opart];
                        V out;
                        out.x = e ? vold : vnew;
                        out.y = e ? vnew : vold;
                        buf_st2(out, buf_rsrc(pout + (size_t)z * plane), cb);
                    }
                });
            });
        }
    }
}

// ---------------------------------------------------------------- z-marching residual kernels
//
// A workgroup (CBX x CBY threads) owns a tile of columns and marches up a chunk
// of planes; each thread keeps its column's p at planes k-1, k, k+1 and the
// z-face below in registers and loads everything of plane k+1 one step ahead,
// so every array is read from HBM about once (the y-neighbour rows at the tile
// edge hit L2 when the neighbouring tile runs on the same XCD, see xcd_tile).

constexpr int CBX = 64, CBY = 4;

struct ColGrid {
    int tiles_x, tiles_y, kc;
};

// Values of one cell's stencil at one plane: own p, 4 in-plane neighbours,
// right-hand side and the 5 faces that are not carried from the plane below.
template <class T>
struct Plane1 {
    T p, pw, pe, ps, pn, b, wx0, wx1, wy0, wy1, wz1;
};

template <class T>
__device__ __forceinline__ Plane1<T> load_plane1(const Lvl<T>& L, const T* __restrict__ p, const T* __restrict__ b,
                                                 int i, int j, int k) {
    Plane1<T> v;
    const int nx = L.nx, ny = L.ny;
    const size_t c = cidx(i, j, k, nx, ny);
    v.p = p[c];
    v.pw = i > 0 ? p[c - 1] : T(0);
    v.pe = i < nx - 1 ? p[c + 1] : T(0);
    v.ps = j > 0 ? p[c - nx] : T(0);
    v.pn = j < ny - 1 ? p[c + nx] : T(0);
    v.b = b[c];
    T wz0;
    faces6(L, i, j, k, c, v.wx0, v.wx1, v.wy0, v.wy1, wz0, v.wz1);
    return v;
}

// Residual r = b - L p along each column; MODE 0: partial sums of r^2 and p;
// MODE 1 (FP64 refinement): also writes r32 = float(r * scal_inv_s[0]);
// MODE 2 (Krylov solve): also writes r64 = r.
template <class T, int MODE>
__global__ void __launch_bounds__(CBX* CBY) k_resid_col(Lvl<T> L, const T* __restrict__ p, const T* __restrict__ b,
                                                       ColGrid G, const double* __restrict__ scal_inv_s,
                                                       float* __restrict__ r32, double* __restrict__ part,
                                                       T* __restrict__ r64, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    p = rb(p, off_);
    b = rb(b, off_);
    scal_inv_s = rb(scal_inv_s, off_);
    r32 = rb(r32, off_);
    part = rb(part, off_);
    r64 = rb(r64, off_);
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int i = tx * CBX + (int)(threadIdx.x % CBX), j = ty * CBY + (int)(threadIdx.x / CBX);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    double a = 0, q = 0;
    const double inv_s = MODE == 1 ? scal_inv_s[0] : 1.0;
    if (i < nx && j < ny && k0 < k1) {
        const size_t plane = (size_t)nx * ny;
        const size_t col = (size_t)j * nx + i;
        T pbelow = k0 > 0 ? p[(size_t)(k0 - 1) * plane + col] : T(0);
        T wz0 = L.fz[(size_t)k0 * plane + col];
        Plane1<T> cur = load_plane1(L, p, b, i, j, k0);
        Plane1<T> nxt = cur;
        for (int k = k0; k < k1; k++) {
            if (k + 1 < nz) nxt = load_plane1(L, p, b, i, j, k + 1);
            const T pabove = k + 1 < nz ? nxt.p : T(0);
            const T s = stencil_sum(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1, cur.pw, cur.pe, cur.ps,
                                    cur.pn, pbelow, pabove);
            const T d = stencil_diag(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1);
            const T r = resid_val(cur.b, s, d, cur.p);
            if (MODE == 1) r32[(size_t)k * plane + col] = (float)((double)r * inv_s);
            if (MODE == 2) r64[(size_t)k * plane + col] = r;
            a += (double)r * (double)r;
            q += (double)cur.p;
            pbelow = cur.p;
            wz0 = cur.wz1;
            cur = nxt;
        }
    }
    // deterministic block partials
    __shared__ double sa[CBX * CBY / 64], sb[CBX * CBY / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        q += __shfl_down(q, off, 64);
    }
    if (threadIdx.x % 64 == 0) { sa[threadIdx.x / 64] = a; sb[threadIdx.x / 64] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < CBX * CBY / 64; w++) { ta += sa[w]; tb += sb[w]; }
        part[2 * tile] = ta;
        part[2 * tile + 1] = tb;
    }
}

// ---------------------------------------------------------------- finest-level residual
//
// r = b - L p on the finest level (FP64), one thread per cell pair (nx even,
// arrays 16-byte aligned), 512 threads per workgroup in plain dispatch order:
// where it writes the residual this one-pass stencil measured faster than
// marching columns, the neighbouring rows and planes coming from the caches
// (the norm alone is faster in columns).  A neighbour across
// a wall is read at the cell itself and multiplied by a zero face.  MODE as
// k_resid_col (0: partial sums of r^2 and p; 1: also r32 = float(r * inv_s);
// 2: also r64 = r); one pair of partial sums per workgroup.  The stencil is
// evaluated in the same order as the other residual kernels (same results).
constexpr int RES_FLAT_THREADS = 512;
template <int MODE>
__global__ void __launch_bounds__(RES_FLAT_THREADS)
    k_resid_flat(Lvl<double> L, const double* __restrict__ p, const double* __restrict__ b, uint32_t units,
                 const double* __restrict__ scal_inv_s, float* __restrict__ r32, double* __restrict__ part,
                 double* __restrict__ r64, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    p = rb(p, off_);
    b = rb(b, off_);
    scal_inv_s = rb(scal_inv_s, off_);
    r32 = rb(r32, off_);
    part = rb(part, off_);
    r64 = rb(r64, off_);
    const uint32_t t = (uint32_t)bid_ * RES_FLAT_THREADS + threadIdx.x;
    double a = 0, q = 0;
    if (t < units) {
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        const uint32_t ux = (uint32_t)nx / 2, r = t / ux;
        const int i = (int)(t - r * ux) * 2, j = (int)(r % (uint32_t)ny), k = (int)(r / (uint32_t)ny);
        const size_t plane = (size_t)nx * ny, c = (size_t)r * nx + i;
        const double2 pc = *reinterpret_cast<const double2*>(p + c);
        const double pw = p[i > 0 ? c - 1 : c], pe = p[i + 2 < nx ? c + 2 : c + 1];
        const double2 ps = *reinterpret_cast<const double2*>(p + (j > 0 ? c - nx : c));
        const double2 pn = *reinterpret_cast<const double2*>(p + (j + 1 < ny ? c + nx : c));
        const double2 pd = *reinterpret_cast<const double2*>(p + (k > 0 ? c - plane : c));
        const double2 pu = *reinterpret_cast<const double2*>(p + (k + 1 < nz ? c + plane : c));
        const double2 bb = *reinterpret_cast<const double2*>(b + c);
        const double2 fx = *reinterpret_cast<const double2*>(L.fx + c);
        const double fxu = i + 2 < nx ? L.fx[c + 2] : 0.0;
        const double2 fy = *reinterpret_cast<const double2*>(L.fy + c);
        const double2 fyu = j + 1 < ny ? *reinterpret_cast<const double2*>(L.fy + c + nx) : make_double2(0.0, 0.0);
        const double2 fz = *reinterpret_cast<const double2*>(L.fz + c);
        const double2 fzu = k + 1 < nz ? *reinterpret_cast<const double2*>(L.fz + c + plane) : make_double2(0.0, 0.0);
        const double s0 = stencil_sum(fx.x, fx.y, fy.x, fyu.x, fz.x, fzu.x, pw, pc.y, ps.x, pn.x, pd.x, pu.x);
        const double d0 = stencil_diag(fx.x, fx.y, fy.x, fyu.x, fz.x, fzu.x);
        const double s1 = stencil_sum(fx.y, fxu, fy.y, fyu.y, fz.y, fzu.y, pc.x, pe, ps.y, pn.y, pd.y, pu.y);
        const double d1 = stencil_diag(fx.y, fxu, fy.y, fyu.y, fz.y, fzu.y);
        const double r0 = resid_val(bb.x, s0, d0, pc.x), r1 = resid_val(bb.y, s1, d1, pc.y);
        if (MODE == 1) {
            const double inv_s = scal_inv_s[0];
            *reinterpret_cast<float2*>(r32 + c) = make_float2((float)(r0 * inv_s), (float)(r1 * inv_s));
        }
        if (MODE == 2) *reinterpret_cast<double2*>(r64 + c) = make_double2(r0, r1);
        a = r0 * r0;
        a += r1 * r1;
        q = pc.x;
        q += pc.y;
    }
    __shared__ double sa[RES_FLAT_THREADS / 64], sb[RES_FLAT_THREADS / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        q += __shfl_down(q, off, 64);
    }
    if (threadIdx.x % 64 == 0) { sa[threadIdx.x / 64] = a; sb[threadIdx.x / 64] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < RES_FLAT_THREADS / 64; w++) { ta += sa[w]; tb += sb[w]; }
        part[2 * bid_] = ta;
        part[2 * bid_ + 1] = tb;
    }
}

// ---------------------------------------------------------------- cell-pair residual kernels
//
// Residual kernels for nx divisible by NC = 2 or 4 (every level but possibly
// the finest has even nx): a thread owns NC consecutive cells of a row, so
// their values, right-hand side and faces are vector loads and one load
// instruction serves NC cells.  Every load is unconditional and no loaded value
// is masked (see cell_offsets), so the loads of a plane stay in flight together.
// Latency is hidden by occupancy (few registers per thread) rather than by
// loading planes further ahead, which measured no faster here.

// NC consecutive values as one vector load (NC = 2 or 4; 16 bytes at most; NC = 1 a scalar).
template <class T, int NC>
struct VecN;
template <>
struct VecN<float, 2> {
    using type = float2;
};
template <>
struct VecN<float, 4> {
    using type = float4;
};
template <>
struct VecN<double, 2> {
    using type = double2;
};

template <class T, int NC>
__device__ __forceinline__ void load_n(const T* src, T (&d)[NC]) {
    if constexpr (NC == 1) {
        d[0] = *src;
    } else {
        const typename VecN<T, NC>::type v = *reinterpret_cast<const typename VecN<T, NC>::type*>(src);
        if constexpr (NC == 2) {
            d[0] = v.x;
            d[1] = v.y;
        } else {
            d[0] = v.x;
            d[1] = v.y;
            d[2] = v.z;
            d[3] = v.w;
        }
    }
}

// One plane of NC cells of a row: own values, in-plane neighbours, right-hand
// side and faces (lower x, y and z faces, the upper x face of the last cell and
// the upper y faces; the upper z faces are the next plane's lower ones).
template <class T, int NC>
struct Cells1 {
    T p[NC], ps[NC], pn[NC], b[NC], fx[NC], fy[NC], fyu[NC], fz[NC];
    T pw, pe, fxu;
};

// Offsets (within a plane) of the loads of cells i = NC*I .. NC*I+NC-1 of row j.
// A neighbour across a wall is read where the face that multiplies it is a
// stored lower wall face, i.e. exactly 0: across a lower wall the cells
// themselves; across the upper x wall the first cell of the row, across the
// upper y wall row 0 (their lower faces are walls).  No value needs masking.
struct CellOff {
    int c, w, e, s, n;
};

template <int NC>
__device__ __forceinline__ CellOff cell_offsets(int I, int j, int nx, int ny) {
    CellOff o;
    o.c = j * nx + NC * I;
    o.w = I > 0 ? o.c - 1 : o.c;
    o.e = NC * I + NC < nx ? o.c + NC : j * nx;
    o.s = j > 0 ? o.c - nx : o.c;
    o.n = j + 1 < ny ? o.c + nx : NC * I;
    return o;
}

// The plane above k for the z-marching kernels: at the top wall plane 0, whose
// lower z faces are walls (0), so the upper z face of the top plane reads as 0.
__device__ __forceinline__ int plane_above(int k, int nz) { return k + 1 < nz ? k + 1 : 0; }

template <class T, int NC>
__device__ __forceinline__ Cells1<T, NC> load_cells1(const Lvl<T>& L, const T* __restrict__ p,
                                                     const T* __restrict__ b, const CellOff& o, int k) {
    const size_t base = (size_t)k * L.nx * L.ny;
    Cells1<T, NC> v;
    load_n(p + base + o.c, v.p);
    v.pw = p[base + o.w];
    v.pe = p[base + o.e];
    load_n(p + base + o.s, v.ps);
    load_n(p + base + o.n, v.pn);
    load_n(b + base + o.c, v.b);
    load_n(L.fx + base + o.c, v.fx);
    v.fxu = L.fx[base + o.e];
    load_n(L.fy + base + o.c, v.fy);
    load_n(L.fy + base + o.n, v.fyu);
    load_n(L.fz + base + o.c, v.fz);
    return v;
}

// Residuals r = b - (s - d p) of the cells on plane k, given p below (pb) and
// the plane above (its p and lower z faces, loaded from plane_above).
template <class T, int NC>
__device__ __forceinline__ void cells_residual(const Cells1<T, NC>& c, const T (&pb)[NC],
                                               const Cells1<T, NC>& up, T (&r)[NC]) {
#pragma unroll
    for (int e = 0; e < NC; e++) {
        const T w1 = e + 1 < NC ? c.fx[e + 1] : c.fxu;
        const T pw = e > 0 ? c.p[e - 1] : c.pw;
        const T pe = e + 1 < NC ? c.p[e + 1] : c.pe;
        const T s = stencil_sum(c.fx[e], w1, c.fy[e], c.fyu[e], c.fz[e], up.fz[e], pw, pe, c.ps[e], c.pn[e], pb[e],
                                up.p[e]);
        const T d = stencil_diag(c.fx[e], w1, c.fy[e], c.fyu[e], c.fz[e], up.fz[e]);
        r[e] = resid_val(c.b[e], s, d, c.p[e]);
    }
}

// k_resid_col for nx divisible by NC.  Tiles of CBX cell groups x CBY rows, one
// wavefront per row.  The wavefronts of a workgroup meet at a barrier before
// every plane, so a row's neighbour rows (the other wavefronts' own rows) are
// read while they are still in the caches: left to drift apart over a long
// column, they were not (1024^3: 1.46x the algorithmic fetch, and the nine
// finest-level residuals of a solve took 97.6 ms against 83.6 ms in step).
template <class T, int NC, int MODE>
__global__ void __launch_bounds__(CBX* CBY) k_resid_cells(Lvl<T> L, const T* __restrict__ p,
                                                         const T* __restrict__ b, ColGrid G,
                                                         const double* __restrict__ scal_inv_s,
                                                         float* __restrict__ r32, double* __restrict__ part,
                                                         T* __restrict__ r64, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    p = rb(p, off_);
    b = rb(b, off_);
    scal_inv_s = rb(scal_inv_s, off_);
    r32 = rb(r32, off_);
    part = rb(part, off_);
    r64 = rb(r64, off_);
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int I = tx * CBX + (int)(threadIdx.x % CBX), j = ty * CBY + (int)(threadIdx.x / CBX);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    double a = 0, q = 0;
    const double inv_s = MODE == 1 ? scal_inv_s[0] : 1.0;
    const bool active = NC * I < nx && j < ny;
    if (k0 < k1) {   // the same for the whole workgroup
        const size_t plane = (size_t)nx * ny;
        // threads outside the grid load at cell (0, 0) and keep nothing
        const CellOff o = cell_offsets<NC>(active ? I : 0, active ? j : 0, nx, ny);
        T pb[NC];
        load_n(p + (size_t)max(k0 - 1, 0) * plane + o.c, pb);
        Cells1<T, NC> cur = load_cells1<T, NC>(L, p, b, o, k0);
        for (int k = k0; k < k1; k++) {
            __syncthreads();
            const Cells1<T, NC> nxt = load_cells1<T, NC>(L, p, b, o, plane_above(k, nz));
            T r[NC];
            cells_residual(cur, pb, nxt, r);
            if (active && MODE == 1) {
                float w[NC];
#pragma unroll
                for (int e = 0; e < NC; e++) w[e] = (float)((double)r[e] * inv_s);
                if constexpr (NC == 2)
                    *reinterpret_cast<float2*>(r32 + (size_t)k * plane + o.c) = make_float2(w[0], w[1]);
                else
                    *reinterpret_cast<float4*>(r32 + (size_t)k * plane + o.c) = make_float4(w[0], w[1], w[2], w[3]);
            }
            if (active && MODE == 2) {
#pragma unroll
                for (int e = 0; e < NC; e++) r64[(size_t)k * plane + o.c + e] = r[e];
            }
#pragma unroll
            for (int e = 0; e < NC; e++) {
                if (active) {
                    a += (double)r[e] * (double)r[e];
                    q += (double)cur.p[e];
                }
                pb[e] = cur.p[e];
            }
            cur = nxt;
        }
    }
    __shared__ double sa[CBX * CBY / 64], sb[CBX * CBY / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        q += __shfl_down(q, off, 64);
    }
    if (threadIdx.x % 64 == 0) { sa[threadIdx.x / 64] = a; sb[threadIdx.x / 64] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < CBX * CBY / 64; w++) { ta += sa[w]; tb += sb[w]; }
        part[2 * tile] = ta;
        part[2 * tile + 1] = tb;
    }
}

// Residual restricted to the next level, rc(I,J,K) = 1/2 * (sum of the 8 child
// residuals), for nx divisible by NC (every restricted level has even nx).
// Tiles of CBX cell groups x CBY rows, one wavefront per row: a thread holds
// the x-children of NC/2 coarse columns and sums them over the plane pair 2K,
// 2K+1; the y partner (next row, next wavefront) is added through LDS.  kc is
// even.
template <class T, int NC>
__global__ void __launch_bounds__(CBX* CBY) k_resid_restrict_cells(Lvl<T> L, const T* __restrict__ p,
                                                                  const T* __restrict__ b, ColGrid G,
                                                                  T* __restrict__ rc, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    p = rb(p, off_);
    b = rb(b, off_);
    rc = rb(rc, off_);
    static_assert(CBY % 2 == 0, "row pairs");
    constexpr int NQ = NC / 2;   // coarse columns per thread
    __shared__ T part[CBY][NQ][CBX];
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int cnx = nx / 2, cny = ny / 2;
    const int li = threadIdx.x % CBX, lj = threadIdx.x / CBX;
    const int I = tx * CBX + li, j = ty * CBY + lj;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    const bool active = NC * I < nx && j < ny;   // ny even: a row pair is all in or all out
    const size_t plane = (size_t)nx * ny;
    const CellOff o = cell_offsets<NC>(active ? I : 0, active ? j : 0, nx, ny);
    T pb[NC] = {};
    Cells1<T, NC> cur{};
    if (active && k0 < k1) {
        load_n(p + (size_t)max(k0 - 1, 0) * plane + o.c, pb);
        cur = load_cells1<T, NC>(L, p, b, o, k0);
    }
    T acc[NQ] = {};
    for (int k = k0; k < k1; k++) {
        if (!(k & 1)) __syncthreads();   // the row wavefronts in step every plane (odd planes below)
        if (active) {
            const Cells1<T, NC> nxt = load_cells1<T, NC>(L, p, b, o, plane_above(k, nz));
            T r[NC];
            cells_residual(cur, pb, nxt, r);
#pragma unroll
            for (int c = 0; c < NQ; c++) acc[c] += r[2 * c] + r[2 * c + 1];
#pragma unroll
            for (int e = 0; e < NC; e++) pb[e] = cur.p[e];
            cur = nxt;
        }
        if (k & 1) {
#pragma unroll
            for (int c = 0; c < NQ; c++) part[lj][c][li] = acc[c];
            __syncthreads();
            if (active && !(lj & 1)) {
                T v[NQ];
#pragma unroll
                for (int c = 0; c < NQ; c++) v[c] = T(0.5) * (acc[c] + part[lj + 1][c][li]);
                T* dst = rc + cidx(NQ * I, j >> 1, k >> 1, cnx, cny);
                if constexpr (NQ == 1)
                    dst[0] = v[0];
                else
                    *reinterpret_cast<typename Vec2<T>::type*>(dst) = typename Vec2<T>::type{v[0], v[1]};
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < NQ; c++) acc[c] = 0;
        }
    }
}

// Flux-conserving prolongation and correction (pro_plane / pro_face /
// pro_child), z-marching over coarse planes.  Thread (I, j) owns the fine cell
// pair i = 2I, 2I+1 of fine row j: both are children of coarse column I with
// the same y side (Jy) and opposite x sides (I-1 for the even child, I+1 for the
// odd one, clamped = wall mirror).  Each step handles the two fine planes 2K,
// 2K+1 of coarse plane K: the corners on the face K-1/2 were computed in the
// previous step (as face K+1/2 of plane K-1).  The coarse plane K+1 and the fine
// planes of the next step are loaded one step ahead.  G.kc counts coarse planes.
template <class T>
__global__ void __launch_bounds__(CBX* CBY) k_prolong_col(const T* __restrict__ ec, const T* __restrict__ ac,
                                                         int cnx, int cny, int cnz, ColGrid G, T* __restrict__ ef, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    ec = rb(ec, off_);
    ac = rb(ac, off_);
    ef = rb(ef, off_);
    using V = typename Vec2<T>::type;
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int nx = 2 * cnx, ny = 2 * cny;
    const int I = tx * CBX + (int)(threadIdx.x % CBX), j = ty * CBY + (int)(threadIdx.x / CBX);
    const int K0 = chunk * G.kc, K1 = min(cnz, K0 + G.kc);
    if (I >= cnx || j >= ny || K0 >= K1) return;
    const int J = j >> 1;
    const int Im = max(I - 1, 0), Ip = min(I + 1, cnx - 1);
    const int Jy = (j & 1) ? min(J + 1, cny - 1) : max(J - 1, 0);
    const size_t cplane = (size_t)cnx * cny;
    const size_t rJ = (size_t)J * cnx, rY = (size_t)Jy * cnx;
    auto load = [&](int K) {
        const size_t base = (size_t)K * cplane;
        return pro_plane<T>(ac[base + rJ + I], ac[base + rJ + Im], ac[base + rJ + Ip], ac[base + rY + I],
                            ac[base + rY + Im], ac[base + rY + Ip], ec[base + rJ + I], ec[base + rJ + Im],
                            ec[base + rJ + Ip], ec[base + rY + I], ec[base + rY + Im], ec[base + rY + Ip]);
    };
    const size_t fplane = (size_t)nx * ny;
    const size_t fcol = (size_t)j * nx + 2 * I;
    ProPlane<T> c0 = load(K0), cp = load(min(K0 + 1, cnz - 1));
    ProFace<T> fl = pro_face(load(max(K0 - 1, 0)), c0);   // face K0 - 1/2 (wall: mirror)
    V n0 = *reinterpret_cast<const V*>(ef + (size_t)(2 * K0) * fplane + fcol);
    V n1 = *reinterpret_cast<const V*>(ef + (size_t)(2 * K0 + 1) * fplane + fcol);
    for (int K = K0; K < K1; K++) {
        V f0 = n0, f1 = n1;
        const ProPlane<T> cq = K + 1 < K1 ? load(min(K + 2, cnz - 1)) : cp;
        if (K + 1 < K1) {
            n0 = *reinterpret_cast<const V*>(ef + (size_t)(2 * K + 2) * fplane + fcol);
            n1 = *reinterpret_cast<const V*>(ef + (size_t)(2 * K + 3) * fplane + fcol);
        }
        const ProFace<T> fu = pro_face(c0, cp);   // face K + 1/2 (wall: mirror)
        f0.x += pro_child(c0, fl, 0) * T(0.125);
        f0.y += pro_child(c0, fl, 1) * T(0.125);
        f1.x += pro_child(c0, fu, 0) * T(0.125);
        f1.y += pro_child(c0, fu, 1) * T(0.125);
        *reinterpret_cast<V*>(ef + (size_t)(2 * K) * fplane + fcol) = f0;
        *reinterpret_cast<V*>(ef + (size_t)(2 * K + 1) * fplane + fcol) = f1;
        fl = fu;
        c0 = cp;
        cp = cq;
    }
}

// FP64 update p = (p - mean) + s * e32, the mean being shift_sum[0] / N (the
// mean-zero projection of the previous iterate, folded into this pass) and s
// = scal_s[0] the scale the residual was divided by.
__global__ void k_refine_update(double* __restrict__ p, const float* __restrict__ e, const double* __restrict__ scal_s,
                                size_t n, const double* __restrict__ shift_sum, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    p = rb(p, off_);
    e = rb(e, off_);
    scal_s = rb(scal_s, off_);
    shift_sum = rb(shift_sum, off_);
    const double c = shift_sum[0] / (double)n;
    const double s = scal_s[0];
    for (size_t t = (size_t)bid_ * blockDim.x + threadIdx.x; t < n; t += (size_t)nb_ * blockDim.x)
        p[t] = (p[t] - c) + s * (double)e[t];
}

// The same update, one thread per value pair (n even, p 16-byte aligned), 512
// threads per workgroup: the streaming form that measured fastest here.
__global__ void __launch_bounds__(512) k_refine_update2(double* __restrict__ p, const float* __restrict__ e,
                                                        const double* __restrict__ scal_s, size_t n,
                                                        const double* __restrict__ shift_sum, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    p = rb(p, off_);
    e = rb(e, off_);
    scal_s = rb(scal_s, off_);
    shift_sum = rb(shift_sum, off_);
    const size_t t = (size_t)bid_ * 512 + threadIdx.x;
    if (2 * t >= n) return;
    const double c = shift_sum[0] / (double)n;
    const double s = scal_s[0];
    double2 v = *reinterpret_cast<const double2*>(p + 2 * t);
    const float2 w = *reinterpret_cast<const float2*>(e + 2 * t);
    v.x = (v.x - c) + s * (double)w.x;
    v.y = (v.y - c) + s * (double)w.y;
    *reinterpret_cast<double2*>(p + 2 * t) = v;
}

// p -= sum/n for n values (n even, p 16-byte aligned), one thread per pair.
__global__ void __launch_bounds__(512) k_sub_mean2(double* __restrict__ p, const double* __restrict__ sum, size_t n, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    p = rb(p, off_);
    sum = rb(sum, off_);
    const size_t t = (size_t)bid_ * 512 + threadIdx.x;
    if (2 * t >= n) return;
    const double mean = sum[0] / (double)n;
    double2 v = *reinterpret_cast<const double2*>(p + 2 * t);
    v.x = v.x - mean;
    v.y = v.y - mean;
    *reinterpret_cast<double2*>(p + 2 * t) = v;
}

// dst = src for n values (the device-to-device copy inside a cycle, as a kernel
// so that a cycle holds kernels only).
template <class T>
__global__ void k_copy(T* __restrict__ dst, const T* __restrict__ src, size_t n, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    dst = rb(dst, off_);
    src = rb(src, off_);
    for (size_t t = (size_t)bid_ * blockDim.x + threadIdx.x; t < n; t += (size_t)nb_ * blockDim.x) dst[t] = src[t];
}

// out[2 s], out[2 s + 1] = the problem's scalars src[0], src[1], for the problem
// of slot s (slot 0 for a single problem); out is an address, not an offset.
// One block of one wavefront per problem.
__global__ void k_gather2(const double* __restrict__ src, double* __restrict__ out, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    const int slot = bt.base ? (int)blockIdx.x / bt.per : 0;
    src = rb(src, off_);
    if (threadIdx.x < 2) out[2 * slot + threadIdx.x] = src[threadIdx.x];
}

// ---------------------------------------------------------------- Krylov acceleration
//
// Flexible conjugate gradients on A = -L, preconditioned by one V-cycle from a
// zero guess (FP64).  Per iteration, after z = V(r): k_fcg_dots (z.q, r.z),
// k_fcg_beta, k_fcg_direction (q = L s for the new direction s = z + beta s_old,
// and s.q), k_fcg_update (s and p), then the residual pass r = b - L p (MODE 2).
// The scalars stay in device memory: scal[10] = z.q, scal[11] = r.z,
// scal[12] = s.q, scal[14] = beta, so an iteration needs no host round trip.

// Partial sums of z.q and r.z over the cells (column grid, k strided by gridDim.z).
__global__ void __launch_bounds__(BX* BY) k_fcg_dots(const double* __restrict__ z, const double* __restrict__ q,
                                                    const double* __restrict__ r, int nx, int ny, int nz,
                                                    double* __restrict__ part, Bt bt) {
    int kz_, nkz_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.z, gridDim.z, kz_, nkz_, off_)) return;
    z = rb(z, off_);
    q = rb(q, off_);
    r = rb(r, off_);
    part = rb(part, off_);
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, b = 0;
    if (i < nx && j < ny)
        for (int k = kz_; k < nz; k += nkz_) {
            const size_t c = cidx(i, j, k, nx, ny);
            a += z[c] * q[c];
            b += r[c] * z[c];
        }
    block_partials2(a, b, part, flat_bid(kz_));
}

// beta = -(z.q) / (s.q) with the previous direction's s.q; 0 before the first
// direction (s.q is reset to 0 when a solve starts).
__global__ void k_fcg_beta(double* __restrict__ scal, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    scal = rb(scal, off_);
    if (threadIdx.x == 0) {
        const double sq = scal[12];
        scal[14] = sq == 0.0 ? 0.0 : -scal[10] / sq;
    }
}

// One plane of NC cells of the combination v = z + beta s_old (fma, the same
// expression k_fcg_update stores), with neighbours and faces as load_cells1.
template <int NC>
__device__ __forceinline__ Cells1<double, NC> load_comb(const Lvl<double>& L, const double* __restrict__ z,
                                                        const double* __restrict__ so, double beta,
                                                        const CellOff& o, int k) {
    const Cells1<double, NC> a = load_cells1<double, NC>(L, z, z, o, k);
    const Cells1<double, NC> b = load_cells1<double, NC>(L, so, so, o, k);
    Cells1<double, NC> v = a;
#pragma unroll
    for (int e = 0; e < NC; e++) {
        v.p[e] = fma(beta, b.p[e], a.p[e]);
        v.ps[e] = fma(beta, b.ps[e], a.ps[e]);
        v.pn[e] = fma(beta, b.pn[e], a.pn[e]);
        v.b[e] = 0.0;
    }
    v.pw = fma(beta, b.pw, a.pw);
    v.pe = fma(beta, b.pe, a.pe);
    return v;
}

// q = L s for the new direction s = z + beta s_old (s itself is not stored
// here, so no thread overwrites a value its neighbours still read), with
// partial sums of s.q.  nx divisible by NC; tiles as k_resid_cells.
template <int NC>
__global__ void __launch_bounds__(CBX* CBY) k_fcg_direction(Lvl<double> L, const double* __restrict__ z,
                                                           const double* __restrict__ so,
                                                           const double* __restrict__ scal, ColGrid G,
                                                           double* __restrict__ q, double* __restrict__ part, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    L = L.rebased(off_);
    z = rb(z, off_);
    so = rb(so, off_);
    scal = rb(scal, off_);
    q = rb(q, off_);
    part = rb(part, off_);
    const int tile = xcd_tile(bid_, nb_);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int I = tx * CBX + (int)(threadIdx.x % CBX), j = ty * CBY + (int)(threadIdx.x / CBX);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    const double beta = scal[14];
    double a = 0;
    const bool active = NC * I < nx && j < ny;
    if (k0 < k1) {   // the same for the whole workgroup
        const size_t plane = (size_t)nx * ny;
        // threads outside the grid load at cell (0, 0) and keep nothing
        const CellOff o = cell_offsets<NC>(active ? I : 0, active ? j : 0, nx, ny);
        double vb[NC];
        {
            const size_t cb = (size_t)max(k0 - 1, 0) * plane + o.c;
#pragma unroll
            for (int e = 0; e < NC; e++) vb[e] = fma(beta, so[cb + e], z[cb + e]);
        }
        Cells1<double, NC> cur = load_comb<NC>(L, z, so, beta, o, k0);
        for (int k = k0; k < k1; k++) {
            __syncthreads();   // the row wavefronts in step (as in k_resid_cells)
            const Cells1<double, NC> nxt = load_comb<NC>(L, z, so, beta, o, plane_above(k, nz));
            double r[NC];
            cells_residual(cur, vb, nxt, r);   // r = 0 - L s
#pragma unroll
            for (int e = 0; e < NC; e++) {
                const double qv = -r[e];
                if (active) {
                    q[(size_t)k * plane + o.c + e] = qv;
                    a += cur.p[e] * qv;
                }
                vb[e] = cur.p[e];
            }
            cur = nxt;
        }
    }
    __shared__ double sa[CBX * CBY / 64];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (threadIdx.x % 64 == 0) sa[threadIdx.x / 64] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0;
        for (int w = 0; w < CBX * CBY / 64; w++) ta += sa[w];
        part[2 * tile] = ta;
        part[2 * tile + 1] = 0.0;
    }
}

// s = z + beta s_old (stored), p += alpha s with alpha = (r.z) / (s.q).
__global__ void k_fcg_update(const double* __restrict__ z, double* __restrict__ s, double* __restrict__ p,
                             const double* __restrict__ scal, size_t n, Bt bt) {
    int bid_, nb_;
    uintptr_t off_;
    if (!bt_enter(bt, blockIdx.x, gridDim.x, bid_, nb_, off_)) return;
    z = rb(z, off_);
    s = rb(s, off_);
    p = rb(p, off_);
    scal = rb(scal, off_);
    const double beta = scal[14], alpha = scal[11] / scal[12];
    size_t t = (size_t)bid_ * blockDim.x + threadIdx.x;
    for (; t < n; t += (size_t)nb_ * blockDim.x) {
        const double sv = fma(beta, s[t], z[t]);
        s[t] = sv;
        p[t] = fma(alpha, sv, p[t]);
    }
}

}  // namespace mgk
