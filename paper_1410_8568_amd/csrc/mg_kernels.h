// Device kernels of the multigrid pressure solve (gfx950).
//
// Every kernel here is bandwidth-bound stencil or transfer work; none is a dense
// contraction, so none uses MFMA.  Arrays are [k][j][i] with i fastest; x-faces
// [nz][ny][nx+1], y-faces [nz][ny+1][nx], z-faces [nz+1][ny][nx]; wall faces are
// stored as 0, so the stencil needs no boundary branches on the coefficients
// (out-of-grid neighbour values are read as 0 instead).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgk {

constexpr int BX = 64;   // threads along i (one wavefront)
constexpr int BY = 4;    // rows per block
constexpr int RED_THREADS = 256;
constexpr int FIN_THREADS = 1024;

__device__ __forceinline__ size_t cidx(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * nx + i;
}
__device__ __forceinline__ size_t fxi(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * (nx + 1) + i;
}
__device__ __forceinline__ size_t fyi(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * (ny + 1) + j) * nx + i;
}
__device__ __forceinline__ size_t fzi(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * nx + i;
}

template <class T>
struct Lvl {
    int nx, ny, nz;
    const T* bx;
    const T* by;
    const T* bz;
};

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

// Neighbour sum s = sum_f beta_f p_nb and diagonal d = sum_f beta_f for cell
// (i,j,k); out-of-grid neighbours read as 0 (their face coefficient is 0).
template <class T>
__device__ __forceinline__ void nbsum(const Lvl<T>& L, const T* __restrict__ p, int i, int j, int k,
                                      T& s, T& d) {
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const size_t c = cidx(i, j, k, nx, ny);
    T w0 = L.bx[fxi(i, j, k, nx, ny)], w1 = L.bx[fxi(i + 1, j, k, nx, ny)];
    T w2 = L.by[fyi(i, j, k, nx, ny)], w3 = L.by[fyi(i, j + 1, k, nx, ny)];
    T w4 = L.bz[fzi(i, j, k, nx, ny)], w5 = L.bz[fzi(i, j, k + 1, nx, ny)];
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
__device__ __forceinline__ int flat_bid() {
    return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// 2-D block (BX x BY) variant writing two partial sums per block.
__device__ __forceinline__ void block_partials2(double a, double b, double* __restrict__ part) {
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
        const int bid = flat_bid();
        part[2 * bid] = ta;
        part[2 * bid + 1] = tb;
    }
}

// out[q] = sum over blocks of part[2*blk+q] (q = 0,1), fixed order.  One block.
__global__ void __launch_bounds__(FIN_THREADS) k_finish2(const double* __restrict__ part, int nblk,
                                                         double* __restrict__ out) {
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
                                                  double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, b = 0;
    if (i < nx && j < ny)
        for (int k = blockIdx.z; k < nz; k += gridDim.z) {
            double v = (double)x[cidx(i, j, k, nx, ny)];
            a += v;
            b += v * v;
        }
    block_partials2(a, b, part);
}

// y = x - sum/n (sum read from device memory); partial sums of y and y^2.
__global__ void __launch_bounds__(BX* BY) k_project(const double* __restrict__ x, double* __restrict__ y,
                                                   const double* __restrict__ sum, int nx, int ny, int nz,
                                                   double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    const double mean = sum[0] / ((double)nx * ny * nz);
    double a = 0, b = 0;
    if (i < nx && j < ny)
        for (int k = blockIdx.z; k < nz; k += gridDim.z) {
            size_t c = cidx(i, j, k, nx, ny);
            double v = x[c] - mean;
            y[c] = v;
            a += v;
            b += v * v;
        }
    block_partials2(a, b, part);
}

// x -= sum/n (sum from device memory).
template <class T>
__global__ void __launch_bounds__(BX* BY) k_sub_mean(T* __restrict__ x, const double* __restrict__ sum,
                                                    int nx, int ny, int nz) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const double mean = sum[0] / ((double)nx * ny * nz);
    for (int k = blockIdx.z; k < nz; k += gridDim.z) {
        size_t c = cidx(i, j, k, nx, ny);
        x[c] = (T)((double)x[c] - mean);
    }
}

template <class T>
__global__ void k_fill(T* __restrict__ x, size_t n, T v) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t < n; t += (size_t)gridDim.x * blockDim.x) x[t] = v;
}

__global__ void k_cast_d2f(const double* __restrict__ x, float* __restrict__ y, size_t n) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; t < n; t += (size_t)gridDim.x * blockDim.x) y[t] = (float)x[t];
}

// ---------------------------------------------------------------- setup

// Copy caller faces with walls forced to 0; count non-finite or non-positive
// interior coefficients into *bad.
__global__ void k_copy_faces(const double* __restrict__ src, double* __restrict__ dst, int n0, int n1,
                             int n2, int axis, int* __restrict__ bad) {
    // array dims [n2][n1][n0]; the face index along `axis` (0: n0, 1: n1, 2: n2) is a wall
    // at 0 and at its extent - 1
    size_t total = (size_t)n0 * n1 * n2;
    int nbad = 0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        int i0 = (int)(t % n0);
        size_t r = t / n0;
        int i1 = (int)(r % n1);
        int i2 = (int)(r / n1);
        int f = axis == 0 ? i0 : (axis == 1 ? i1 : i2);
        int ext = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
        double v = 0.0;
        if (f > 0 && f < ext - 1) {
            v = src[t];
            if (!(v > 0.0) || !(v < 1e300)) nbad++;
        }
        dst[t] = v;
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Coarse faces = mean of the 2 x 2 fine faces they cover, ((f00+f10)+(f01+f11))/4.
__global__ void k_coarsen_x(const double* __restrict__ f, double* __restrict__ c, int fnx, int fny, int cnx,
                            int cny, int cnz) {
    size_t total = (size_t)(cnx + 1) * cny * cnz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        int I = (int)(t % (cnx + 1));
        size_t r = t / (cnx + 1);
        int J = (int)(r % cny), K = (int)(r / cny);
        double s0 = f[fxi(2 * I, 2 * J, 2 * K, fnx, fny)] + f[fxi(2 * I, 2 * J + 1, 2 * K, fnx, fny)];
        double s1 = f[fxi(2 * I, 2 * J, 2 * K + 1, fnx, fny)] + f[fxi(2 * I, 2 * J + 1, 2 * K + 1, fnx, fny)];
        c[t] = 0.25 * (s0 + s1);
    }
}

__global__ void k_coarsen_y(const double* __restrict__ f, double* __restrict__ c, int fnx, int fny, int cnx,
                            int cny, int cnz) {
    size_t total = (size_t)cnx * (cny + 1) * cnz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        int I = (int)(t % cnx);
        size_t r = t / cnx;
        int J = (int)(r % (cny + 1)), K = (int)(r / (cny + 1));
        double s0 = f[fyi(2 * I, 2 * J, 2 * K, fnx, fny)] + f[fyi(2 * I + 1, 2 * J, 2 * K, fnx, fny)];
        double s1 = f[fyi(2 * I, 2 * J, 2 * K + 1, fnx, fny)] + f[fyi(2 * I + 1, 2 * J, 2 * K + 1, fnx, fny)];
        c[t] = 0.25 * (s0 + s1);
    }
}

__global__ void k_coarsen_z(const double* __restrict__ f, double* __restrict__ c, int fnx, int fny, int cnx,
                            int cny, int cnz) {
    size_t total = (size_t)cnx * cny * (cnz + 1);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        int I = (int)(t % cnx);
        size_t r = t / cnx;
        int J = (int)(r % cny), K = (int)(r / cny);
        double s0 = f[fzi(2 * I, 2 * J, 2 * K, fnx, fny)] + f[fzi(2 * I + 1, 2 * J, 2 * K, fnx, fny)];
        double s1 = f[fzi(2 * I, 2 * J + 1, 2 * K, fnx, fny)] + f[fzi(2 * I + 1, 2 * J + 1, 2 * K, fnx, fny)];
        c[t] = 0.25 * (s0 + s1);
    }
}

// Cell weight = mean of beta over the cell's interior faces (x-, x+, y-, y+, z-, z+).
__global__ void k_cell_weights(const double* __restrict__ bx, const double* __restrict__ by,
                               const double* __restrict__ bz, double* __restrict__ a, int nx, int ny, int nz) {
    size_t total = (size_t)nx * ny * nz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(t % nx);
        size_t r = t / nx;
        int j = (int)(r % ny), k = (int)(r / ny);
        double s = 0;
        int cnt = 0;
        if (i > 0) { s += bx[fxi(i, j, k, nx, ny)]; cnt++; }
        if (i < nx - 1) { s += bx[fxi(i + 1, j, k, nx, ny)]; cnt++; }
        if (j > 0) { s += by[fyi(i, j, k, nx, ny)]; cnt++; }
        if (j < ny - 1) { s += by[fyi(i, j + 1, k, nx, ny)]; cnt++; }
        if (k > 0) { s += bz[fzi(i, j, k, nx, ny)]; cnt++; }
        if (k < nz - 1) { s += bz[fzi(i, j, k + 1, nx, ny)]; cnt++; }
        a[t] = cnt ? s / cnt : 1.0;
    }
}

// Dense inverse of B = -L + (sigma/n) 1 1^T on the coarsest grid (one block,
// B in global memory, n <= 512): assemble, then in-place Gauss-Jordan without
// pivoting (B is symmetric positive definite, every pivot is positive).
// *bad is incremented if a pivot is not positive.
__global__ void __launch_bounds__(FIN_THREADS) k_coarse_invert(const double* __restrict__ bx,
                                                               const double* __restrict__ by,
                                                               const double* __restrict__ bz, int nx, int ny,
                                                               int nz, double* __restrict__ B,
                                                               int* __restrict__ bad) {
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
        double dg = 0;
        if (i > 0) { double w = bx[fxi(i, j, k, nx, ny)]; dg += w; B[(size_t)c * n + c - 1] = -w; }
        if (i < nx - 1) { double w = bx[fxi(i + 1, j, k, nx, ny)]; dg += w; B[(size_t)c * n + c + 1] = -w; }
        if (j > 0) { double w = by[fyi(i, j, k, nx, ny)]; dg += w; B[(size_t)c * n + c - nx] = -w; }
        if (j < ny - 1) { double w = by[fyi(i, j + 1, k, nx, ny)]; dg += w; B[(size_t)c * n + c + nx] = -w; }
        if (k > 0) { double w = bz[fzi(i, j, k, nx, ny)]; dg += w; B[(size_t)c * n + c - nx * ny] = -w; }
        if (k < nz - 1) { double w = bz[fzi(i, j, k + 1, nx, ny)]; dg += w; B[(size_t)c * n + c + nx * ny] = -w; }
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
                                                   int colour) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= L.nx || j >= L.ny) return;
    for (int k = blockIdx.z; k < L.nz; k += gridDim.z) {
        if (((i + j + k) & 1) != colour) continue;
        T s, d;
        nbsum(L, p, i, j, k, s, d);
        size_t c = cidx(i, j, k, L.nx, L.ny);
        p[c] = (s - b[c]) / d;
    }
}

// Residual r = b - L p restricted: rc(I,J,K) = 1/2 * sum of the 8 child residuals.
template <class T>
__global__ void __launch_bounds__(BX* BY) k_residual_restrict(Lvl<T> L, const T* __restrict__ p,
                                                             const T* __restrict__ b, T* __restrict__ rc) {
    const int cnx = L.nx / 2, cny = L.ny / 2, cnz = L.nz / 2;
    const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y;
    if (I >= cnx || J >= cny) return;
    for (int K = blockIdx.z; K < cnz; K += gridDim.z) {
        T acc = 0;
        for (int c = 0; c < 2; c++)
            for (int bb = 0; bb < 2; bb++)
                for (int a = 0; a < 2; a++) {
                    int i = 2 * I + a, j = 2 * J + bb, k = 2 * K + c;
                    T s, d;
                    nbsum(L, p, i, j, k, s, d);
                    size_t cc = cidx(i, j, k, L.nx, L.ny);
                    acc += b[cc] - (s - d * p[cc]);
                }
        rc[cidx(I, J, K, cnx, cny)] = T(0.5) * acc;
    }
}

// Flux-conserving prolongation and correction: fine cell in octant s of coarse
// cell C gets (1/8) * sum over T subset of {x,y,z} of the weight-averaged coarse
// error over the 2^|T| coarse cells sharing the octant corner T (wall mirror
// by index clamping).
template <class T>
__global__ void __launch_bounds__(BX* BY) k_prolong_add(const T* __restrict__ ec, const T* __restrict__ ac,
                                                       int cnx, int cny, int cnz, T* __restrict__ ef) {
    const int nx = 2 * cnx, ny = 2 * cny, nz = 2 * cnz;
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const int I = i >> 1, J = j >> 1;
    const int Ix = (i & 1) ? min(I + 1, cnx - 1) : max(I - 1, 0);
    const int Jy = (j & 1) ? min(J + 1, cny - 1) : max(J - 1, 0);
    for (int k = blockIdx.z; k < nz; k += gridDim.z) {
        const int K = k >> 1;
        const int Kz = (k & 1) ? min(K + 1, cnz - 1) : max(K - 1, 0);
        T av[8], wv[8];
#pragma unroll
        for (int dl = 0; dl < 8; dl++) {
            int ci = (dl & 1) ? Ix : I, cj = (dl & 2) ? Jy : J, ck = (dl & 4) ? Kz : K;
            size_t m = cidx(ci, cj, ck, cnx, cny);
            av[dl] = ac[m];
            wv[dl] = ac[m] * ec[m];
        }
        T total = 0;
#pragma unroll
        for (int Tm = 0; Tm < 8; Tm++) {
            T num = 0, den = 0;
#pragma unroll
            for (int dl = 0; dl < 8; dl++) {
                if (dl & ~Tm) continue;
                num += wv[dl];
                den += av[dl];
            }
            total += num / den;
        }
        size_t c = cidx(i, j, k, nx, ny);
        ef[c] += total / T(8);
    }
}

// Convergence check: partial sums of r^2 (r = b - L p) and of p, FP64 accumulation.
template <class T>
__global__ void __launch_bounds__(BX* BY) k_resid_norm(Lvl<T> L, const T* __restrict__ p,
                                                      const T* __restrict__ b, double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, q = 0;
    if (i < L.nx && j < L.ny)
        for (int k = blockIdx.z; k < L.nz; k += gridDim.z) {
            T s, d;
            nbsum(L, p, i, j, k, s, d);
            size_t c = cidx(i, j, k, L.nx, L.ny);
            double r = (double)(b[c] - (s - d * p[c]));
            a += r * r;
            q += (double)p[c];
        }
    block_partials2(a, q, part);
}

// Exact coarsest solve e = -B^{-1} (r - mean r), FP64 arithmetic; one block.
template <class T>
__global__ void __launch_bounds__(512) k_coarse_solve(const double* __restrict__ Binv, int n,
                                                     const T* __restrict__ r, T* __restrict__ e) {
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
    if (t < n) {
        double acc = 0;
        for (int jj = 0; jj < n; jj++) acc += Binv[(size_t)jj * n + t] * rs[jj];
        e[t] = (T)(-acc);
    }
}

// Workgroup barrier that only orders LDS traffic: waits for this wave's
// outstanding LDS operations, not for its global loads, so loads issued for the
// next plane stay in flight across it.  (Global results are only consumed by
// the issuing thread, after the compiler's own wait.)
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Map the dispatch order of workgroups onto tiles so that each XCD works on a
// contiguous range of tiles: workgroup w is dispatched to XCD w % 8, and XCD x
// receives logical tiles [start_x, start_x + count_x).  Neighbouring tiles then
// share one L2, where their halo re-reads hit.
__device__ __forceinline__ int xcd_tile(int w, int nwg) {
    const int q = nwg >> 3, r = nwg & 7, x = w & 7, m = w >> 3;
    return x * q + min(x, r) + m;
}

// One full red-black Gauss-Seidel sweep (colour c0 first, then 1 - c0) in a
// single pass over HBM, out of place (pin -> pout, so tiles never race).
//
// A workgroup owns a TX x TY column of cells and marches upward through a chunk
// of kc planes.  Planes of pin are staged in LDS with a 2-cell ring; the first
// colour is updated on the tile plus a 1-cell ring (the ring values are the
// same ones the neighbouring tile computes, bit for bit), so the second colour
// can be updated on the tile from LDS alone.  At step t the first colour is
// updated on plane t and the second colour on plane t-1, which is then final
// and written out.  Thread (li, lj) owns ring-1 column (li, lj) and keeps that
// column's face coefficients and right-hand side for two planes in registers.
// Below plane k0 and above k1-1 the first colour is recomputed redundantly
// (planes k0-1 and k1) so chunks are independent.  The global loads of plane
// t+2 (pin) and t+1 (faces, b) are issued before the compute of step t and
// written to LDS at the start of step t+1.
template <class T, int TX, int TY>
__global__ void __launch_bounds__((TX + 2) * (TY + 2)) k_rb_sweep(Lvl<T> L, const T* __restrict__ pin,
                                                                  T* __restrict__ pout, const T* __restrict__ b,
                                                                  int c0, int kc, int tiles_x, int tiles_y) {
    constexpr int W = TX + 4, H = TY + 4, NT = (TX + 2) * (TY + 2), NS = 5;
    constexpr int NP = (H * W + NT - 1) / NT;  // ring cells loaded per thread
    __shared__ T sp[NS][H][W];
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, chunk = tile / (tiles_x * tiles_y);
    const int i0 = tx * TX, j0 = ty * TY;
    const int k0 = chunk * kc, k1 = min(nz, k0 + kc);
    const int tid = threadIdx.x;
    const int li = tid % (TX + 2), lj = tid / (TX + 2);
    const int gi = i0 + li - 1, gj = j0 + lj - 1;
    const bool incell = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
    const bool interior = incell && li >= 1 && li <= TX && lj >= 1 && lj <= TY;
    const size_t plane = (size_t)nx * ny;

    // the ring cells this thread stages: offsets into a plane (-1 = outside the grid)
    long roff[NP];
    int rpos[NP];
#pragma unroll
    for (int u = 0; u < NP; u++) {
        const int q = tid + u * NT;
        rpos[u] = q < H * W ? q : -1;
        const int qi = q % W, qj = q / W;
        const int ii = i0 + qi - 2, jj = j0 + qj - 2;
        roff[u] = (q < H * W && ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? (long)jj * nx + ii : -1;
    }
    T* const spf = &sp[0][0][0];
    auto slot = [](int k) { return (k + 2 * NS) % NS; };
    auto fetch_ring = [&](int k, T* v) {
        const bool kin = k >= 0 && k < nz;
#pragma unroll
        for (int u = 0; u < NP; u++) v[u] = (kin && roff[u] >= 0) ? pin[(size_t)k * plane + roff[u]] : T(0);
    };
    auto store_ring = [&](int k, const T* v) {
        T* dst = spf + slot(k) * (H * W);
#pragma unroll
        for (int u = 0; u < NP; u++)
            if (rpos[u] >= 0) dst[rpos[u]] = v[u];
    };
    struct FB {
        T w0, w1, w2, w3, w4, w5, bb;
    };
    auto fetch_fb = [&](int k) {
        FB f{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
        if (incell && k >= 0 && k < nz) {
            f.w0 = L.bx[fxi(gi, gj, k, nx, ny)];
            f.w1 = L.bx[fxi(gi + 1, gj, k, nx, ny)];
            f.w2 = L.by[fyi(gi, gj, k, nx, ny)];
            f.w3 = L.by[fyi(gi, gj + 1, k, nx, ny)];
            f.w4 = L.bz[fzi(gi, gj, k, nx, ny)];
            f.w5 = L.bz[fzi(gi, gj, k + 1, nx, ny)];
            f.bb = b[(size_t)k * plane + (size_t)gj * nx + gi];
        }
        return f;
    };

    T ring[NP];
    fetch_ring(k0 - 2, ring);
    store_ring(k0 - 2, ring);
    fetch_ring(k0 - 1, ring);
    store_ring(k0 - 1, ring);
    fetch_ring(k0, ring);              // plane t+1 for the first step
    FB fnext = fetch_fb(k0 - 1);       // plane t for the first step
    FB fcur, fprev = fnext;
    for (int t = k0 - 1; t <= k1; t++) {
        store_ring(t + 1, ring);
        fcur = fnext;
        lds_barrier();
        fetch_ring(t + 2, ring);       // in flight during this step
        fnext = fetch_fb(t + 1);
        if (incell && t >= 0 && t < nz && (((gi + gj + t) & 1) == c0)) {
            T(*c)[W] = sp[slot(t)];
            const T s = stencil_sum(fcur.w0, fcur.w1, fcur.w2, fcur.w3, fcur.w4, fcur.w5, c[lj + 1][li],
                                    c[lj + 1][li + 2], c[lj][li + 1], c[lj + 2][li + 1],
                                    sp[slot(t - 1)][lj + 1][li + 1], sp[slot(t + 1)][lj + 1][li + 1]);
            c[lj + 1][li + 1] = (s - fcur.bb) / stencil_diag(fcur.w0, fcur.w1, fcur.w2, fcur.w3, fcur.w4, fcur.w5);
        }
        lds_barrier();
        const int tp = t - 1;
        if (interior && tp >= k0 && tp < k1) {
            T(*c)[W] = sp[slot(tp)];
            T v;
            if (((gi + gj + tp) & 1) != c0) {
                const T s = stencil_sum(fprev.w0, fprev.w1, fprev.w2, fprev.w3, fprev.w4, fprev.w5, c[lj + 1][li],
                                        c[lj + 1][li + 2], c[lj][li + 1], c[lj + 2][li + 1],
                                        sp[slot(tp - 1)][lj + 1][li + 1], sp[slot(tp + 1)][lj + 1][li + 1]);
                v = (s - fprev.bb) / stencil_diag(fprev.w0, fprev.w1, fprev.w2, fprev.w3, fprev.w4, fprev.w5);
            } else {
                v = c[lj + 1][li + 1];
            }
            pout[(size_t)tp * plane + (size_t)gj * nx + gi] = v;
        }
        fprev = fcur;
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
    v.wx0 = L.bx[fxi(i, j, k, nx, ny)];
    v.wx1 = L.bx[fxi(i + 1, j, k, nx, ny)];
    v.wy0 = L.by[fyi(i, j, k, nx, ny)];
    v.wy1 = L.by[fyi(i, j + 1, k, nx, ny)];
    v.wz1 = L.bz[fzi(i, j, k + 1, nx, ny)];
    return v;
}

// Residual r = b - L p along each column; MODE 0: partial sums of r^2 and p;
// MODE 1 (FP64 refinement): also writes r32 = float(r * inv_s).
template <class T, int MODE>
__global__ void __launch_bounds__(CBX* CBY) k_resid_col(Lvl<T> L, const T* __restrict__ p, const T* __restrict__ b,
                                                       ColGrid G, double inv_s, float* __restrict__ r32,
                                                       double* __restrict__ part) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int i = tx * CBX + (int)(threadIdx.x % CBX), j = ty * CBY + (int)(threadIdx.x / CBX);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    double a = 0, q = 0;
    if (i < nx && j < ny && k0 < k1) {
        const size_t plane = (size_t)nx * ny;
        const size_t col = (size_t)j * nx + i;
        T pbelow = k0 > 0 ? p[(size_t)(k0 - 1) * plane + col] : T(0);
        T wz0 = L.bz[fzi(i, j, k0, nx, ny)];
        Plane1<T> cur = load_plane1(L, p, b, i, j, k0);
        Plane1<T> nxt = cur;
        for (int k = k0; k < k1; k++) {
            if (k + 1 < nz) nxt = load_plane1(L, p, b, i, j, k + 1);
            const T pabove = k + 1 < nz ? nxt.p : T(0);
            const T s = stencil_sum(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1, cur.pw, cur.pe, cur.ps,
                                    cur.pn, pbelow, pabove);
            const T d = stencil_diag(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1);
            const T r = cur.b - (s - d * cur.p);
            if (MODE == 1) r32[(size_t)k * plane + col] = (float)((double)r * inv_s);
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

// Residual restricted to the next level.  A wavefront covers 32 x 2 fine
// columns (lane l: i = i0 + l % 32, j = j0 + l / 32), so the 2 x 2 children of
// a coarse column sit in lanes l, l^1, l^32, l^33; each thread marches up its
// column, sums its residuals over the plane pair 2K, 2K+1, and the four sums are
// combined with lane shuffles.  rc(I,J,K) = 1/2 * (sum of the 8 child residuals).
// Tiles are 32 x 8 fine columns (4 wavefronts); kc (planes per chunk) is even.
constexpr int RBX = 32, RBY = 8;

template <class T>
__global__ void __launch_bounds__(256) k_resid_restrict_col(Lvl<T> L, const T* __restrict__ p,
                                                           const T* __restrict__ b, ColGrid G,
                                                           T* __restrict__ rc) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, chunk = tile / (G.tiles_x * G.tiles_y);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int cnx = nx / 2, cny = ny / 2;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int i = tx * RBX + lane % 32, j = ty * RBY + 2 * wave + lane / 32;
    const int k0 = chunk * G.kc, k1 = min(nz, k0 + G.kc);
    const bool active = i < nx && j < ny;   // nx, ny even: a 2x2 group is all in or all out
    const size_t plane = (size_t)nx * ny;
    const size_t col = (size_t)j * nx + i;
    T pbelow = T(0), wz0 = T(0);
    Plane1<T> cur{}, nxt{};
    if (active && k0 < k1) {
        pbelow = k0 > 0 ? p[(size_t)(k0 - 1) * plane + col] : T(0);
        wz0 = L.bz[fzi(i, j, k0, nx, ny)];
        cur = load_plane1(L, p, b, i, j, k0);
    }
    T acc = 0;
    for (int k = k0; k < k1; k++) {
        if (active) {
            if (k + 1 < nz) nxt = load_plane1(L, p, b, i, j, k + 1);
            const T pabove = k + 1 < nz ? nxt.p : T(0);
            const T s = stencil_sum(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1, cur.pw, cur.pe, cur.ps, cur.pn,
                                    pbelow, pabove);
            const T d = stencil_diag(cur.wx0, cur.wx1, cur.wy0, cur.wy1, wz0, cur.wz1);
            acc += cur.b - (s - d * cur.p);
            pbelow = cur.p;
            wz0 = cur.wz1;
            cur = nxt;
        }
        if (k & 1) {
            T v = acc;
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 32, 64);
            if (active && !(i & 1) && !(j & 1)) rc[cidx(i >> 1, j >> 1, k >> 1, cnx, cny)] = T(0.5) * v;
            acc = 0;
        }
    }
}

// FP64 refinement residual: r = b - L p (FP64), r32 = float(r * inv_s), partial sums
// of r^2 and of p.
__global__ void __launch_bounds__(BX* BY) k_refine_residual(Lvl<double> L, const double* __restrict__ p,
                                                           const double* __restrict__ b, double inv_s,
                                                           float* __restrict__ r32, double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, q = 0;
    if (i < L.nx && j < L.ny)
        for (int k = blockIdx.z; k < L.nz; k += gridDim.z) {
            double s, d;
            nbsum(L, p, i, j, k, s, d);
            size_t c = cidx(i, j, k, L.nx, L.ny);
            double r = b[c] - (s - d * p[c]);
            r32[c] = (float)(r * inv_s);
            a += r * r;
            q += p[c];
        }
    block_partials2(a, q, part);
}

// FP64 update p += s * e32; partial sums of the updated p (for the mean) and of e^2.
__global__ void __launch_bounds__(BX* BY) k_refine_update(double* __restrict__ p, const float* __restrict__ e,
                                                         double s, int nx, int ny, int nz,
                                                         double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double a = 0, q = 0;
    if (i < nx && j < ny)
        for (int k = blockIdx.z; k < nz; k += gridDim.z) {
            size_t c = cidx(i, j, k, nx, ny);
            double v = p[c] + s * (double)e[c];
            p[c] = v;
            a += v;
            q += (double)e[c] * (double)e[c];
        }
    block_partials2(a, q, part);
}

}  // namespace mgk
