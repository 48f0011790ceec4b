// libplbm device code for gfx950: the fused collide-and-stream step of the
// parametric lattice Boltzmann method (arXiv:1402.5487, Eq. srt with the
// equilibrium of Eq. eqdist / Eq. rdr), initialisation, moments and the FP64
// invariant reductions, plus the C-ABI launchers that validate and enqueue
// them.
//
// Design (memory-bound streaming kernel):
//  * SoA planes, pull scheme: each node gathers population k from
//    src_k(x - v_k) and writes its post-collision value to dst_k(x), so every
//    plane is read once and written once per step, all with wave-contiguous
//    (coalesced) addresses; A/B buffers make the step race-free.
//  * One thread per node column inside a 256 x TY tile (four wave64 side by
//    side); each thread walks TY rows.  Tiles are numbered so that each of
//    the eight XCDs gets a contiguous band of rows: neighbouring tiles, whose
//    shifted windows share cache lines at their edges, meet in the same L2.
//  * Interior tiles address each plane as one scalar base plus one 32-bit lane
//    offset; only tiles touching the periodic seam wrap indices.
//  * Arithmetic per node: column/row sums give rho, j, and sum f|v|^2; the
//    Maxwell moments follow mu_(n+1) = u mu_n + n theta mu_(n-1); the 1D rules
//    are r = C mu per axis; f_eq = rho r^x_i r^y_j; the relaxation is folded
//    into a_i = omega rho r^x_i so each population costs one multiply and one
//    FMA.  FP64 storage computes in FP64; the other forms compute in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "plbm_internal.h"

namespace {

constexpr int Q = 5;            // velocities per axis compiled into the kernels
constexpr int NQ = Q * Q;       // populations of the 2D tensor-product model
constexpr int TX = 256;         // tile width = threads per block
constexpr int TY = 8;           // tile height (rows walked by each thread)
constexpr int NXCD = 8;         // accelerator complex dies on MI355X
constexpr int RED_THREADS = 256;

struct KParams {
    int nx, ny;
    int tiles_x, ntiles;
    int interior_x0, interior_x1;   // tile-x range whose windows never wrap
    int interior_y0, interior_y1;   // tile-y range whose windows never wrap
    int sx[Q];                      // integer velocities
    double v[Q];
    float vf[Q];
    double c[NQ];                   // c[i*Q + j]
    float cf[NQ];
    double omega;
    float omegaf;
    float base[NQ], scale[NQ], inv_scale[NQ];   // 16-bit deviation storage
    long long plane;                // elements per plane (2D) / padded row (1D)
};

// ---------------------------------------------------------------------------
// Storage forms
// ---------------------------------------------------------------------------
struct StF64 {
    using T = double;
    using C = double;
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &) { return f; }
    static __device__ __forceinline__ C coef(int i, const KParams &p) { return p.c[i]; }
    static __device__ __forceinline__ C vel(int i, const KParams &p) { return p.v[i]; }
    static __device__ __forceinline__ C om(const KParams &p) { return p.omega; }
};

struct StF32 {
    using T = float;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &) { return f; }
    static __device__ __forceinline__ C coef(int i, const KParams &p) { return p.cf[i]; }
    static __device__ __forceinline__ C vel(int i, const KParams &p) { return p.vf[i]; }
    static __device__ __forceinline__ C om(const KParams &p) { return p.omegaf; }
};

// f_k = base_k + scale_k * h_k, h stored as IEEE half; scales are powers of
// two, so only the half rounding (round to nearest even) and the subtraction
// of the base round.
struct StF16 {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        return fmaf(p.scale[k], (float)__builtin_bit_cast(_Float16, h), p.base[k]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p) {
        return __builtin_bit_cast(uint16_t, (_Float16)((f - p.base[k]) * p.inv_scale[k]));
    }
    static __device__ __forceinline__ C coef(int i, const KParams &p) { return p.cf[i]; }
    static __device__ __forceinline__ C vel(int i, const KParams &p) { return p.vf[i]; }
    static __device__ __forceinline__ C om(const KParams &p) { return p.omegaf; }
};

struct StBF16 {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        return fmaf(p.scale[k], __uint_as_float((uint32_t)h << 16), p.base[k]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p) {
        return __builtin_bit_cast(uint16_t, (__bf16)((f - p.base[k]) * p.inv_scale[k]));
    }
    static __device__ __forceinline__ C coef(int i, const KParams &p) { return p.cf[i]; }
    static __device__ __forceinline__ C vel(int i, const KParams &p) { return p.vf[i]; }
    static __device__ __forceinline__ C om(const KParams &p) { return p.omegaf; }
};

// ---------------------------------------------------------------------------
// Per-node arithmetic
// ---------------------------------------------------------------------------

// rho, rho u_x, rho u_y and sum f |v|^2 of 25 populations via column and row
// sums (population k = i + Q j moves with (v_i, v_j)).
template <class S>
__device__ __forceinline__ void sums2d(const typename S::C (&f)[NQ], const KParams &p,
                                       typename S::C &rho, typename S::C &jx,
                                       typename S::C &jy, typename S::C &e)
{
    using C = typename S::C;
    C col[Q], row[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        col[i] = f[i];
        row[i] = f[Q * i];
    }
#pragma unroll
    for (int j = 1; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < Q; ++i) col[i] += f[i + Q * j];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 1; i < Q; ++i) row[j] += f[i + Q * j];
    rho = col[0];
    jx = C(0);
    jy = C(0);
    e = C(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) rho += col[i];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C vi = S::vel(i, p);
        jx = fma(col[i], vi, jx);
        jy = fma(row[i], vi, jy);
        e = fma(col[i] + row[i], vi * vi, e);
    }
}

// 1D rule of Eq. rdr: r_i = sum_j c_ij mu_j with the Maxwell moments of
// (u, theta) built by the recurrence mu_(n+1) = u mu_n + n theta mu_(n-1).
template <class S>
__device__ __forceinline__ void rule1d(typename S::C u, typename S::C theta, const KParams &p,
                                       typename S::C (&r)[Q])
{
    using C = typename S::C;
    C mu[Q];
    mu[0] = C(1);
    mu[1] = u;
#pragma unroll
    for (int n = 1; n + 1 < Q; ++n) mu[n + 1] = fma(u, mu[n], C(n) * theta * mu[n - 1]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C s = S::coef(i * Q, p);
#pragma unroll
        for (int j = 1; j < Q; ++j) s = fma(S::coef(i * Q + j, p), mu[j], s);
        r[i] = s;
    }
}

// In place: f <- (1 - omega) f + omega f_eq (Eq. srt, collision half).
template <class S>
__device__ __forceinline__ void collide2d(typename S::C (&f)[NQ], const KParams &p)
{
    using C = typename S::C;
    C rho, jx, jy, e;
    sums2d<S>(f, p, rho, jx, jy, e);
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv;
    const C theta = C(0.5) * (e * inv - ux * ux - uy * uy);
    C rx[Q], ry[Q];
    rule1d<S>(ux, theta, p, rx);
    rule1d<S>(uy, theta, p, ry);
    const C w = S::om(p);
    const C keep = C(1) - w;
    const C wr = w * rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) rx[i] *= wr;
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i + Q * j] = fma(keep, f[i + Q * j], rx[i] * ry[j]);
}

// ---------------------------------------------------------------------------
// Reductions (FP64): wave64 butterfly, then LDS across the block's waves.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <int NV>
__device__ __forceinline__ void block_sums_store(double (&acc)[NV], double *out)
{
    __shared__ double red[NV][TX / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double s = wave_sum(acc[m]);
        if (lane == 0) red[m][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < TX / 64; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

// Deterministic second pass: one block adds the per-block partials in a fixed
// order with Neumaier compensation and writes NV doubles.
template <int NV>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_partials(const double *__restrict__ part,
                                                                 int nblocks, double *__restrict__ out)
{
    __shared__ double sh[RED_THREADS][2];
    for (int m = 0; m < NV; ++m) {
        double s = 0.0, comp = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
            double t = part[(size_t)b * NV + m];
            double u = s + t;
            comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
            s = u;
        }
        sh[threadIdx.x][0] = s;
        sh[threadIdx.x][1] = comp;
        __syncthreads();
        if (threadIdx.x == 0) {
            double S = 0.0, Cc = 0.0;
            for (int t = 0; t < RED_THREADS; ++t) {
                double a = sh[t][0];
                double u = S + a;
                Cc += (fabs(S) >= fabs(a)) ? (S - u) + a : (a - u) + S;
                S = u;
                Cc += sh[t][1];
            }
            out[m] = S + Cc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Tile mapping
// ---------------------------------------------------------------------------
// Blocks are dispatched round-robin over the XCDs (block b runs on XCD b % 8).
// Give XCD x the contiguous tile range [start(x), start(x+1)).
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int x = b % NXCD, local = b / NXCD;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    return x * per + min(x, rem) + local;
}

// ---------------------------------------------------------------------------
// 2D fused step
// ---------------------------------------------------------------------------
template <class S, bool SUMS>
__global__ __launch_bounds__(TX) void k_step2d(const typename S::T *__restrict__ src,
                                               typename S::T *__restrict__ dst, KParams p,
                                               double *__restrict__ partials)
{
    using T = typename S::T;
    using C = typename S::C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tyi = tile / p.tiles_x, txi = tile - tyi * p.tiles_x;
    const int x = txi * TX + threadIdx.x;
    const int y0 = tyi * TY;
    const bool interior = txi >= p.interior_x0 && txi < p.interior_x1 &&
                          tyi >= p.interior_y0 && tyi < p.interior_y1;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int nx = p.nx, ny = p.ny;

    if (interior) {
        // No wrap: plane k of the source is read at (x - vx, y - vy), i.e. a
        // uniform base plus the node's own offset.
#pragma unroll 1
        for (int r = 0; r < TY; ++r) {
            const int y = y0 + r;
            const unsigned o = (unsigned)(y * nx + x);
            C f[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                // integer arithmetic: the shifted base may precede the buffer
                const T *pk = reinterpret_cast<const T *>(
                    reinterpret_cast<uintptr_t>(src) +
                    (uintptr_t)((k * p.plane - (long long)(p.sx[k / Q] * nx + p.sx[k % Q])) *
                                (long long)sizeof(T)));
                f[k] = S::dec(pk[o], k, p);
            }
            collide2d<S>(f, p);
#pragma unroll
            for (int k = 0; k < NQ; ++k)
                __builtin_nontemporal_store(S::enc(f[k], k, p), dst + k * p.plane + o);
            if constexpr (SUMS) {
                // invariants of what was stored (decoded again for 16-bit forms)
                C g[NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) g[k] = S::dec(S::enc(f[k], k, p), k, p);
                C rho, jx, jy, e;
                sums2d<S>(g, p, rho, jx, jy, e);
                acc[0] += rho; acc[1] += jx; acc[2] += jy; acc[3] += e;
            }
        }
    } else if (x < nx) {
#pragma unroll 1
        for (int r = 0; r < TY; ++r) {
            const int y = y0 + r;
            if (y >= ny) break;
            C f[NQ];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                int ys = y - p.sx[j];
                ys += (ys < 0) ? ny : 0;
                ys -= (ys >= ny) ? ny : 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    int xs = x - p.sx[i];
                    xs += (xs < 0) ? nx : 0;
                    xs -= (xs >= nx) ? nx : 0;
                    const int k = i + Q * j;
                    f[k] = S::dec(src[k * p.plane + (long long)ys * nx + xs], k, p);
                }
            }
            collide2d<S>(f, p);
            const long long o = (long long)y * nx + x;
#pragma unroll
            for (int k = 0; k < NQ; ++k)
                __builtin_nontemporal_store(S::enc(f[k], k, p), dst + k * p.plane + o);
            if constexpr (SUMS) {
                C g[NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) g[k] = S::dec(S::enc(f[k], k, p), k, p);
                C rho, jx, jy, e;
                sums2d<S>(g, p, rho, jx, jy, e);
                acc[0] += rho; acc[1] += jx; acc[2] += jy; acc[3] += e;
            }
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// 2D initialisation: the buffer whose pull is f_eq.  Node x computes its own
// equilibrium and scatters population k to x - v_k, so that pulling it back
// from x - v_k returns f_eq_k(x).  The equilibrium is evaluated in FP64 and
// rounded once into the storage type.
// ---------------------------------------------------------------------------
struct Fp64Math {
    using C = double;
    static __device__ __forceinline__ C coef(int i, const KParams &p) { return p.c[i]; }
    static __device__ __forceinline__ C vel(int i, const KParams &p) { return p.v[i]; }
};

__device__ __forceinline__ void equilibrium2d(double rho, double ux, double uy, double th,
                                              const KParams &p, double (&feq)[NQ])
{
    double rx[Q], ry[Q];
    rule1d<Fp64Math>(ux, th, p, rx);
    rule1d<Fp64Math>(uy, th, p, ry);
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < Q; ++i) feq[i + Q * j] = rho * rx[i] * ry[j];
}

template <class S>
__global__ __launch_bounds__(TX) void k_init2d(const double *__restrict__ rho,
                                               const double *__restrict__ ux,
                                               const double *__restrict__ uy,
                                               const double *__restrict__ th,
                                               typename S::T *__restrict__ dst, KParams p)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= p.nx) return;
    const long long n = (long long)y * p.nx + x;
    double feq[NQ];
    equilibrium2d(rho[n], ux[n], uy[n], th[n], p, feq);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        int yd = y - p.sx[j];
        yd += (yd < 0) ? p.ny : 0;
        yd -= (yd >= p.ny) ? p.ny : 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xd = x - p.sx[i];
            xd += (xd < 0) ? p.nx : 0;
            xd -= (xd >= p.nx) ? p.nx : 0;
            const int k = i + Q * j;
            dst[k * p.plane + (long long)yd * p.nx + xd] = S::enc((typename S::C)feq[k], k, p);
        }
    }
}

// ---------------------------------------------------------------------------
// 2D moments of the pulled (pre-collision) state, in FP64.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(TX) void k_moments2d(const typename S::T *__restrict__ src, KParams p,
                                                  double *__restrict__ rho, double *__restrict__ ux,
                                                  double *__restrict__ uy, double *__restrict__ th,
                                                  double *__restrict__ partials)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        double f[NQ];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            int ys = y - p.sx[j];
            ys += (ys < 0) ? p.ny : 0;
            ys -= (ys >= p.ny) ? p.ny : 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int xs = x - p.sx[i];
                xs += (xs < 0) ? p.nx : 0;
                xs -= (xs >= p.nx) ? p.nx : 0;
                const int k = i + Q * j;
                f[k] = (double)S::dec(src[k * p.plane + (long long)ys * p.nx + xs], k, p);
            }
        }
        double r, jx, jy, e;
        sums2d<Fp64Math>(f, p, r, jx, jy, e);
        const double inv = 1.0 / r;
        const double u = jx * inv, w = jy * inv;
        const long long n = (long long)y * p.nx + x;
        if (rho) rho[n] = r;
        if (ux) ux[n] = u;
        if (uy) uy[n] = w;
        if (th) th[n] = 0.5 * (e * inv - u * u - w * w);
        acc[0] = r; acc[1] = jx; acc[2] = jy; acc[3] = e;
    }
    if (partials)
        block_sums_store<4>(acc, partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4);
}

// ---------------------------------------------------------------------------
// 1D (D1Q5) kernels on the ghost-padded layout: node x at x + 3.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ void collide1d(typename S::C (&f)[Q], const KParams &p)
{
    using C = typename S::C;
    C rho = f[0], j = C(0), e = C(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) rho += f[i];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const C vi = S::vel(i, p);
        j = fma(f[i], vi, j);
        e = fma(f[i], vi * vi, e);
    }
    const C inv = C(1) / rho;
    const C u = j * inv;
    const C theta = e * inv - u * u;
    C r[Q];
    rule1d<S>(u, theta, p, r);
    const C w = S::om(p);
    const C keep = C(1) - w, wr = w * rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = fma(keep, f[i], wr * r[i]);
}

template <class S, bool SUMS>
__global__ __launch_bounds__(TX) void k_step1d(const typename S::T *__restrict__ src,
                                               typename S::T *__restrict__ dst, KParams p,
                                               double *__restrict__ partials)
{
    using C = typename S::C;
    const int x = blockIdx.x * TX + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        C f[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k)
            f[k] = S::dec(src[k * p.plane + x + PLBM_GHOST - p.sx[k]], k, p);
        collide1d<S>(f, p);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const auto h = S::enc(f[k], k, p);
            dst[k * p.plane + x + PLBM_GHOST] = h;
            // zero-gradient ends: ghosts take the edge node's post-collision value
            if (x == 0)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * p.plane + g] = h;
            if (x == p.nx - 1)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * p.plane + p.nx + PLBM_GHOST + g] = h;
        }
        if constexpr (SUMS) {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double g = (double)S::dec(S::enc(f[k], k, p), k, p);
                const double vk = p.v[k];
                acc[0] += g; acc[1] += g * vk; acc[3] += g * vk * vk;
            }
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

template <class S>
__global__ __launch_bounds__(TX) void k_init1d(const double *__restrict__ rho,
                                               const double *__restrict__ ux,
                                               const double *__restrict__ th,
                                               typename S::T *__restrict__ dst, KParams p)
{
    // padded index q holds node y = q - 3; population k there must be
    // f_eq_k(y + v_k) so that the pull at y + v_k returns it.
    const int q = blockIdx.x * TX + threadIdx.x;
    if (q >= p.nx + 2 * PLBM_GHOST) return;
    const int y = q - PLBM_GHOST;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int s = y + p.sx[k];
        s = s < 0 ? 0 : (s >= p.nx ? p.nx - 1 : s);   // never pulled; kept finite
        double r[Q];
        rule1d<Fp64Math>(ux[s], th[s], p, r);
        dst[k * p.plane + q] = S::enc((typename S::C)(rho[s] * r[k]), k, p);
    }
}

template <class S>
__global__ __launch_bounds__(TX) void k_moments1d(const typename S::T *__restrict__ src, KParams p,
                                                  double *__restrict__ rho, double *__restrict__ ux,
                                                  double *__restrict__ th,
                                                  double *__restrict__ partials)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        double r = 0.0, j = 0.0, e = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const double f = (double)S::dec(src[k * p.plane + x + PLBM_GHOST - p.sx[k]], k, p);
            r += f;
            j += f * p.v[k];
            e += f * p.v[k] * p.v[k];
        }
        const double u = j / r;
        if (rho) rho[x] = r;
        if (ux) ux[x] = u;
        if (th) th[x] = e / r - u * u;
        acc[0] = r; acc[1] = j; acc[3] = e;
    }
    if (partials) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// Deviation scales: per-plane max |f_eq_k - rho0 w_k| over the nodes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TX) void k_devmax2d(const double *__restrict__ rho,
                                                 const double *__restrict__ ux,
                                                 const double *__restrict__ uy,
                                                 const double *__restrict__ th, KParams p,
                                                 const double *__restrict__ base,
                                                 double *__restrict__ partials)
{
    __shared__ double red[NQ][TX / 64];
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y;
    double m[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) m[k] = 0.0;
    if (x < p.nx) {
        const long long n = (long long)y * p.nx + x;
        double feq[NQ];
        equilibrium2d(rho[n], ux[n], uy[n], th[n], p, feq);
#pragma unroll
        for (int k = 0; k < NQ; ++k) m[k] = fabs(feq[k] - base[k]);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double v = m[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double v = 0.0;
        for (int w = 0; w < TX / 64; ++w) v = fmax(v, red[threadIdx.x][w]);
        partials[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NQ + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void rest_weights(const plbm_desc *d, double (&w1)[Q])
{
    // r_i(u = 0, theta0): mu = (1, 0, theta0, 0, 3 theta0^2)
    const double t = d->theta0;
    const double mu[Q] = {1.0, 0.0, t, 0.0, 3.0 * t * t};
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int j = 0; j < Q; ++j) s += d->c[i * Q + j] * mu[j];
        w1[i] = s;
    }
}

int make_params(const plbm_desc *d, KParams &p)
{
    int rc = plbm::validate(d);
    if (rc != PLBM_OK) return rc;
    if (d->q1d != Q) return PLBM_EUNSUPPORTED;
    if (d->dim == 1 && d->storage >= PLBM_F16DEV) return PLBM_EUNSUPPORTED;
    std::memset(&p, 0, sizeof(p));
    p.nx = d->nx;
    p.ny = d->ny;
    int maxs = 0;
    for (int i = 0; i < Q; ++i) {
        p.sx[i] = (int)d->v[i];
        p.v[i] = d->v[i];
        p.vf[i] = (float)d->v[i];
        maxs = std::max(maxs, std::abs(p.sx[i]));
    }
    for (int i = 0; i < NQ; ++i) {
        p.c[i] = d->c[i];
        p.cf[i] = (float)d->c[i];
    }
    p.omega = d->omega;
    p.omegaf = (float)d->omega;
    if (d->dim == 1) {
        p.plane = d->nx + 2 * PLBM_GHOST;
    } else {
        p.plane = (long long)d->nx * d->ny;
        p.tiles_x = (d->nx + TX - 1) / TX;
        const int tiles_y = (d->ny + TY - 1) / TY;
        p.ntiles = p.tiles_x * tiles_y;
        // a tile is interior when its shifted windows stay inside the lattice
        p.interior_x0 = (maxs + TX - 1) / TX;
        p.interior_x1 = std::max(0, (d->nx - maxs) / TX);   // (t+1)*TX + maxs <= nx
        p.interior_y0 = (maxs + TY - 1) / TY;
        p.interior_y1 = std::max(0, (d->ny - maxs) / TY);
    }
    if (d->storage >= PLBM_F16DEV) {
        double w1[Q];
        rest_weights(d, w1);
        for (int j = 0; j < Q; ++j)
            for (int i = 0; i < Q; ++i) {
                const int k = i + Q * j;
                p.base[k] = (float)(d->rho0 * w1[i] * w1[j]);
                p.scale[k] = d->scale[k];
                p.inv_scale[k] = 1.0f / d->scale[k];
            }
    }
    return PLBM_OK;
}

thread_local char g_last_error[160] = "";

int hip_ok(hipError_t e)
{
    if (e == hipSuccess) return PLBM_OK;
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d)", hipGetErrorString(e), (int)e);
    return PLBM_EHIP;
}

// The runtime's last-error slot is per thread and sticky: clear whatever an
// earlier, unrelated call left there before launching, then read it back.
inline void clear_launch_error() { (void)hipGetLastError(); }
inline int launch_status() { return hip_ok(hipGetLastError()); }

// Finish a partial-sum reduction: second pass, copy the 4 doubles to the host,
// synchronise, check finiteness.
int finish_sums(double *dev, int nblocks, double *host, hipStream_t st)
{
    double *out = dev + (size_t)nblocks * 4;
    clear_launch_error();
    hipLaunchKernelGGL(k_reduce_partials<4>, dim3(1), dim3(RED_THREADS), 0, st, dev, nblocks, out);
    int rc = launch_status();
    if (rc == PLBM_OK)
        rc = hip_ok(hipMemcpyAsync(host, out, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = hip_ok(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    for (int m = 0; m < 4; ++m)
        if (!std::isfinite(host[m])) return PLBM_ENONFINITE;
    return PLBM_OK;
}

template <class S, bool SUMS>
int launch_step(const KParams &p, const plbm_desc *d, const void *src, void *dst, double *partials,
                hipStream_t st, int &nblocks)
{
    using T = typename S::T;
    clear_launch_error();
    if (d->dim == 2) {
        nblocks = p.ntiles;
        hipLaunchKernelGGL((k_step2d<S, SUMS>), dim3(p.ntiles), dim3(TX), 0, st,
                           (const T *)src, (T *)dst, p, partials);
    } else {
        nblocks = (p.nx + TX - 1) / TX;
        hipLaunchKernelGGL((k_step1d<S, SUMS>), dim3(nblocks), dim3(TX), 0, st,
                           (const T *)src, (T *)dst, p, partials);
    }
    return launch_status();
}

template <class S>
int run_steps(const KParams &p, const plbm_desc *d, void *fa, void *fb, int nsteps, double *sums,
              hipStream_t st)
{
    int nb = 0;
    for (int s = 0; s < nsteps; ++s) {
        const void *src = (s & 1) ? fb : fa;
        void *dst = (s & 1) ? fa : fb;
        const bool last = (s == nsteps - 1);
        if (last && sums) {
            const int nblocks = d->dim == 2 ? p.ntiles : (p.nx + TX - 1) / TX;
            double *part = nullptr;
            int rc = hip_ok(
                hipMallocAsync((void **)&part, ((size_t)nblocks + 1) * 4 * sizeof(double), st));
            if (rc != PLBM_OK) return rc;
            rc = launch_step<S, true>(p, d, src, dst, part, st, nb);
            if (rc == PLBM_OK) rc = finish_sums(part, nb, sums, st);
            (void)hipFreeAsync(part, st);
            return rc;
        }
        int rc = launch_step<S, false>(p, d, src, dst, nullptr, st, nb);
        if (rc != PLBM_OK) return rc;
    }
    return PLBM_OK;
}

template <class S>
int launch_init(const KParams &p, const plbm_desc *d, const double *rho, const double *ux,
                const double *uy, const double *th, void *f, hipStream_t st)
{
    using T = typename S::T;
    clear_launch_error();
    if (d->dim == 2) {
        hipLaunchKernelGGL(k_init2d<S>, dim3((p.nx + TX - 1) / TX, p.ny), dim3(TX), 0, st, rho, ux,
                           uy, th, (T *)f, p);
    } else {
        hipLaunchKernelGGL(k_init1d<S>, dim3((p.nx + 2 * PLBM_GHOST + TX - 1) / TX), dim3(TX), 0,
                           st, rho, ux, th, (T *)f, p);
    }
    return launch_status();
}

template <class S>
int launch_moments(const KParams &p, const plbm_desc *d, const void *f, double *rho, double *ux,
                   double *uy, double *th, double *partials, hipStream_t st, int &nblocks)
{
    using T = typename S::T;
    clear_launch_error();
    if (d->dim == 2) {
        dim3 g((p.nx + TX - 1) / TX, p.ny);
        nblocks = (int)(g.x * g.y);
        hipLaunchKernelGGL(k_moments2d<S>, g, dim3(TX), 0, st, (const T *)f, p, rho, ux, uy, th,
                           partials);
    } else {
        nblocks = (p.nx + TX - 1) / TX;
        hipLaunchKernelGGL(k_moments1d<S>, dim3(nblocks), dim3(TX), 0, st, (const T *)f, p, rho, ux,
                           th, partials);
    }
    return launch_status();
}

#define PLBM_DISPATCH(storage, FN, ...)                                                  \
    switch (storage) {                                                                   \
    case PLBM_F64: return FN<StF64>(__VA_ARGS__);                                        \
    case PLBM_F32: return FN<StF32>(__VA_ARGS__);                                        \
    case PLBM_F16DEV: return FN<StF16>(__VA_ARGS__);                                     \
    case PLBM_BF16DEV: return FN<StBF16>(__VA_ARGS__);                                   \
    default: return PLBM_EINVAL;                                                         \
    }

int init_dispatch(const KParams &p, const plbm_desc *d, const double *rho, const double *ux,
                  const double *uy, const double *th, void *f, hipStream_t st)
{
    PLBM_DISPATCH(d->storage, launch_init, p, d, rho, ux, uy, th, f, st);
}

int step_dispatch(const KParams &p, const plbm_desc *d, void *fa, void *fb, int n, double *sums,
                  hipStream_t st)
{
    PLBM_DISPATCH(d->storage, run_steps, p, d, fa, fb, n, sums, st);
}

int moments_dispatch(const KParams &p, const plbm_desc *d, const void *f, double *rho, double *ux,
                     double *uy, double *th, double *part, hipStream_t st, int &nb)
{
    PLBM_DISPATCH(d->storage, launch_moments, p, d, f, rho, ux, uy, th, part, st, nb);
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int plbm_init(const plbm_desc *d, const double *rho, const double *ux,
                         const double *uy, const double *theta, void *f, void *stream)
{
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !theta || !f || (d->dim == 2 && !uy)) return PLBM_EINVAL;
    return init_dispatch(p, d, rho, ux, uy, theta, f, as_stream(stream));
}

extern "C" int plbm_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *sums,
                         void *stream)
{
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f_a || !f_b || f_a == f_b || nsteps < 0) return PLBM_EINVAL;
    if (nsteps == 0) {
        if (sums) return plbm_moments(d, f_a, nullptr, nullptr, nullptr, nullptr, sums, stream);
        return PLBM_OK;
    }
    return step_dispatch(p, d, f_a, f_b, nsteps, sums, as_stream(stream));
}

extern "C" int plbm_moments(const plbm_desc *d, const void *f, double *rho, double *ux,
                            double *uy, double *theta, double *sums, void *stream)
{
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f) return PLBM_EINVAL;
    hipStream_t st = as_stream(stream);
    int nb = 0;
    if (!sums) return moments_dispatch(p, d, f, rho, ux, uy, theta, nullptr, st, nb);
    const int nblocks = d->dim == 2 ? ((p.nx + TX - 1) / TX) * p.ny : (p.nx + TX - 1) / TX;
    double *part = nullptr;
    rc = hip_ok(hipMallocAsync((void **)&part, ((size_t)nblocks + 1) * 4 * sizeof(double), st));
    if (rc != PLBM_OK) return rc;
    rc = moments_dispatch(p, d, f, rho, ux, uy, theta, part, st, nb);
    if (rc == PLBM_OK) rc = finish_sums(part, nb, sums, st);
    (void)hipFreeAsync(part, st);
    return rc;
}

extern "C" int plbm_dev_scales(plbm_desc *d, const double *rho, const double *ux,
                               const double *uy, const double *theta, void *stream)
{
    if (!d || d->dim != 2 || d->storage < PLBM_F16DEV) return PLBM_EINVAL;
    // validation with provisional unit scales
    for (int k = 0; k < NQ; ++k) d->scale[k] = 1.0f;
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !uy || !theta) return PLBM_EINVAL;
    hipStream_t st = as_stream(stream);
    double w1[Q], base[NQ];
    rest_weights(d, w1);
    for (int j = 0; j < Q; ++j)
        for (int i = 0; i < Q; ++i) base[i + Q * j] = d->rho0 * w1[i] * w1[j];
    dim3 g((p.nx + TX - 1) / TX, p.ny);
    const size_t nb = (size_t)g.x * g.y;
    double *buf = nullptr;
    const size_t bytes = (NQ + nb * NQ) * sizeof(double);
    rc = hip_ok(hipMallocAsync((void **)&buf, bytes, st));
    if (rc != PLBM_OK) return rc;
    rc = hip_ok(hipMemcpyAsync(buf, base, NQ * sizeof(double), hipMemcpyHostToDevice, st));
    if (rc == PLBM_OK) {
        clear_launch_error();
        hipLaunchKernelGGL(k_devmax2d, g, dim3(TX), 0, st, rho, ux, uy, theta, p, buf, buf + NQ);
        rc = launch_status();
    }
    double *host = rc == PLBM_OK ? new double[nb * NQ] : nullptr;
    if (rc == PLBM_OK)
        rc = hip_ok(hipMemcpyAsync(host, buf + NQ, nb * NQ * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = hip_ok(hipStreamSynchronize(st));
    (void)hipFreeAsync(buf, st);
    if (rc == PLBM_OK) {
        for (int k = 0; k < NQ; ++k) {
            double m = 0.0;
            for (size_t b = 0; b < nb; ++b) m = std::fmax(m, host[b * NQ + k]);
            if (!std::isfinite(m)) { rc = PLBM_ENONFINITE; break; }
            // smallest e with m <= 2^e * 2^10
            int e = m > 0.0 ? (int)std::ceil(std::log2(m)) - 10 : -30;
            if (m > 0.0 && std::ldexp(1.0, e + 10) < m) e += 1;
            d->scale[k] = (float)std::ldexp(1.0, e);
        }
    }
    delete[] host;
    return rc;
}

extern "C" const char *plbm_last_hip_error(void) { return g_last_error; }
