// libplbm device code for general on-lattice velocity sets (Sec. 2.2): any
// q1d = 3..7 distinct integer velocities with |v| <= 3, in any order, with
// the full Lagrange table of Eq. rdr, r_i = sum_n c_in mu_n, and the Maxwell
// moments mu_0..mu_(q1d-1) from the recurrence mu_(n+1) = u mu_n +
// n theta mu_(n-1).  Sets of up to four velocities are isothermal models (the
// moments at the fixed reference temperature theta0, as for the
// three-velocity family), sets of five or more thermal ones (the local
// temperature, one for all axes).  This path takes every descriptor the
// symmetric kernels do not: asymmetric sets, D1Q4 and q1d = 6, 7.
//
// D1: padded layout k (nx + 6) + x + 3 with zero-gradient ghost ends; D2: the
// tensor product on a periodic lattice, row-interleaved layout
// (y q + k) nx + x with q = q1d^2 and k = i + q1d j.  Same streaming design
// as the specialised steps: one 256-node row segment per workgroup,
// XCD-contiguous tiles, a scalar row base per y velocity and a lane offset
// per x velocity (x wrap folded in), non-temporal stores.  FP64 storage
// computes in FP64, FP32 in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "plbm_device.h"
#include "plbm_internal.h"

namespace {

constexpr int GMAX = 7;                 // most distinct velocities with |v| <= 3
constexpr int MAX_GRID_G = 1 << 22;

struct GenParams {
    int dim, nx, ny, q1d;
    int tiles_x, ntiles;                // 2D: row segments; 1D: node segments
    int iso;                            // 1: moments at theta0
    int sx[GMAX];                       // integer velocities (streaming shifts)
    double v64[GMAX], c64[GMAX * GMAX], theta0, omega;   // c[i * q1d + n]
    float v32[GMAX], c32[GMAX * GMAX], theta0f, omegaf;
};

template <typename C>
struct GenView;
template <>
struct GenView<double> {
    static __device__ __forceinline__ const double *v(const GenParams &p) { return p.v64; }
    static __device__ __forceinline__ const double *c(const GenParams &p) { return p.c64; }
    static __device__ __forceinline__ double theta0(const GenParams &p) { return p.theta0; }
    static __device__ __forceinline__ double omega(const GenParams &p) { return p.omega; }
};
template <>
struct GenView<float> {
    static __device__ __forceinline__ const float *v(const GenParams &p) { return p.v32; }
    static __device__ __forceinline__ const float *c(const GenParams &p) { return p.c32; }
    static __device__ __forceinline__ float theta0(const GenParams &p) { return p.theta0f; }
    static __device__ __forceinline__ float omega(const GenParams &p) { return p.omegaf; }
};

__device__ __forceinline__ int wrap_g(int s, int n)
{
    s += (s < 0) ? n : 0;
    s -= (s >= n) ? n : 0;
    return s;
}

// r = C mu(u, theta) for the Q1-velocity set (Eq. rdr).
template <int Q1, typename C>
__device__ __forceinline__ void rule_gen(C u, C theta, const GenParams &p, C (&r)[Q1])
{
    const C *c = GenView<C>::c(p);
    C mu[Q1];
    mu[0] = C(1);
    mu[1] = u;
#pragma unroll
    for (int n = 1; n + 1 < Q1; ++n) mu[n + 1] = fma(u, mu[n], C(n) * theta * mu[n - 1]);
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
        C s = c[i * Q1];
#pragma unroll
        for (int n = 1; n < Q1; ++n) s = fma(c[i * Q1 + n], mu[n], s);
        r[i] = s;
    }
}

// rho, rho u_x, rho u_y, sum f |v|^2 of the Q1^2 populations via column and
// row sums.
template <int Q1, typename C>
__device__ __forceinline__ void sums_gen2d(const C (&f)[Q1 * Q1], const GenParams &p, C &rho, C &jx, C &jy,
                                           C &e)
{
    const C *v = GenView<C>::v(p);
    C col[Q1], row[Q1];
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
        col[i] = f[i];
        row[i] = f[Q1 * i];
    }
#pragma unroll
    for (int j = 1; j < Q1; ++j)
#pragma unroll
        for (int i = 0; i < Q1; ++i) col[i] += f[i + Q1 * j];
#pragma unroll
    for (int j = 0; j < Q1; ++j)
#pragma unroll
        for (int i = 1; i < Q1; ++i) row[j] += f[i + Q1 * j];
    rho = col[0];
    jx = v[0] * col[0];
    jy = v[0] * row[0];
    e = v[0] * v[0] * (col[0] + row[0]);
#pragma unroll
    for (int i = 1; i < Q1; ++i) {
        rho += col[i];
        jx = fma(v[i], col[i], jx);
        jy = fma(v[i], row[i], jy);
        e = fma(v[i] * v[i], col[i] + row[i], e);
    }
}

// Launch shape measured on MI355X at 4096^2 (KH rest state): non-temporal
// loads help up to five velocities per axis (D2Q16 FP32 0.80 of 8 TB/s) and
// cost 3-9 % at seven (D2Q49), where cached loads reach 0.76 (FP32) and 0.74
// (FP64); an LDS reservation of 40 KB (D2Q16 FP32) or 53 KB (otherwise)
// caps the resident workgroups at the best measured count.
template <int Q1>
constexpr bool gen_nt_loads() { return Q1 <= 5; }
// Sets whose first velocity is 0 (Z0): only that column is loaded
// non-temporally, since it reads exactly the wave's own nodes while the
// shifted columns' window edges are read again by the neighbouring wave.
#ifndef PLBM_GEN_Z0_NT
#define PLBM_GEN_Z0_NT 1
#endif
template <int Q1, bool Z0>
constexpr unsigned gen_nt_mask()
{
    return (Z0 && PLBM_GEN_Z0_NT) ? 1u : (gen_nt_loads<Q1>() ? (1u << Q1) - 1 : 0u);
}
template <int Q1, typename T>
constexpr size_t gen_lds_cap() { return (sizeof(T) == 4 && Q1 <= 4) ? 40 * 1024 : 53 * 1024; }

template <bool NT, typename T>
__device__ __forceinline__ T load_g(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Pull-gather of node (xb, y): f_k = src_k(x - v_i, y - v_j), k = i + Q1 j.
template <int Q1, typename T, typename C, bool Z0 = false>
__device__ __forceinline__ void gather_gen2d(const T *__restrict__ src, const GenParams &p, int xb, int y,
                                             C (&f)[Q1 * Q1])
{
    const int nx = p.nx;
    const long long rowelems = (long long)Q1 * Q1 * nx;
    const int xc = min(xb, nx - 1);
    unsigned lo[Q1];
#pragma unroll
    for (int i = 0; i < Q1; ++i) lo[i] = (unsigned)(wrap_g(xc - p.sx[i], nx) + i * nx);
#pragma unroll
    for (int j = 0; j < Q1; ++j) {
        const int ys = wrap_g(y - p.sx[j], p.ny);
        const T *base = src + (ys * rowelems + (long long)(Q1 * j) * nx);
#pragma unroll
        for (int i = 0; i < Q1; ++i) {
            if ((gen_nt_mask<Q1, Z0>() >> i) & 1) f[i + Q1 * j] = (C)load_g<true>(&base[lo[i]]);
            else f[i + Q1 * j] = (C)load_g<false>(&base[lo[i]]);
        }
    }
}

template <int Q1, typename C>
__device__ __forceinline__ void collide_gen2d(C (&f)[Q1 * Q1], const GenParams &p)
{
    C rho, jx, jy, e;
    sums_gen2d<Q1, C>(f, p, rho, jx, jy, e);
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv;
    const C theta = p.iso ? GenView<C>::theta0(p) : C(0.5) * (e * inv - ux * ux - uy * uy);
    C rx[Q1], ry[Q1];
    rule_gen<Q1, C>(ux, theta, p, rx);
    rule_gen<Q1, C>(uy, theta, p, ry);
    const C w = GenView<C>::omega(p);
    const C wr = w * rho, keep = C(1) - w;
#pragma unroll
    for (int i = 0; i < Q1; ++i) rx[i] *= wr;
#pragma unroll
    for (int j = 0; j < Q1; ++j)
#pragma unroll
        for (int i = 0; i < Q1; ++i) f[i + Q1 * j] = fma(keep, f[i + Q1 * j], rx[i] * ry[j]);
}

template <int Q1, typename T, bool SUMS, bool Z0>
__global__ __launch_bounds__(TX) void k_step_gen2d(const T *__restrict__ src, T *__restrict__ dst, GenParams p,
                                                   double *__restrict__ partials)
{
    using C = T;
    constexpr int NG = Q1 * Q1;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long rowelems = (long long)NG * p.nx;
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int tile = slot; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int xb = (tile - y * p.tiles_x) * TX + threadIdx.x;
        C f[NG];
        gather_gen2d<Q1, T, C, Z0>(src, p, xb, y, f);
        collide_gen2d<Q1, C>(f, p);
        if (xb < p.nx) {
            if constexpr (SUMS) {
                C g[NG];
#pragma unroll
                for (int k = 0; k < NG; ++k) g[k] = (C)(T)f[k];
                C rho, jx, jy, e;
                sums_gen2d<Q1, C>(g, p, rho, jx, jy, e);
                acc[0] += rho;
                acc[1] += jx;
                acc[2] += jy;
                acc[3] += e;
            }
            T *out = dst + (y * rowelems + xb);
#pragma unroll
            for (int k = 0; k < NG; ++k) store_stream((T)f[k], out + (long long)k * p.nx);
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// Initial state: f_eq of node (x, y) in FP64, written to (x - v_i, y - v_j).
template <int Q1, typename T>
__global__ __launch_bounds__(TX) void k_init_gen2d(const double *__restrict__ rho, const double *__restrict__ ux,
                                                   const double *__restrict__ uy, const double *__restrict__ th,
                                                   T *__restrict__ dst, GenParams p)
{
    constexpr int NG = Q1 * Q1;
    const long long rowelems = (long long)NG * p.nx;
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int x = (tile - y * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        const long long n = (long long)y * p.nx + x;
        const double theta = p.iso ? p.theta0 : th[n];
        double rx[Q1], ry[Q1];
        rule_gen<Q1, double>(ux[n], theta, p, rx);
        rule_gen<Q1, double>(uy[n], theta, p, ry);
#pragma unroll
        for (int j = 0; j < Q1; ++j) {
            const int yd = wrap_g(y - p.sx[j], p.ny);
#pragma unroll
            for (int i = 0; i < Q1; ++i) {
                const int xd = wrap_g(x - p.sx[i], p.nx);
                dst[yd * rowelems + (long long)(i + Q1 * j) * p.nx + xd] = (T)(rho[n] * rx[i] * ry[j]);
            }
        }
    }
}

// Fields of the pulled state (2 rho theta = sum f |v - u|^2) and FP64 sums.
template <int Q1, typename T>
__global__ __launch_bounds__(TX) void k_moments_gen2d(const T *__restrict__ src, GenParams p,
                                                      double *__restrict__ rho, double *__restrict__ ux,
                                                      double *__restrict__ uy, double *__restrict__ th,
                                                      double *__restrict__ partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int x = (tile - y * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        double f[Q1 * Q1];
        gather_gen2d<Q1, T, double>(src, p, x, y, f);
        double r, jx, jy, e;
        sums_gen2d<Q1, double>(f, p, r, jx, jy, e);
        const long long n = (long long)y * p.nx + x;
        const double u = jx / r, w = jy / r;
        if (rho) rho[n] = r;
        if (ux) ux[n] = u;
        if (uy) uy[n] = w;
        if (th) th[n] = 0.5 * (e / r - u * u - w * w);
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += e;
    }
    if (partials) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// 1D: pull f_k = src_k(x - v_k) from the padded rows, relax, write at x; the
// three ghost nodes at each end take the edge node's post-collision values.
// ---------------------------------------------------------------------------
template <int Q1, typename T, bool SUMS>
__global__ __launch_bounds__(TX) void k_step_gen1d(const T *__restrict__ src, T *__restrict__ dst, GenParams p,
                                                   double *__restrict__ partials)
{
    using C = T;
    const C *v = GenView<C>::v(p);
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int x = tile * TX + threadIdx.x;
        if (x >= p.nx) continue;
        C f[Q1];
#pragma unroll
        for (int k = 0; k < Q1; ++k) f[k] = (C)src[k * ps + x + PLBM_GHOST - p.sx[k]];
        C rho = f[0], j = v[0] * f[0], e = v[0] * v[0] * f[0];
#pragma unroll
        for (int k = 1; k < Q1; ++k) {
            rho += f[k];
            j = fma(v[k], f[k], j);
            e = fma(v[k] * v[k], f[k], e);
        }
        const C u = j / rho;
        const C theta = p.iso ? GenView<C>::theta0(p) : e / rho - u * u;
        C r[Q1];
        rule_gen<Q1, C>(u, theta, p, r);
        const C w = GenView<C>::omega(p);
        const C wr = w * rho, keep = C(1) - w;
#pragma unroll
        for (int k = 0; k < Q1; ++k) {
            const T h = (T)fma(keep, f[k], wr * r[k]);
            dst[k * ps + x + PLBM_GHOST] = h;
            if (x == 0)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * ps + g] = h;
            if (x == p.nx - 1)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * ps + p.nx + PLBM_GHOST + g] = h;
            if constexpr (SUMS) {
                const double vk = p.v64[k];
                acc[0] += (double)h;
                acc[1] += (double)h * vk;
                acc[3] += (double)h * vk * vk;
            }
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// Padded index q holds node q - 3; its population k is f_eq_k of node
// q - 3 + v_k (clamped into the lattice), so the first pull returns f_eq.
template <int Q1, typename T>
__global__ __launch_bounds__(TX) void k_init_gen1d(const double *__restrict__ rho, const double *__restrict__ ux,
                                                   const double *__restrict__ th, T *__restrict__ dst, GenParams p)
{
    const int q = blockIdx.x * TX + threadIdx.x;
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    if (q >= ps) return;
#pragma unroll
    for (int k = 0; k < Q1; ++k) {
        int s = q - PLBM_GHOST + p.sx[k];
        s = s < 0 ? 0 : (s >= p.nx ? p.nx - 1 : s);
        double r[Q1];
        rule_gen<Q1, double>(ux[s], p.iso ? p.theta0 : th[s], p, r);
        dst[k * ps + q] = (T)(rho[s] * r[k]);
    }
}

template <int Q1, typename T>
__global__ __launch_bounds__(TX) void k_moments_gen1d(const T *__restrict__ src, GenParams p,
                                                      double *__restrict__ rho, double *__restrict__ ux,
                                                      double *__restrict__ th, double *__restrict__ partials)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        double r = 0.0, j = 0.0, e = 0.0;
#pragma unroll
        for (int k = 0; k < Q1; ++k) {
            const double f = (double)src[k * ps + x + PLBM_GHOST - p.sx[k]];
            r += f;
            j = fma(p.v64[k], f, j);
            e = fma(p.v64[k] * p.v64[k], f, e);
        }
        const double u = j / r;
        if (rho) rho[x] = r;
        if (ux) ux[x] = u;
        if (th) th[x] = e / r - u * u;
        acc[0] = r;
        acc[1] = j;
        acc[3] = e;
    }
    if (partials) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int gen_hip(hipError_t e)
{
    if (e == hipSuccess) return PLBM_OK;
    plbm::note_hip_error(hipGetErrorString(e), (int)e);
    return PLBM_EHIP;
}

int gen_launch_status() { return gen_hip(hipGetLastError()); }

// Descriptor checks of the general path: dims 1 and 2, FP64 or FP32, q1d
// 3..7, a table that is the Lagrange table of v (sum_n c_in v_k^n = delta_ik
// to 1e-9 of its scale), theta0 > 0 for the isothermal sets.
int gen_params(const plbm_desc *d, GenParams &p)
{
    int rc = plbm::validate(d);
    if (rc != PLBM_OK) return rc;
    if (d->dim != 1 && d->dim != 2) return PLBM_EINVAL;
    if (d->q1d < 3 || d->q1d > GMAX) return PLBM_EUNSUPPORTED;
    if (d->storage != PLBM_F64 && d->storage != PLBM_F32) return PLBM_EUNSUPPORTED;
    const int q = d->q1d;
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < q; ++k) {
            double s = 0.0, pw = 1.0, mag = 0.0;
            for (int n = 0; n < q; ++n) {
                s += d->c[i * q + n] * pw;
                mag += std::fabs(d->c[i * q + n] * pw);
                pw *= d->v[k];
            }
            if (!(std::fabs(s - (i == k ? 1.0 : 0.0)) <= 1e-9 * std::fmax(1.0, mag))) return PLBM_EINVAL;
        }
    const bool iso = q <= 4;
    if (iso && (!(d->theta0 > 0.0) || !std::isfinite(d->theta0))) return PLBM_EINVAL;
    std::memset(&p, 0, sizeof(p));
    p.dim = d->dim;
    p.nx = d->nx;
    p.ny = d->ny;
    p.q1d = q;
    p.iso = iso ? 1 : 0;
    p.tiles_x = (d->nx + TX - 1) / TX;
    const long long nt = d->dim == 2 ? (long long)p.tiles_x * d->ny : p.tiles_x;
    if (nt > 0x7fffffffLL) return PLBM_EINVAL;
    p.ntiles = (int)nt;
    for (int i = 0; i < q; ++i) {
        p.sx[i] = (int)d->v[i];
        p.v64[i] = d->v[i];
        p.v32[i] = (float)d->v[i];
    }
    for (int i = 0; i < q * q; ++i) {
        p.c64[i] = d->c[i];
        p.c32[i] = (float)d->c[i];
    }
    p.theta0 = d->theta0;
    p.theta0f = (float)d->theta0;
    p.omega = d->omega;
    p.omegaf = (float)d->omega;
    return PLBM_OK;
}

inline int grid_g(const GenParams &p) { return std::min(p.ntiles, MAX_GRID_G); }

int gen_finish_sums(double *dev, int nblocks, double *host, hipStream_t st)
{
    double *out = dev + (size_t)nblocks * 4;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_reduce_partials<4>, dim3(1), dim3(RED_THREADS), 0, st, dev, nblocks, out);
    int rc = gen_launch_status();
    if (rc == PLBM_OK) rc = gen_hip(hipMemcpyAsync(host, out, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = gen_hip(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    for (int m = 0; m < 4; ++m)
        if (!std::isfinite(host[m])) return PLBM_ENONFINITE;
    return PLBM_OK;
}

template <int Q1, typename T, bool SUMS>
void gen_launch(const GenParams &p, const T *src, T *dst, double *part, hipStream_t st)
{
    if (p.dim == 2 && p.sx[0] == 0)
        hipLaunchKernelGGL((k_step_gen2d<Q1, T, SUMS, true>), dim3(grid_g(p)), dim3(TX), (gen_lds_cap<Q1, T>()), st,
                           src, dst, p, part);
    else if (p.dim == 2)
        hipLaunchKernelGGL((k_step_gen2d<Q1, T, SUMS, false>), dim3(grid_g(p)), dim3(TX), (gen_lds_cap<Q1, T>()), st,
                           src, dst, p, part);
    else
        hipLaunchKernelGGL((k_step_gen1d<Q1, T, SUMS>), dim3(grid_g(p)), dim3(TX), 0, st, src, dst, p, part);
}

template <int Q1, typename T>
int gen_run(const GenParams &p, void *fa, void *fb, int nsteps, double *sums, hipStream_t st)
{
    const int grid = grid_g(p);
    for (int s = 0; s < nsteps; ++s) {
        const T *src = static_cast<const T *>((s & 1) ? fb : fa);
        T *dst = static_cast<T *>((s & 1) ? fa : fb);
        (void)hipGetLastError();
        if (s == nsteps - 1 && sums) {
            double *part = nullptr;
            int rc = gen_hip(hipMallocAsync((void **)&part, ((size_t)grid + 1) * 4 * sizeof(double), st));
            if (rc != PLBM_OK) return rc;
            gen_launch<Q1, T, true>(p, src, dst, part, st);
            rc = gen_launch_status();
            if (rc == PLBM_OK) rc = gen_finish_sums(part, grid, sums, st);
            (void)hipFreeAsync(part, st);
            return rc;
        }
        gen_launch<Q1, T, false>(p, src, dst, nullptr, st);
        const int rc = gen_launch_status();
        if (rc != PLBM_OK) return rc;
    }
    return PLBM_OK;
}

template <int Q1, typename T>
int gen_init_t(const GenParams &p, const double *rho, const double *ux, const double *uy, const double *th, void *f,
               hipStream_t st)
{
    (void)hipGetLastError();
    if (p.dim == 2)
        hipLaunchKernelGGL((k_init_gen2d<Q1, T>), dim3(grid_g(p)), dim3(TX), 0, st, rho, ux, uy, th, (T *)f, p);
    else
        hipLaunchKernelGGL((k_init_gen1d<Q1, T>), dim3((unsigned)((p.nx + 2 * PLBM_GHOST + TX - 1) / TX)), dim3(TX),
                           0, st, rho, ux, th, (T *)f, p);
    return gen_launch_status();
}

template <int Q1, typename T>
int gen_moments_t(const GenParams &p, const void *f, double *rho, double *ux, double *uy, double *th,
                  double *sums, hipStream_t st)
{
    const int grid = p.dim == 2 ? grid_g(p) : p.tiles_x;
    double *part = nullptr;
    int rc = PLBM_OK;
    if (sums) {
        rc = gen_hip(hipMallocAsync((void **)&part, ((size_t)grid + 1) * 4 * sizeof(double), st));
        if (rc != PLBM_OK) return rc;
    }
    (void)hipGetLastError();
    if (p.dim == 2)
        hipLaunchKernelGGL((k_moments_gen2d<Q1, T>), dim3(grid), dim3(TX), 0, st, (const T *)f, p, rho, ux, uy, th,
                           part);
    else
        hipLaunchKernelGGL((k_moments_gen1d<Q1, T>), dim3(grid), dim3(TX), 0, st, (const T *)f, p, rho, ux, th, part);
    rc = gen_launch_status();
    if (rc == PLBM_OK && sums) rc = gen_finish_sums(part, grid, sums, st);
    if (part) (void)hipFreeAsync(part, st);
    return rc;
}

#define PLBM_GEN_DISPATCH(p, storage, FN, ...)                                            \
    do {                                                                                  \
        const bool f64_ = (storage) == PLBM_F64;                                          \
        switch ((p).q1d) {                                                                \
        case 3: return f64_ ? FN<3, double>(__VA_ARGS__) : FN<3, float>(__VA_ARGS__);     \
        case 4: return f64_ ? FN<4, double>(__VA_ARGS__) : FN<4, float>(__VA_ARGS__);     \
        case 5: return f64_ ? FN<5, double>(__VA_ARGS__) : FN<5, float>(__VA_ARGS__);     \
        case 6: return f64_ ? FN<6, double>(__VA_ARGS__) : FN<6, float>(__VA_ARGS__);     \
        case 7: return f64_ ? FN<7, double>(__VA_ARGS__) : FN<7, float>(__VA_ARGS__);     \
        default: return PLBM_EUNSUPPORTED;                                                \
        }                                                                                 \
    } while (0)

} // namespace

namespace plbm {

bool gen_handles(const plbm_desc *d)
{
    if (!d || d->dim < 1 || d->dim > 2 || d->q1d < 3 || d->q1d > GMAX) return false;
    const double *v = d->v;
    if (d->q1d == 3) return !(v[0] == 0.0 && v[1] > 0.0 && v[2] == -v[1]);
    if (d->q1d == 5) return !(v[0] == 0.0 && v[2] == -v[1] && v[4] == -v[3]);
    return true;
}

int gen_init(const plbm_desc *d, const double *rho, const double *ux, const double *uy, const double *theta,
             void *f, void *stream)
{
    GenParams p;
    const int rc = gen_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !f || (p.dim == 2 && !uy) || (!p.iso && !theta)) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PLBM_GEN_DISPATCH(p, d->storage, gen_init_t, p, rho, ux, uy, theta, f, st);
}

int gen_step(const plbm_desc *d, void *fa, void *fb, int nsteps, double *sums, void *stream)
{
    GenParams p;
    const int rc = gen_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!fa || !fb || fa == fb || nsteps < 0) return PLBM_EINVAL;
    if (nsteps == 0) return sums ? gen_moments(d, fa, nullptr, nullptr, nullptr, nullptr, sums, stream) : PLBM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PLBM_GEN_DISPATCH(p, d->storage, gen_run, p, fa, fb, nsteps, sums, st);
}

int gen_moments(const plbm_desc *d, const void *f, double *rho, double *ux, double *uy, double *theta,
                double *sums, void *stream)
{
    GenParams p;
    const int rc = gen_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PLBM_GEN_DISPATCH(p, d->storage, gen_moments_t, p, f, rho, ux, uy, theta, sums, st);
}

} // namespace plbm
