// libplbm device code for the three-dimensional tensor-product model D3Q125
// (Sec. 2.4): the symmetric five-velocity 1D rule {0, +-a, +-b} of Eq. rdr
// along each axis, f_eq_k = rho r_i(u_x) r_j(u_y) r_l(u_z) for
// k = i + 5 j + 25 l, one temperature for all axes (3 rho theta =
// sum f |v - u|^2), SRT relaxation (Eq. srt), periodic in x, y and z.
//
// Pull scheme with A/B buffers holding post-collision populations; layout
// ((z ny + y) 125 + k) nx + x, i.e. lattice row (y, z) stores its 125
// population rows one after another.  One 256-node row segment per
// workgroup, tiles numbered contiguously per XCD.  Each node pulls its 125
// populations through 25 wave-uniform row bases (one per source row
// (y - v_j, z - v_l)) and 5 lane byte offsets (one per v_i, the periodic wrap
// in x folded in), so every load is a scalar base plus a 32-bit vector
// offset.  Non-temporal stores, cached loads.  FP64 storage computes in
// FP64, FP32 in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "plbm_device.h"
#include "plbm_internal.h"

namespace {

// Measured on MI355X at 256^3: non-temporal loads lose 1.5 % (FP64) and
// 9 % (FP32) here, unlike the 2D step.  FP64 holds 125 populations per lane
// and runs one wave per SIMD whatever the LDS; FP32 (164 VGPRs) is fastest
// with one workgroup per CU (0.73 of 8 TB/s against 0.69 at three).
// Non-temporal loads for the x-velocity columns in this mask (bit i: v_i;
// the other columns use PLBM_Q125_NT_LOAD).  Column 0 (v = 0) reads exactly
// the wave's own nodes: 1.8 % (FP32) and 1.3 % (FP64) faster at 256^3 than
// no non-temporal load; all columns non-temporal lose 9 % and 1.5 %.
#ifndef PLBM_Q125_NT_MASK
#define PLBM_Q125_NT_MASK 1
#endif
#ifndef PLBM_Q125_NT_LOAD
#define PLBM_Q125_NT_LOAD 0
#endif
#ifndef PLBM_Q125_LDS_F64
#define PLBM_Q125_LDS_F64 0
#endif
#ifndef PLBM_Q125_LDS_F32
#define PLBM_Q125_LDS_F32 (160 * 1024)
#endif

constexpr int N125 = Q * Q * Q;
constexpr int MAX_GRID3 = 1 << 22;   // workgroups per launch; larger grids loop

struct P3 {
    int nx, ny, nz;
    int tiles_x, ntiles;          // ntiles = tiles_x * ny * nz row segments
    int sx[Q];                    // integer velocities (streaming shifts)
    SymRule<double> r64;
    SymRule<float> r32;
};

template <typename C>
__device__ __forceinline__ const SymRule<C> &rule_of(const P3 &p);
template <>
__device__ __forceinline__ const SymRule<double> &rule_of<double>(const P3 &p) { return p.r64; }
template <>
__device__ __forceinline__ const SymRule<float> &rule_of<float>(const P3 &p) { return p.r32; }

__device__ __forceinline__ int wrap(int s, int n)
{
    s += (s < 0) ? n : 0;
    s -= (s >= n) ? n : 0;
    return s;
}

// rho, rho u and sum f |v|^2 of 125 populations from the three marginals
// X_i = sum_(j,l) f, Y_j = sum_(i,l) f, Z_l = sum_(i,j) f.
template <typename C>
__device__ __forceinline__ void sums125(const C (&f)[N125], const SymRule<C> &R, C &rho, C &jx, C &jy,
                                        C &jz, C &e)
{
    C P[Q * Q], X[Q], Y[Q], Z[Q];
#pragma unroll
    for (int m = 0; m < Q * Q; ++m)
        P[m] = ((f[m] + f[m + 25]) + (f[m + 50] + f[m + 75])) + f[m + 100];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        C s = f[25 * l];
#pragma unroll
        for (int m = 1; m < Q * Q; ++m) s += f[m + 25 * l];
        Z[l] = s;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        X[i] = ((P[i] + P[i + 5]) + (P[i + 10] + P[i + 15])) + P[i + 20];
        Y[i] = ((P[5 * i] + P[5 * i + 1]) + (P[5 * i + 2] + P[5 * i + 3])) + P[5 * i + 4];
    }
    rho = (X[0] + (X[1] + X[2])) + (X[3] + X[4]);
    jx = fma(R.a, X[1] - X[2], R.b * (X[3] - X[4]));
    jy = fma(R.a, Y[1] - Y[2], R.b * (Y[3] - Y[4]));
    jz = fma(R.a, Z[1] - Z[2], R.b * (Z[3] - Z[4]));
    e = fma(R.a2, (X[1] + X[2]) + (Y[1] + Y[2]) + (Z[1] + Z[2]),
            R.b2 * ((X[3] + X[4]) + (Y[3] + Y[4]) + (Z[3] + Z[4])));
}

template <typename T>
__device__ __forceinline__ T load_pop(const T *base, unsigned byte_off)
{
    const T *q = reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
    if constexpr (PLBM_Q125_NT_LOAD) return __builtin_nontemporal_load(q);
    else return *q;
}

// Pull of node (xb, y, z): f_k = src_k(x - v_i, y - v_j, z - v_l).  Lanes
// past the ragged right edge read column nx - 1 (their results are dropped).
template <typename T, typename C>
__device__ __forceinline__ void gather125(const T *__restrict__ src, const P3 &p, int xb, int y, int z,
                                          C (&f)[N125])
{
    const int nx = p.nx;
    const long long rowelems = (long long)N125 * nx;
    unsigned lo[Q];
    const int xc = min(xb, nx - 1);
#pragma unroll
    for (int i = 0; i < Q; ++i)   // unsigned: the FP64 offsets pass 2^31 for nx near 2^26
        lo[i] = ((unsigned)wrap(xc - p.sx[i], nx) + (unsigned)i * (unsigned)nx) * (unsigned)sizeof(T);
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const int zs = wrap(z - p.sx[l], p.nz);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const int ys = wrap(y - p.sx[j], p.ny);
            const T *base = src + (((long long)zs * p.ny + ys) * rowelems + (long long)(Q * j + 25 * l) * nx);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if ((PLBM_Q125_NT_MASK >> i) & 1)
                    f[i + Q * j + 25 * l] = (C)__builtin_nontemporal_load(
                        reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + lo[i]));
                else
                    f[i + Q * j + 25 * l] = (C)load_pop(base, lo[i]);
            }
        }
    }
}

// f <- (1 - omega) f + omega rho r^x_i r^y_j r^z_l (Eq. srt, collision half).
template <typename C>
__device__ __forceinline__ void collide125(C (&f)[N125], const SymRule<C> &R)
{
    C rho, jx, jy, jz, e;
    sums125<C>(f, R, rho, jx, jy, jz, e);
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const C theta = (e * inv - (ux * ux + uy * uy + uz * uz)) * (C(1) / C(3));
    C rx[Q], ry[Q], rz[Q];
    rule_sym<C>(ux, theta, R, rx);
    rule_sym<C>(uy, theta, R, ry);
    rule_sym<C>(uz, theta, R, rz);
    const C wr = R.omega * rho, keep = C(1) - R.omega;
#pragma unroll
    for (int i = 0; i < Q; ++i) rx[i] *= wr;
#pragma unroll
    for (int l = 0; l < Q; ++l)
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const C t = ry[j] * rz[l];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int k = i + Q * j + 25 * l;
                f[k] = fma(keep, f[k], rx[i] * t);
            }
        }
}

// One step over the row segments tile = (z ny + y) tiles_x + tx.  Optional
// FP64 block sums of what is stored: (sum f, sum f v_x, sum f v_y,
// sum f |v|^2, sum f v_z).
template <typename T, bool SUMS>
__global__ __launch_bounds__(TX) void k_step3d(const T *__restrict__ src, T *__restrict__ dst, P3 p,
                                               double *__restrict__ partials)
{
    using C = T;
    const SymRule<C> &R = rule_of<C>(p);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const long long rowelems = (long long)N125 * p.nx;
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int tile = slot; tile < p.ntiles; tile += gridDim.x) {
        const int row = tile / p.tiles_x;
        const int z = row / p.ny, y = row - z * p.ny;
        const int xb = (tile - row * p.tiles_x) * TX + threadIdx.x;
        C f[N125];
        gather125<T, C>(src, p, xb, y, z, f);
        collide125<C>(f, R);
        if (xb < p.nx) {
            if constexpr (SUMS) {
                C g[N125];
#pragma unroll
                for (int k = 0; k < N125; ++k) g[k] = (C)(T)f[k];
                C rho, jx, jy, jz, e;
                sums125<C>(g, R, rho, jx, jy, jz, e);
                acc[0] += rho;
                acc[1] += jx;
                acc[2] += jy;
                acc[3] += e;
                acc[4] += jz;
            }
            T *base = dst + ((long long)row * rowelems + xb);
#pragma unroll
            for (int k = 0; k < N125; ++k) store_stream((T)f[k], base + (long long)k * p.nx);
        }
    }
    if constexpr (SUMS) block_sums_store<5>(acc, partials + (size_t)blockIdx.x * 5);
}

// Initial state: node (x, y, z) evaluates f_eq(rho, u, theta) in FP64 and
// writes population k to (x - v_i, y - v_j, z - v_l), so the first pull
// returns exactly f_eq.
template <typename T>
__global__ __launch_bounds__(TX) void k_init3d(const double *__restrict__ rho, const double *__restrict__ ux,
                                               const double *__restrict__ uy, const double *__restrict__ uz,
                                               const double *__restrict__ th, T *__restrict__ dst, P3 p)
{
    const long long rowelems = (long long)N125 * p.nx;
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int row = tile / p.tiles_x;
        const int z = row / p.ny, y = row - z * p.ny;
        const int x = (tile - row * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        const long long n = (long long)row * p.nx + x;
        double rx[Q], ry[Q], rz[Q];
        rule_sym<double>(ux[n], th[n], p.r64, rx);
        rule_sym<double>(uy[n], th[n], p.r64, ry);
        rule_sym<double>(uz[n], th[n], p.r64, rz);
        const double r = rho[n];
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            const int zd = wrap(z - p.sx[l], p.nz);
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int yd = wrap(y - p.sx[j], p.ny);
                T *base = dst + ((long long)zd * p.ny + yd) * rowelems;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int xd = wrap(x - p.sx[i], p.nx);
                    const int k = i + Q * j + 25 * l;
                    base[(long long)k * p.nx + xd] = (T)(r * rx[i] * ry[j] * rz[l]);
                }
            }
        }
    }
}

// Macroscopic fields of the pulled state (3 rho theta = sum f |v - u|^2) and
// optional FP64 block sums in the order of the step's.
template <typename T>
__global__ __launch_bounds__(TX) void k_moments3d(const T *__restrict__ src, P3 p, double *__restrict__ rho,
                                                  double *__restrict__ ux, double *__restrict__ uy,
                                                  double *__restrict__ uz, double *__restrict__ th,
                                                  double *__restrict__ partials)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int row = tile / p.tiles_x;
        const int z = row / p.ny, y = row - z * p.ny;
        const int x = (tile - row * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        double f[N125];
        gather125<T, double>(src, p, x, y, z, f);
        double r, jx, jy, jz, e;
        sums125<double>(f, p.r64, r, jx, jy, jz, e);
        const long long n = (long long)row * p.nx + x;
        const double u = jx / r, v = jy / r, w = jz / r;
        if (rho) rho[n] = r;
        if (ux) ux[n] = u;
        if (uy) uy[n] = v;
        if (uz) uz[n] = w;
        if (th) th[n] = (e / r - (u * u + v * v + w * w)) / 3.0;
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += e;
        acc[4] += jz;
    }
    if (partials) block_sums_store<5>(acc, partials + (size_t)blockIdx.x * 5);
}

int q125_hip(hipError_t e)
{
    if (e == hipSuccess) return PLBM_OK;
    plbm::note_hip_error(hipGetErrorString(e), (int)e);
    return PLBM_EHIP;
}

int q125_launch_status() { return q125_hip(hipGetLastError()); }

// dim 3, q1d 5, FP64 or FP32, the symmetric set (0, a, -a, b, -b) with the
// reduced table of its Lagrange polynomials.
int q125_params(const plbm_desc *d, P3 &p)
{
    int rc = plbm::validate(d);
    if (rc != PLBM_OK) return rc;
    if (d->dim != 3 || d->q1d != Q) return PLBM_EINVAL;
    if (d->storage != PLBM_F64 && d->storage != PLBM_F32) return PLBM_EUNSUPPORTED;
    std::memset(&p, 0, sizeof(p));
    rc = sym_rule(d, p.r64);
    if (rc != PLBM_OK) return rc;
    const SymRule<double> &R = p.r64;
    p.r32 = SymRule<float>{(float)R.a,   (float)R.b,   (float)R.a2,  (float)R.b2,  (float)R.c02,
                           (float)R.c04, (float)R.c11, (float)R.c12, (float)R.c13, (float)R.c14,
                           (float)R.c31, (float)R.c32, (float)R.c33, (float)R.c34, (float)R.omega};
    p.nx = d->nx;
    p.ny = d->ny;
    p.nz = d->nz;
    p.tiles_x = (d->nx + TX - 1) / TX;
    const long long nt = (long long)p.tiles_x * d->ny * d->nz;
    if (nt > 0x7fffffffLL) return PLBM_EINVAL;
    p.ntiles = (int)nt;
    for (int i = 0; i < Q; ++i) p.sx[i] = (int)d->v[i];
    return PLBM_OK;
}

inline int grid_of(const P3 &p) { return std::min(p.ntiles, MAX_GRID3); }

template <typename T>
constexpr size_t lds_cap() { return sizeof(T) == 8 ? PLBM_Q125_LDS_F64 : PLBM_Q125_LDS_F32; }

int q125_finish_sums(double *dev, int nblocks, double *host, hipStream_t st)
{
    double *out = dev + (size_t)nblocks * 5;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_reduce_partials<5>, dim3(1), dim3(RED_THREADS), 0, st, dev, nblocks, out);
    int rc = q125_launch_status();
    if (rc == PLBM_OK) rc = q125_hip(hipMemcpyAsync(host, out, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = q125_hip(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    for (int m = 0; m < 5; ++m)
        if (!std::isfinite(host[m])) return PLBM_ENONFINITE;
    return PLBM_OK;
}

template <typename T>
int q125_run(const P3 &p, void *fa, void *fb, int nsteps, double *sums, hipStream_t st)
{
    const int grid = grid_of(p);
    for (int s = 0; s < nsteps; ++s) {
        const T *src = static_cast<const T *>((s & 1) ? fb : fa);
        T *dst = static_cast<T *>((s & 1) ? fa : fb);
        (void)hipGetLastError();
        if (s == nsteps - 1 && sums) {
            double *part = nullptr;
            int rc = q125_hip(hipMallocAsync((void **)&part, ((size_t)grid + 1) * 5 * sizeof(double), st));
            if (rc != PLBM_OK) return rc;
            hipLaunchKernelGGL((k_step3d<T, true>), dim3(grid), dim3(TX), lds_cap<T>(), st, src, dst, p, part);
            rc = q125_launch_status();
            if (rc == PLBM_OK) rc = q125_finish_sums(part, grid, sums, st);
            (void)hipFreeAsync(part, st);
            return rc;
        }
        hipLaunchKernelGGL((k_step3d<T, false>), dim3(grid), dim3(TX), lds_cap<T>(), st, src, dst, p, nullptr);
        const int rc = q125_launch_status();
        if (rc != PLBM_OK) return rc;
    }
    return PLBM_OK;
}

} // namespace

namespace plbm {

int q125_step(const plbm_desc *d, void *fa, void *fb, int nsteps, double *sums, void *stream)
{
    P3 p;
    const int rc = q125_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!fa || !fb || fa == fb || nsteps < 0) return PLBM_EINVAL;
    if (nsteps == 0)
        return sums ? plbm_moments3(d, fa, nullptr, nullptr, nullptr, nullptr, nullptr, sums, stream) : PLBM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (d->storage == PLBM_F64) return q125_run<double>(p, fa, fb, nsteps, sums, st);
    return q125_run<float>(p, fa, fb, nsteps, sums, st);
}

} // namespace plbm

extern "C" int plbm_init3(const plbm_desc *d, const double *rho, const double *ux, const double *uy,
                          const double *uz, const double *theta, void *f, void *stream)
{
    P3 p;
    const int rc = q125_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !uy || !uz || !theta || !f) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (d->storage == PLBM_F64)
        hipLaunchKernelGGL(k_init3d<double>, dim3(grid_of(p)), dim3(TX), 0, st, rho, ux, uy, uz, theta,
                           (double *)f, p);
    else
        hipLaunchKernelGGL(k_init3d<float>, dim3(grid_of(p)), dim3(TX), 0, st, rho, ux, uy, uz, theta,
                           (float *)f, p);
    return q125_launch_status();
}

extern "C" int plbm_moments3(const plbm_desc *d, const void *f, double *rho, double *ux, double *uy,
                             double *uz, double *theta, double *sums, void *stream)
{
    P3 p;
    int rc = q125_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int grid = grid_of(p);
    double *part = nullptr;
    if (sums) {
        rc = q125_hip(hipMallocAsync((void **)&part, ((size_t)grid + 1) * 5 * sizeof(double), st));
        if (rc != PLBM_OK) return rc;
    }
    (void)hipGetLastError();
    if (d->storage == PLBM_F64)
        hipLaunchKernelGGL(k_moments3d<double>, dim3(grid), dim3(TX), 0, st, (const double *)f, p, rho, ux, uy, uz,
                           theta, part);
    else
        hipLaunchKernelGGL(k_moments3d<float>, dim3(grid), dim3(TX), 0, st, (const float *)f, p, rho, ux, uy, uz,
                           theta, part);
    rc = q125_launch_status();
    if (rc == PLBM_OK && sums) rc = q125_finish_sums(part, grid, sums, st);
    if (part) (void)hipFreeAsync(part, st);
    return rc;
}
