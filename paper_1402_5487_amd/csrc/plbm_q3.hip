// libplbm device code for the isothermal three-velocity family: the 1D rule
// of Eq. 1d3v (velocities {0, +a, -a}, a^2 = zeta theta0) on D1Q3 lattices
// with zero-gradient ends, and its tensor product D2Q9 on periodic lattices.  It is the Lagrange rule of Eq. rdr with the Maxwell
// moments of a fixed reference temperature: mu_0 = 1, mu_1 = u,
// mu_2 = theta0 + u^2, so for the symmetric set
//   r_0 = 1 + c02 mu_2,   r_(+-a) = c12 mu_2 +- c11 mu_1
// with c02 = -1/a^2, c11 = 1/(2a), c12 = 1/(2a^2) (the Lagrange polynomials
// through 0 and +-a).  zeta = 3 gives the LBGK D2Q9 equilibrium in product
// form, zeta = 4 the parametric model of Table 3vel.
//
// Same streaming design as the D2Q25 step: pull scheme with A/B buffers,
// row-interleaved layout (y * 9 + k) * nx + x (1D: k * (nx + 6) + x + 3, three
// ghost nodes per end as for D1Q5), one 256-node row segment per
// workgroup with XCD-contiguous tile numbering, a scalar row base per y
// velocity plus a 32-bit lane offset per x velocity (the periodic wrap in x
// folded into the offsets), non-temporal stores (and loads for 4- and
// 8-byte populations).  FP64 storage computes in FP64, FP32 in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "plbm_device.h"
#include "plbm_internal.h"

namespace {

constexpr int Q3 = 3;
constexpr int N9 = Q3 * Q3;

// LDS reserved per workgroup as a residency cap (measured on MI355X at
// 4096^2: 9 loads per lane need more resident waves in FP32 than in FP64;
// FP32 0.78 of peak at 10-20 KB against 0.54 at 80 KB, FP64 best at 53 KB)
#ifndef PLBM_Q9_LDS_F64
#define PLBM_Q9_LDS_F64 (53 * 1024)
#endif
#ifndef PLBM_Q9_LDS_F32
#define PLBM_Q9_LDS_F32 (16 * 1024)
#endif

template <typename C>
struct Rule3 {
    C a, a2;                 // velocity magnitude and its square
    C c02, c11, c12;         // reduced Lagrange table of {0, +a, -a}
    C theta0, omega;
};

struct Q9Params {
    int dim;
    int nx, ny, tiles_x, ntiles;
    int sx[Q3];              // streaming shifts (0, +a, -a)
    Rule3<double> r64;
    Rule3<float> r32;
};

template <typename C>
__device__ __forceinline__ const Rule3<C> &rule_of(const Q9Params &p);
template <>
__device__ __forceinline__ const Rule3<double> &rule_of<double>(const Q9Params &p) { return p.r64; }
template <>
__device__ __forceinline__ const Rule3<float> &rule_of<float>(const Q9Params &p) { return p.r32; }

// isothermal 1D rule: mu_2 = theta0 + u^2
template <typename C>
__device__ __forceinline__ void rule3(C u, const Rule3<C> &R, C (&r)[Q3])
{
    const C m2 = fma(u, u, R.theta0);
    const C e = R.c12 * m2, o = R.c11 * u;
    r[0] = fma(R.c02, m2, C(1));
    r[1] = e + o;
    r[2] = e - o;
}

// rho, rho u_x, rho u_y and sum f |v|^2 via column and row sums
template <typename C>
__device__ __forceinline__ void sums9(const C (&f)[N9], const Rule3<C> &R, C &rho, C &jx, C &jy, C &e)
{
    C col[Q3], row[Q3];
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        col[i] = f[i] + f[i + Q3] + f[i + 2 * Q3];
        row[i] = f[Q3 * i] + f[Q3 * i + 1] + f[Q3 * i + 2];
    }
    rho = col[0] + (col[1] + col[2]);
    jx = R.a * (col[1] - col[2]);
    jy = R.a * (row[1] - row[2]);
    e = R.a2 * ((col[1] + col[2]) + (row[1] + row[2]));
}

// Non-temporal loads for the velocity columns in this mask (bit i: v_i).
// Column 0 (v = 0) reads exactly the wave's own nodes; the shifted columns'
// edge lines are read again by the neighbouring wave from L2.  Column 0
// alone is 0.8 % faster than all columns (FP32 at 4096^2).
#ifndef PLBM_Q3_NT_MASK
#define PLBM_Q3_NT_MASK 1
#endif

template <typename T>
__device__ __forceinline__ void store_pop(T v, T *p)
{
    if constexpr (PLBM_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Pull-gather of node (xb, y): f_k = src_k(x - v_i, y - v_j), k = i + 3 j.
template <typename T, typename C>
__device__ __forceinline__ void gather9(const T *__restrict__ src, const Q9Params &p, int xb, int y, C (&f)[N9])
{
    const int nx = p.nx, ny = p.ny;
    const long long rowelems = (long long)N9 * nx;
    unsigned lo[Q3];
    const int xc = min(xb, nx - 1);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        int xs = xc - p.sx[i];
        xs += (xs < 0) ? nx : 0;
        xs -= (xs >= nx) ? nx : 0;
        lo[i] = (unsigned)(xs + i * nx);
    }
#pragma unroll
    for (int j = 0; j < Q3; ++j) {
        int ys = y - p.sx[j];
        ys += (ys < 0) ? ny : 0;
        ys -= (ys >= ny) ? ny : 0;
        const T *base = src + (ys * rowelems + (long long)(Q3 * j) * nx);
#pragma unroll
        for (int i = 0; i < Q3; ++i) {
            if ((PLBM_Q3_NT_MASK >> i) & 1) f[i + Q3 * j] = (C)__builtin_nontemporal_load(&base[lo[i]]);
            else f[i + Q3 * j] = (C)base[lo[i]];
        }
    }
}

// One step (Eq. srt): gather, moments, isothermal equilibrium f_eq =
// rho r^x_i r^y_j, relax, store at x.  Optional FP64 block sums of what is
// stored (sum f, sum f v_x, sum f v_y, sum f |v|^2).
template <typename T, typename C, bool SUMS>
__global__ __launch_bounds__(TX) void k_step_q9(const T *__restrict__ src, T *__restrict__ dst, Q9Params p,
                                                double *__restrict__ partials)
{
    const Rule3<C> &R = rule_of<C>(p);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long rowelems = (long long)N9 * p.nx;
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int tile = slot; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int xb = (tile - y * p.tiles_x) * TX + threadIdx.x;
        C f[N9];
        gather9<T, C>(src, p, xb, y, f);
        C rho, jx, jy, e;
        sums9<C>(f, R, rho, jx, jy, e);
        const C inv = C(1) / rho;
        C rx[Q3], ry[Q3];
        rule3<C>(jx * inv, R, rx);
        rule3<C>(jy * inv, R, ry);
        const C wr = R.omega * rho, keep = C(1) - R.omega;
#pragma unroll
        for (int i = 0; i < Q3; ++i) rx[i] *= wr;
#pragma unroll
        for (int j = 0; j < Q3; ++j)
#pragma unroll
            for (int i = 0; i < Q3; ++i) f[i + Q3 * j] = fma(keep, f[i + Q3 * j], rx[i] * ry[j]);
        if (xb < p.nx) {
            if constexpr (SUMS) {
                C g[N9];
#pragma unroll
                for (int k = 0; k < N9; ++k) g[k] = (C)(T)f[k];
                sums9<C>(g, R, rho, jx, jy, e);
                acc[0] += rho;
                acc[1] += jx;
                acc[2] += jy;
                acc[3] += e;
            }
            T *out = dst + (y * rowelems + xb);
#pragma unroll
            for (int k = 0; k < N9; ++k) store_pop((T)f[k], out + (long long)k * p.nx);
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// Initial state: node x evaluates f_eq(rho, u; theta0) in FP64 and writes
// population k to x - v_k, so the first pull returns exactly f_eq.
template <typename T>
__global__ __launch_bounds__(TX) void k_init_q9(const double *__restrict__ rho, const double *__restrict__ ux,
                                                const double *__restrict__ uy, T *__restrict__ dst, Q9Params p)
{
    const long long rowelems = (long long)N9 * p.nx;
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int x = (tile - y * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        const long long n = (long long)y * p.nx + x;
        double rx[Q3], ry[Q3];
        rule3<double>(ux[n], p.r64, rx);
        rule3<double>(uy[n], p.r64, ry);
#pragma unroll
        for (int j = 0; j < Q3; ++j) {
            int yd = y - p.sx[j];
            yd += (yd < 0) ? p.ny : 0;
            yd -= (yd >= p.ny) ? p.ny : 0;
#pragma unroll
            for (int i = 0; i < Q3; ++i) {
                int xd = x - p.sx[i];
                xd += (xd < 0) ? p.nx : 0;
                xd -= (xd >= p.nx) ? p.nx : 0;
                dst[yd * rowelems + (long long)(i + Q3 * j) * p.nx + xd] = (T)(rho[n] * rx[i] * ry[j]);
            }
        }
    }
}

// Macroscopic fields of the pulled state (2 rho theta = sum f |v - u|^2) and
// optional FP64 block sums.
template <typename T>
__global__ __launch_bounds__(TX) void k_moments_q9(const T *__restrict__ src, Q9Params p, double *__restrict__ rho,
                                                   double *__restrict__ ux, double *__restrict__ uy,
                                                   double *__restrict__ th, double *__restrict__ partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int tile = blockIdx.x; tile < p.ntiles; tile += gridDim.x) {
        const int y = tile / p.tiles_x;
        const int x = (tile - y * p.tiles_x) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        double f[N9];
        gather9<T, double>(src, p, x, y, f);
        double r, jx, jy, e;
        sums9<double>(f, p.r64, r, jx, jy, e);
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
// D1Q3: padded layout k * (nx + 6) + x + 3.  Step: pull f_k = src_k(x - v_k),
// relax to rho r(u), write at x; the ghost nodes at each end take the edge
// node's post-collision populations (zero-gradient ends, as for D1Q5).
// ---------------------------------------------------------------------------
template <typename T, typename C, bool SUMS>
__global__ __launch_bounds__(TX) void k_step_q3_1d(const T *__restrict__ src, T *__restrict__ dst, Q9Params p,
                                                   double *__restrict__ partials)
{
    const Rule3<C> &R = rule_of<C>(p);
    const int x = blockIdx.x * TX + threadIdx.x;
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        C f[Q3];
#pragma unroll
        for (int k = 0; k < Q3; ++k) f[k] = (C)src[k * ps + x + PLBM_GHOST - p.sx[k]];
        const C rho = f[0] + (f[1] + f[2]);
        const C u = R.a * (f[1] - f[2]) / rho;
        C r[Q3];
        rule3<C>(u, R, r);
        const C wr = R.omega * rho, keep = C(1) - R.omega;
#pragma unroll
        for (int k = 0; k < Q3; ++k) {
            const T h = (T)fma(keep, f[k], wr * r[k]);
            dst[k * ps + x + PLBM_GHOST] = h;
            if (x == 0)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * ps + g] = h;
            if (x == p.nx - 1)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * ps + p.nx + PLBM_GHOST + g] = h;
            if constexpr (SUMS) {
                const double vk = (double)p.sx[k];
                acc[0] += (double)h;
                acc[1] += (double)h * vk;
                acc[3] += (double)h * vk * vk;
            }
        }
    }
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// Padded index q holds node y = q - 3; population k there is f_eq_k of node
// y + v_k (clamped into the lattice), so the pull at y + v_k returns f_eq.
template <typename T>
__global__ __launch_bounds__(TX) void k_init_q3_1d(const double *__restrict__ rho, const double *__restrict__ ux,
                                                   T *__restrict__ dst, Q9Params p)
{
    const int q = blockIdx.x * TX + threadIdx.x;
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    if (q >= ps) return;
    const int y = q - PLBM_GHOST;
#pragma unroll
    for (int k = 0; k < Q3; ++k) {
        int s = y + p.sx[k];
        s = s < 0 ? 0 : (s >= p.nx ? p.nx - 1 : s);
        double r[Q3];
        rule3<double>(ux[s], p.r64, r);
        dst[k * ps + q] = (T)(rho[s] * r[k]);
    }
}

// rho, u and rho theta = sum f (v - u)^2 (one dimension) of the pulled state.
template <typename T>
__global__ __launch_bounds__(TX) void k_moments_q3_1d(const T *__restrict__ src, Q9Params p, double *__restrict__ rho,
                                                      double *__restrict__ ux, double *__restrict__ th,
                                                      double *__restrict__ partials)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const long long ps = (long long)p.nx + 2 * PLBM_GHOST;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < p.nx) {
        double f[Q3];
#pragma unroll
        for (int k = 0; k < Q3; ++k) f[k] = (double)src[k * ps + x + PLBM_GHOST - p.sx[k]];
        const double r = f[0] + (f[1] + f[2]);
        const double j = p.r64.a * (f[1] - f[2]);
        const double e = p.r64.a2 * (f[1] + f[2]);
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

int q9_hip(hipError_t e)
{
    if (e == hipSuccess) return PLBM_OK;
    plbm::note_hip_error(hipGetErrorString(e), (int)e);
    return PLBM_EHIP;
}

int q9_launch_status() { return q9_hip(hipGetLastError()); }

// The descriptor of the three-velocity family: dim 2, q1d 3, FP64 or FP32,
// v = (0, +a, -a) with integer a, theta0 > 0, and a table with the structure
// of the Lagrange polynomials of that set.
int q9_params(const plbm_desc *d, Q9Params &p)
{
    const int rc = plbm::validate(d);
    if (rc != PLBM_OK) return rc;
    if (d->q1d != Q3) return PLBM_EINVAL;
    if (d->storage != PLBM_F64 && d->storage != PLBM_F32) return PLBM_EUNSUPPORTED;
    if (!(d->theta0 > 0.0) || !std::isfinite(d->theta0)) return PLBM_EINVAL;
    const double a = d->v[1];
    if (d->v[0] != 0.0 || !(a > 0.0) || d->v[2] != -a) return PLBM_EUNSUPPORTED;
    const double *c = d->c;
    const double c02 = c[2], c11 = c[Q3 + 1], c12 = c[Q3 + 2];
    auto near = [](double x, double y) { return std::fabs(x - y) <= 1e-12 * std::max(1.0, std::fabs(y)); };
    const bool sym = near(c[0], 1.0) && near(c[1], 0.0) && near(c[Q3], 0.0) && near(c[2 * Q3], 0.0) &&
                     near(c[2 * Q3 + 1], -c11) && near(c[2 * Q3 + 2], c12) && near(c02, -1.0 / (a * a)) &&
                     near(c11, 0.5 / a) && near(c12, 0.5 / (a * a));
    if (!sym) return PLBM_EUNSUPPORTED;
    std::memset(&p, 0, sizeof(p));
    p.dim = d->dim;
    p.nx = d->nx;
    p.ny = d->ny;
    p.tiles_x = (d->nx + TX - 1) / TX;
    p.ntiles = p.tiles_x * d->ny;
    p.sx[0] = 0;
    p.sx[1] = (int)a;
    p.sx[2] = -(int)a;
    p.r64 = Rule3<double>{a, a * a, c02, c11, c12, d->theta0, d->omega};
    p.r32 = Rule3<float>{(float)a, (float)(a * a), (float)c02, (float)c11, (float)c12, (float)d->theta0,
                         (float)d->omega};
    return PLBM_OK;
}

int q9_finish_sums(double *dev, int nblocks, double *host, hipStream_t st)
{
    double *out = dev + (size_t)nblocks * 4;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_reduce_partials<4>, dim3(1), dim3(RED_THREADS), 0, st, dev, nblocks, out);
    int rc = q9_launch_status();
    if (rc == PLBM_OK) rc = q9_hip(hipMemcpyAsync(host, out, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = q9_hip(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    for (int m = 0; m < 4; ++m)
        if (!std::isfinite(host[m])) return PLBM_ENONFINITE;
    return PLBM_OK;
}

template <typename T, typename C, bool SUMS>
void q3_launch(const Q9Params &p, const T *src, T *dst, double *part, hipStream_t st)
{
    if (p.dim == 2) {
        const size_t lds = sizeof(T) == 8 ? PLBM_Q9_LDS_F64 : PLBM_Q9_LDS_F32;
        hipLaunchKernelGGL((k_step_q9<T, C, SUMS>), dim3(grid_for(p.ntiles)), dim3(TX), lds, st, src, dst, p,
                           part);
    } else {
        hipLaunchKernelGGL((k_step_q3_1d<T, C, SUMS>), dim3(p.tiles_x), dim3(TX), 0, st, src, dst, p, part);
    }
}

template <typename T, typename C>
int q9_run(const Q9Params &p, void *fa, void *fb, int nsteps, double *sums, hipStream_t st)
{
    const int nblocks = p.dim == 2 ? grid_for(p.ntiles) : p.tiles_x;
    for (int s = 0; s < nsteps; ++s) {
        const T *src = static_cast<const T *>((s & 1) ? fb : fa);
        T *dst = static_cast<T *>((s & 1) ? fa : fb);
        (void)hipGetLastError();
        if (s == nsteps - 1 && sums) {
            double *part = nullptr;
            int rc = q9_hip(hipMallocAsync((void **)&part, ((size_t)nblocks + 1) * 4 * sizeof(double), st));
            if (rc != PLBM_OK) return rc;
            q3_launch<T, C, true>(p, src, dst, part, st);
            rc = q9_launch_status();
            if (rc == PLBM_OK) rc = q9_finish_sums(part, nblocks, sums, st);
            (void)hipFreeAsync(part, st);
            return rc;
        }
        q3_launch<T, C, false>(p, src, dst, nullptr, st);
        const int rc = q9_launch_status();
        if (rc != PLBM_OK) return rc;
    }
    return PLBM_OK;
}

} // namespace

namespace plbm {

int q3_init(const plbm_desc *d, const double *rho, const double *ux, const double *uy, void *f, void *stream)
{
    Q9Params p;
    const int rc = q9_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !f || (p.dim == 2 && !uy)) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (p.dim == 1) {
        const dim3 g((unsigned)((p.nx + 2 * PLBM_GHOST + TX - 1) / TX));
        if (d->storage == PLBM_F64)
            hipLaunchKernelGGL(k_init_q3_1d<double>, g, dim3(TX), 0, st, rho, ux, (double *)f, p);
        else
            hipLaunchKernelGGL(k_init_q3_1d<float>, g, dim3(TX), 0, st, rho, ux, (float *)f, p);
        return q9_launch_status();
    }
    const dim3 g(grid_for(p.ntiles));
    if (d->storage == PLBM_F64)
        hipLaunchKernelGGL(k_init_q9<double>, g, dim3(TX), 0, st, rho, ux, uy, (double *)f, p);
    else
        hipLaunchKernelGGL(k_init_q9<float>, g, dim3(TX), 0, st, rho, ux, uy, (float *)f, p);
    return q9_launch_status();
}

int q3_step(const plbm_desc *d, void *fa, void *fb, int nsteps, double *sums, void *stream)
{
    Q9Params p;
    const int rc = q9_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!fa || !fb || fa == fb || nsteps < 0) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (nsteps == 0) return sums ? q3_moments(d, fa, nullptr, nullptr, nullptr, nullptr, sums, stream) : PLBM_OK;
    if (d->storage == PLBM_F64) return q9_run<double, double>(p, fa, fb, nsteps, sums, st);
    return q9_run<float, float>(p, fa, fb, nsteps, sums, st);
}

int q3_moments(const plbm_desc *d, const void *f, double *rho, double *ux, double *uy, double *theta,
               double *sums, void *stream)
{
    Q9Params p;
    int rc = q9_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 g(p.dim == 2 ? grid_for(p.ntiles) : p.tiles_x);
    const int nblocks = (int)g.x;
    double *part = nullptr;
    if (sums) {
        rc = q9_hip(hipMallocAsync((void **)&part, ((size_t)nblocks + 1) * 4 * sizeof(double), st));
        if (rc != PLBM_OK) return rc;
    }
    (void)hipGetLastError();
    if (p.dim == 1) {
        if (d->storage == PLBM_F64)
            hipLaunchKernelGGL(k_moments_q3_1d<double>, g, dim3(TX), 0, st, (const double *)f, p, rho, ux, theta,
                               part);
        else
            hipLaunchKernelGGL(k_moments_q3_1d<float>, g, dim3(TX), 0, st, (const float *)f, p, rho, ux, theta,
                               part);
    } else if (d->storage == PLBM_F64) {
        hipLaunchKernelGGL(k_moments_q9<double>, g, dim3(TX), 0, st, (const double *)f, p, rho, ux, uy, theta, part);
    } else {
        hipLaunchKernelGGL(k_moments_q9<float>, g, dim3(TX), 0, st, (const float *)f, p, rho, ux, uy, theta, part);
    }
    rc = q9_launch_status();
    if (rc == PLBM_OK && sums) rc = q9_finish_sums(part, nblocks, sums, st);
    if (part) (void)hipFreeAsync(part, st);
    return rc;
}

} // namespace plbm
