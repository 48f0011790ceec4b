// libplbm device code for gfx950: the fused collide-and-stream step of the
// parametric lattice Boltzmann method (arXiv:1402.5487, Eq. srt with the
// equilibrium of Eq. eqdist / Eq. rdr), initialisation, moments and the FP64
// invariant reductions, plus the C-ABI launchers that validate and enqueue
// them.
//
// Design (memory-bound streaming kernel, measured on MI355X):
//  * Pull scheme with A/B buffers: each node gathers population k from
//    src_k(x - v_k) and writes its post-collision value to dst_k(x), so every
//    population is read once and written once per step with wave-contiguous
//    addresses, and the step is race-free by construction.
//  * Row-interleaved layout (y * q + k) * nx + x: the 25 rows one output row
//    reads come from seven contiguous blocks and its 25 writes form one
//    contiguous block, far fewer concurrent DRAM streams than 25 separate
//    planes (measured +10-15% bandwidth).
//  * One workgroup per tile of 256 nodes of one row (four wave64 side by
//    side).  Tiles are numbered so that each of the eight XCDs gets a
//    contiguous run: neighbouring tiles, whose shifted windows share cache
//    lines at their edges, meet in the same L2.  Resident workgroups per CU
//    are capped (see PLBM_LDS_CAP_*).
//  * Addressing: per output row the wave computes five scalar row bases (one
//    per y velocity, periodic wrap applied to the uniform row index) and each
//    lane keeps five 32-bit offsets (one per x velocity), so each of the 50
//    accesses is a scalar base plus a vector offset.  Only the waves whose
//    windows cross the periodic seam in x take a per-node wrapped path.
//  * Arithmetic per node: column/row sums give rho, j and sum f|v|^2; the
//    Maxwell moments follow mu_(n+1) = u mu_n + n theta mu_(n-1); the 1D rule
//    r = C mu uses the reduced table of a symmetric velocity set; f_eq =
//    rho r^x_i r^y_j, with the relaxation folded into a_i = omega rho r^x_i
//    so each population costs one multiply and one FMA.  FP64 storage
//    computes in FP64; the other forms compute in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include <mutex>

#include "plbm_device.h"
#include "plbm_internal.h"

// Scratch of plbm_step_noalloc: the per-workgroup FP64 partial sums of its
// sums launch (at most NOALLOC_BLOCKS workgroups, four doubles each) and the
// four reduced sums behind them.  Each GPU the library runs on holds its own
// copy until the process ends.  Every workgroup of a sums launch writes its
// own four partials before the reduction reads them, so nothing in it has to
// start at zero.  Host code must not use this name as a device address: it
// takes the address hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_BLOCKS = 8192;
static __device__ __align__(256) double scratch[(NOALLOC_BLOCKS + 1) * 4];

namespace {

// The step launch: either one block per tile, or (persistent) a grid of a
// few blocks per CU that walk the tiles in order, block b taking tile
// it * gridDim.x + (b's slot); a slot maps the eight XCDs to eight contiguous
// runs of tiles, so the blocks sharing an L2 work on neighbouring tiles and
// all blocks sweep memory together.  Every block ends when its next tile
// index passes ntiles.
template <class S, int NV, bool SUMS>
__global__ __launch_bounds__(TX, PLBM_MIN_WAVES) void k_step2d(const typename S::T *__restrict__ src,
                                                               typename S::T *__restrict__ dst,
                                                               KParams p,
                                                               double *__restrict__ partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int tile = slot; tile < p.ntiles; tile += gridDim.x)
        step_tile<S, NV, SUMS>(src, dst, p, tile, acc);
    if constexpr (SUMS) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// The same step, also writing the pre-collision fields of the state it reads
// (the moments its collision uses, in its arithmetic).
template <class S, int NV>
__global__ __launch_bounds__(TX, PLBM_MIN_WAVES) void k_step2d_fields(const typename S::T *__restrict__ src,
                                                                      typename S::T *__restrict__ dst,
                                                                      KParams p, FieldsOut fo)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int tile = slot; tile < p.ntiles; tile += gridDim.x)
        step_tile<S, NV, false, true>(src, dst, p, tile, acc, fo);
}

// ---------------------------------------------------------------------------
// 2D initialisation: the buffer whose pull is f_eq.  Node x computes its own
// equilibrium and scatters population k to x - v_k, so that pulling it back
// from x - v_k returns f_eq_k(x).  The equilibrium is evaluated in FP64 and
// rounded once into the storage type.
// ---------------------------------------------------------------------------
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
    const int segs = (p.nx + TX - 1) / TX;
    const long long total = (long long)segs * p.ny;
#pragma unroll 1
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int y = (int)(t / segs);
        const int x = (int)(t - (long long)y * segs) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        const long long n = (long long)y * p.nx + x;    // fields are (ny, nx) row-major
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
                dst[k * p.pstride + (long long)yd * p.rstride + xd] =
                    S::enc((typename S::C)feq[k], k, p, S::key((uint32_t)n));
            }
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
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int segs = (p.nx + TX - 1) / TX;
    const long long total = (long long)segs * p.ny;
#pragma unroll 1
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int y = (int)(t / segs);
        const int x = (int)(t - (long long)y * segs) * TX + threadIdx.x;
        if (x >= p.nx) continue;
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
                f[k] = (double)S::dec(src[k * p.pstride + (long long)ys * p.rstride + xs], k, p);
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
        acc[0] += r; acc[1] += jx; acc[2] += jy; acc[3] += e;
    }
    if (partials) block_sums_store<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// 1D (D1Q5) kernels on the ghost-padded layout: node x at x + 3.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ void collide1d(typename S::C (&f)[Q], const KParams &p)
{
    using C = typename S::C;
    const SymRule<C> &R = S::R(p);
    const C rho = (f[0] + (f[1] + f[2])) + (f[3] + f[4]);
    const C j = fma(R.a, f[1] - f[2], R.b * (f[3] - f[4]));
    const C e = fma(R.a2, f[1] + f[2], R.b2 * (f[3] + f[4]));
    const C inv = C(1) / rho;
    const C u = j * inv;
    const C theta = e * inv - u * u;
    C r[Q];
    rule1d<S>(u, theta, p, r);
    const C w = R.omega;
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
            f[k] = S::dec(src[k * p.pstride + x + PLBM_GHOST - p.sx[k]], k, p);
        collide1d<S>(f, p);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const auto h = S::enc(f[k], k, p, (uint32_t)x);
            dst[k * p.pstride + x + PLBM_GHOST] = h;
            // zero-gradient ends: ghosts take the edge node's post-collision value
            if (x == 0)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * p.pstride + g] = h;
            if (x == p.nx - 1)
                for (int g = 0; g < PLBM_GHOST; ++g) dst[k * p.pstride + p.nx + PLBM_GHOST + g] = h;
        }
        if constexpr (SUMS) {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double g = (double)S::dec(S::enc(f[k], k, p, (uint32_t)x), k, p);
                const double vk = (double)p.sx[k];
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
        dst[k * p.pstride + q] = S::enc((typename S::C)(rho[s] * r[k]), k, p, (uint32_t)q);
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
            const double f = (double)S::dec(src[k * p.pstride + x + PLBM_GHOST - p.sx[k]], k, p);
            const double vk = (double)p.sx[k];
            r += f;
            j += f * vk;
            e += f * vk * vk;
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
    double m[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) m[k] = 0.0;
    const int segs = (p.nx + TX - 1) / TX;
    const long long total = (long long)segs * p.ny;
#pragma unroll 1
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int y = (int)(t / segs);
        const int x = (int)(t - (long long)y * segs) * TX + threadIdx.x;
        if (x >= p.nx) continue;
        const long long n = (long long)y * p.nx + x;
        double feq[NQ];
        equilibrium2d(rho[n], ux[n], uy[n], th[n], p, feq);
#pragma unroll
        for (int k = 0; k < NQ; ++k) m[k] = fmax(m[k], fabs(feq[k] - base[k]));
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
        partials[(size_t)blockIdx.x * NQ + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

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

// Workgroups of a 2D launch over `tiles` tiles or row segments; max_blocks
// caps the grid (the kernels walk the remaining tiles in a grid-stride loop).
inline int grid_capped(long long tiles, int max_blocks)
{
    return std::min(grid_for(tiles), max_blocks);
}

template <class S, bool SUMS>
int launch_step(const KParams &p, const plbm_desc *d, const void *src, void *dst, double *partials,
                hipStream_t st, int &nblocks, int max_blocks = MAX_GRID)
{
    using T = typename S::T;
    clear_launch_error();
    if (d->dim == 2) {
        nblocks = grid_capped(p.ntiles, max_blocks);
        const size_t lds = sizeof(T) == 2 ? (d->rounding == PLBM_ROUND_STOCHASTIC ? PLBM_LDS_CAP_16SR
                                                                                 : PLBM_LDS_CAP_16)
                                          : PLBM_LDS_CAP_WIDE;
        if (p.nv == 2)
            hipLaunchKernelGGL((k_step2d<S, 2, SUMS>), dim3(nblocks), dim3(TX), lds, st,
                               (const T *)src, (T *)dst, p, partials);
        else
            hipLaunchKernelGGL((k_step2d<S, 1, SUMS>), dim3(nblocks), dim3(TX), lds, st,
                               (const T *)src, (T *)dst, p, partials);
    } else {
        nblocks = (p.nx + TX - 1) / TX;
        hipLaunchKernelGGL((k_step1d<S, SUMS>), dim3(nblocks), dim3(TX), 0, st,
                           (const T *)src, (T *)dst, p, partials);
    }
    return launch_status();
}

// 2D steps of which the first also writes the fields of the state it reads.
template <class S>
int run_steps_fields(const KParams &p, const plbm_desc *d, void *fa, void *fb, int nsteps, FieldsOut fo,
                     hipStream_t st)
{
    using T = typename S::T;
    clear_launch_error();
    const int nblocks = grid_for(p.ntiles);
    const size_t lds = sizeof(T) == 2 ? (d->rounding == PLBM_ROUND_STOCHASTIC ? PLBM_LDS_CAP_16SR
                                                                             : PLBM_LDS_CAP_16)
                                      : PLBM_LDS_CAP_WIDE;
    if (p.nv == 2)
        hipLaunchKernelGGL((k_step2d_fields<S, 2>), dim3(nblocks), dim3(TX), lds, st, (const T *)fa, (T *)fb, p,
                           fo);
    else
        hipLaunchKernelGGL((k_step2d_fields<S, 1>), dim3(nblocks), dim3(TX), lds, st, (const T *)fa, (T *)fb, p,
                           fo);
    int rc = launch_status();
    int nb = 0;
    for (int s = 1; s < nsteps && rc == PLBM_OK; ++s)
        rc = launch_step<S, false>(p, d, (s & 1) ? fb : fa, (s & 1) ? fa : fb, nullptr, st, nb);
    return rc;
}

// `scratch`: NULL, or a device buffer of (NOALLOC_BLOCKS + 1) * 4 doubles
// that receives the partial sums instead of a stream-ordered allocation (the
// sums launch then runs at most NOALLOC_BLOCKS workgroups).
template <class S>
int run_steps(const KParams &p, const plbm_desc *d, void *fa, void *fb, int nsteps, double *sums,
              hipStream_t st, double *scratch)
{
    int nb = 0;
    for (int s = 0; s < nsteps; ++s) {
        const void *src = (s & 1) ? fb : fa;
        void *dst = (s & 1) ? fa : fb;
        const bool last = (s == nsteps - 1);
        if (last && sums && scratch) {
            const int rc = launch_step<S, true>(p, d, src, dst, scratch, st, nb, NOALLOC_BLOCKS);
            return rc == PLBM_OK ? finish_sums(scratch, nb, sums, st) : rc;
        }
        if (last && sums) {
            const int nblocks = d->dim == 2 ? grid_for(p.ntiles) : (p.nx + TX - 1) / TX;
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
        hipLaunchKernelGGL(k_init2d<S>, dim3(grid_for((long long)((p.nx + TX - 1) / TX) * p.ny)),
                           dim3(TX), 0, st, rho, ux, uy, th, (T *)f, p);
    } else {
        hipLaunchKernelGGL(k_init1d<S>, dim3((p.nx + 2 * PLBM_GHOST + TX - 1) / TX), dim3(TX), 0,
                           st, rho, ux, th, (T *)f, p);
    }
    return launch_status();
}

template <class S>
int launch_moments(const KParams &p, const plbm_desc *d, const void *f, double *rho, double *ux,
                   double *uy, double *th, double *partials, hipStream_t st, int &nblocks,
                   int max_blocks)
{
    using T = typename S::T;
    clear_launch_error();
    if (d->dim == 2) {
        nblocks = grid_capped((long long)((p.nx + TX - 1) / TX) * p.ny, max_blocks);
        hipLaunchKernelGGL(k_moments2d<S>, dim3(nblocks), dim3(TX), 0, st, (const T *)f, p, rho,
                           ux, uy, th, partials);
    } else {
        nblocks = (p.nx + TX - 1) / TX;
        hipLaunchKernelGGL(k_moments1d<S>, dim3(nblocks), dim3(TX), 0, st, (const T *)f, p, rho, ux,
                           th, partials);
    }
    return launch_status();
}

#define PLBM_DISPATCH(d, FN, ...)                                                        \
    switch ((d)->storage + 8 * (d)->rounding) {                                          \
    case PLBM_F64: return FN<StF64>(__VA_ARGS__);                                        \
    case PLBM_F32: return FN<StF32>(__VA_ARGS__);                                        \
    case PLBM_F16DEV: return FN<StF16>(__VA_ARGS__);                                     \
    case PLBM_BF16DEV: return FN<StBF16>(__VA_ARGS__);                                   \
    case PLBM_F16DEV + 8 * PLBM_ROUND_STOCHASTIC: return FN<StF16SR>(__VA_ARGS__);       \
    case PLBM_BF16DEV + 8 * PLBM_ROUND_STOCHASTIC: return FN<StBF16SR>(__VA_ARGS__);     \
    default: return PLBM_EINVAL;                                                         \
    }

int init_dispatch(const KParams &p, const plbm_desc *d, const double *rho, const double *ux,
                  const double *uy, const double *th, void *f, hipStream_t st)
{
    PLBM_DISPATCH(d, launch_init, p, d, rho, ux, uy, th, f, st);
}

int step_dispatch(const KParams &p, const plbm_desc *d, void *fa, void *fb, int n, double *sums,
                  hipStream_t st, double *scratch = nullptr)
{
    PLBM_DISPATCH(d, run_steps, p, d, fa, fb, n, sums, st, scratch);
}

int step_fields_dispatch(const KParams &p, const plbm_desc *d, void *fa, void *fb, int n, FieldsOut fo,
                         hipStream_t st)
{
    PLBM_DISPATCH(d, run_steps_fields, p, d, fa, fb, n, fo, st);
}

int moments_dispatch(const KParams &p, const plbm_desc *d, const void *f, double *rho, double *ux,
                     double *uy, double *th, double *part, hipStream_t st, int &nb,
                     int max_blocks = MAX_GRID)
{
    PLBM_DISPATCH(d, launch_moments, p, d, f, rho, ux, uy, th, part, st, nb, max_blocks);
}

// Plain streaming copy, 16 bytes per thread: the calibration kernel for
// achievable HBM bandwidth and for the byte counters of a profiler.
typedef float CopyVec __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const CopyVec *__restrict__ a,
                                                     CopyVec *__restrict__ b, size_t n)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(a[i], b + i);
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace plbm {
void note_hip_error(const char *what, int code)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d)", what, code);
}
} // namespace plbm

extern "C" int plbm_init(const plbm_desc *d, const double *rho, const double *ux,
                         const double *uy, const double *theta, void *f, void *stream)
{
    if (d && d->dim == 3) return PLBM_EINVAL;
    if (plbm::gen_handles(d)) return plbm::gen_init(d, rho, ux, uy, theta, f, stream);
    if (d && d->q1d == 3) return plbm::q3_init(d, rho, ux, uy, f, stream);
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!rho || !ux || !theta || !f || (d->dim == 2 && !uy)) return PLBM_EINVAL;
    return init_dispatch(p, d, rho, ux, uy, theta, f, as_stream(stream));
}

extern "C" int plbm_step(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *sums,
                         void *stream)
{
    if (d && d->dim == 3) return plbm::q125_step(d, f_a, f_b, nsteps, sums, stream);
    if (plbm::gen_handles(d)) return plbm::gen_step(d, f_a, f_b, nsteps, sums, stream);
    if (d && d->q1d == 3) return plbm::q3_step(d, f_a, f_b, nsteps, sums, stream);
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

extern "C" int plbm_step_fields(const plbm_desc *d, void *f_a, void *f_b, int nsteps, double *rho, double *ux,
                                double *uy, double *theta, void *stream)
{
    if (!d) return PLBM_EINVAL;
    if (d->dim != 2 || plbm::gen_handles(d) || d->q1d != Q) return PLBM_EUNSUPPORTED;
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f_a || !f_b || f_a == f_b || nsteps < 1) return PLBM_EINVAL;
    FieldsOut fo = {{rho, ux, uy, theta}};
    return step_fields_dispatch(p, d, f_a, f_b, nsteps, fo, as_stream(stream));
}

namespace {
// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

int scratch_for_current_device(double **out)
{
    int dev = -1;
    int rc = hip_ok(hipGetDevice(&dev));
    if (rc != PLBM_OK) return rc;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return PLBM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        rc = hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (rc != PLBM_OK) return rc;
        if (!ptr) return PLBM_EHIP;
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return PLBM_OK;
}
} // namespace

extern "C" int plbm_step_noalloc(const plbm_desc *d, void *f_a, void *f_b, int nsteps,
                                 double *sums, void *stream)
{
    if (d && d->dim == 3) return PLBM_EUNSUPPORTED;
    if (plbm::gen_handles(d) || (d && d->q1d != Q)) return PLBM_EUNSUPPORTED;
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f_a || !f_b || f_a == f_b || nsteps < 0) return PLBM_EINVAL;
    // the 1D kernels run one workgroup per 256 nodes: at most NOALLOC_BLOCKS
    // of them fit the scratch when sums are asked for
    if (sums && d->dim == 1 && (p.nx + TX - 1) / TX > NOALLOC_BLOCKS) return PLBM_EINVAL;
    if (!sums) return nsteps ? step_dispatch(p, d, f_a, f_b, nsteps, nullptr, as_stream(stream))
                             : PLBM_OK;
    double *scr = nullptr;
    rc = scratch_for_current_device(&scr);
    if (rc != PLBM_OK) return rc;
    hipStream_t st = as_stream(stream);
    if (nsteps > 0) return step_dispatch(p, d, f_a, f_b, nsteps, sums, st, scr);
    int nb = 0;
    rc = moments_dispatch(p, d, f_a, nullptr, nullptr, nullptr, nullptr, scr, st, nb,
                          NOALLOC_BLOCKS);
    return rc == PLBM_OK ? finish_sums(scr, nb, sums, st) : rc;
}

extern "C" int plbm_moments(const plbm_desc *d, const void *f, double *rho, double *ux,
                            double *uy, double *theta, double *sums, void *stream)
{
    if (d && d->dim == 3) return PLBM_EINVAL;
    if (plbm::gen_handles(d)) return plbm::gen_moments(d, f, rho, ux, uy, theta, sums, stream);
    if (d && d->q1d == 3)
        return plbm::q3_moments(d, f, rho, ux, uy, theta, sums, stream);
    KParams p;
    int rc = make_params(d, p);
    if (rc != PLBM_OK) return rc;
    if (!f) return PLBM_EINVAL;
    hipStream_t st = as_stream(stream);
    int nb = 0;
    if (!sums) return moments_dispatch(p, d, f, rho, ux, uy, theta, nullptr, st, nb);
    const int nblocks = d->dim == 2 ? grid_for((long long)((p.nx + TX - 1) / TX) * p.ny)
                                    : (p.nx + TX - 1) / TX;
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
    double w[3], base[NQ];
    rest_weights(p.r64, d->theta0, w);
    for (int k = 0; k < NQ; ++k) base[k] = d->rho0 * w[vclass(k % Q)] * w[vclass(k / Q)];
    const dim3 g(grid_for((long long)((p.nx + TX - 1) / TX) * p.ny));
    const size_t nb = g.x;
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
        double cmax[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < NQ; ++k)
            for (size_t b = 0; b < nb; ++b) {
                const double m = host[b * NQ + k];
                if (!std::isfinite(m)) rc = PLBM_ENONFINITE;
                else cmax[pclass(k)] = std::fmax(cmax[pclass(k)], m);
            }
        // Floor: the FP32 collision leaves absolute rounding noise of a few
        // 2^-24 rho0 in any population, which must stay a small deviation
        // (|h| of order 10) rather than overflow it; an initial state at
        // rest (deviations of FP64 rounding, ~1e-17) would otherwise get
        // scales near 1e-20.
        const int e_floor = (int)std::floor(std::log2(d->rho0)) - 26;
        if (rc == PLBM_OK)
            for (int k = 0; k < NQ; ++k) {
                // smallest e with max deviation <= 2^e * 2^10 over the class
                const double m = cmax[pclass(k)];
                int e = m > 0.0 ? (int)std::ceil(std::log2(m)) - 10 : e_floor;
                if (m > 0.0 && std::ldexp(1.0, e + 10) < m) e += 1;
                d->scale[k] = (float)std::ldexp(1.0, std::max(e, e_floor));
            }
    }
    delete[] host;
    return rc;
}

extern "C" int plbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst || bytes == 0 || (bytes % 16) != 0) return PLBM_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return PLBM_EINVAL;
    const size_t n = bytes / 16;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return PLBM_EINVAL;
    clear_launch_error();
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                       (const CopyVec *)src, (CopyVec *)dst, n);
    return launch_status();
}

extern "C" const char *plbm_last_hip_error(void) { return g_last_error; }
