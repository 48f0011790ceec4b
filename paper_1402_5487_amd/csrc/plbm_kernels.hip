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

#include "plbm_internal.h"

namespace {

#ifndef PLBM_TILE_Y
#define PLBM_TILE_Y 1
#endif
#ifndef PLBM_MIN_WAVES
#define PLBM_MIN_WAVES 1
#endif
#ifndef PLBM_NT_STORE
#define PLBM_NT_STORE 1
#endif
#ifndef PLBM_XCD_REMAP
#define PLBM_XCD_REMAP 1
#endif
#ifndef PLBM_NV_F64
#define PLBM_NV_F64 1
#endif
#ifndef PLBM_NV_F32
#define PLBM_NV_F32 1
#endif
#ifndef PLBM_NV_16
#define PLBM_NV_16 1
#endif
// Resident-workgroup cap of the 2D step, set by reserving LDS per workgroup
// (160 KB per CU).  Fewer concurrent workgroups mean fewer DRAM rows open at
// once; on MI355X at 4096^2 two workgroups per CU (8 waves) were fastest for
// FP64 and FP32 storage and four for the 16-bit forms.
#ifndef PLBM_LDS_CAP_WIDE
#define PLBM_LDS_CAP_WIDE (80 * 1024)
#endif
#ifndef PLBM_LDS_CAP_16
#define PLBM_LDS_CAP_16 (40 * 1024)
#endif

constexpr int Q = 5;            // velocities per axis compiled into the kernels
constexpr int NQ = Q * Q;       // populations of the 2D tensor-product model
constexpr int TX = 256;         // tile width = threads per block
constexpr int TY = PLBM_TILE_Y; // tile height (rows walked by each thread)
constexpr int NXCD = 8;         // accelerator complex dies on MI355X
constexpr int RED_THREADS = 256;

// The paper's thermal velocity set is symmetric, v = (0, +a, -a, +b, -b)
// (Sec. 2.4).  For such a set the Lagrange polynomials satisfy
// L_(-v)(x) = L_v(-x) and L_0 is even, so the 5 x 5 table reduces to ten
// numbers: r_0 = mu_0 + c02 mu_2 + c04 mu_4 and
// r_(+-a) = (c12 mu_2 + c14 mu_4) +- (c11 mu_1 + c13 mu_3), likewise for +-b
// with c3j.  The host checks the structure of the table it is given.
template <typename C>
struct SymRule {
    C a, b, a2, b2;                  // velocities and their squares
    C c02, c04;                      // row of v = 0 (c00 = 1, odd terms 0)
    C c11, c12, c13, c14;            // row of v = +a
    C c31, c32, c33, c34;            // row of v = +b
    C omega;
};

// Velocity index -> symmetry class (0: v = 0, 1: +-a, 2: +-b); a 2D
// population's class is (class of i, class of j), nine in all.  The 16-bit
// forms share one base and one scale per class.
__host__ __device__ constexpr int vclass(int i) { return (i + 1) / 2; }
__host__ __device__ constexpr int pclass(int k) { return vclass(k % 5) * 3 + vclass(k / 5); }

struct KParams {
    int nx, ny;
    int tiles_x, ntiles;
    int xmargin;                    // nodes a vector window may reach past its wave
    int nv;                         // nodes per thread along x in the 2D step
    int sx[Q];                      // integer velocities (streaming shifts)
    SymRule<double> r64;
    SymRule<float> r32;
    // 16-bit deviation storage per class c: f = base + scale * h,
    // h = f * inv + nbi with inv = 1/scale, nbi = -base * inv
    float dbase[9], dscale[9], dinv[9], dnbi[9];
    long long pstride;              // elements between populations (1D: padded row)
    long long rstride;              // elements between rows (2D)
};

// ---------------------------------------------------------------------------
// Storage forms
// ---------------------------------------------------------------------------
struct StF64 {
    using T = double;
    using C = double;
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &) { return f; }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r64; }
};

struct StF32 {
    using T = float;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &) { return f; }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

// f_k = base + scale * h_k, h stored as IEEE half; scales are powers of two,
// so the encode fma(f, 1/scale, -base/scale) rounds exactly like
// (f - base)/scale, and only the half rounding (to nearest even) and the
// FP32 subtraction of the base round.
struct StF16 {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        const int c = pclass(k);
        return fmaf((float)__builtin_bit_cast(_Float16, h), p.dscale[c], p.dbase[c]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p) {
        const int c = pclass(k);
        return __builtin_bit_cast(uint16_t, (_Float16)fmaf(f, p.dinv[c], p.dnbi[c]));
    }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

struct StBF16 {
    using T = uint16_t;
    using C = float;
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        const int c = pclass(k);
        return fmaf(__uint_as_float((uint32_t)h << 16), p.dscale[c], p.dbase[c]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p) {
        const int c = pclass(k);
        return __builtin_bit_cast(uint16_t, (__bf16)fmaf(f, p.dinv[c], p.dnbi[c]));
    }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

// FP64 arithmetic on FP64 inputs (initialisation, moments, scale search).
struct Fp64Math {
    using C = double;
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r64; }
};

// ---------------------------------------------------------------------------
// Per-node arithmetic
// ---------------------------------------------------------------------------

// rho, rho u_x, rho u_y and sum f |v|^2 of 25 populations via column sums
// (same x velocity) and row sums (same y velocity); population k = i + Q j
// moves with (v_i, v_j).
template <class S>
__device__ __forceinline__ void sums2d(const typename S::C (&f)[NQ], const KParams &p,
                                       typename S::C &rho, typename S::C &jx,
                                       typename S::C &jy, typename S::C &e)
{
    using C = typename S::C;
    const SymRule<C> &R = S::R(p);
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
    rho = (col[0] + (col[1] + col[2])) + (col[3] + col[4]);
    jx = fma(R.a, col[1] - col[2], R.b * (col[3] - col[4]));
    jy = fma(R.a, row[1] - row[2], R.b * (row[3] - row[4]));
    e = fma(R.a2, (col[1] + col[2]) + (row[1] + row[2]),
            R.b2 * ((col[3] + col[4]) + (row[3] + row[4])));
}

// 1D rule of Eq. rdr for the symmetric set: Maxwell moments of (u, theta)
// by mu_(n+1) = u mu_n + n theta mu_(n-1), then r = C mu in its reduced form.
template <class S>
__device__ __forceinline__ void rule1d(typename S::C u, typename S::C theta, const KParams &p,
                                       typename S::C (&r)[Q])
{
    using C = typename S::C;
    const SymRule<C> &R = S::R(p);
    const C m1 = u;
    const C m2 = fma(u, u, theta);
    const C m3 = fma(u, m2, C(2) * theta * u);
    const C m4 = fma(u, m3, C(3) * theta * m2);
    const C e1 = fma(R.c12, m2, R.c14 * m4), o1 = fma(R.c11, m1, R.c13 * m3);
    const C e3 = fma(R.c32, m2, R.c34 * m4), o3 = fma(R.c31, m1, R.c33 * m3);
    r[0] = fma(R.c02, m2, fma(R.c04, m4, C(1)));
    r[1] = e1 + o1;
    r[2] = e1 - o1;
    r[3] = e3 + o3;
    r[4] = e3 - o3;
}

// In place: f <- (1 - omega) f + omega f_eq (Eq. srt, collision half), with
// f_eq = rho r^x_i r^y_j (tensor product, Eq. eqdist).
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
    const C w = S::R(p).omega;
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
    if (!PLBM_XCD_REMAP) return b;
    const int x = b % NXCD, local = b / NXCD;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    return x * per + min(x, rem) + local;
}

// ---------------------------------------------------------------------------
// 2D fused step
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void store_stream(T v, T *p)
{
    if constexpr (PLBM_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Loads and stores of NV consecutive nodes of one population row.  `base`
// is a wave-uniform byte pointer, `off` the lane's byte offset (the node's
// x, shifted by the population's velocity for loads).  FP32/FP64 use one
// vector access with element alignment (dword-aligned multi-dword accesses
// are native); a 16-bit pair always loads the two enclosing aligned dwords
// and byte-aligns them (shift 0 or 2 bytes), so no load sits behind a branch.
template <class T, int NV>
struct Lane {
    typedef T V __attribute__((ext_vector_type(NV), aligned(sizeof(T))));
    using Raw = V;
    // byte offset of element x - s for the load (x: first node of the lane)
    static __device__ __forceinline__ int load_off(int x, int s) { return (x - s) * (int)sizeof(T); }
    static __device__ __forceinline__ Raw load(const T *base, unsigned off, int)
    {
        return *reinterpret_cast<const V *>(&base[off / sizeof(T)]);
    }
    static __device__ __forceinline__ T get(const Raw &r, int m) { return r[m]; }
    static __device__ __forceinline__ Raw pack(const T (&e)[NV])
    {
        Raw r;
#pragma unroll
        for (int m = 0; m < NV; ++m) r[m] = e[m];
        return r;
    }
    static __device__ __forceinline__ void store(T *base, unsigned off, const T (&v)[NV])
    {
        V w;
#pragma unroll
        for (int m = 0; m < NV; ++m) w[m] = v[m];
        V *q = reinterpret_cast<V *>(&base[off / sizeof(T)]);
        if constexpr (PLBM_NT_STORE)
            __builtin_nontemporal_store(w, q);
        else
            *q = w;
    }
};

template <>
struct Lane<uint16_t, 1> {
    using Raw = uint16_t;
    static __device__ __forceinline__ int load_off(int x, int s) { return (x - s) * 2; }
    static __device__ __forceinline__ Raw load(const uint16_t *base, unsigned off, int)
    {
        return base[off / 2];
    }
    static __device__ __forceinline__ uint16_t get(const Raw &r, int) { return r; }
    static __device__ __forceinline__ Raw pack(const uint16_t (&e)[1]) { return e[0]; }
    static __device__ __forceinline__ void store(uint16_t *base, unsigned off, const uint16_t (&v)[1])
    {
        uint16_t *q = &base[off / 2];
        if constexpr (PLBM_NT_STORE) __builtin_nontemporal_store(v[0], q);
        else *q = v[0];
    }
};

template <>
struct Lane<uint16_t, 2> {
    using Raw = uint32_t;   // element x - s in the low half, x - s + 1 in the high half
    typedef uint32_t U2 __attribute__((ext_vector_type(2), aligned(4)));
    // x is even and rows start on 4-byte boundaries: the pair begins at the
    // aligned dword holding element x - s - (s & 1)
    static __device__ __forceinline__ int load_off(int x, int s) { return (x - s - (s & 1)) * 2; }
    static __device__ __forceinline__ Raw load(const uint16_t *base, unsigned off, int s)
    {
        const U2 d = *reinterpret_cast<const U2 *>(&base[off / 2]);
        return __builtin_amdgcn_alignbyte(d.y, d.x, (s & 1) * 2);
    }
    static __device__ __forceinline__ uint16_t get(const Raw &r, int m)
    {
        return (uint16_t)(m == 0 ? (r & 0xffffu) : (r >> 16));
    }
    static __device__ __forceinline__ Raw pack(const uint16_t (&e)[2])
    {
        return (uint32_t)e[0] | ((uint32_t)e[1] << 16);
    }
    static __device__ __forceinline__ void store(uint16_t *base, unsigned off, const uint16_t (&v)[2])
    {
        const uint32_t w = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        uint32_t *q = reinterpret_cast<uint32_t *>(&base[off / 2]);
        if constexpr (PLBM_NT_STORE)
            __builtin_nontemporal_store(w, q);
        else
            *q = w;
    }
};

template <class S>
__device__ __forceinline__ void accumulate_sums(const typename S::C (&f)[NQ], const KParams &p,
                                                double (&acc)[4])
{
    // invariants of what is stored (decoded again for the 16-bit forms)
    using C = typename S::C;
    C g[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) g[k] = S::dec(S::enc(f[k], k, p), k, p);
    C rho, jx, jy, e;
    sums2d<S>(g, p, rho, jx, jy, e);
    acc[0] += rho;
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += e;
}

// One fused step over a tile of (TX * NV) x TY nodes.  Layout: element
// (k, y, x) at (y * NQ + k) * nx + x, so the five populations k = i + Q j
// that share a y velocity are five consecutive rows of nx.  Per output row y
// and per j the wave computes one scalar base (source row y - v_j, wrapped);
// per i each lane keeps one 32-bit byte offset (its x, shifted by v_i, plus
// i rows) that is the same for every output row.  All 25 loads and 25
// stores are therefore (scalar base) + (vector offset).  Only waves whose
// windows cross the periodic seam in x or the ragged right edge take the
// per-node path with wrapped indices.
template <class S, int NV, bool SUMS>
__device__ __forceinline__ void step_tile(const typename S::T *__restrict__ src,
                                          typename S::T *__restrict__ dst, const KParams &p,
                                          int tile, double (&acc)[4])
{
    using T = typename S::T;
    using C = typename S::C;
    using L = Lane<T, NV>;
    const int tyi = tile / p.tiles_x, txi = tile - tyi * p.tiles_x;
    const int xb = txi * (TX * NV) + threadIdx.x * NV;
    const int y0 = tyi * TY;
    const int nx = p.nx, ny = p.ny;
    const long long rowelems = (long long)NQ * nx;
    // first node of this wave; its windows span [wx - xmargin, wx + 64 NV + xmargin)
    const int wx = __builtin_amdgcn_readfirstlane(xb);
    const bool fast = wx >= p.xmargin && wx + 64 * NV + p.xmargin <= nx;
    const int rows = min(TY, ny - y0);

    // lane byte offsets, row-invariant: loads of population column i
    // (shifted by v_i), and stores.  Kept as 32-bit byte counts and indexed
    // as (offset / sizeof(T)) so that every access is a scalar base plus a
    // 32-bit vector offset.
    unsigned lo[Q], so[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        lo[i] = (unsigned)(L::load_off(xb, p.sx[i]) + i * nx * (int)sizeof(T));
        so[i] = (unsigned)((xb + i * nx) * (int)sizeof(T));
        asm volatile("" : "+v"(lo[i]), "+v"(so[i]));
    }

#pragma unroll 1
    for (int r = 0; r < rows; ++r) {
        const int y = y0 + r;
        typename L::Raw raw[NQ];
        if (fast) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                int ys = y - p.sx[j];
                ys += (ys < 0) ? ny : 0;
                ys -= (ys >= ny) ? ny : 0;
                const T *base = src + (ys * rowelems + (long long)(Q * j) * nx);
#pragma unroll
                for (int i = 0; i < Q; ++i) raw[i + Q * j] = L::load(base, lo[i], p.sx[i]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                int ys = y - p.sx[j];
                ys += (ys < 0) ? ny : 0;
                ys -= (ys >= ny) ? ny : 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const T *row = src + ((long long)ys * NQ + i + Q * j) * nx;
                    T e[NV];
#pragma unroll
                    for (int m = 0; m < NV; ++m) {
                        int xs = xb + m - p.sx[i];
                        xs += (xs < 0) ? nx : 0;
                        xs -= (xs >= nx) ? nx : 0;
                        xs = min(xs, nx - 1);      // lanes past the ragged edge
                        e[m] = row[xs];
                    }
                    raw[i + Q * j] = L::pack(e);
                }
            }
        }
        T out[NQ][NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            C f[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) f[k] = S::dec(L::get(raw[k], m), k, p);
            collide2d<S>(f, p);
#pragma unroll
            for (int k = 0; k < NQ; ++k) out[k][m] = S::enc(f[k], k, p);
            if constexpr (SUMS) {
                if (fast || xb + m < nx) accumulate_sums<S>(f, p, acc);
            }
        }
        if (fast) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                T *base = dst + (y * rowelems + (long long)(Q * j) * nx);
#pragma unroll
                for (int i = 0; i < Q; ++i) L::store(base, so[i], out[i + Q * j]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                T *row = dst + ((long long)y * NQ + k) * nx;
#pragma unroll
                for (int m = 0; m < NV; ++m)
                    if (xb + m < nx) store_stream(out[k][m], row + (xb + m));
            }
        }
    }
}

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
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= p.nx) return;
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
            dst[k * p.pstride + (long long)yd * p.rstride + xd] = S::enc((typename S::C)feq[k], k, p);
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
            const auto h = S::enc(f[k], k, p);
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
                const double g = (double)S::dec(S::enc(f[k], k, p), k, p);
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
        dst[k * p.pstride + q] = S::enc((typename S::C)(rho[s] * r[k]), k, p);
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

// Reduced table of a symmetric velocity set v = (0, a, -a, b, -b), or
// PLBM_EUNSUPPORTED when the set or its table lacks that structure.
int sym_rule(const plbm_desc *d, SymRule<double> &R)
{
    const double *v = d->v, *c = d->c;
    if (v[0] != 0.0 || v[2] != -v[1] || v[4] != -v[3]) return PLBM_EUNSUPPORTED;
    double big = 0.0;
    for (int i = 0; i < NQ; ++i) big = std::fmax(big, std::fabs(c[i]));
    const double tol = 1e-12 * std::fmax(1.0, big);
    auto C = [&](int i, int j) { return c[i * Q + j]; };
    bool ok = std::fabs(C(0, 0) - 1.0) <= tol && std::fabs(C(0, 1)) <= tol &&
              std::fabs(C(0, 3)) <= tol && std::fabs(C(1, 0)) <= tol && std::fabs(C(3, 0)) <= tol;
    for (int j = 0; j < Q && ok; ++j) {
        const double sg = (j & 1) ? -1.0 : 1.0;
        ok = std::fabs(C(2, j) - sg * C(1, j)) <= tol && std::fabs(C(4, j) - sg * C(3, j)) <= tol;
    }
    if (!ok) return PLBM_EUNSUPPORTED;
    R.a = v[1];
    R.b = v[3];
    R.a2 = v[1] * v[1];
    R.b2 = v[3] * v[3];
    R.c02 = C(0, 2);
    R.c04 = C(0, 4);
    R.c11 = C(1, 1);
    R.c12 = C(1, 2);
    R.c13 = C(1, 3);
    R.c14 = C(1, 4);
    R.c31 = C(3, 1);
    R.c32 = C(3, 2);
    R.c33 = C(3, 3);
    R.c34 = C(3, 4);
    R.omega = d->omega;
    return PLBM_OK;
}

// Rest-state weights r_i(u = 0, theta0) per velocity class, from the reduced
// table: mu = (1, 0, theta0, 0, 3 theta0^2).
void rest_weights(const SymRule<double> &R, double theta0, double (&w)[3])
{
    const double m2 = theta0, m4 = 3.0 * theta0 * theta0;
    w[0] = 1.0 + R.c02 * m2 + R.c04 * m4;
    w[1] = R.c12 * m2 + R.c14 * m4;
    w[2] = R.c32 * m2 + R.c34 * m4;
}

// Tile grid for NV nodes per thread and the margin that decides which waves
// may use the unwrapped vector loads.
void set_tiling(KParams &p, int nv, int maxs)
{
    p.nv = nv;
    const int txn = TX * nv;
    p.tiles_x = (p.nx + txn - 1) / txn;
    const int tiles_y = (p.ny + TY - 1) / TY;
    p.ntiles = p.tiles_x * tiles_y;
    // a wave starting at wx reads elements wx - maxs - 1 .. wx + 64 nv + maxs
    // (the extra element: paired 16-bit loads of odd shifts)
    p.xmargin = maxs + 1;
}

int make_params(const plbm_desc *d, KParams &p)
{
    int rc = plbm::validate(d);
    if (rc != PLBM_OK) return rc;
    if (d->q1d != Q) return PLBM_EUNSUPPORTED;
    if (d->dim == 1 && d->storage >= PLBM_F16DEV) return PLBM_EUNSUPPORTED;
    std::memset(&p, 0, sizeof(p));
    rc = sym_rule(d, p.r64);
    if (rc != PLBM_OK) return rc;
    const SymRule<double> &R = p.r64;
    p.r32 = SymRule<float>{(float)R.a,   (float)R.b,   (float)R.a2,  (float)R.b2,  (float)R.c02,
                           (float)R.c04, (float)R.c11, (float)R.c12, (float)R.c13, (float)R.c14,
                           (float)R.c31, (float)R.c32, (float)R.c33, (float)R.c34, (float)R.omega};
    p.nx = d->nx;
    p.ny = d->ny;
    int maxs = 0;
    for (int i = 0; i < Q; ++i) {
        p.sx[i] = (int)d->v[i];
        maxs = std::max(maxs, std::abs(p.sx[i]));
    }
    if (d->dim == 1) {
        p.pstride = d->nx + 2 * PLBM_GHOST;
        p.nv = 1;
    } else {
        // row-interleaved layout: row y holds the 25 population rows of nx
        p.pstride = d->nx;
        p.rstride = (long long)NQ * d->nx;
        int nv = d->storage == PLBM_F64 ? PLBM_NV_F64
                                        : (d->storage == PLBM_F32 ? PLBM_NV_F32 : PLBM_NV_16);
        if (d->nx & 1) nv = 1;        // paired nodes need rows that start on even elements
        set_tiling(p, nv, maxs);
    }
    if (d->storage >= PLBM_F16DEV) {
        double w[3];
        rest_weights(R, d->theta0, w);
        for (int c = 0; c < 9; ++c) {
            p.dbase[c] = (float)(d->rho0 * w[c / 3] * w[c % 3]);
            p.dscale[c] = 0.0f;
        }
        for (int k = 0; k < NQ; ++k) {
            const int c = pclass(k);
            if (p.dscale[c] == 0.0f) p.dscale[c] = d->scale[k];
            else if (p.dscale[c] != d->scale[k]) return PLBM_EINVAL;   // one scale per class
        }
        for (int c = 0; c < 9; ++c) {
            int e = 0;
            if (std::frexp(p.dscale[c], &e) != 0.5f) return PLBM_EINVAL;   // powers of two only
            p.dinv[c] = 1.0f / p.dscale[c];
            p.dnbi[c] = -p.dbase[c] * p.dinv[c];
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
        const size_t lds = sizeof(T) == 2 ? PLBM_LDS_CAP_16 : PLBM_LDS_CAP_WIDE;
        if (p.nv == 2)
            hipLaunchKernelGGL((k_step2d<S, 2, SUMS>), dim3(p.ntiles), dim3(TX), lds, st,
                               (const T *)src, (T *)dst, p, partials);
        else
            hipLaunchKernelGGL((k_step2d<S, 1, SUMS>), dim3(p.ntiles), dim3(TX), lds, st,
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
    double w[3], base[NQ];
    rest_weights(p.r64, d->theta0, w);
    for (int k = 0; k < NQ; ++k) base[k] = d->rho0 * w[vclass(k % Q)] * w[vclass(k / Q)];
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
        double cmax[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < NQ; ++k)
            for (size_t b = 0; b < nb; ++b) {
                const double m = host[b * NQ + k];
                if (!std::isfinite(m)) rc = PLBM_ENONFINITE;
                else cmax[pclass(k)] = std::fmax(cmax[pclass(k)], m);
            }
        if (rc == PLBM_OK)
            for (int k = 0; k < NQ; ++k) {
                // smallest e with max deviation <= 2^e * 2^10 over the class
                const double m = cmax[pclass(k)];
                int e = m > 0.0 ? (int)std::ceil(std::log2(m)) - 10 : -30;
                if (m > 0.0 && std::ldexp(1.0, e + 10) < m) e += 1;
                d->scale[k] = (float)std::ldexp(1.0, e);
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
