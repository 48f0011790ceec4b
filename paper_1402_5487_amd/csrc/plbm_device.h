// Device building blocks of libplbm shared by the single-lattice and the
// batched kernels: launch constants, the reduced equilibrium rule, storage
// forms, per-node arithmetic, reductions, tile mapping and the row stepper.
// Internal header (not part of the C ABI); every includer gets its own copy
// in an anonymous namespace.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "plbm_internal.h"

namespace {


#ifndef PLBM_TILE_Y
#define PLBM_TILE_Y 1
#endif
#ifndef PLBM_MIN_WAVES
#define PLBM_MIN_WAVES 1
#endif
// Non-temporal loads for 4- and 8-byte populations in the paired-node
// paths (each is read once).  The one-node-per-lane 2D step chooses per
// velocity column instead (PLBM_NT_WIDE_MASK, PLBM_NT16_MASK).
#ifndef PLBM_NT_LOAD
#define PLBM_NT_LOAD 1
#endif
#ifndef PLBM_NT_STORE
#define PLBM_NT_STORE 1
#endif
// 16-bit forms: non-temporal loads for the population columns in this mask
// (bit i: velocity v_i).  Column 0 (v = 0) reads exactly the wave's own
// nodes; the shifted columns' edge lines are also read by the neighbouring
// wave and are better kept in L2.  Measured at 4096^2: column 0 alone
// 1.5-2 % faster (3-4 % with stochastic rounding), all columns 1-2 % slower.
// 4- and 8-byte forms, one node per lane: the same per-column mask.
// Column 0 alone beats all columns non-temporal by 2.6 % (FP32) and 1.4 %
// (FP64) at 4096^2, and by 4 % in the batch of small lattices, whose
// windows share more edge lines; no non-temporal column is slower still.
#ifndef PLBM_NT_WIDE_MASK
#define PLBM_NT_WIDE_MASK 1
#endif
#ifndef PLBM_NT16_MASK
#define PLBM_NT16_MASK 1
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
// FP64 and FP32 storage and five for the 16-bit forms (0.6-1.1 % faster than
// four; three are 25 % slower).  Stochastic rounding adds ALU work per
// population and also wants five (5.5 % faster than four).
#ifndef PLBM_LDS_CAP_WIDE
#define PLBM_LDS_CAP_WIDE (80 * 1024)
#endif
#ifndef PLBM_LDS_CAP_16
#define PLBM_LDS_CAP_16 (32 * 1024)
#endif
#ifndef PLBM_LDS_CAP_16SR
#define PLBM_LDS_CAP_16SR (27 * 1024)
#endif

constexpr int Q = 5;            // velocities per axis compiled into the kernels
constexpr int NQ = Q * Q;       // populations of the 2D tensor-product model
#ifndef PLBM_TX
#define PLBM_TX 256
#endif
constexpr int TX = PLBM_TX;     // tile width = threads per block
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
    // per-node key of the stochastic rounding (unused by the other forms)
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return node; }
    static constexpr bool row_prio_pair = false;   // see StF16
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &, uint32_t = 0) { return f; }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r64; }
};

struct StF32 {
    using T = float;
    using C = float;
    // per-node key of the stochastic rounding (unused by the other forms)
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return node; }
    static constexpr bool row_prio_pair = false;   // see StF16
    static __device__ __forceinline__ C dec(T h, int, const KParams &) { return h; }
    static __device__ __forceinline__ T enc(C f, int, const KParams &, uint32_t = 0) { return f; }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

// f_k = base + scale * h_k, h stored as IEEE half; scales are powers of two,
// so the encode fma(f, 1/scale, -base/scale) rounds exactly like
// (f - base)/scale, and only the half rounding (to nearest even) and the
// FP32 subtraction of the base round.
struct StF16 {
    using T = uint16_t;
    using C = float;
    // per-node key of the stochastic rounding (unused by the other forms)
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return node; }
    // an s_setprio 1 / 0 pair at the head of each row (see step_rows)
    static constexpr bool row_prio_pair = true;
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        const int c = pclass(k);
        return fmaf((float)__builtin_bit_cast(_Float16, h), p.dscale[c], p.dbase[c]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p, uint32_t = 0) {
        const int c = pclass(k);
        return __builtin_bit_cast(uint16_t, (_Float16)fmaf(f, p.dinv[c], p.dnbi[c]));
    }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

struct StBF16 {
    using T = uint16_t;
    using C = float;
    // per-node key of the stochastic rounding (unused by the other forms)
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return node; }
    static constexpr bool row_prio_pair = true;    // see StF16
    static __device__ __forceinline__ C dec(T h, int k, const KParams &p) {
        const int c = pclass(k);
        return fmaf(__uint_as_float((uint32_t)h << 16), p.dscale[c], p.dbase[c]);
    }
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p, uint32_t = 0) {
        const int c = pclass(k);
        return __builtin_bit_cast(uint16_t, (__bf16)fmaf(f, p.dinv[c], p.dnbi[c]));
    }
    static __device__ __forceinline__ const SymRule<C> &R(const KParams &p) { return p.r32; }
};

// Stochastic rounding of the stored deviation: h = (f - base) / scale (exact
// in FP32, as above) goes to one of its two neighbours in the 16-bit format
// with probability proportional to its distance from the other, so the
// stored value is unbiased.  Round to nearest loses every per-step change
// smaller than half an ulp of the deviation (2^-11 of it in FP16, 2^-8 in
// BF16): a slowly decaying wave then decays at the wrong rate or not at all.
// The random bits depend on the node, the population and the value's own
// bits, so results are deterministic and independent of how the steps are
// split into calls.
//  - per node, once: a 32-bit key from the node index (two multiply-xorshift
//    rounds, the finaliser of MurmurHash3);
//  - per population: the low 24 bits of the value's bits xor the key, times
//    a 24-bit odd constant of its own population (one full-rate 24 x 24
//    multiply, low 32 bits kept); bits 16-31 of that product depend on all
//    24 input bits and serve as the random bits.  An odd multiplier maps
//    distinct 24-bit inputs to distinct products, so for a fixed value and
//    keys spread over the nodes the random bits spread evenly and the
//    rounding is unbiased to within sampling noise (measured: over 2^18
//    nodes the share rounded up matches the distance to the lower neighbour
//    within six standard errors on every plane).  (The high half of the
//    48-bit product would not do: it only spans [0, multiplier / 2^8).)
__device__ __forceinline__ uint32_t sr_node_key(uint32_t node)
{
    uint32_t h = node * 0x9E3779B1u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    return h;
}

// The key as one register: left to itself the compiler keeps the last
// xorshift's two operands apart and pays a second xor per population.
__device__ __forceinline__ uint32_t sr_key_reg(uint32_t h)
{
    asm volatile("" : "+v"(h));
    return h;
}

__device__ __forceinline__ uint32_t sr_word(uint32_t key, int k, uint32_t vbits)
{
    // odd 24-bit multipliers, one per population (k < 25)
    const uint32_t mult = 0x9E3779u + 0x2A62D6u * (uint32_t)k | 1u;
    return (uint32_t)__umul24(vbits ^ key, mult & 0xffffffu);
}

// gfx950 converts FP32 to FP16 or BF16 with stochastic rounding in one
// instruction (v_cvt_sr_f16_f32, v_cvt_sr_bf16_f32) that takes a 32-bit
// random word; a probe of both over normal, subnormal, overflowing, infinite
// and NaN inputs and 20 random words matched the following description.
//  - BF16: the word's top 16 bits are added below BF16's kept bits of the
//    FP32 pattern and the sum truncated; infinities and NaNs are unchanged.
//    The value rounds up with probability frac(h / ulp).
//  - FP16, normal range: the word's top 13 bits are added below FP16's 11
//    kept bits, the sum truncated and converted (exact there).  Past the top
//    of the range the sum reaches 65536 and becomes infinity of h's sign, with
//    the probability that keeps the rounding unbiased, so the sums still
//    report the overflow.  Below the normal range (|h| < 2^-14, a deviation
//    under 2^-24 of the class's largest) the random bits are aligned to the
//    subnormal step, so those values are rounded stochastically too.  NaNs
//    stay NaN.
typedef _Float16 plbm_f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 plbm_bf16x2 __attribute__((ext_vector_type(2)));

struct StF16SR : StF16 {
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return sr_key_reg(sr_node_key(node)); }
    static constexpr bool row_prio_pair = false;
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p, uint32_t key) {
        const int c = pclass(k);
        const float v = fmaf(f, p.dinv[c], p.dnbi[c]);
        const uint32_t vb = __float_as_uint(v);
        // the upper half of the destination is kept from the first operand:
        // v's own register, which is dead after this, so no zeroing move
        const plbm_f16x2 r =
            __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(plbm_f16x2, vb), v, sr_word(key, k, vb), false);
        return __builtin_bit_cast(uint16_t, r[0]);
    }
};

struct StBF16SR : StBF16 {
    static __device__ __forceinline__ uint32_t key(uint32_t node) { return sr_key_reg(sr_node_key(node)); }
    static constexpr bool row_prio_pair = false;
    static __device__ __forceinline__ T enc(C f, int k, const KParams &p, uint32_t key) {
        const int c = pclass(k);
        const float v = fmaf(f, p.dinv[c], p.dnbi[c]);
        const uint32_t vb = __float_as_uint(v);
        const plbm_bf16x2 r =
            __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(plbm_bf16x2, vb), v, sr_word(key, k, vb), false);
        return __builtin_bit_cast(uint16_t, r[0]);
    }
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
template <typename C>
__device__ __forceinline__ void rule_sym(C u, C theta, const SymRule<C> &R, C (&r)[Q])
{
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

template <class S>
__device__ __forceinline__ void rule1d(typename S::C u, typename S::C theta, const KParams &p,
                                       typename S::C (&r)[Q])
{
    rule_sym<typename S::C>(u, theta, S::R(p), r);
}

// 1 / rho: correctly rounded in FP64; in FP32 the hardware reciprocal
// (within 1 ulp), one instruction instead of a ten-instruction division, in
// a step whose FP32 arithmetic already rounds each moment by several ulps.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// In place: f <- (1 - omega) f + omega f_eq (Eq. srt, collision half), with
// f_eq = rho r^x_i r^y_j (tensor product, Eq. eqdist).  mom receives the
// node's (rho, u_x, u_y, theta) before the collision.
template <class S>
__device__ __forceinline__ void collide2d(typename S::C (&f)[NQ], const KParams &p, typename S::C (&mom)[4])
{
    using C = typename S::C;
    C rho, jx, jy, e;
    sums2d<S>(f, p, rho, jx, jy, e);
    const C inv = recip(rho);
    const C ux = jx * inv, uy = jy * inv;
    const C theta = C(0.5) * (e * inv - ux * ux - uy * uy);
    mom[0] = rho;
    mom[1] = ux;
    mom[2] = uy;
    mom[3] = theta;
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

template <class S>
__device__ __forceinline__ void collide2d(typename S::C (&f)[NQ], const KParams &p)
{
    typename S::C mom[4];
    collide2d<S>(f, p, mom);
}

// Optional per-node outputs of a step: (rho, u_x, u_y, theta) planes of the
// state it reads, row-major (ny, nx); a NULL plane is not written.
struct FieldsOut {
    double *p[4];
};

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
// Launch grids
// ---------------------------------------------------------------------------
// A dispatch counts its work-items in 32 bits and gridDim.y is at most 65536,
// so every lattice kernel runs a one-dimensional grid of at most MAX_GRID
// workgroups that walks its row segments, tile = y * tiles_x + tx.
constexpr int MAX_GRID = 1 << 22;
inline int grid_for(long long tiles) { return (int)std::min<long long>(tiles, MAX_GRID); }

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
        const V *q = reinterpret_cast<const V *>(&base[off / sizeof(T)]);
        if constexpr (PLBM_NT_LOAD && sizeof(T) >= 4) return __builtin_nontemporal_load(q);
        else return *q;
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
                                                double (&acc)[4], uint32_t salt)
{
    // invariants of what is stored (decoded again for the 16-bit forms)
    using C = typename S::C;
    C g[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) g[k] = S::dec(S::enc(f[k], k, p, salt), k, p);
    C rho, jx, jy, e;
    sums2d<S>(g, p, rho, jx, jy, e);
    acc[0] += rho;
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += e;
}

// Fused step of `nrows` rows y_first + r * y_step for the lane's node(s)
// starting at x = xb.  Layout: element (k, y, x) at (y * NQ + k) * nx + x,
// so the five populations k = i + Q j that share a y velocity are five
// consecutive rows of nx.  Per output row y and per j the wave computes one
// scalar base (source row y - v_j, wrapped); per i each lane keeps one
// 32-bit byte offset (its source column plus i rows) that is the same for
// every output row.  All 25 loads and 25 stores are therefore (scalar base)
// + (vector offset).  With paired nodes (NV = 2) the waves whose windows
// cross the periodic seam in x or the ragged right edge take a per-node path
// with wrapped indices instead.
template <class S, int NV, bool SUMS, bool FIELDS = false>
__device__ __forceinline__ void step_rows(const typename S::T *__restrict__ src,
                                          typename S::T *__restrict__ dst, const KParams &p,
                                          int xb, int y_first, int y_step, int nrows,
                                          double (&acc)[4], const FieldsOut &fo = FieldsOut{})
{
    using T = typename S::T;
    using C = typename S::C;
    using L = Lane<T, NV>;
    const int nx = p.nx, ny = p.ny;
    const long long rowelems = (long long)NQ * nx;
    // first node of this wave; its windows span [wx - xmargin, wx + 64 NV + xmargin)
    const int wx = __builtin_amdgcn_readfirstlane(xb);
    const bool fast = wx >= p.xmargin && wx + 64 * NV + p.xmargin <= nx;

    // lane byte offsets, row-invariant: loads of population column i
    // (shifted by v_i), and stores.  Kept as 32-bit byte counts and indexed
    // as (offset / sizeof(T)) so that every access is a scalar base plus a
    // 32-bit vector offset.
    // With one node per lane the periodic wrap in x is folded into these
    // offsets (the source column of lane x is (x - v_i) mod nx), so every
    // wave takes the vector path and only waves past the ragged right edge
    // mask their stores.
    unsigned lo[Q], so[Q];
    // unsigned arithmetic: with nx up to 2^26 the FP64 offsets pass 2^31
    const unsigned x0 = (unsigned)xb * (unsigned)sizeof(T);
    if (NV == 1 && fast) {
        // interior waves (all but the two at the seam): no lane wraps, so
        // each offset is the lane's own plus a wave-uniform constant
#pragma unroll
        for (int i = 0; i < Q; ++i)
            lo[i] = x0 + (unsigned)(i * nx - p.sx[i]) * (unsigned)sizeof(T);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xs;
            if constexpr (NV == 1) {
                xs = min(xb, nx - 1) - p.sx[i];
                xs += (xs < 0) ? nx : 0;
                xs -= (xs >= nx) ? nx : 0;
                xs *= (int)sizeof(T);
            } else {
                xs = L::load_off(xb, p.sx[i]);
            }
            lo[i] = (unsigned)xs + (unsigned)i * (unsigned)nx * (unsigned)sizeof(T);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        so[i] = x0 + (unsigned)i * (unsigned)nx * (unsigned)sizeof(T);
        asm volatile("" : "+v"(lo[i]), "+v"(so[i]));
    }
    const bool full = NV == 1 ? (wx + 64 <= nx) : fast;

#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
        const int y = y_first + r * y_step;
        if (y >= ny) break;
        typename L::Raw raw[NQ];
        // The round-to-nearest 16-bit forms put an s_setprio 1 / s_setprio 0
        // pair around the loads.  The compiler sinks the loads (and the whole
        // row) into the branch that stores it, past lanes beyond a ragged
        // edge, so both land ahead of that branch and the wave's priority is
        // not raised while the loads issue.  The pair stays for the code it
        // leaves: it bounds the scalar code motion at the row head, and the
        // 4096^2 step built with it ran 0.5 % faster (0.759 against 0.755 of
        // 8 TB/s in paired runs).  Skipping the edge lanes first, so that the
        // pair does bracket the loads, ran at 0.747-0.750; the other forms
        // ran no faster with the pair either way.
        if constexpr (S::row_prio_pair) __builtin_amdgcn_s_setprio(1);
        if (NV == 1 || fast) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                int ys = y - p.sx[j];
                ys += (ys < 0) ? ny : 0;
                ys -= (ys >= ny) ? ny : 0;
                const T *base = src + (ys * rowelems + (long long)(Q * j) * nx);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if constexpr (NV == 1) {
                        // non-temporal for the columns in the mask, ordinary otherwise
                        constexpr unsigned mask = sizeof(T) == 2 ? PLBM_NT16_MASK : PLBM_NT_WIDE_MASK;
                        const auto *q = reinterpret_cast<const typename L::Raw *>(&base[lo[i] / sizeof(T)]);
                        if ((mask >> i) & 1) {
                            raw[i + Q * j] = __builtin_nontemporal_load(q);
                            continue;
                        }
                        raw[i + Q * j] = *q;
                    } else {
                        raw[i + Q * j] = L::load(base, lo[i], p.sx[i]);
                    }
                }
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
        if constexpr (S::row_prio_pair) __builtin_amdgcn_s_setprio(0);
        T out[NQ][NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            C f[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) f[k] = S::dec(L::get(raw[k], m), k, p);
            if constexpr (FIELDS) {
                C mom[4];
                collide2d<S>(f, p, mom);
                if (full || xb + m < nx) {
                    const long long n = (long long)y * nx + (xb + m);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (fo.p[q]) fo.p[q][n] = (double)mom[q];
                }
            } else {
                collide2d<S>(f, p);
            }
            const uint32_t salt = S::key((uint32_t)y * (uint32_t)nx + (uint32_t)(xb + m));   // the node
#pragma unroll
            for (int k = 0; k < NQ; ++k) out[k][m] = S::enc(f[k], k, p, salt);
            if constexpr (SUMS) {
                if (full || xb + m < nx) accumulate_sums<S>(f, p, acc, salt);
            }
        }
        if (full) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                T *base = dst + (y * rowelems + (long long)(Q * j) * nx);
#pragma unroll
                for (int i = 0; i < Q; ++i) L::store(base, so[i], out[i + Q * j]);
            }
        } else if (NV == 1) {
            if (xb < nx) {
#pragma unroll
                for (int j = 0; j < Q; ++j) {
                    T *base = dst + (y * rowelems + (long long)(Q * j) * nx);
#pragma unroll
                    for (int i = 0; i < Q; ++i) L::store(base, so[i], out[i + Q * j]);
                }
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

// One tile of the single-lattice launch: TX * NV nodes of each of TY rows.
template <class S, int NV, bool SUMS, bool FIELDS = false>
__device__ __forceinline__ void step_tile(const typename S::T *__restrict__ src,
                                          typename S::T *__restrict__ dst, const KParams &p,
                                          int tile, double (&acc)[4], const FieldsOut &fo = FieldsOut{})
{
    const int tyi = tile / p.tiles_x, txi = tile - tyi * p.tiles_x;
    const int xb = txi * (TX * NV) + threadIdx.x * NV;
    step_rows<S, NV, SUMS, FIELDS>(src, dst, p, xb, tyi * TY, 1, TY, acc, fo);
}

// ---------------------------------------------------------------------------
// Host-side parameter setup
// ---------------------------------------------------------------------------
// Reduced table of a symmetric velocity set v = (0, a, -a, b, -b), or
// PLBM_EUNSUPPORTED when the set or its table lacks that structure.
inline int sym_rule(const plbm_desc *d, SymRule<double> &R)
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
inline void rest_weights(const SymRule<double> &R, double theta0, double (&w)[3])
{
    const double m2 = theta0, m4 = 3.0 * theta0 * theta0;
    w[0] = 1.0 + R.c02 * m2 + R.c04 * m4;
    w[1] = R.c12 * m2 + R.c14 * m4;
    w[2] = R.c32 * m2 + R.c34 * m4;
}

// Tile grid for NV nodes per thread and the margin that decides which waves
// may use the unwrapped vector loads.
inline void set_tiling(KParams &p, int nv, int maxs)
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

inline int make_params(const plbm_desc *d, KParams &p)
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

} // namespace
