// libplbm learned closure: a 3-layer 3x3 convolutional network (25 -> 32 ->
// 32 -> 25 channels, ReLU between layers, periodic padding) that maps a coarse
// lattice's normalised post-collision populations to a correction of them,
// with hand-written BF16 MFMA kernels for inference and training.
//
//  * Activations are NHWC bf16 with the channel count padded to 32: one node
//    is 64 contiguous bytes.  Weights (FP32 master copy owned by the caller)
//    are cast to two bf16 copies, [tap][out][in] for the forward pass and
//    [tap][in][out] for the input gradient.
//  * Convolution = implicit GEMM on v_mfma_f32_32x32x16_bf16: one wave
//    computes 32 nodes of a row x 32 channels; K = 9 taps x 32 channels is
//    18 MFMAs, each fed by one 16-byte load per lane of the (shifted) input
//    node and one of the weights.  The input gradient is the same kernel with
//    the taps mirrored and the transposed weights; the ReLU derivative is
//    applied in its epilogue.
//  * Weight gradient: a workgroup stages, row by row, the dZ row and the
//    three input rows it needs in LDS node-major and reads MFMA operands
//    with transposing LDS reads; each wave accumulates 32 x 32 x (64 nodes)
//    MFMA products for its taps; block partials are summed in a fixed order
//    (deterministic).
//  * Projection, loss and apply are per-node kernels: the projection removes
//    the correction's mass, momentum and energy (the invariants of the
//    collision), orthogonally in the metric of the output scales, so an
//    applied correction conserves them exactly.  The loss streams the
//    correction (pull form) and compares the conserved densities it adds
//    with a target increment error; its gradient is the adjoint (push) of
//    the same streaming followed by the projection.  Apply hands those
//    moments to the next step as a shift of the equilibrium, so the corrected
//    node keeps the plain step's non-equilibrium part.
//  * Training through corrected coarse steps: FP64 adjoints (vector-Jacobian
//    products) of the fused step, the apply and the rollout loss, as
//    separate calls and fused into two node passes per corrected step.
//  * The coarse lattice may hold FP32 or FP64 populations; the network reads
//    and corrects either.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "plbm_device.h"
#include "plbm_internal.h"

struct plbm_closure;

namespace {

constexpr int CH = 32;          // padded channels
constexpr int CREAL = 25;       // populations
constexpr int TAPS = 9;
constexpr int LAYER_W = TAPS * CH * CH;
constexpr int LAYER_P = LAYER_W + CH;          // weights + bias, per layer
constexpr int NPARAM = 3 * LAYER_P;
#ifndef PLBM_WG_ROWS
#define PLBM_WG_ROWS 16
#endif
#ifndef PLBM_CONV_BLOCKS
#define PLBM_CONV_BLOCKS 256       // target block count of the convolution launches
#endif
#ifndef PLBM_CONV_MAX_ROWS
#define PLBM_CONV_MAX_ROWS 16      // most output rows per convolution block
#endif
#ifndef PLBM_CONV_WAVES
#define PLBM_CONV_WAVES 2          // waves per SIMD the convolution's registers must allow
#endif
#ifndef PLBM_CONV_BROWS_DIV
#define PLBM_CONV_BROWS_DIV 2      // input-gradient blocks take rows / this
#endif
constexpr int WG_ROWS = PLBM_WG_ROWS;          // rows per weight-gradient block
constexpr int WG_SEG = 64;                     // nodes per weight-gradient row segment

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16;

// Up to MAX_FRAMES buffer pointers, passed by value in the kernel arguments
// (no host-to-device copy of pointer tables).
constexpr int MAX_FRAMES = 64;
struct PtrList {
    void *p[MAX_FRAMES];
};

// Normalisation and projection.  With D = diag(s) (output scales) and
// Phi = (1, vx, vy, |v|^2), B = D Phi and G = B^T B, the projection in
// normalised coordinates is Ph = I - B G^-1 B^T: symmetric, idempotent, and
// the physical correction D Ph y has zero mass, momentum and energy.  It is
// the orthogonal projection in the metric sum_k (x_k / s_k)^2, so each
// population absorbs a share proportional to its own scale.
struct ClNorm {
    float in_mean[CREAL], in_inv[CREAL];    // x = (P - mean) * inv
    float out_scale[CREAL];                 // s_k
    float ginv[16];                         // G^-1
    float vx[CREAL], vy[CREAL];
    int ivx[CREAL], ivy[CREAL];             // the same velocities as node offsets
    float mw2[4];                           // loss weights 1 / sigma_m^2
};

__device__ __forceinline__ u16 bf16_bits(float f) { return __builtin_bit_cast(u16, (__bf16)f); }
__device__ __forceinline__ float bf16_val(u16 h) { return __uint_as_float((uint32_t)h << 16); }

// v <- Ph v = v - B G^-1 B^T v (normalised coordinates), in place
__device__ __forceinline__ void project(float (&v)[CREAL], const ClNorm &nm)
{
    float m[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        const float vx = nm.vx[k], vy = nm.vy[k], sv = nm.out_scale[k] * v[k];
        m[0] += sv;
        m[1] += vx * sv;
        m[2] += vy * sv;
        m[3] += (vx * vx + vy * vy) * sv;
    }
    float a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a[i] = nm.ginv[4 * i] * m[0] + nm.ginv[4 * i + 1] * m[1] + nm.ginv[4 * i + 2] * m[2] +
               nm.ginv[4 * i + 3] * m[3];
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        const float vx = nm.vx[k], vy = nm.vy[k];
        v[k] -= nm.out_scale[k] * (a[0] + a[1] * vx + a[2] * vy + a[3] * (vx * vx + vy * vy));
    }
}

// ---------------------------------------------------------------------------
// population buffer (row layout (y*25 + k)*nx + x, FP32 or FP64) -> normalised
// NHWC bf16; the difference from the mean is taken in the buffer's precision.
// A block takes 256 nodes of a row: thread t reads node t of each plane
// (coalesced), packs channel pairs into LDS rows of 17 words (a stride
// coprime with the 64 banks), and the block then stores the 256 x 64 bytes
// as consecutive 16-byte chunks, one per lane.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_cl_input(PtrList post, int nx, int ny, ClNorm nm,
                                                  const float *__restrict__ noise, float amp,
                                                  u16 *__restrict__ x0)
{
    __shared__ uint32_t tile[256][17];
    const int f = blockIdx.z;
    const int y = blockIdx.y;
    const int xb = blockIdx.x * 256;
    const int x = xb + threadIdx.x;
    if (x < nx) {
        const T *P = static_cast<const T *>(post.p[f]);
        float v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            v[c] = 0.f;
            if (c < CREAL) {
                v[c] = (float)(P[((size_t)y * CREAL + c) * nx + x] - (T)nm.in_mean[c]) * nm.in_inv[c];
                if (noise) v[c] += amp * noise[(((size_t)f * CREAL + c) * ny + y) * nx + x];
            }
        }
#pragma unroll
        for (int c = 0; c < CH; c += 2)
            tile[threadIdx.x][c / 2] = (uint32_t)bf16_bits(v[c]) | ((uint32_t)bf16_bits(v[c + 1]) << 16);
    }
    __syncthreads();
    const int nodes = min(256, nx - xb);
    u16 *dst = x0 + (((size_t)f * ny + y) * nx + xb) * CH;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = r * 256 + threadIdx.x;          // 16-byte chunk: node i / 4, quarter i % 4
        const int n = i >> 2, q = i & 3;
        if (n < nodes)
            reinterpret_cast<uint4 *>(dst)[i] =
                make_uint4(tile[n][4 * q], tile[n][4 * q + 1], tile[n][4 * q + 2], tile[n][4 * q + 3]);
    }
}

// ---------------------------------------------------------------------------
// 3x3 periodic convolution as implicit GEMM on 32x32x16 bf16 MFMA.
// MODE 0: forward hidden layer  out = bf16(relu(conv + bias))
// MODE 1: forward last layer    out = f32(conv + bias)
// MODE 2: input gradient        out = bf16(conv_mirrored(dz, W^T) * (act > 0))
// MODE 3: network-input gradient out = f32(conv_mirrored(dz, W^T))  (no ReLU below)
// ---------------------------------------------------------------------------
// A block covers 4 waves x 32 nodes of `rows` consecutive rows; each lane
// keeps its 18 weight operands in registers across the rows (the weights
// are the same for every node, and reloading them per row made the L1 read
// traffic several times the activations').  The A operands of the three
// input rows an output row reads (3 columns x 2 channel halves each) form a
// ring in registers: the next output row reuses two of them and loads one
// new input row, issued while the current row's MFMAs run (three times
// fewer operand loads; the forward pass is 20 % faster).  conv_rows() picks
// the row count that leaves about 256 blocks, at most 16 rows each
// (measured best at 8 frames of 256^2; a single frame keeps one row per
// block).
inline int conv_rows(int nx, int ny, int frames)
{
    const long long blocks1 = (long long)((nx / 32 + 3) / 4) * ny * frames;
    return (int)std::max<long long>(1, std::min<long long>(PLBM_CONV_MAX_ROWS, blocks1 / PLBM_CONV_BLOCKS));
}

// A operands of one input row: columns x - 1, x, x + 1 (periodic) of the
// lane's node, channel halves 0..15 and 16..31
__device__ __forceinline__ void cl_load_row(const u16 *__restrict__ in, size_t fbase, int nx, int ny,
                                            int ys, const int (&xs)[3], int kh, bf16x8 (&a)[3][2])
{
    ys += (ys < 0) ? ny : 0;
    ys -= (ys >= ny) ? ny : 0;
    const u16 *row = in + (fbase + (size_t)ys * nx) * CH + 8 * kh;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            a[d][h] = *reinterpret_cast<const bf16x8 *>(row + (size_t)xs[d] * CH + h * 16);
}

// Output row y with input rows y - 1, y, y + 1 in ring slots P, P + 1, P + 2
// (mod 3).  The taps reading row y - 1 go first; when `more`, input row
// y + 2 is then loaded into slot P while the other six MFMA pairs run.
template <int MODE, int P>
__device__ __forceinline__ void cl_conv_row(bf16x8 (&A)[3][3][2], const bf16x8 (&bw)[TAPS][2],
                                            const u16 *__restrict__ in, const u16 *__restrict__ act,
                                            void *__restrict__ out, size_t fbase, int nx, int ny, int y,
                                            int x0, const int (&xs)[3], int l, float bj, bool more)
{
    const int kh = l >> 5, j = l & 31;
    f32x16 acc = {};
#pragma unroll
    for (int r = 0; r < 3; ++r) {                 // input row y - 1 + r, ring slot P + r
#pragma unroll
        for (int d = 0; d < 3; ++d) {             // input column x - 1 + d
            // tap (ty, tx) of the kernel: the forward pass reads input y + ty - 1,
            // the input gradient (mirrored kernel) input y - ty + 1
            const int t = (MODE >= 2) ? (2 - r) * 3 + (2 - d) : r * 3 + d;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[(P + r) % 3][d][h], bw[t][h], acc, 0, 0, 0);
        }
        if (r == 0 && more) cl_load_row(in, fbase, nx, ny, y + 2, xs, kh, A[P]);
    }
    // D[i][j]: i = node 8*(r/4) + 4*(l/32) + r%4, j = channel l%32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r / 4) + 4 * (l >> 5) + (r & 3);
        const size_t node = fbase + (size_t)y * nx + x0 + i;
        float v = acc[r] + bj;
        if (MODE == 0) {
            reinterpret_cast<u16 *>(out)[node * CH + j] = bf16_bits(fmaxf(v, 0.f));
        } else if (MODE == 1 || MODE == 3) {
            reinterpret_cast<float *>(out)[node * CH + j] = v;
        } else {
            const float a = bf16_val(act[node * CH + j]);
            reinterpret_cast<u16 *>(out)[node * CH + j] = bf16_bits(a > 0.f ? v : 0.f);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256, PLBM_CONV_WAVES) void k_cl_conv(const u16 *__restrict__ in, const u16 *__restrict__ wb,
                                                 const float *__restrict__ bias,
                                                 const u16 *__restrict__ act, void *__restrict__ out,
                                                 int nx, int ny, int rows)
{
    const int f = blockIdx.z;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int x0 = (blockIdx.x * 4 + wv) * 32;       // first node of this wave
    const int ybeg = blockIdx.y * rows;
    if (x0 >= nx || ybeg >= ny) return;
    const int yend = min(ybeg + rows, ny);
    const int row_i = l & 31, kh = l >> 5;            // A: node row_i, channels 8*kh..
    const size_t fbase = (size_t)f * ny * nx;
    // B: column (output channel) l & 31, k = 8*kh.. within each half
    bf16x8 bw[TAPS][2];
#pragma unroll
    for (int t = 0; t < TAPS; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            bw[t][h] = *reinterpret_cast<const bf16x8 *>(wb + ((size_t)t * CH + (l & 31)) * CH + h * 16 + 8 * kh);
    const float bj = (MODE >= 2) ? 0.f : bias[l & 31];
    int xs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int x = x0 + row_i + d - 1;
        x += (x < 0) ? nx : 0;
        x -= (x >= nx) ? nx : 0;
        xs[d] = x;
    }
    bf16x8 A[3][3][2];
    cl_load_row(in, fbase, nx, ny, ybeg - 1, xs, kh, A[0]);
    cl_load_row(in, fbase, nx, ny, ybeg, xs, kh, A[1]);
    cl_load_row(in, fbase, nx, ny, ybeg + 1, xs, kh, A[2]);
#pragma unroll 1
    for (int y = ybeg; y < yend; y += 3) {
        cl_conv_row<MODE, 0>(A, bw, in, act, out, fbase, nx, ny, y, x0, xs, l, bj, y + 1 < yend);
        if (y + 1 >= yend) break;
        cl_conv_row<MODE, 1>(A, bw, in, act, out, fbase, nx, ny, y + 1, x0, xs, l, bj, y + 2 < yend);
        if (y + 2 >= yend) break;
        cl_conv_row<MODE, 2>(A, bw, in, act, out, fbase, nx, ny, y + 2, x0, xs, l, bj, y + 3 < yend);
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][o][i] = sum_p dz[p][o] * a[p + d_t][i], db[o] = sum_p dz[p][o].
// A 32x32x16 MFMA takes 8 consecutive nodes of one channel per lane (the
// contraction runs over nodes).  dz and the input rows y-1, y, y+1 sit in
// LDS node-major, as they are in memory (16-byte writes), and each operand
// is read with two of gfx950's transposing LDS reads (ds_read_b64_tr_b16).
// Within each group of 16 lanes such a read gives lane 4a + b the b-th
// 16-bit element of the 8-byte chunks that lanes a, a + 4, a + 8, a + 12
// address.  Lane j of a group addresses node q + j/4, channels c + 4 (j%4),
// so lane 4a + b receives nodes q .. q + 3 of channel c + 4a + b: the
// operand layout.  An x shift of the input is an offset of the node index.
// The input rows form a ring in LDS, so each row of the block loads one new
// input row.  Block = WG_SEG nodes x WG_ROWS rows of one frame; wave w owns
// taps w and w+4 and the nodes 16 w .. 16 w + 15 of tap 8, whose four
// partials are summed through LDS in a fixed order (nine MFMAs per row on
// every wave; with all of tap 8 on wave 0 its SIMD did twelve).  The next
// row's global loads are issued before the current row's MFMAs.
// ---------------------------------------------------------------------------
constexpr int WG_AN = WG_SEG + 2;               // nodes of one input row: x0 - 1 .. x0 + WG_SEG
constexpr int WG_AVEC = WG_AN * CH / 8;         // 16-byte vectors of one input row

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16;

// One input row (vectors t and 256 + t of this thread) and one dz row
// segment (node t/4, channels 8 (t%4) ..).
struct WgRegs {
    uint4 dz, a0, a1;
};

// vector i of an input row: node x0 - 1 + i / 4, channels 8 (i % 4) ..
__device__ __forceinline__ uint4 wg_load_vec(const u16 *__restrict__ a, size_t fbase, int nx, int x0, int y,
                                             int i)
{
    int xs = x0 + (i >> 2) - 1;
    xs += (xs < 0) ? nx : 0;
    xs -= (xs >= nx) ? nx : 0;
    return *reinterpret_cast<const uint4 *>(a + (fbase + (size_t)y * nx + xs) * CH + (i & 3) * 8);
}

__device__ __forceinline__ void wg_load_a(const u16 *__restrict__ a, size_t fbase, int nx, int ny, int x0, int y,
                                          uint4 &v0, uint4 &v1)
{
    y += (y < 0) ? ny : 0;
    y -= (y >= ny) ? ny : 0;
    v0 = wg_load_vec(a, fbase, nx, x0, y, threadIdx.x);
    if (threadIdx.x + 256 < WG_AVEC) v1 = wg_load_vec(a, fbase, nx, x0, y, threadIdx.x + 256);
}

// input row -> LDS slot, node-major (node m is x0 - 1 + m)
__device__ __forceinline__ void wg_store_a(u16 (*slot)[CH], const uint4 &v0, const uint4 &v1)
{
    const int i = threadIdx.x;
    *reinterpret_cast<uint4 *>(&slot[i >> 2][(i & 3) * 8]) = v0;
    if (i + 256 < WG_AVEC) *reinterpret_cast<uint4 *>(&slot[(i + 256) >> 2][((i + 256) & 3) * 8]) = v1;
}

// MFMA operand of lane l from a node-major LDS array: nodes
// n0 + 8 (l / 32) .. + 7 of channel l % 32
__device__ __forceinline__ bf16x8 wg_operand(const u16 (*rows)[CH], int n0, int l)
{
    const int j = l & 15;
    const int node = n0 + 8 * (l >> 5) + (j >> 2);
    const int ch = 16 * ((l >> 4) & 1) + 4 * (j & 3);
    const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16 *)&rows[node][ch]);
    const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16 *)&rows[node + 4][ch]);
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

__global__ __launch_bounds__(256) void k_cl_wgrad(const u16 *__restrict__ a, const u16 *__restrict__ dz,
                                                  int nx, int ny, float *__restrict__ part)
{
    __shared__ __attribute__((aligned(16))) u16 sdz[WG_SEG][CH];
    // a ring of three input rows: row yy sits in slot (yy - y0 + 1) % 3
    __shared__ __attribute__((aligned(16))) u16 sa[3][WG_AN][CH];
    __shared__ float bred[4][4][8];
    __shared__ float red8[4][16][64];    // the four waves' partials of tap 8
    const int f = blockIdx.z;
    const int segs = nx / WG_SEG;
    const int x0 = (blockIdx.x % segs) * WG_SEG;
    const int y0 = (blockIdx.x / segs) * WG_ROWS;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, t = threadIdx.x;
    const size_t fbase = (size_t)f * ny * nx;
    const int rows = min(WG_ROWS, ny - y0);
    f32x16 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = f32x16{};
    float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // node t/4, channels 8 (t%4) ..
    {
        uint4 v0 = {}, v1 = {};
        wg_load_a(a, fbase, nx, ny, x0, y0 - 1, v0, v1);
        wg_store_a(sa[0], v0, v1);
        wg_load_a(a, fbase, nx, ny, x0, y0, v0, v1);
        wg_store_a(sa[1], v0, v1);
    }
    WgRegs R = {};
    R.dz = *reinterpret_cast<const uint4 *>(dz + (fbase + (size_t)y0 * nx + x0 + (t >> 2)) * CH + (t & 3) * 8);
    wg_load_a(a, fbase, nx, ny, x0, y0 + 1, R.a0, R.a1);

#pragma unroll 1
    for (int r = 0; r < rows; ++r) {
        const int y = y0 + r;
        __syncthreads();                 // the previous row's LDS reads are done
        *reinterpret_cast<uint4 *>(&sdz[t >> 2][(t & 3) * 8]) = R.dz;
        {
            const uint32_t w4[4] = {R.dz.x, R.dz.y, R.dz.z, R.dz.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) bsum[k] += bf16_val((u16)(w4[k >> 1] >> (16 * (k & 1))));
        }
        wg_store_a(sa[(r + 2) % 3], R.a0, R.a1);   // row y + 1
        __syncthreads();
        if (r + 1 < rows) {
            R.dz = *reinterpret_cast<const uint4 *>(dz + (fbase + (size_t)(y + 1) * nx + x0 + (t >> 2)) * CH +
                                                    (t & 3) * 8);
            wg_load_a(a, fbase, nx, ny, x0, y + 2, R.a0, R.a1);
        }
        // A = dz^T (row o = l&31, k = nodes), B = a_t (col i = l&31, k = nodes).
        // Wave w takes taps w and w + 4 over all 64 nodes and tap 8 over
        // nodes 16 w .. 16 w + 15 (nine MFMAs per row on every wave).
#pragma unroll
        for (int kc = 0; kc < WG_SEG / 16; ++kc) {
            const bf16x8 av = wg_operand(sdz, kc * 16, l);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q == 2 && kc != wv) continue;
                const int tap = q == 2 ? 8 : wv + 4 * q;
                const int dy = tap / 3, dx = tap % 3;    // input row y + dy - 1, node x + dx - 1
                const int slot = (r + dy) % 3;
                // output node x0 + n reads input node x0 + n + dx - 1, LDS node n + dx
                const bf16x8 bv = wg_operand(sa[slot], kc * 16 + dx, l);
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red8[wv][r][l] = acc[2][r];
    // bias: sum the per-thread channel sums over the 16 nodes of the wave
    // (lanes 4 n + q), then over the four waves, in a fixed order
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) bsum[k] += __shfl_xor(bsum[k], off, 64);
    }
    if (l < 4) {
#pragma unroll
        for (int k = 0; k < 8; ++k) bred[wv][l][k] = bsum[k];
    }
    __syncthreads();
    // partials: [block][t][o][i] then [block][bias o]
    const size_t nblk = (size_t)gridDim.x * gridDim.y * gridDim.z;
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int tap = wv + 4 * q;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 8 * (r / 4) + 4 * (l >> 5) + (r & 3);
            part[blk * LAYER_W + ((size_t)tap * CH + o) * CH + (l & 31)] = acc[q][r];
        }
    }
    // tap 8: the four partials summed in a fixed order (red8 was written
    // before the barrier above)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int idx = k * 256 + t, r = idx >> 6, ll = idx & 63;
        const int o = 8 * (r / 4) + 4 * (ll >> 5) + (r & 3);
        part[blk * LAYER_W + ((size_t)8 * CH + o) * CH + (ll & 31)] =
            (red8[0][r][ll] + red8[1][r][ll]) + (red8[2][r][ll] + red8[3][r][ll]);
    }
    if (t < CH) {
        const int q = t >> 3, k = t & 7;
        part[nblk * LAYER_W + blk * CH + t] = (bred[0][q][k] + bred[1][q][k]) + (bred[2][q][k] + bred[3][q][k]);
    }
}

// Sum the block partials in a fixed order into the flat gradient of one
// layer, in two passes: slice z of the first pass sums blocks z, z + WR_SLICES,
// ... ; the second sums the slices in order.  Deterministic, and wide enough
// to keep the memory system busy (the partials of 16 row bands x 8 frames are
// several MB).
constexpr int WR_SLICES = 32;

__device__ __forceinline__ float part_at(const float *part, int nblk, int b, int i)
{
    return i < LAYER_W ? part[(size_t)b * LAYER_W + i] : part[(size_t)nblk * LAYER_W + (size_t)b * CH + (i - LAYER_W)];
}

__global__ __launch_bounds__(256) void k_cl_wgrad_slices(const float *__restrict__ part, int nblk,
                                                         float *__restrict__ slices)
{
    const int i = blockIdx.x * 256 + threadIdx.x, z = blockIdx.y;
    if (i >= LAYER_P) return;
    float s = 0.f;
    for (int b = z; b < nblk; b += WR_SLICES) s += part_at(part, nblk, b, i);
    slices[(size_t)z * LAYER_P + i] = s;
}

__global__ __launch_bounds__(256) void k_cl_wgrad_reduce(const float *__restrict__ slices,
                                                         float *__restrict__ grad, int accumulate)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= LAYER_P) return;
    float s = 0.f;
#pragma unroll 8
    for (int z = 0; z < WR_SLICES; ++z) s += slices[(size_t)z * LAYER_P + i];
    grad[i] = accumulate ? grad[i] + s : s;
}

// ---------------------------------------------------------------------------
// Moment-form loss.  Physical correction c = s * Ph y (planes [f][k][y][x]);
// the corrected buffer streamed in the pull form adds to node x the conserved
// densities m(x) = sum_k Phi_k (c_k(x - v_k) - c_k(x)) (flux form: the second
// term is zero for a moment-free c, and with it the domain totals of m vanish
// exactly although c is stored in FP32); with the target increment error
// d (planes [j][y][x] per frame) the residual is r = m - d and
//   L = (1/N) sum_x [sum_j w_j r_j^2 + beta |Ph y|^2],   w_j = 1 / sigma_j^2.
// The moments fix only 4 of a node's 21 free correction components; the
// minimum-norm term picks the smallest correction that explains them.
// dL/dc_k(x) = sum_j Phi_jk (a_j(x + v_k) - a_j(x)) with a = (2/N) w r (the
// push); the a_j(x) part lies in the span Ph removes, so
// dL/dy = Ph (s * push + (2 beta / N) y) since Ph is symmetric idempotent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cl_corr(const float *__restrict__ y3, int nx, int ny, ClNorm nm,
                                                 float reg, float *__restrict__ C, float *__restrict__ lpart)
{
    __shared__ float red[4];
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    float lsum = 0.f;
    if (x < nx) {
        const size_t plane = (size_t)nx * ny;
        const size_t node = ((size_t)f * ny + y) * nx + x;
        float d[CREAL];
#pragma unroll
        for (int k = 0; k < CREAL; ++k) d[k] = y3[node * CH + k];
        project(d, nm);
#pragma unroll
        for (int k = 0; k < CREAL; ++k) {
            lsum += d[k] * d[k];
            C[((size_t)f * CREAL + k) * plane + (size_t)y * nx + x] = nm.out_scale[k] * d[k];
        }
        lsum *= reg;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0)
        lpart[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] =
            (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_cl_mloss(const float *__restrict__ C, PtrList target, int nx, int ny,
                                                  ClNorm nm, float inv_n, float *__restrict__ A,
                                                  float *__restrict__ lpart)
{
    __shared__ float red[4];
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    float lsum = 0.f;
    if (x < nx) {
        const size_t plane = (size_t)nx * ny;
        float m[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < CREAL; ++k) {
            int xs = x - nm.ivx[k], ys = y - nm.ivy[k];
            xs += xs < 0 ? nx : (xs >= nx ? -nx : 0);
            ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
            const float *ck = C + ((size_t)f * CREAL + k) * plane;
            const float c = ck[(size_t)ys * nx + xs] - ck[(size_t)y * nx + x];
            const float vx = nm.vx[k], vy = nm.vy[k];
            m[0] += c;
            m[1] += vx * c;
            m[2] += vy * c;
            m[3] += (vx * vx + vy * vy) * c;
        }
        const float *d = static_cast<const float *>(target.p[f]);
        const size_t at = (size_t)y * nx + x;
        float a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float r = m[j] - d[j * plane + at];
            lsum += nm.mw2[j] * r * r;
            a[j] = 2.f * inv_n * nm.mw2[j] * r;
        }
        // node-interleaved, so that the push gathers one 16-byte vector per neighbour
        reinterpret_cast<float4 *>(A)[(size_t)f * plane + at] = make_float4(a[0], a[1], a[2], a[3]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0)
        lpart[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] +=
            (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_cl_mgrad(const float *__restrict__ A, const float *__restrict__ y3,
                                                  int nx, int ny, ClNorm nm, float reg2n,
                                                  u16 *__restrict__ dy3)
{
    // the node's bf16 row goes through LDS, so that the block's 256 x 64
    // bytes are stored as consecutive 16-byte chunks (as in k_cl_input)
    __shared__ uint32_t tile[256][17];
    const int f = blockIdx.z, y = blockIdx.y;
    const int xb = blockIdx.x * 256;
    const int x = xb + threadIdx.x;
    if (x < nx) {
        const size_t plane = (size_t)nx * ny;
        const size_t node = ((size_t)f * ny + y) * nx + x;
        float t[CREAL];
#pragma unroll
        for (int k = 0; k < CREAL; ++k) {
            int xs = x + nm.ivx[k], ys = y + nm.ivy[k];
            xs += xs < 0 ? nx : (xs >= nx ? -nx : 0);
            ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
            const float4 a = reinterpret_cast<const float4 *>(A)[(size_t)f * plane + (size_t)ys * nx + xs];
            const float vx = nm.vx[k], vy = nm.vy[k];
            t[k] = nm.out_scale[k] * (a.x + vx * a.y + vy * a.z + (vx * vx + vy * vy) * a.w);
        }
        if (reg2n != 0.f) {                           // the minimum-norm term, when asked for
#pragma unroll
            for (int k = 0; k < CREAL; ++k) t[k] += reg2n * y3[node * CH + k];
        }
        project(t, nm);
#pragma unroll
        for (int c = 0; c < CH; c += 2) {
            const float a = c < CREAL ? t[c] : 0.f;
            const float b = c + 1 < CREAL ? t[c + 1] : 0.f;
            tile[threadIdx.x][c / 2] = (uint32_t)bf16_bits(a) | ((uint32_t)bf16_bits(b) << 16);
        }
    }
    __syncthreads();
    const int nodes = min(256, nx - xb);
    u16 *dst = dy3 + (((size_t)f * ny + y) * nx + xb) * CH;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = r * 256 + threadIdx.x;
        const int n = i >> 2, q = i & 3;
        if (n < nodes)
            reinterpret_cast<uint4 *>(dst)[i] =
                make_uint4(tile[n][4 * q], tile[n][4 * q + 1], tile[n][4 * q + 2], tile[n][4 * q + 3]);
    }
}

// Increment error d = (cons(truth_now) - cons(truth_prev)) - (cons(model_now)
// - cons(model_prev)), cons(rho, u, theta) = (rho, rho u, rho (2 theta + |u|^2)),
// in FP64, rounded once to FP32 planes [j][node].
struct Fields16 {
    const double *p[16];
};

__device__ __forceinline__ void cons4(const Fields16 &F, int b, size_t i, double (&c)[4])
{
    const double r = F.p[b][i], u = F.p[b + 1][i], w = F.p[b + 2][i], t = F.p[b + 3][i];
    c[0] = r;
    c[1] = r * u;
    c[2] = r * w;
    c[3] = r * (2.0 * t + u * u + w * w);
}

__global__ __launch_bounds__(256) void k_cl_target(Fields16 F, size_t n, float *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double tp[4], tn[4], mp[4], mn[4];
    cons4(F, 0, i, tp);
    cons4(F, 4, i, tn);
    cons4(F, 8, i, mp);
    cons4(F, 12, i, mn);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j * n + i] = (float)((tn[j] - tp[j]) - (mn[j] - mp[j]));
}

// ---------------------------------------------------------------------------
// Apply, as an equilibrium shift.  The correction's streamed moments
// g(x) = sum_k Phi_k (c_k(x - v_k) - c_k(x)) are the change of node x's conserved
// densities; they are given to the populations f = pull(P) of the next step
// as  f <- f + f_eq(m + g) - f_eq(m)  (m the node's own moments), so the
// node's moments become m + g exactly and its non-equilibrium part f - f_eq
// is the plain step's.  In the pull layout population k of node x is stored
// at x - v_k.
//
// 1. k_cl_corr_apply: c = s * Ph y where every normalised component is
//    finite and within bound, else c = 0 (fallback, counted in *skipped);
// 2. k_cl_shift: per node, m from the pulled populations (FP64), g from c,
//    delta = f_eq(m + g) - f_eq(m) (zero if the shifted density or
//    temperature would not be positive), added in place to the populations
//    it pulled: the slot of population k at x - v_k is read and written by
//    node x alone, so no other thread touches it.  The sum is rounded once
//    to the storage type (FP64 lattices conserve the totals to FP64 rounding).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cl_corr_apply(const float *__restrict__ y3, int nx, int ny, ClNorm nm,
                                                       float bound, float *__restrict__ C,
                                                       unsigned *__restrict__ skipped)
{
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const size_t plane = (size_t)nx * ny;
    const size_t node = ((size_t)f * ny + y) * nx + x;
    float d[CREAL];
#pragma unroll
    for (int k = 0; k < CREAL; ++k) d[k] = y3[node * CH + k];
    project(d, nm);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < CREAL; ++k) ok = ok && (fabsf(d[k]) <= bound);
    if (!ok && skipped) atomicAdd(skipped, 1u);
#pragma unroll
    for (int k = 0; k < CREAL; ++k)
        C[((size_t)f * CREAL + k) * plane + (size_t)y * nx + x] = ok ? nm.out_scale[k] * d[k] : 0.f;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_shift(PtrList post, const float *__restrict__ C, int nx, int ny,
                                                  ClNorm nm, KParams kp)
{
    // no fused multiply-adds: the two equilibria below are evaluated by the
    // same rounded operations, so a zero moment change gives a zero shift
#pragma clang fp contract(off)
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const size_t plane = (size_t)nx * ny;
    T *P = static_cast<T *>(post.p[f]);
    double fp[NQ];
    double g[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        int xs = x - nm.ivx[k], ys = y - nm.ivy[k];
        xs += xs < 0 ? nx : (xs >= nx ? -nx : 0);
        ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
        fp[k] = (double)P[((size_t)ys * CREAL + k) * nx + xs];
        const float *ck = C + ((size_t)f * CREAL + k) * plane;
        const double c = (double)ck[(size_t)ys * nx + xs] - (double)ck[(size_t)y * nx + x];
        const double vx = nm.vx[k], vy = nm.vy[k];
        g[0] += c;
        g[1] += vx * c;
        g[2] += vy * c;
        g[3] += (vx * vx + vy * vy) * c;
    }
    double rho, jx, jy, e;
    sums2d<Fp64Math>(fp, kp, rho, jx, jy, e);
    const double r1 = rho + g[0];
    const double ux0 = jx / rho, uy0 = jy / rho;
    const double th0 = 0.5 * (e / rho - ux0 * ux0 - uy0 * uy0);
    const double ux1 = (jx + g[1]) / r1, uy1 = (jy + g[2]) / r1;
    const double th1 = 0.5 * ((e + g[3]) / r1 - ux1 * ux1 - uy1 * uy1);
    const bool ok = r1 > 0.0 && th1 > 0.0 && isfinite(th1) && isfinite(ux1) && isfinite(uy1);
    if (!ok) return;                                  // the node keeps its populations
    double a0[Q], b0[Q], a1[Q], b1[Q];
    rule1d<Fp64Math>(ux0, th0, kp, a0);
    rule1d<Fp64Math>(uy0, th0, kp, b0);
    rule1d<Fp64Math>(ux1, th1, kp, a1);
    rule1d<Fp64Math>(uy1, th1, kp, b1);
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int k = i + Q * j;
            int xs = x - nm.ivx[k], ys = y - nm.ivy[k];
            xs += xs < 0 ? nx : (xs >= nx ? -nx : 0);
            ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
            const double dlt = r1 * a1[i] * b1[j] - rho * a0[i] * b0[j];
            P[((size_t)ys * CREAL + k) * nx + xs] = (T)fp[k] + (T)dlt;
        }
}

// ---------------------------------------------------------------------------
// Training through coarse steps: adjoints (vector-Jacobian products, FP64).
// With Phi_k = (1, v_x, v_y, |v|^2), m = Phi^T f the conserved densities
// (rho, j_x, j_y, E) and F(m) the tensor-product equilibrium (Eq. eqdist with
// r = C mu of Eq. rdr; rho, u = j / rho, 2 theta = E / rho - |u|^2):
//   step   P' = (1 - w) S + w F(m(S)),  S = pull(P)
//          dL/dP = push((1 - w) lam + w Phi J_F(m)^T lam)
//   shift  P' = P + push(F(m + g) - F(m)),  m = m(pull(P)),
//          g = Phi^T (pull(c) - c)
//          dL/dP = lam + push(Phi (J_F(m + g) - J_F(m))^T Lam),
//          dL/dg = J_F(m + g)^T Lam,  Lam = pull(lam)
//   loss   L = scale sum_x sum_j w_j (m_j(pull(P))(x) - cons_j(R)(x))^2
//          dL/dP = push(Phi a),  a = 2 scale w r
// Adjoint buffers have the population layout (y * 25 + k) * nx + x in FP64.
// ---------------------------------------------------------------------------

// r, dr/du and dr/dtheta of the symmetric 1D rule: the Maxwell moments and
// their derivatives d mu_n/du = n mu_(n-1), d mu_n/dtheta = n (n-1)/2 mu_(n-2)
// go through the same linear map r = C mu (without its constant for the
// derivatives).
__device__ __forceinline__ void rule_lin(const SymRule<double> &R, double m1, double m2, double m3, double m4,
                                         double c0, double (&r)[Q])
{
    const double e1 = R.c12 * m2 + R.c14 * m4, o1 = R.c11 * m1 + R.c13 * m3;
    const double e3 = R.c32 * m2 + R.c34 * m4, o3 = R.c31 * m1 + R.c33 * m3;
    r[0] = c0 + R.c02 * m2 + R.c04 * m4;
    r[1] = e1 + o1;
    r[2] = e1 - o1;
    r[3] = e3 + o3;
    r[4] = e3 - o3;
}

__device__ __forceinline__ void rule_derivs(const SymRule<double> &R, double u, double th, double (&r)[Q],
                                            double (&ru)[Q], double (&rt)[Q])
{
    const double m2 = u * u + th, m3 = u * m2 + 2.0 * th * u, m4 = u * m3 + 3.0 * th * m2;
    rule_lin(R, u, m2, m3, m4, 1.0, r);
    rule_lin(R, 1.0, 2.0 * u, 3.0 * m2, 4.0 * m3, 0.0, ru);
    rule_lin(R, 0.0, 1.0, 3.0 * u, 6.0 * m2, 0.0, rt);
}

// a = J_F(m)^T lam for conserved densities m and cotangents lam[k = i + 5 j]
__device__ __forceinline__ void feq_vjp(const SymRule<double> &R, const double (&m)[4], const double (&lam)[NQ],
                                        double (&a)[4])
{
    const double rho = m[0], inv = 1.0 / rho;
    const double ux = m[1] * inv, uy = m[2] * inv;
    const double th = 0.5 * (m[3] * inv - ux * ux - uy * uy);
    double rx[Q], rxu[Q], rxt[Q], ry[Q], ryu[Q], ryt[Q];
    rule_derivs(R, ux, th, rx, rxu, rxt);
    rule_derivs(R, uy, th, ry, ryu, ryt);
    double gr = 0.0, gu = 0.0, gw = 0.0, gt = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        double lr = 0.0, lu = 0.0, lt = 0.0;        // sum over i of lam_ij (r_i, r'_i, rdot_i)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double l = lam[i + Q * j];
            lr += l * rx[i];
            lu += l * rxu[i];
            lt += l * rxt[i];
        }
        gr += ry[j] * lr;
        gu += ry[j] * lu;
        gw += ryu[j] * lr;
        gt += ry[j] * lt + ryt[j] * lr;
    }
    gu *= rho;
    gw *= rho;
    gt *= rho;
    a[0] = gr - (gu * ux + gw * uy) * inv + 0.5 * gt * (ux * ux + uy * uy - 2.0 * th) * inv;
    a[1] = (gu - gt * ux) * inv;
    a[2] = (gw - gt * uy) * inv;
    a[3] = 0.5 * gt * inv;
}

__device__ __forceinline__ int wrap(int i, int n)
{
    i += i < 0 ? n : 0;
    return i - (i >= n ? n : 0);
}

// Step adjoint at node x: from l = dL/dP'(x) and the conserved densities of
// S(x) = pull(P)(x), mu = (1 - w) l + w Phi J^T l, scattered to
// dL/dP(x - v_k)_k = mu_k (each target written exactly once).
// Conserved densities of S(x) = pull(P)(x)
template <typename T>
__device__ __forceinline__ void step_moments(const T *__restrict__ P, int x, int y, int nx, int ny,
                                             const KParams &kp, double (&m)[4])
{
    m[0] = m[1] = m[2] = m[3] = 0.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int vx = kp.sx[k % Q], vy = kp.sx[k / Q];
        const double f = (double)P[((size_t)wrap(y - vy, ny) * NQ + k) * nx + wrap(x - vx, nx)];
        m[0] += f;
        m[1] += vx * f;
        m[2] += vy * f;
        m[3] += (vx * vx + vy * vy) * f;
    }
}

// Step adjoint at node x: from l = dL/dP'(x) and the conserved densities m
// of S(x), mu = (1 - w) l + w Phi J^T l, scattered to dL/dP(x - v_k)_k =
// mu_k (each target written exactly once).
__device__ __forceinline__ void step_vjp_scatter(const double (&m)[4], const double (&l)[NQ],
                                                 double *__restrict__ out, int x, int y, int nx, int ny,
                                                 const KParams &kp)
{
    double a[4];
    feq_vjp(kp.r64, m, l, a);
    const double w = kp.r64.omega;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int vx = kp.sx[k % Q], vy = kp.sx[k / Q];
        const double phi_a = a[0] + vx * a[1] + vy * a[2] + (vx * vx + vy * vy) * a[3];
        out[((size_t)wrap(y - vy, ny) * NQ + k) * nx + wrap(x - vx, nx)] = (1.0 - w) * l[k] + w * phi_a;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_step_vjp(const T *__restrict__ P, const double *__restrict__ lam,
                                                  double *__restrict__ out, int nx, int ny, KParams kp)
{
    const int y = blockIdx.y, x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    double m[4], l[NQ];
    step_moments(P, x, y, nx, ny, kp, m);
#pragma unroll
    for (int k = 0; k < NQ; ++k) l[k] = lam[((size_t)y * NQ + k) * nx + x];
    step_vjp_scatter(m, l, out, x, y, nx, ny, kp);
}

// Phi_k . a for a per-node moment cotangent a = (a_rho, a_jx, a_jy, a_E)
__device__ __forceinline__ double phi_dot(double vx, double vy, const double *__restrict__ a)
{
    return a[0] + vx * a[1] + vy * a[2] + (vx * vx + vy * vy) * a[3];
}

// Up to MAX_FRAMES sets of (rho, u_x, u_y, theta) planes.
struct TruthList {
    const double *p[4 * MAX_FRAMES];
};

// Rollout loss at node x: residual r = m(pull(P))(x) - cons(R)(x) per
// moment; a = 2 scale w r, returns scale sum_j w_j r_j^2.
template <typename T>
__device__ __forceinline__ double rloss_node(const T *__restrict__ P, const TruthList &truth, int f, int x, int y,
                                             int nx, int ny, const ClNorm &nm, double scale, double (&a)[4])
{
    double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        const double v = (double)P[((size_t)wrap(y - nm.ivy[k], ny) * CREAL + k) * nx + wrap(x - nm.ivx[k], nx)];
        const double vx = nm.ivx[k], vy = nm.ivy[k];
        m[0] += v;
        m[1] += vx * v;
        m[2] += vy * v;
        m[3] += (vx * vx + vy * vy) * v;
    }
    const size_t at = (size_t)y * nx + x;
    const double r0 = truth.p[4 * f][at], u = truth.p[4 * f + 1][at], w = truth.p[4 * f + 2][at],
                 t = truth.p[4 * f + 3][at];
    const double c[4] = {r0, r0 * u, r0 * w, r0 * (2.0 * t + u * u + w * w)};
    double lsum = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double r = m[j] - c[j];
        lsum += scale * (double)nm.mw2[j] * r * r;
        a[j] = 2.0 * scale * (double)nm.mw2[j] * r;
    }
    return lsum;
}

// Sum of one value per thread over a 256-thread block, in a fixed order;
// the result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double (&red)[4])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Rollout loss at one step: a = 2 scale w r (double4 per node) and the
// loss partials scale w r^2 per block.
template <typename T>
__global__ __launch_bounds__(256) void k_cl_rloss(PtrList post, TruthList truth, int nx, int ny, ClNorm nm,
                                                  double scale, double *__restrict__ A,
                                                  double *__restrict__ lpart)
{
    __shared__ double red[4];
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    double lsum = 0.0;
    if (x < nx) {
        double a[4];
        lsum = rloss_node(static_cast<const T *>(post.p[f]), truth, f, x, y, nx, ny, nm, scale, a);
        double *dst = A + ((size_t)f * ny * nx + (size_t)y * nx + x) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[j] = a[j];
    }
    const double tot = block_sum256(lsum, red);
    if (threadIdx.x == 0)
        lpart[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// lam(y)_k += Phi_k . a(y + v_k): the push of per-node moment cotangents
__global__ __launch_bounds__(256) void k_cl_push4(const double *__restrict__ A, PtrList lam, int nx, int ny,
                                                  ClNorm nm)
{
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    double *L = static_cast<double *>(lam.p[f]);
    const double *Af = A + (size_t)f * ny * nx * 4;
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        const double *a = Af + ((size_t)wrap(y + nm.ivy[k], ny) * nx + wrap(x + nm.ivx[k], nx)) * 4;
        L[((size_t)y * CREAL + k) * nx + x] += phi_dot(nm.ivx[k], nm.ivy[k], a);
    }
}

// Shift adjoint at node x from Lam = l (the adjoint of the shifted state,
// already pulled): m from pull(P), g from c (as k_cl_shift); writes
// a_g = J_F(m + g)^T Lam as the moment cotangent of the correction (float4,
// read by k_cl_mgrad) and a_m = a_g - J_F(m)^T Lam (double4, the state
// path).  Nodes the forward left unshifted (density or temperature not
// positive) pass nothing.
template <typename T>
__device__ __forceinline__ void shift_vjp_node(const T *__restrict__ P, const double (&l)[NQ],
                                               const float *__restrict__ C, int f, int x, int y, int nx, int ny,
                                               const ClNorm &nm, const KParams &kp, float *__restrict__ Ag,
                                               double (&am)[4], size_t node)
{
    const size_t plane = (size_t)nx * ny;
    double m[4] = {0.0, 0.0, 0.0, 0.0}, g[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CREAL; ++k) {
        const int xs = wrap(x - nm.ivx[k], nx), ys = wrap(y - nm.ivy[k], ny);
        const double v = (double)P[((size_t)ys * CREAL + k) * nx + xs];
        const float *ck = C + ((size_t)f * CREAL + k) * plane;
        const double c = (double)ck[(size_t)ys * nx + xs] - (double)ck[(size_t)y * nx + x];
        const double vx = nm.ivx[k], vy = nm.ivy[k], v2 = vx * vx + vy * vy;
        m[0] += v;
        m[1] += vx * v;
        m[2] += vy * v;
        m[3] += v2 * v;
        g[0] += c;
        g[1] += vx * c;
        g[2] += vy * c;
        g[3] += v2 * c;
    }
    double m1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) m1[j] = m[j] + g[j];
    const double ux1 = m1[1] / m1[0], uy1 = m1[2] / m1[0];
    const double th1 = 0.5 * (m1[3] / m1[0] - ux1 * ux1 - uy1 * uy1);
    const bool ok = m1[0] > 0.0 && th1 > 0.0 && isfinite(th1);
    double ag[4] = {0.0, 0.0, 0.0, 0.0}, a0[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
        feq_vjp(kp.r64, m1, l, ag);
        feq_vjp(kp.r64, m, l, a0);
    }
    reinterpret_cast<float4 *>(Ag)[node] = make_float4((float)ag[0], (float)ag[1], (float)ag[2], (float)ag[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) am[j] = ag[j] - a0[j];
}

template <typename T>
__global__ __launch_bounds__(256) void k_cl_shift_vjp(PtrList post, PtrList lam, const float *__restrict__ C,
                                                      int nx, int ny, ClNorm nm, KParams kp,
                                                      float *__restrict__ Ag, double *__restrict__ Am)
{
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const double *L = static_cast<const double *>(lam.p[f]);
    double l[NQ];
#pragma unroll
    for (int k = 0; k < CREAL; ++k)
        l[k] = L[((size_t)wrap(y - nm.ivy[k], ny) * CREAL + k) * nx + wrap(x - nm.ivx[k], nx)];
    const size_t node = (size_t)f * ny * nx + (size_t)y * nx + x;
    double am[4];
    shift_vjp_node(static_cast<const T *>(post.p[f]), l, C, f, x, y, nx, ny, nm, kp, Ag, am, node);
#pragma unroll
    for (int j = 0; j < 4; ++j) Am[node * 4 + j] = am[j];
}

// The network input is the normalised post-collision buffer at the node
// itself, x_k = (P_k - mean_k) * inv_k: lam(x)_k += inv_k dL/dx_k.
__global__ __launch_bounds__(256) void k_cl_input_vjp(const float *__restrict__ dx, PtrList lam, int nx, int ny,
                                                      ClNorm nm)
{
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    double *L = static_cast<double *>(lam.p[f]);
    const size_t node = ((size_t)f * ny + y) * nx + x;
#pragma unroll
    for (int k = 0; k < CREAL; ++k)
        L[((size_t)y * CREAL + k) * nx + x] += (double)nm.in_inv[k] * (double)dx[node * CH + k];
}

// ---------------------------------------------------------------------------
// One backward step of rollout training in two passes (plbm_closure_rollout_vjp).
// With lam_in = dL/dQ_s from the later steps (Q_s the state after the apply
// of step s), the loss at Q_s adds push(Phi A_L) and the apply's state path
// push(Phi a_m); the network input adds inv * dx.  Seen through the pull at
// node x, a pushed moment cotangent is the node's own: pull(push(Phi A))(x)_k
// = Phi_k . A(x).  So
//   k_cl_rstep_shift: A_L(x) from Q_s, Lam_k = lam_in(x - v_k)_k + Phi_k . A_L(x)
//     (as k_cl_rloss + k_cl_push4 compute it), then the shift adjoint
//     (a_g, a_m) from Lam; stores A = A_L + a_m per node;
//   k_cl_rstep_step:  l_k(x) = (lam_in(x)_k + Phi_k . A(x + v_k)) + inv_k dx_k(x),
//     then the step adjoint to lam_out = dL/dQ_(s-1),
// without the three read-modify-write passes over lam that the separate
// calls make (the two pushes are summed per node before they are pushed,
// a different rounding of the same terms).  Loss partials are added to the
// block's slot when acc_loss (the segment's loss stays on the device).
// Scheduling barriers between the phases keep the compiler from hoisting
// every load of the kernel at once (that took 256 VGPRs and one wave per
// SIMD).
// ---------------------------------------------------------------------------
template <typename T, bool LIN>
__global__ __launch_bounds__(256) void k_cl_rstep_shift(PtrList after, TruthList truth, PtrList pre, PtrList lam_in,
                                                        const float *__restrict__ C, int nx, int ny, ClNorm nm,
                                                        KParams kp, double scale, int acc_loss,
                                                        float *__restrict__ Ag, double *__restrict__ A,
                                                        double *__restrict__ lpart)
{
    __shared__ double red[4];
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    double lsum = 0.0;
    if (x < nx) {
        double a[4];
        lsum = rloss_node(static_cast<const T *>(after.p[f]), truth, f, x, y, nx, ny, nm, scale, a);
        __builtin_amdgcn_sched_barrier(0);
        const double *L = static_cast<const double *>(lam_in.p[f]);
        double l[NQ];
#pragma unroll
        for (int k = 0; k < CREAL; ++k) {
            const double in = LIN ? L[((size_t)wrap(y - nm.ivy[k], ny) * CREAL + k) * nx + wrap(x - nm.ivx[k], nx)]
                                  : 0.0;
            l[k] = in + phi_dot(nm.ivx[k], nm.ivy[k], a);
        }
        __builtin_amdgcn_sched_barrier(0);
        const size_t node = (size_t)f * ny * nx + (size_t)y * nx + x;
        double am[4];
        shift_vjp_node(static_cast<const T *>(pre.p[f]), l, C, f, x, y, nx, ny, nm, kp, Ag, am, node);
        reinterpret_cast<double4 *>(A)[node] = make_double4(a[0] + am[0], a[1] + am[1], a[2] + am[2], a[3] + am[3]);
    }
    const double tot = block_sum256(lsum, red);
    if (threadIdx.x == 0) {
        const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        lpart[b] = acc_loss ? lpart[b] + tot : tot;
    }
}

template <typename T, bool LIN>
__global__ __launch_bounds__(256) void k_cl_rstep_step(PtrList before, PtrList lam_in, const double *__restrict__ A,
                                                       const float *__restrict__ dx, PtrList lam_out, int nx,
                                                       int ny, ClNorm nm, KParams kp)
{
    const int f = blockIdx.z, y = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const size_t fbase = (size_t)f * ny * nx;
    const double *L = static_cast<const double *>(lam_in.p[f]);
    double m[4];
    step_moments(static_cast<const T *>(before.p[f]), x, y, nx, ny, kp, m);
    __builtin_amdgcn_sched_barrier(0);
    // the node's 25 input-gradient channels: seven 16-byte loads of its 128-byte row
    const float4 *d4 = reinterpret_cast<const float4 *>(dx + (fbase + (size_t)y * nx + x) * CH);
    double l[NQ];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const float4 t = d4[q];
        const float d[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * q + e;
            if (k >= CREAL) break;
            const size_t nb = fbase + (size_t)wrap(y + nm.ivy[k], ny) * nx + wrap(x + nm.ivx[k], nx);
            const double4 av = reinterpret_cast<const double4 *>(A)[nb];
            const double a[4] = {av.x, av.y, av.z, av.w};
            double v = LIN ? L[((size_t)y * CREAL + k) * nx + x] : 0.0;
            v += phi_dot(nm.ivx[k], nm.ivy[k], a);
            l[k] = v + (double)nm.in_inv[k] * (double)d[e];
        }
        __builtin_amdgcn_sched_barrier(0);     // four neighbours' loads in flight at a time
    }
    __builtin_amdgcn_sched_barrier(0);
    step_vjp_scatter(m, l, static_cast<double *>(lam_out.p[f]), x, y, nx, ny, kp);
}

// FP32 parameters -> bf16 [t][o][i] (forward) and [t][i][o] (input gradient)
__global__ __launch_bounds__(256) void k_cl_cast(const float *__restrict__ params, u16 *__restrict__ wf,
                                                 u16 *__restrict__ wt)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 3 * LAYER_W) return;
    const int layer = e / LAYER_W, r = e % LAYER_W;
    const int t = r / (CH * CH), o = (r / CH) % CH, i = r % CH;
    const u16 h = bf16_bits(params[(size_t)layer * LAYER_P + r]);
    wf[e] = h;
    wt[(size_t)layer * LAYER_W + ((size_t)t * CH + i) * CH + o] = h;
}

__global__ __launch_bounds__(256) void k_cl_adam(float *__restrict__ p, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v, float lr,
                                                 float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NPARAM) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Restriction: 4x4 block means of rho, rho u and E = rho (2 theta + |u|^2)
// of FP64 fine fields -> coarse (rho, u, theta).
__global__ __launch_bounds__(256) void k_restrict(const double *__restrict__ rho, const double *__restrict__ ux,
                                                  const double *__restrict__ uy,
                                                  const double *__restrict__ th, int fnx, int fny,
                                                  int factor, double *__restrict__ crho,
                                                  double *__restrict__ cux, double *__restrict__ cuy,
                                                  double *__restrict__ cth)
{
    const int cnx = fnx / factor;
    const int X = blockIdx.x * 256 + threadIdx.x, Y = blockIdx.y;
    if (X >= cnx) return;
    double r = 0, jx = 0, jy = 0, e = 0;
    for (int dy = 0; dy < factor; ++dy)
        for (int dx = 0; dx < factor; ++dx) {
            const size_t n = (size_t)(Y * factor + dy) * fnx + X * factor + dx;
            const double rr = rho[n], u = ux[n], w = uy[n];
            r += rr;
            jx += rr * u;
            jy += rr * w;
            e += rr * (2.0 * th[n] + u * u + w * w);
        }
    const double inv = 1.0 / r;
    const double u = jx * inv, w = jy * inv;
    const size_t c = (size_t)Y * cnx + X;
    crho[c] = r / (factor * factor);
    cux[c] = u;
    cuy[c] = w;
    cth[c] = 0.5 * (e * inv - u * u - w * w);
}

int ck(hipError_t e) { return e == hipSuccess ? PLBM_OK : PLBM_EHIP; }

} // namespace

struct plbm_closure {
    int nx = 0, ny = 0, frames = 0;
    bool f64 = false;                          // coarse populations FP64 (else FP32)
    ClNorm nm;
    u16 *wf = nullptr, *wt = nullptr;          // bf16 weights
    u16 *x0 = nullptr, *a1 = nullptr, *a2 = nullptr;
    float *y3 = nullptr;
    u16 *dy3 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    float *part = nullptr;                     // weight-gradient partials
    float *slices = nullptr;                   // their first-pass sums
    float *lpart = nullptr;                    // loss partials
    float *corr = nullptr;                     // c = s * Ph y, planes [f][k][y][x]
    float *mres = nullptr;                     // (2/N) w r, [f][y][x][j]
    double *adj4 = nullptr;                    // per-node moment cotangents (adjoints), [f][y][x][j]
    float *dx = nullptr;                       // gradient of the network input, NHWC x 32
    double *lpart64 = nullptr;                 // rollout-loss partials
    KParams kp;                                // the coarse lattice's rule
    int nwblk = 0, nlblk = 0;
    int frames_in_fwd = 0;
    const float *cast_from = nullptr;
};

namespace {

// G = sum_k s_k^2 phi_k phi_k^T and its inverse (double, Gauss-Jordan)
int set_projection(ClNorm &nm)
{
    double G[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) G[i][j] = (j - 4 == i) ? 1.0 : 0.0;
    for (int k = 0; k < CREAL; ++k) {
        const double vx = nm.vx[k], vy = nm.vy[k], s2 = (double)nm.out_scale[k] * nm.out_scale[k];
        const double phi[4] = {1.0, vx, vy, vx * vx + vy * vy};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) G[i][j] += s2 * phi[i] * phi[j];
    }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (std::fabs(G[r][col]) > std::fabs(G[piv][col])) piv = r;
        for (int j = 0; j < 8; ++j) std::swap(G[col][j], G[piv][j]);
        const double d = G[col][col];
        if (!(std::fabs(d) > 0.0)) return PLBM_ESINGULAR;
        for (int j = 0; j < 8; ++j) G[col][j] /= d;
        for (int r = 0; r < 4; ++r)
            if (r != col) {
                const double fct = G[r][col];
                for (int j = 0; j < 8; ++j) G[r][j] -= fct * G[col][j];
            }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) nm.ginv[4 * i + j] = (float)G[i][4 + j];
    return PLBM_OK;
}

template <typename P>
int make_list(PtrList &l, const P *host, int n)
{
    std::memset(&l, 0, sizeof(l));
    for (int i = 0; i < n; ++i) {
        if (!host[i]) return PLBM_EINVAL;
        l.p[i] = const_cast<void *>(static_cast<const void *>(host[i]));
    }
    return PLBM_OK;
}

void reduce_wgrad(plbm_closure *c, int nwblk, float *grad, hipStream_t st, int accumulate = 0)
{
    hipLaunchKernelGGL(k_cl_wgrad_slices, dim3((LAYER_P + 255) / 256, WR_SLICES), dim3(256), 0, st, c->part,
                       nwblk, c->slices);
    hipLaunchKernelGGL(k_cl_wgrad_reduce, dim3((LAYER_P + 255) / 256), dim3(256), 0, st, c->slices, grad,
                       accumulate);
}

// From dy3 (the gradient of the network output): the weight gradients of the
// three layers (written, or added to `grads` when accumulate), dz2 and dz1,
// and with input_grad the gradient of the network input into c->dx.
void layers_backward(plbm_closure *c, int frames, float *grads, int accumulate, hipStream_t st,
                     bool input_grad = false)
{
    const int crows = conv_rows(c->nx, c->ny, frames);
    // the input-gradient pass (with its ReLU mask read) is fastest at half the rows
    const int brows = std::max(1, crows / PLBM_CONV_BROWS_DIV);
    const dim3 gb((c->nx / 32 + 3) / 4, (c->ny + brows - 1) / brows, frames);
    const dim3 gw((c->nx / WG_SEG) * ((c->ny + WG_ROWS - 1) / WG_ROWS), 1, frames);
    const int nwblk = (int)(gw.x * gw.z);
    // layer 3: dW3 from a2 and dy3; dz2 = (W3^T dy3) * (a2 > 0)
    hipLaunchKernelGGL(k_cl_wgrad, gw, dim3(256), 0, st, c->a2, c->dy3, c->nx, c->ny, c->part);
    reduce_wgrad(c, nwblk, grads + 2 * LAYER_P, st, accumulate);
    hipLaunchKernelGGL(k_cl_conv<2>, gb, dim3(256), 0, st, c->dy3, c->wt + 2 * LAYER_W, nullptr, c->a2,
                       c->dz2, c->nx, c->ny, brows);
    // layer 2
    hipLaunchKernelGGL(k_cl_wgrad, gw, dim3(256), 0, st, c->a1, c->dz2, c->nx, c->ny, c->part);
    reduce_wgrad(c, nwblk, grads + LAYER_P, st, accumulate);
    hipLaunchKernelGGL(k_cl_conv<2>, gb, dim3(256), 0, st, c->dz2, c->wt + LAYER_W, nullptr, c->a1, c->dz1,
                       c->nx, c->ny, brows);
    // layer 1
    hipLaunchKernelGGL(k_cl_wgrad, gw, dim3(256), 0, st, c->x0, c->dz1, c->nx, c->ny, c->part);
    reduce_wgrad(c, nwblk, grads, st, accumulate);
    if (input_grad)
        hipLaunchKernelGGL(k_cl_conv<3>, gb, dim3(256), 0, st, c->dz1, c->wt, nullptr, nullptr, c->dx, c->nx,
                           c->ny, brows);
}

int cast_weights(plbm_closure *c, const float *params, hipStream_t st)
{
    hipLaunchKernelGGL(k_cl_cast, dim3((3 * LAYER_W + 255) / 256), dim3(256), 0, st, params, c->wf, c->wt);
    return ck(hipGetLastError());
}

} // namespace

extern "C" int plbm_closure_create(const plbm_desc *coarse, int frames, plbm_closure **out)
{
    if (!coarse || !out || frames < 1 || frames > MAX_FRAMES) return PLBM_EINVAL;
    *out = nullptr;
    if (coarse->dim != 2 || (coarse->storage != PLBM_F32 && coarse->storage != PLBM_F64))
        return PLBM_EUNSUPPORTED;
    const int rc0 = plbm::validate(coarse);
    if (rc0 != PLBM_OK) return rc0;
    if (coarse->nx % WG_SEG != 0 || coarse->nx < WG_SEG) return PLBM_EUNSUPPORTED;
    // the closure kernels launch one grid row per lattice row
    if (coarse->ny > 65535) return PLBM_EUNSUPPORTED;
    KParams kp;
    const int rck = make_params(coarse, kp);
    if (rck != PLBM_OK) return rck;
    plbm_closure *c = new plbm_closure();
    c->nx = coarse->nx;
    c->ny = coarse->ny;
    c->frames = frames;
    c->f64 = coarse->storage == PLBM_F64;
    c->kp = kp;
    std::memset(&c->nm, 0, sizeof(c->nm));
    for (int k = 0; k < CREAL; ++k) {
        const double vx = coarse->v[k % 5], vy = coarse->v[k / 5];
        // streaming offsets of the loss: whole nodes, one periodic wrap at most
        if (vx != std::rint(vx) || vy != std::rint(vy) || std::fabs(vx) >= coarse->nx ||
            std::fabs(vy) >= coarse->ny) {
            delete c;
            return PLBM_EUNSUPPORTED;
        }
        c->nm.vx[k] = (float)vx;
        c->nm.vy[k] = (float)vy;
        c->nm.ivx[k] = (int)vx;
        c->nm.ivy[k] = (int)vy;
        c->nm.in_inv[k] = 1.f;
        c->nm.out_scale[k] = 1.f;
    }
    for (int j = 0; j < 4; ++j) c->nm.mw2[j] = 1.f;
    if (set_projection(c->nm) != PLBM_OK) {
        delete c;
        return PLBM_ESINGULAR;
    }

    const size_t nodes = (size_t)frames * c->nx * c->ny;
    c->nwblk = frames * ((c->nx / WG_SEG) * ((c->ny + WG_ROWS - 1) / WG_ROWS));
    c->nlblk = frames * c->ny * ((c->nx + 255) / 256);
    bool ok = hipMalloc((void **)&c->wf, 3 * LAYER_W * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->wt, 3 * LAYER_W * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->x0, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->a1, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->a2, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->y3, nodes * CH * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->dy3, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->dz2, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->dz1, nodes * CH * sizeof(u16)) == hipSuccess &&
              hipMalloc((void **)&c->part, (size_t)c->nwblk * (LAYER_W + CH) * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->lpart, (size_t)c->nlblk * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->slices, (size_t)WR_SLICES * LAYER_P * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->corr, nodes * CREAL * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->mres, nodes * 4 * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->adj4, nodes * 4 * sizeof(double)) == hipSuccess &&
              hipMalloc((void **)&c->dx, nodes * CH * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&c->lpart64, (size_t)c->nlblk * sizeof(double)) == hipSuccess;
    if (!ok) {
        plbm_closure_destroy(c);
        return PLBM_EHIP;
    }
    *out = c;
    return PLBM_OK;
}

extern "C" int plbm_closure_destroy(plbm_closure *c)
{
    if (!c) return PLBM_EINVAL;
    (void)hipDeviceSynchronize();
    void *ptrs[] = {c->wf, c->wt, c->x0, c->a1, c->a2, c->y3, c->dy3, c->dz2, c->dz1, c->part,
                    c->lpart, c->corr, c->mres, c->slices, c->adj4, c->dx, c->lpart64};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
    return PLBM_OK;
}

extern "C" int plbm_closure_set_norm(plbm_closure *c, const float *in_mean, const float *in_scale,
                                     const float *out_scale, const float *moment_scale)
{
    if (!c || !in_mean || !in_scale || !out_scale || !moment_scale) return PLBM_EINVAL;
    ClNorm nm = c->nm;
    for (int j = 0; j < 4; ++j) {
        if (!(moment_scale[j] > 0.f) || !std::isfinite(moment_scale[j])) return PLBM_EINVAL;
        const double w = 1.0 / ((double)moment_scale[j] * moment_scale[j]);
        if (!std::isfinite((float)w)) return PLBM_EINVAL;
        nm.mw2[j] = (float)w;
    }
    for (int k = 0; k < CREAL; ++k) {
        if (!(in_scale[k] > 0.f) || !(out_scale[k] > 0.f) || !std::isfinite(in_mean[k]) ||
            !std::isfinite(in_scale[k]) || !std::isfinite(out_scale[k]))
            return PLBM_EINVAL;
        nm.in_mean[k] = in_mean[k];
        nm.in_inv[k] = 1.0f / in_scale[k];
        nm.out_scale[k] = out_scale[k];
    }
    const int rc = set_projection(nm);
    if (rc != PLBM_OK) return rc;
    c->nm = nm;
    return PLBM_OK;
}

extern "C" int plbm_closure_forward(plbm_closure *c, const float *params, const void *const *post,
                                    int frames, const float *noise, float noise_amp, void *stream)
{
    if (!c || !params || !post || frames < 1 || frames > c->frames || !std::isfinite(noise_amp))
        return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PtrList pl;
    int rc = make_list(pl, post, frames);
    if (rc != PLBM_OK) return rc;
    (void)hipGetLastError();
    rc = cast_weights(c, params, st);
    if (rc != PLBM_OK) return rc;
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    const int crows = conv_rows(c->nx, c->ny, frames);
    const dim3 gc((c->nx / 32 + 3) / 4, (c->ny + crows - 1) / crows, frames);
    if (c->f64)
        hipLaunchKernelGGL(k_cl_input<double>, gn, dim3(256), 0, st, pl, c->nx, c->ny, c->nm, noise, noise_amp,
                           c->x0);
    else
        hipLaunchKernelGGL(k_cl_input<float>, gn, dim3(256), 0, st, pl, c->nx, c->ny, c->nm, noise, noise_amp,
                           c->x0);
    // bias of layer l: params + l * LAYER_P + LAYER_W
    hipLaunchKernelGGL(k_cl_conv<0>, gc, dim3(256), 0, st, c->x0, c->wf, params + LAYER_W, nullptr, c->a1,
                       c->nx, c->ny, crows);
    hipLaunchKernelGGL(k_cl_conv<0>, gc, dim3(256), 0, st, c->a1, c->wf + LAYER_W, params + LAYER_P + LAYER_W,
                       nullptr, c->a2, c->nx, c->ny, crows);
    hipLaunchKernelGGL(k_cl_conv<1>, gc, dim3(256), 0, st, c->a2, c->wf + 2 * LAYER_W,
                       params + 2 * LAYER_P + LAYER_W, nullptr, c->y3, c->nx, c->ny, crows);
    c->frames_in_fwd = frames;
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_backward(plbm_closure *c, const float *params, const float *const *target,
                                     float reg, float *grads, double *loss, void *stream)
{
    if (!c || !params || !target || !grads || c->frames_in_fwd < 1 || !(reg >= 0.f) || !std::isfinite(reg))
        return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int frames = c->frames_in_fwd;
    PtrList tl;
    int rc = make_list(tl, target, frames);
    if (rc != PLBM_OK) return rc;
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    const float inv_n = 1.0f / ((float)frames * c->nx * c->ny);
    hipLaunchKernelGGL(k_cl_corr, gn, dim3(256), 0, st, c->y3, c->nx, c->ny, c->nm, reg, c->corr, c->lpart);
    hipLaunchKernelGGL(k_cl_mloss, gn, dim3(256), 0, st, c->corr, tl, c->nx, c->ny, c->nm, inv_n, c->mres,
                       c->lpart);
    hipLaunchKernelGGL(k_cl_mgrad, gn, dim3(256), 0, st, c->mres, c->y3, c->nx, c->ny, c->nm, 2.f * reg * inv_n,
                       c->dy3);
    layers_backward(c, frames, grads, 0, st);
    rc = ck(hipGetLastError());
    if (rc != PLBM_OK || !loss) return rc;
    const int nl = (int)(gn.x * gn.y * gn.z);
    std::vector<float> h(nl);
    rc = ck(hipMemcpyAsync(h.data(), c->lpart, nl * sizeof(float), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = ck(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    double s = 0.0;
    for (float v : h) s += v;
    *loss = s * inv_n;
    return std::isfinite(*loss) ? PLBM_OK : PLBM_ENONFINITE;
}

extern "C" int plbm_closure_adam(plbm_closure *c, float *params, const float *grads, float *m, float *v,
                                 int t, float lr, float b1, float b2, float eps, void *stream)
{
    if (!c || !params || !grads || !m || !v || t < 1) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_cl_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, grads, m, v, lr, b1,
                       b2, eps, c1, c2);
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_apply(plbm_closure *c, void *const *post, int frames, float bound,
                                  unsigned *skipped, void *stream)
{
    if (!c || !post || frames < 1 || frames != c->frames_in_fwd || !(bound > 0.f)) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PtrList pl;
    const int rc = make_list(pl, post, frames);
    if (rc != PLBM_OK) return rc;
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    hipLaunchKernelGGL(k_cl_corr_apply, gn, dim3(256), 0, st, c->y3, c->nx, c->ny, c->nm, bound, c->corr, skipped);
    if (c->f64)
        hipLaunchKernelGGL(k_cl_shift<double>, gn, dim3(256), 0, st, pl, c->corr, c->nx, c->ny, c->nm, c->kp);
    else
        hipLaunchKernelGGL(k_cl_shift<float>, gn, dim3(256), 0, st, pl, c->corr, c->nx, c->ny, c->nm, c->kp);
    return ck(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Training through coarse steps (adjoints)
// ---------------------------------------------------------------------------
extern "C" int plbm_step_vjp(const plbm_desc *d, const void *post, const double *lam, double *out,
                             void *stream)
{
    if (!d || d->dim != 2 || (d->storage != PLBM_F64 && d->storage != PLBM_F32)) return PLBM_EUNSUPPORTED;
    if (plbm::gen_handles(d) || d->q1d != Q) return PLBM_EUNSUPPORTED;
    KParams kp;
    const int rc = make_params(d, kp);
    if (rc != PLBM_OK) return rc;
    if (!post || !lam || !out || lam == out || d->ny > 65535) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const dim3 g((d->nx + 255) / 256, d->ny);
    if (d->storage == PLBM_F64)
        hipLaunchKernelGGL(k_step_vjp<double>, g, dim3(256), 0, st, static_cast<const double *>(post), lam, out,
                           d->nx, d->ny, kp);
    else
        hipLaunchKernelGGL(k_step_vjp<float>, g, dim3(256), 0, st, static_cast<const float *>(post), lam, out,
                           d->nx, d->ny, kp);
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_rollout_loss(plbm_closure *c, void *const *post, const double *const *truth,
                                         int frames, double scale, double *const *lam, double *loss,
                                         void *stream)
{
    if (!c || !post || !truth || frames < 1 || frames > c->frames || !(scale > 0.0) || !std::isfinite(scale))
        return PLBM_EINVAL;
    PtrList pl, ll;
    int rc = make_list(pl, post, frames);
    if (rc != PLBM_OK) return rc;
    if (lam) {
        rc = make_list(ll, lam, frames);
        if (rc != PLBM_OK) return rc;
    }
    TruthList tl;
    for (int i = 0; i < 4 * frames; ++i) {
        if (!truth[i]) return PLBM_EINVAL;
        tl.p[i] = truth[i];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    if (c->f64)
        hipLaunchKernelGGL(k_cl_rloss<double>, gn, dim3(256), 0, st, pl, tl, c->nx, c->ny, c->nm, scale, c->adj4,
                           c->lpart64);
    else
        hipLaunchKernelGGL(k_cl_rloss<float>, gn, dim3(256), 0, st, pl, tl, c->nx, c->ny, c->nm, scale, c->adj4,
                           c->lpart64);
    if (lam) hipLaunchKernelGGL(k_cl_push4, gn, dim3(256), 0, st, c->adj4, ll, c->nx, c->ny, c->nm);
    rc = ck(hipGetLastError());
    if (rc != PLBM_OK || !loss) return rc;
    const int nl = (int)(gn.x * gn.y * gn.z);
    std::vector<double> h(nl);
    rc = ck(hipMemcpyAsync(h.data(), c->lpart64, nl * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = ck(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    double sum = 0.0;
    for (double v : h) sum += v;
    *loss = sum;
    return std::isfinite(sum) ? PLBM_OK : PLBM_ENONFINITE;
}

extern "C" int plbm_closure_apply_vjp(plbm_closure *c, void *const *post, double *const *lam, int frames,
                                      void *stream)
{
    if (!c || !post || !lam || frames < 1 || frames != c->frames_in_fwd) return PLBM_EINVAL;
    PtrList pl, ll;
    int rc = make_list(pl, post, frames);
    if (rc == PLBM_OK) rc = make_list(ll, lam, frames);
    if (rc != PLBM_OK) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    // the correction of the last forward pass, without the fallback bound
    hipLaunchKernelGGL(k_cl_corr_apply, gn, dim3(256), 0, st, c->y3, c->nx, c->ny, c->nm, INFINITY, c->corr,
                       nullptr);
    if (c->f64)
        hipLaunchKernelGGL(k_cl_shift_vjp<double>, gn, dim3(256), 0, st, pl, ll, c->corr, c->nx, c->ny, c->nm,
                           c->kp, c->mres, c->adj4);
    else
        hipLaunchKernelGGL(k_cl_shift_vjp<float>, gn, dim3(256), 0, st, pl, ll, c->corr, c->nx, c->ny, c->nm,
                           c->kp, c->mres, c->adj4);
    hipLaunchKernelGGL(k_cl_push4, gn, dim3(256), 0, st, c->adj4, ll, c->nx, c->ny, c->nm);
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_backward_vjp(plbm_closure *c, const float *params, float reg, float *grads,
                                         int accumulate, double *const *lam, void *stream)
{
    if (!c || !params || !grads || c->frames_in_fwd < 1 || !(reg >= 0.f) || !std::isfinite(reg))
        return PLBM_EINVAL;
    const int frames = c->frames_in_fwd;
    PtrList ll;
    if (lam) {
        const int rc = make_list(ll, lam, frames);
        if (rc != PLBM_OK) return rc;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    const float inv_n = 1.0f / ((float)frames * c->nx * c->ny);
    hipLaunchKernelGGL(k_cl_mgrad, gn, dim3(256), 0, st, c->mres, c->y3, c->nx, c->ny, c->nm, 2.f * reg * inv_n,
                       c->dy3);
    layers_backward(c, frames, grads, accumulate ? 1 : 0, st, lam != nullptr);
    if (lam) hipLaunchKernelGGL(k_cl_input_vjp, gn, dim3(256), 0, st, c->dx, ll, c->nx, c->ny, c->nm);
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_rollout_vjp(plbm_closure *c, const plbm_desc *coarse, const float *params, float reg,
                                        float *grads, int accumulate, void *const *after,
                                        const double *const *truth, double scale, void *const *pre,
                                        const void *const *before, const double *const *lam_in,
                                        double *const *lam_out, int frames, double *loss, void *stream)
{
    if (!c || !coarse || !params || !grads || !after || !truth || !pre || frames < 1 ||
        frames != c->frames_in_fwd || !(scale > 0.0) || !std::isfinite(scale) || !(reg >= 0.f) ||
        !std::isfinite(reg))
        return PLBM_EINVAL;
    // the coarse lattice the step adjoint runs on: the closure's shape, storage and velocities
    if (coarse->dim != 2 || coarse->nx != c->nx || coarse->ny != c->ny ||
        (coarse->storage == PLBM_F64) != c->f64 || (coarse->storage != PLBM_F64 && coarse->storage != PLBM_F32) ||
        plbm::gen_handles(coarse) || coarse->q1d != Q)
        return PLBM_EINVAL;
    KParams kp;
    int rc = make_params(coarse, kp);
    if (rc != PLBM_OK) return rc;
    for (int k = 0; k < CREAL; ++k)
        if (kp.sx[k % Q] != c->nm.ivx[k] || kp.sx[k / Q] != c->nm.ivy[k]) return PLBM_EINVAL;
    PtrList al, pl, bl, li, lo;
    rc = make_list(al, after, frames);
    if (rc == PLBM_OK) rc = make_list(pl, pre, frames);
    if (rc != PLBM_OK) return rc;
    std::memset(&li, 0, sizeof(li));
    if (lam_in) {
        rc = make_list(li, lam_in, frames);
        if (rc != PLBM_OK) return rc;
    }
    if (lam_out) {
        if (!before) return PLBM_EINVAL;
        rc = make_list(bl, before, frames);
        if (rc == PLBM_OK) rc = make_list(lo, lam_out, frames);
        if (rc != PLBM_OK) return rc;
        for (int i = 0; i < frames; ++i)
            if (lam_in && lam_in[i] == lam_out[i]) return PLBM_EINVAL;
    }
    TruthList tl;
    for (int i = 0; i < 4 * frames; ++i) {
        if (!truth[i]) return PLBM_EINVAL;
        tl.p[i] = truth[i];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const dim3 gn((c->nx + 255) / 256, c->ny, frames);
    const float inv_n = 1.0f / ((float)frames * c->nx * c->ny);
    // the correction of the last forward pass, without the fallback bound
    hipLaunchKernelGGL(k_cl_corr_apply, gn, dim3(256), 0, st, c->y3, c->nx, c->ny, c->nm, INFINITY, c->corr,
                       nullptr);
    // lam_in == NULL (zero) and FP32 / FP64 storage are template cases
    auto shift_kernel = c->f64 ? (lam_in ? k_cl_rstep_shift<double, true> : k_cl_rstep_shift<double, false>)
                               : (lam_in ? k_cl_rstep_shift<float, true> : k_cl_rstep_shift<float, false>);
    hipLaunchKernelGGL(shift_kernel, gn, dim3(256), 0, st, al, tl, pl, li, c->corr, c->nx, c->ny, c->nm, c->kp,
                       scale, accumulate ? 1 : 0, c->mres, c->adj4, c->lpart64);
    hipLaunchKernelGGL(k_cl_mgrad, gn, dim3(256), 0, st, c->mres, c->y3, c->nx, c->ny, c->nm, 2.f * reg * inv_n,
                       c->dy3);
    layers_backward(c, frames, grads, accumulate ? 1 : 0, st, lam_out != nullptr);
    if (lam_out) {
        auto step_kernel = c->f64 ? (lam_in ? k_cl_rstep_step<double, true> : k_cl_rstep_step<double, false>)
                                  : (lam_in ? k_cl_rstep_step<float, true> : k_cl_rstep_step<float, false>);
        hipLaunchKernelGGL(step_kernel, gn, dim3(256), 0, st, bl, li, c->adj4, c->dx, lo, c->nx, c->ny, c->nm, kp);
    }
    rc = ck(hipGetLastError());
    if (rc != PLBM_OK || !loss) return rc;
    const int nl = (int)(gn.x * gn.y * gn.z);
    std::vector<double> h(nl);
    rc = ck(hipMemcpyAsync(h.data(), c->lpart64, nl * sizeof(double), hipMemcpyDeviceToHost, st));
    if (rc == PLBM_OK) rc = ck(hipStreamSynchronize(st));
    if (rc != PLBM_OK) return rc;
    double sum = 0.0;
    for (double v : h) sum += v;
    *loss = sum;
    return std::isfinite(sum) ? PLBM_OK : PLBM_ENONFINITE;
}

extern "C" int plbm_closure_activation(const plbm_closure *c, int which, const void **ptr, size_t *bytes)
{
    if (!c || !ptr) return PLBM_EINVAL;
    const size_t nodes = (size_t)c->frames * c->nx * c->ny;
    const void *p = nullptr;
    size_t b = nodes * CH * sizeof(u16);
    switch (which) {
    case 0: p = c->x0; break;
    case 1: p = c->a1; break;
    case 2: p = c->a2; break;
    case 3: p = c->y3; b = nodes * CH * sizeof(float); break;
    case 4: p = c->dy3; break;
    case 5: p = c->dz2; break;
    case 6: p = c->dz1; break;
    case 7: p = c->corr; b = nodes * CREAL * sizeof(float); break;
    case 8: p = c->mres; b = nodes * 4 * sizeof(float); break;
    case 10: p = c->adj4; b = nodes * 4 * sizeof(double); break;
    case 11: p = c->dx; b = nodes * CH * sizeof(float); break;
    default: return PLBM_EINVAL;
    }
    *ptr = p;
    if (bytes) *bytes = b;
    return PLBM_OK;
}

extern "C" int plbm_restrict(const double *rho, const double *ux, const double *uy, const double *theta,
                             int fnx, int fny, int factor, double *crho, double *cux, double *cuy,
                             double *ctheta, void *stream)
{
    if (!rho || !ux || !uy || !theta || !crho || !cux || !cuy || !ctheta) return PLBM_EINVAL;
    if (factor < 1 || fnx < factor || fny < factor || fnx % factor || fny % factor) return PLBM_EINVAL;
    if (fny / factor > 65535) return PLBM_EINVAL;     // one grid row per coarse row
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int cnx = fnx / factor, cny = fny / factor;
    hipLaunchKernelGGL(k_restrict, dim3((cnx + 255) / 256, cny), dim3(256), 0, st, rho, ux, uy, theta, fnx,
                       fny, factor, crho, cux, cuy, ctheta);
    return ck(hipGetLastError());
}

extern "C" int plbm_closure_target(const double *const *fields, size_t nodes, float *out, void *stream)
{
    if (!fields || !out || nodes == 0 || nodes > ((size_t)1 << 30)) return PLBM_EINVAL;
    Fields16 F;
    for (int i = 0; i < 16; ++i) {
        if (!fields[i]) return PLBM_EINVAL;
        F.p[i] = fields[i];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_cl_target, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, st, F, nodes, out);
    return ck(hipGetLastError());
}
