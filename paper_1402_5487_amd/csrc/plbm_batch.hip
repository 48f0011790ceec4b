// libplbm batching form: many independent D2Q25 lattices of uneven sizes and
// parameters advanced by one launch per step.
//
//  * All lattices live in one device pool, two FP32 population buffers each,
//    in the row-interleaved layout of the single-lattice step.
//  * A host-built work list holds every tile of every lattice.  A tile is W
//    nodes wide (64, 128 or 256: one to four waves per row) and 256/W rows
//    per pass, R passes (1, 2, 4 or 8); its shape is chosen per size class.
//    Each entry carries its lattice's buffers and parameters.  One kernel
//    launch walks the whole list, each block taking tile
//    it * gridDim.x + (XCD-contiguous slot), so a grid of one block per tile
//    and a persistent grid of a few blocks per CU are the same kernel.
//  * The per-node work is the single-lattice row stepper with the lattice's
//    own size and relaxation constant.
//  * plbm_batch_step replays a captured hipGraph of `graph_steps` consecutive
//    steps (alternating buffers), so the host issues one graph launch per
//    graph_steps steps.  No memset is recorded in the graph.
//  * Lattices of one size form a shape group: back to back in the pool, one
//    tile shape, so a tile index decodes arithmetically from a table passed
//    as a kernel argument (up to 48 sizes; beyond that a work list in device
//    memory names every tile).
//  * plbm_batch_autotune times a few tile policies (per-class shapes) with
//    the grid / occupancy options on the whole batch and keeps the choice in
//    a small JSON cache keyed by (architecture, storage, size class).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "plbm_device.h"
#include "plbm_internal.h"

struct plbm_batch;

namespace {

struct BLat {
    float *buf[2];
    int nx, ny;
    float omega;
    int pad;
};

// A work-list entry carries its lattice's buffers and parameters, so a block
// needs one scalar load before it starts streaming.
struct BTile {
    float *buf[2];
    int nx, ny;
    float omega;
    int x0, y0;
    int shape;          // log2(W / 64) in bits 0..1, R in bits 8..15
};


__device__ __forceinline__ void batch_tile(const BTile &t, const KParams &proto, int parity)
{
    KParams q = proto;
    q.nx = t.nx;
    q.ny = t.ny;
    q.r32.omega = t.omega;
    const int lw = t.shape & 3, R = (t.shape >> 8) & 0xff;
    const int wpr = 1 << lw;                       // waves per row
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xb = t.x0 + (w & (wpr - 1)) * 64 + lane;
    const int y_first = t.y0 + (w >> lw);
    const int y_step = 4 >> lw;                    // rows per pass
    double acc[4];
    // select the buffers without indexing t.buf by a runtime value: such an
    // index makes the compiler place the tile in LDS (10 KB per workgroup)
    float *const b0 = t.buf[0], *const b1 = t.buf[1];
    step_rows<StF32, 1, false>(parity ? b1 : b0, parity ? b0 : b1, q, xb, y_first, y_step, R, acc);
}

__global__ __launch_bounds__(TX) void k_step_batch(const BTile *__restrict__ tiles, int ntiles,
                                                   KParams proto, int parity)
{
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int i = slot; i < ntiles; i += gridDim.x) {
        const BTile t = tiles[i];
        batch_tile(t, proto, parity);
    }
}

// Shape groups: the lattices of one size (nx, ny) sit back to back in the
// pool with a uniform stride and share a tile shape, so a tile index decodes
// arithmetically into (group, lattice, x0, y0) from a table passed as a
// kernel argument.  A workgroup then starts streaming at once: the only
// memory read besides the populations is the lattice's relaxation constant,
// which nothing waits for until the collision.  (A work-list entry read from
// global memory first costs about half the throughput at 256-node tiles.)
constexpr int MAX_GROUPS = 48;

struct BGroup {
    long long base;         // pool element offset of the group's first buffer 0
    long long stride;       // elements from one lattice's buffer 0 to the next
    long long half;         // elements from a lattice's buffer 0 to its buffer 1
    int first_lat;          // position of the group's first lattice in the omega table
    int tiles_x, tiles_per_lat;
    int nx, ny;
    int shape;              // log2(W / 64) in bits 0..1, R in bits 8..15
};

struct BGroups {
    int count, ntiles;
    int first[MAX_GROUPS];  // first tile of each group; INT_MAX past count
    BGroup g[MAX_GROUPS];
};

__global__ __launch_bounds__(TX) void k_step_groups(float *__restrict__ pool, const float *__restrict__ omegas,
                                                    BGroups G, KParams proto, int parity)
{
    const int slot = xcd_tile(blockIdx.x, gridDim.x);
#pragma unroll 1
    for (int t = slot; t < G.ntiles; t += gridDim.x) {
        int gi = 0;
#pragma unroll
        for (int k = 1; k < MAX_GROUPS; ++k) gi += (t >= G.first[k]) ? 1 : 0;
        const BGroup &gr = G.g[gi];
        const int local = t - G.first[gi];
        const int lat = local / gr.tiles_per_lat;
        const int lt = local - lat * gr.tiles_per_lat;
        const int ty = lt / gr.tiles_x, tx = lt - ty * gr.tiles_x;
        const int lw = gr.shape & 3, R = (gr.shape >> 8) & 0xff;
        BTile tile;
        tile.buf[0] = pool + gr.base + (long long)lat * gr.stride;
        tile.buf[1] = tile.buf[0] + gr.half;
        tile.nx = gr.nx;
        tile.ny = gr.ny;
        tile.omega = omegas[gr.first_lat + lat];
        tile.x0 = tx * (64 << lw);
        tile.y0 = ty * ((4 >> lw) * R);
        tile.shape = gr.shape;
        batch_tile(tile, proto, parity);
    }
}

__global__ void k_fill(float *p, size_t n, float v)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int hipck(hipError_t e) { return e == hipSuccess ? PLBM_OK : PLBM_EHIP; }

struct ShapeChoice {
    int w = 256, r = 1;
};

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

} // namespace

struct plbm_batch {
    plbm_desc proto;                 // velocity set, table, storage
    KParams kp;                      // kernel parameters shared by all lattices
    std::vector<plbm_lattice_spec> specs;
    std::vector<BLat> lats;          // host copy of the lattice table
    BTile *d_tiles = nullptr;        // work list (when the sizes exceed MAX_GROUPS)
    int ntiles = 0;
    // shape groups: lattices of one size, contiguous in the pool
    bool grouped = false;
    std::vector<std::vector<int>> group_lats;   // lattice indices per group
    std::vector<long long> group_base;          // pool offset of each group
    float *d_omega = nullptr;        // omega per lattice, in group order
    BGroups groups;
    float *pool = nullptr;
    size_t pool_elems = 0;
    int parity = 0;                  // buffer holding the current state
    std::map<int, ShapeChoice> shape;   // per size class (max(nx, ny))
    int grid_mode = 0;               // 0: one block per tile; k > 0: k blocks per CU
    int lds = 80 * 1024;             // LDS reserved per block (occupancy cap)
    int cus = 256;
    int graph_steps = 8;
    hipStream_t capture = nullptr;
    hipGraphExec_t exec = nullptr;
    bool tuned = false;
};

namespace {

int size_class(const plbm_lattice_spec &s) { return std::max(s.nx, s.ny); }

// one population buffer, rounded up to 64 elements (256-byte alignment)
size_t padded_elems(const plbm_lattice_spec &s)
{
    const size_t n = (size_t)NQ * s.nx * s.ny;
    return (n + 63) / 64 * 64;
}

BTile make_tile(const BLat &L, int x0, int y0, int shape)
{
    BTile t;
    t.buf[0] = L.buf[0];
    t.buf[1] = L.buf[1];
    t.nx = L.nx;
    t.ny = L.ny;
    t.omega = L.omega;
    t.x0 = x0;
    t.y0 = y0;
    t.shape = shape;
    return t;
}

ShapeChoice shape_of(const plbm_batch *b, int cls)
{
    const auto it = b->shape.find(cls);
    return it == b->shape.end() ? ShapeChoice{} : it->second;
}

int shape_bits(const ShapeChoice &sc)
{
    const int lw = sc.w == 64 ? 0 : (sc.w == 128 ? 1 : 2);
    return lw | (sc.r << 8);
}

// The group table for the groups in `which` (all when empty), each with the
// tile shape of its size class, or with `force` when given.
BGroups make_groups(const plbm_batch *b, const std::vector<int> &which, const ShapeChoice *force)
{
    BGroups G;
    std::memset(&G, 0, sizeof(G));
    int tiles = 0, lat0 = 0, n = 0;
    for (size_t gi = 0; gi < b->group_lats.size(); ++gi) {
        const bool take = which.empty() || std::find(which.begin(), which.end(), (int)gi) != which.end();
        const plbm_lattice_spec &sp = b->specs[b->group_lats[gi][0]];
        if (take) {
            const ShapeChoice sc = force ? *force : shape_of(b, size_class(sp));
            const int h = (256 / sc.w) * sc.r;
            BGroup &g = G.g[n];
            g.base = b->group_base[gi];
            g.half = (long long)padded_elems(sp);
            g.stride = 2 * g.half;
            g.first_lat = lat0;
            g.tiles_x = (sp.nx + sc.w - 1) / sc.w;
            g.tiles_per_lat = g.tiles_x * ((sp.ny + h - 1) / h);
            g.nx = sp.nx;
            g.ny = sp.ny;
            g.shape = shape_bits(sc);
            G.first[n] = tiles;
            tiles += g.tiles_per_lat * (int)b->group_lats[gi].size();
            ++n;
        }
        lat0 += (int)b->group_lats[gi].size();
    }
    G.count = n;
    G.ntiles = tiles;
    for (int k = n; k < MAX_GROUPS; ++k) G.first[k] = 0x7fffffff;
    return G;
}

int build_tiles(plbm_batch *b)
{
    if (b->grouped) {
        b->groups = make_groups(b, {}, nullptr);
        b->ntiles = b->groups.ntiles;
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        return PLBM_OK;
    }
    std::vector<BTile> tiles;
    for (size_t i = 0; i < b->specs.size(); ++i) {
        const ShapeChoice sc = b->shape.count(size_class(b->specs[i]))
                                   ? b->shape[size_class(b->specs[i])]
                                   : ShapeChoice{};
        const int lw = sc.w == 64 ? 0 : (sc.w == 128 ? 1 : 2);
        const int h = (256 / sc.w) * sc.r;
        for (int y0 = 0; y0 < b->specs[i].ny; y0 += h)
            for (int x0 = 0; x0 < b->specs[i].nx; x0 += sc.w)
                tiles.push_back(make_tile(b->lats[i], x0, y0, lw | (sc.r << 8)));
    }
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    b->ntiles = (int)tiles.size();
    if (hipMalloc((void **)&b->d_tiles, tiles.size() * sizeof(BTile)) != hipSuccess) return PLBM_EHIP;
    if (hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BTile), hipMemcpyHostToDevice) !=
        hipSuccess)
        return PLBM_EHIP;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    return PLBM_OK;
}

int grid_of(const plbm_batch *b, int ntiles)
{
    if (b->grid_mode <= 0) return grid_for(ntiles);
    return std::min(ntiles, b->grid_mode * b->cus);
}

int launch_batch(plbm_batch *b, const BTile *tiles, int ntiles, int parity, hipStream_t st)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_step_batch, dim3(grid_of(b, ntiles)), dim3(TX), b->lds, st, tiles, ntiles,
                       b->kp, parity);
    return hipck(hipGetLastError());
}

int launch_groups(plbm_batch *b, const BGroups &G, int parity, hipStream_t st)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_step_groups, dim3(grid_of(b, G.ntiles)), dim3(TX), b->lds, st, b->pool, b->d_omega, G,
                       b->kp, parity);
    return hipck(hipGetLastError());
}

// one step of the whole batch in its current form
int launch_step(plbm_batch *b, int parity, hipStream_t st)
{
    return b->grouped ? launch_groups(b, b->groups, parity, st)
                      : launch_batch(b, b->d_tiles, b->ntiles, parity, st);
}

// Cache file: {"entries": [{"arch": "...", "storage": "f32", "class": 64, "w": 128,
// "r": 2}, ...], "grid": {"arch": "...", "mode": 0, "lds": 81920}} -- written by
// this code only, read back with a tolerant scanner.
std::string cache_key(const std::string &arch, int cls)
{
    return arch + "/f32/" + std::to_string(cls);
}

bool read_cache(const char *path, const std::string &arch, std::map<std::string, ShapeChoice> &out,
                int &mode, int &lds, bool &have_grid)
{
    have_grid = false;
    if (!path) return false;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return false;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) txt.append(buf, n);
    std::fclose(fp);
    size_t pos = 0;
    while ((pos = txt.find("{\"arch\": \"", pos)) != std::string::npos) {
        const size_t e = txt.find('}', pos);
        if (e == std::string::npos) break;
        const std::string obj = txt.substr(pos, e - pos + 1);
        pos = e;
        char a[64] = {0}, stor[16] = {0};
        int cls = 0, w = 0, r = 0, m = 0, l = 0;
        if (std::sscanf(obj.c_str(), "{\"arch\": \"%63[^\"]\", \"storage\": \"%15[^\"]\", \"class\": %d, "
                                     "\"w\": %d, \"r\": %d}", a, stor, &cls, &w, &r) == 5) {
            if (std::string(stor) == "f32" && (w == 64 || w == 128 || w == 256) && r >= 1 && r <= 8 &&
                (r & (r - 1)) == 0)
                out[std::string(a) + "/f32/" + std::to_string(cls)] = ShapeChoice{w, r};
        } else if (std::sscanf(obj.c_str(), "{\"arch\": \"%63[^\"]\", \"mode\": %d, \"lds\": %d}", a, &m,
                               &l) == 3) {
            if (arch == a && m >= 0 && m <= 64 && l >= 0 && l <= 160 * 1024) {
                mode = m;
                lds = l;
                have_grid = true;
            }
        }
    }
    return true;
}

void write_cache(const char *path, const std::map<std::string, ShapeChoice> &all,
                 const std::string &arch, int mode, int lds)
{
    if (!path) return;
    FILE *fp = std::fopen(path, "w");
    if (!fp) return;
    std::fprintf(fp, "{\"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : all) {
        const std::string &k = kv.first;
        const size_t s1 = k.find('/'), s2 = k.rfind('/');
        std::fprintf(fp, "  {\"arch\": \"%s\", \"storage\": \"f32\", \"class\": %s, \"w\": %d, \"r\": %d}%s\n",
                     k.substr(0, s1).c_str(), k.substr(s2 + 1).c_str(), kv.second.w, kv.second.r,
                     ++i < all.size() ? "," : "");
    }
    std::fprintf(fp, "],\n \"grid\": {\"arch\": \"%s\", \"mode\": %d, \"lds\": %d}}\n", arch.c_str(), mode,
                 lds);
    std::fclose(fp);
}

// Median-free timing: best of three runs of `reps` launches of `one(parity)`.
template <class F>
int time_runs(F one, int reps, hipStream_t st, float &ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PLBM_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PLBM_EHIP;
    }
    int rc = PLBM_OK;
    ms = 1e30f;
    for (int trial = 0; trial < 3 && rc == PLBM_OK; ++trial) {
        rc = hipck(hipEventRecord(e0, st));
        for (int i = 0; i < reps && rc == PLBM_OK; ++i) rc = one(i & 1);
        if (rc == PLBM_OK) rc = hipck(hipEventRecord(e1, st));
        if (rc == PLBM_OK) rc = hipck(hipEventSynchronize(e1));
        float t = 0.0f;
        if (rc == PLBM_OK) rc = hipck(hipEventElapsedTime(&t, e0, e1));
        if (rc == PLBM_OK) ms = std::min(ms, t / reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

} // namespace

extern "C" int plbm_batch_create(const plbm_desc *proto, const plbm_lattice_spec *specs, int count,
                                 plbm_batch **out)
{
    if (!proto || !specs || !out || count <= 0) return PLBM_EINVAL;
    *out = nullptr;
    if (proto->dim != 2 || proto->storage != PLBM_F32) return PLBM_EUNSUPPORTED;
    plbm_batch *b = new plbm_batch();
    b->proto = *proto;
    b->specs.assign(specs, specs + count);
    size_t elems = 0;
    for (int i = 0; i < count; ++i) {
        plbm_desc d = *proto;
        d.nx = specs[i].nx;
        d.ny = specs[i].ny;
        d.omega = specs[i].omega;
        const int rc = plbm::validate(&d);
        if (rc != PLBM_OK) {
            delete b;
            return rc;
        }
        elems += 2 * padded_elems(specs[i]);
    }
    elems += 64;        // slack so that 16-byte rounded copies stay inside the pool
    plbm_desc d0 = *proto;
    d0.nx = specs[0].nx;
    d0.ny = specs[0].ny;
    d0.omega = specs[0].omega;
    int rc = make_params(&d0, b->kp);
    if (rc != PLBM_OK) {
        delete b;
        return rc;
    }
    b->pool_elems = elems;
    if (hipMalloc((void **)&b->pool, elems * sizeof(float)) != hipSuccess) {
        delete b;
        return PLBM_EHIP;
    }
    // shape groups: lattices of one size, in order of first appearance
    {
        std::map<std::pair<int, int>, int> gid;
        for (int i = 0; i < count; ++i) {
            const auto key = std::make_pair(specs[i].nx, specs[i].ny);
            auto it = gid.find(key);
            if (it == gid.end()) {
                it = gid.emplace(key, (int)b->group_lats.size()).first;
                b->group_lats.emplace_back();
            }
            b->group_lats[it->second].push_back(i);
        }
        b->grouped = (int)b->group_lats.size() <= MAX_GROUPS;
    }
    // pool layout: group by group when grouped (uniform stride inside a
    // group), else in spec order
    std::vector<int> order;
    if (b->grouped) {
        for (const auto &gl : b->group_lats) order.insert(order.end(), gl.begin(), gl.end());
    } else {
        for (int i = 0; i < count; ++i) order.push_back(i);
    }
    b->lats.assign(count, BLat{});
    std::vector<size_t> offset(count, 0);
    size_t off = 0;
    for (int i : order) {
        offset[i] = off;
        off += 2 * padded_elems(specs[i]);
    }
    for (int i = 0; i < count; ++i) {
        BLat &L = b->lats[i];
        const size_t n = padded_elems(specs[i]);
        L.buf[0] = b->pool + offset[i];
        L.buf[1] = b->pool + offset[i] + n;
        L.nx = specs[i].nx;
        L.ny = specs[i].ny;
        L.omega = (float)specs[i].omega;
        L.pad = 0;
    }
    if (b->grouped) {
        for (const auto &gl : b->group_lats) b->group_base.push_back((long long)offset[gl[0]]);
        std::vector<float> om;
        for (int i : order) om.push_back((float)specs[i].omega);
        if (hipMalloc((void **)&b->d_omega, om.size() * sizeof(float)) != hipSuccess ||
            hipMemcpy(b->d_omega, om.data(), om.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            plbm_batch_destroy(b);
            return PLBM_EHIP;
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
        plbm_batch_destroy(b);
        return PLBM_EHIP;
    }
    rc = build_tiles(b);
    if (rc != PLBM_OK) {
        plbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PLBM_OK;
}

extern "C" int plbm_batch_destroy(plbm_batch *b)
{
    if (!b) return PLBM_EINVAL;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_omega) (void)hipFree(b->d_omega);
    if (b->pool) (void)hipFree(b->pool);
    delete b;
    return PLBM_OK;
}

extern "C" int plbm_batch_lattice(const plbm_batch *b, int i, plbm_desc *desc, void **f)
{
    if (!b || i < 0 || i >= (int)b->specs.size()) return PLBM_EINVAL;
    if (desc) {
        *desc = b->proto;
        desc->nx = b->specs[i].nx;
        desc->ny = b->specs[i].ny;
        desc->omega = b->specs[i].omega;
    }
    if (f) *f = b->lats[i].buf[b->parity];
    return PLBM_OK;
}

extern "C" int plbm_batch_init(plbm_batch *b, int i, const double *rho, const double *ux,
                               const double *uy, const double *theta, void *stream)
{
    plbm_desc d;
    void *f = nullptr;
    const int rc = plbm_batch_lattice(b, i, &d, &f);
    if (rc != PLBM_OK) return rc;
    return plbm_init(&d, rho, ux, uy, theta, f, stream);
}

extern "C" int plbm_batch_moments(const plbm_batch *b, int i, double *rho, double *ux, double *uy,
                                  double *theta, double *sums, void *stream)
{
    plbm_desc d;
    void *f = nullptr;
    const int rc = plbm_batch_lattice(b, i, &d, &f);
    if (rc != PLBM_OK) return rc;
    return plbm_moments(&d, f, rho, ux, uy, theta, sums, stream);
}

extern "C" int plbm_batch_set_graph_steps(plbm_batch *b, int steps)
{
    if (!b || steps < 0 || (steps & 1) || steps > 64) return PLBM_EINVAL;
    b->graph_steps = steps;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    return PLBM_OK;
}

extern "C" int plbm_batch_step(plbm_batch *b, int nsteps, void *stream)
{
    if (!b || nsteps < 0) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = PLBM_OK;
    int left = nsteps;
    if (b->graph_steps >= 2 && left >= b->graph_steps) {
        if (!b->exec) {
            // record graph_steps launches (even: the state returns to the same buffer)
            hipGraph_t g = nullptr;
            rc = hipck(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
            if (rc != PLBM_OK) return rc;
            for (int s = 0; s < b->graph_steps && rc == PLBM_OK; ++s)
                rc = launch_step(b, s & 1, b->capture);
            const int rc_end = hipck(hipStreamEndCapture(b->capture, &g));
            if (rc == PLBM_OK) rc = rc_end;
            if (rc == PLBM_OK) rc = hipck(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
            if (g) (void)hipGraphDestroy(g);
            if (rc != PLBM_OK) return rc;
        }
        // the recorded graph starts from buffer 0
        if (b->parity != 0) {
            rc = launch_step(b, b->parity, st);
            if (rc != PLBM_OK) return rc;
            b->parity ^= 1;
            --left;
        }
        while (left >= b->graph_steps) {
            rc = hipck(hipGraphLaunch(b->exec, st));
            if (rc != PLBM_OK) return rc;
            left -= b->graph_steps;
        }
    }
    for (; left > 0; --left) {
        rc = launch_step(b, b->parity, st);
        if (rc != PLBM_OK) return rc;
        b->parity ^= 1;
    }
    return PLBM_OK;
}

extern "C" int plbm_batch_autotune(plbm_batch *b, const char *cache_path, void *stream)
{
    if (!b) return PLBM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const std::string arch = arch_name();
    std::map<std::string, ShapeChoice> cache;
    int mode = b->grid_mode, lds = b->lds;
    bool have_grid = false;
    read_cache(cache_path, arch, cache, mode, lds, have_grid);

    // timing overwrites the populations: start from a harmless uniform state
    {
        const size_t blocks = (b->pool_elems + 255) / 256;
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, b->pool, b->pool_elems,
                           1.0f / NQ);
        int rc = hipck(hipGetLastError());
        if (rc != PLBM_OK) return rc;
    }
    std::map<int, std::vector<int>> classes;
    for (size_t i = 0; i < b->specs.size(); ++i) classes[size_class(b->specs[i])].push_back((int)i);

    bool cached = have_grid;
    for (const auto &kv : classes) cached = cached && cache.count(cache_key(arch, kv.first)) > 0;
    int rc = PLBM_OK;
    bool changed = false;
    if (cached) {
        for (const auto &kv : classes) b->shape[kv.first] = cache[cache_key(arch, kv.first)];
        rc = build_tiles(b);
        if (rc != PLBM_OK) return rc;
    } else {
        // Whole-batch timings of a few tile policies x occupancy caps x grid
        // modes.  (Timing one size class alone is dominated by launch overhead
        // for the small classes, and one class's shape moves the whole batch
        // by less than the timing noise, so shapes are chosen as policies.)
        auto narrow = [](int cls) { return cls <= 64 ? 64 : (cls <= 128 ? 128 : 256); };
        const int npol = 5;
        auto policy = [&](int pi, int cls) {
            switch (pi) {
            case 0: return ShapeChoice{narrow(cls), 1};
            case 1: return ShapeChoice{narrow(cls), 2};
            case 2: return ShapeChoice{64, 1};
            case 3: return ShapeChoice{64, 2};
            default: return ShapeChoice{256, 1};
            }
        };
        const int modes[3] = {0, 2, 4};
        const int ldss[3] = {0, 40 * 1024, 80 * 1024};
        float best = 1e30f;
        int best_pol = 0;
        for (int pi = 0; pi < npol; ++pi) {
            for (const auto &kv : classes) b->shape[kv.first] = policy(pi, kv.first);
            rc = build_tiles(b);
            if (rc != PLBM_OK) return rc;
            for (int mi = 0; mi < 3; ++mi)
                for (int li = 0; li < 3; ++li) {
                    b->grid_mode = modes[mi];
                    b->lds = ldss[li];
                    float ms = 0.0f;
                    rc = time_runs([&](int par) { return launch_step(b, par, st); }, 4, st, ms);
                    if (rc != PLBM_OK) return rc;
                    if (ms < best) {
                        best = ms;
                        best_pol = pi;
                        mode = modes[mi];
                        lds = ldss[li];
                    }
                }
        }
        for (const auto &kv : classes) {
            b->shape[kv.first] = policy(best_pol, kv.first);
            cache[cache_key(arch, kv.first)] = b->shape[kv.first];
        }
        rc = build_tiles(b);
        if (rc != PLBM_OK) return rc;
        changed = true;
    }
    b->grid_mode = mode;
    b->lds = lds;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    b->parity = 0;
    b->tuned = true;
    if (changed) write_cache(cache_path, cache, arch, mode, lds);
    return PLBM_OK;
}

extern "C" int plbm_batch_query(const plbm_batch *b, plbm_batch_info *info)
{
    if (!b || !info) return PLBM_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->count = (int)b->specs.size();
    info->tiles = b->ntiles;
    info->grid_mode = b->grid_mode;
    info->lds_bytes = b->lds;
    info->graph_steps = b->graph_steps;
    info->parity = b->parity;
    long long nodes = 0;
    for (const auto &s : b->specs) nodes += (long long)s.nx * s.ny;
    info->nodes = nodes;
    info->pool_bytes = (long long)(b->pool_elems * sizeof(float));
    int k = 0;
    for (const auto &kv : b->shape) {
        if (k >= PLBM_BATCH_MAX_CLASSES) break;
        info->class_size[k] = kv.first;
        info->class_w[k] = kv.second.w;
        info->class_r[k] = kv.second.r;
        ++k;
    }
    info->classes = k;
    return PLBM_OK;
}
