// Batched stepping of many independent lattices (declared in clbm.h).
//
// Every instance keeps its own geometry, power-law parameters, lid and
// force; all share the storage type and the state layout.  One launch per
// time step covers the tiles of all instances, its workgroups striding over
// them; the grid runs from a persistent few workgroups per CU up to one tile
// per wave (the autotuner's choice, and the default: the hardware dispatcher
// then balances the uneven item costs, which a persistent grid leaves to the
// slowest wave of each workgroup).  Planes layout:
// workgroup b processes tiles b, b + G, b + 2G, ... of a flattened tile list,
// each tile being (instance, z layer, run of bx consecutive nodes of that
// layer in x-fastest order), so small lattices leave no lanes idle except at
// the end of a layer.  Row layout: every wave takes items (instance, row, run
// of 64 x) of a flattened list in the same strided way, so the wave's row is
// uniform and its populations come through scalar row bases, with the face
// rules taken per wave (rows on a y or z face) or per lane (x faces).  k
// consecutive steps are captured into a hipGraph on a library stream and
// replayed on the caller's stream.
#include <algorithm>
#include <vector>

#include "clbm_host.hpp"
#include "clbm_rows.hpp"

namespace clbm {

template <typename T> struct BatchInst {
    Geom g;
    Relax<T> p;
    int64_t base;       // element offset of the instance's state in each pool
    uint32_t tile0;     // first tile of the instance in the flattened list
    uint32_t chunks;    // tiles per z layer (planes), 64-wide runs per row (rows), or packed items per z
                        // layer (rows, packed)
    float inv_nx;       // 1 / nx, for the row of a node within a layer
    int32_t forced;
    uint32_t bytes;     // bytes of the instance's state (row layout, packed items)
};

// Row-layout work item of one wave: the 64-wide run from x0 of row `row`
// (pair = 0), or the short tails from x0 of two inner rows `row` and
// row + pair, one per half of the wave (tails of at most 32 values).
struct alignas(16) RowItem {
    int32_t inst, row, x0, pair;
};

// The collision index of a launch (it keys the stochastic rounding of FP16
// storage) is *step_base + step_off: step_base is set on the stream before
// each run of launches, step_off is the launch's place in that run, so that
// launches captured in a graph draw new rounding bits on every replay.
template <typename S, typename T, int Route, int StAux, bool AnyForced>
__global__ void __launch_bounds__(MaxThreads<T>::value)
batch_step_kernel(const S *__restrict__ A, S *__restrict__ B, const BatchInst<T> *__restrict__ inst,
                  const int32_t *__restrict__ tile_inst, uint32_t ntiles, const uint32_t *__restrict__ step_base,
                  uint32_t step_off) {
    const uint32_t step = *step_base + step_off;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int i = tile_inst[t];
        const Geom g = inst[i].g;
        const int64_t base = inst[i].base;
        const uint32_t local = t - inst[i].tile0;
        const uint32_t chunks = inst[i].chunks;
        const int z = (int)(local / chunks);
        const uint32_t l = (local - (uint32_t)z * chunks) * blockDim.x + threadIdx.x;   // node within the layer
        if (l >= (uint32_t)g.nxy) continue;
        // row y = l / nx: float estimate, corrected to the exact quotient
        int y = (int)((float)l * inst[i].inv_nx);
        if ((uint32_t)y * (uint32_t)g.nx > l) --y;
        if ((uint32_t)(y + 1) * (uint32_t)g.nx <= l) ++y;
        const int x = (int)(l - (uint32_t)y * (uint32_t)g.nx);
        const Relax<T> p = inst[i].p;       // a copy: read once per item, not at each use
        const uint32_t self = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y + (uint32_t)g.nxy * (uint32_t)z;
        T d[Q];
        gather<S, T, 0>(A + base, g, p, x, y, z, self, d);
        if (AnyForced && inst[i].forced)
            collide<T, true, Route, NewtonSteps<S>::value>(d, p, nullptr);
        else
            collide<T, false, Route, NewtonSteps<S>::value>(d, p, nullptr);
        round_state<S, T>(d, p, self, step);
#pragma unroll
        for (int a = 0; a < Q; ++a) Plane<S, StAux>::store(B + base, g, a, self, d[a]);
    }
}

template <typename S, typename T, bool Forced, int Route, int StAux>
__device__ inline void batch_row(const S *A, S *B, const Geom &g, const Relax<T> &p, int x, int y, int z,
                                 uint32_t step) {
    if (y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1)
        row_step<S, T, Forced, 0, StAux, Route, true, XGroupRows<S>::value>(A, B, g, p, x, y, z, step);
    else
        row_step<S, T, Forced, 0, StAux, Route, false, XGroupRows<S>::value>(A, B, g, p, x, y, z, step);
}

template <typename S, typename T, int Route, int StAux, bool AnyForced>
__global__ void __launch_bounds__(MaxThreads<T>::value)
batch_rows_kernel(const S *__restrict__ A, S *__restrict__ B, const BatchInst<T> *__restrict__ inst,
                  const RowItem *__restrict__ items, uint32_t nitems, const uint32_t *__restrict__ step_base,
                  uint32_t step_off) {
    const uint32_t step = __builtin_amdgcn_readfirstlane(*step_base + step_off);
    const uint32_t waves = blockDim.x >> 6;
    // XCD-contiguous order: workgroups wg, wg + 8, ... run on one XCD, so they
    // take consecutive items, and the partial cache lines that neighbouring
    // rows share meet in that XCD's L2
    uint32_t wg = blockIdx.x;
    const uint32_t aligned = gridDim.x & ~7u;
    if (wg < aligned) wg = (wg & 7u) * (aligned >> 3) + (wg >> 3);
    const uint32_t w0 = wg * waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63u);
    for (uint32_t t = w0; t < nitems; t += gridDim.x * waves) {
        const int i = __builtin_amdgcn_readfirstlane(items[t].inst);
        const uint32_t row = (uint32_t)__builtin_amdgcn_readfirstlane(items[t].row);
        const int x0 = __builtin_amdgcn_readfirstlane(items[t].x0);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane(items[t].pair);
        const Geom g = inst[i].g;
        const int64_t base = inst[i].base;
        const int y = (int)(row % (uint32_t)g.ny), z = (int)(row / (uint32_t)g.ny);
        const Relax<T> p = inst[i].p;       // a copy: read once per item, not at each use
        const bool forced = AnyForced && inst[i].forced;
        if (k == 0) {
            const int x = x0 + lane;
            if (x >= g.nx) continue;
            if (forced)
                batch_row<S, T, true, Route, StAux>(A + base, B + base, g, p, x, y, z, step);
            else
                batch_row<S, T, false, Route, StAux>(A + base, B + base, g, p, x, y, z, step);
        } else {
            const int x = x0 + (lane & 31);
            if (x >= g.nx) continue;
            if (forced)
                row_step_pair<S, T, true, 0, StAux, Route>(A + base, B + base, g, p, x, y, z, k, lane >= 32, step);
            else
                row_step_pair<S, T, false, 0, StAux, Route>(A + base, B + base, g, p, x, y, z, k, lane >= 32, step);
        }
    }
}

struct BatchStep {
    const uint32_t *base;   // device: collision index before the first launch of the run
    uint32_t off;           // this launch's place in the run (1, 2, ...)
};

// ---------------------------------------------------------------------------
// Packed items (row layout): a wave takes `passes` passes of 64 consecutive
// nodes of one z layer, so a pass may hold the ends and starts of several
// rows and a lattice of any width fills whole waves.  Each lane addresses its
// own row through one buffer descriptor per instance (byte offset of element
// (19 r + a) nx + x); the offset of direction a's source is the lane's offset
// plus a uniform constant.  A pass whose lanes all lie off the y and z faces
// takes that uniform pull, with the x-face lanes redone; a pass touching a
// face row takes the full wall rule per lane.  Consecutive passes of a layer
// stay in one wave, so the cache lines two neighbouring rows share are read
// and written by the same wave.
// ---------------------------------------------------------------------------
template <typename S, typename T, bool Forced, int Route, int StAux>
__device__ inline void packed_pass(const S *__restrict__ A, S *__restrict__ B, const Geom &g, const Relax<T> &p,
                                   uint32_t bytes, float inv_nx, uint32_t l, int z, uint32_t step) {
    constexpr int es = (int)sizeof(S);
    const bool active = l < (uint32_t)g.nxy;
    // row y = l / nx: float estimate, corrected to the exact quotient (l < 2^22)
    int y = (int)((float)l * inv_nx);
    if ((uint32_t)y * (uint32_t)g.nx > l) --y;
    if ((uint32_t)(y + 1) * (uint32_t)g.nx <= l) ++y;
    const int x = (int)(l - (uint32_t)y * (uint32_t)g.nx);
    const bool face = y == 0 || y >= g.ny - 1 || z == 0 || z == g.nz - 1;
    const bool any_face = __any(active && face);
    if (!active) return;
    const __amdgpu_buffer_rsrc_t ra = row_rsrc(A, __builtin_amdgcn_readfirstlane(bytes));
    const __amdgpu_buffer_rsrc_t rb = row_rsrc(B, __builtin_amdgcn_readfirstlane(bytes));
    const int nx = g.nx, ny = g.ny;
    const int lane_el = (Q * (y + ny * z)) * nx + x;             // element of (a = 0, x) in the row group
    auto own = [&](int a) { return (T)RawBits<S>::template load<0>(ra, (uint32_t)((lane_el + opp(a) * nx) * es)); };
    T d[Q];
    if (!any_face) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const int c = (a - Q * cy(a) - Q * cz(a) * ny) * nx - cx(a);
            d[a] = (T)RawBits<S>::template load<0>(ra, (uint32_t)((lane_el + c) * es));
        }
        if (x == 0 || x == nx - 1) {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                if (!((x == 0 && cx(a) == 1) || (x == nx - 1 && cx(a) == -1))) continue;
                if (g.px) {
                    const int c = (a - Q * cy(a) - Q * cz(a) * ny) * nx - cx(a) + (cx(a) == 1 ? nx : -nx);
                    d[a] = (T)RawBits<S>::template load<0>(ra, (uint32_t)((lane_el + c) * es));
                } else {
                    d[a] = wall_value<T>(own(a), p, a, (g.lid_mask & (cx(a) == 1 ? 1 : 2)) != 0);
                }
            }
        }
    } else {
        d[0] = (T)RawBits<S>::template load<0>(ra, (uint32_t)(lane_el * es));
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
            const bool in_lid = ghost_in_lid(g, sx, sy, sz);
            bool wall = false;
            if (sx < 0 || sx >= nx) { if (g.px) sx = sx < 0 ? sx + nx : sx - nx; else wall = true; }
            if (sy < 0 || sy >= ny) { if (g.py) sy = sy < 0 ? sy + ny : sy - ny; else wall = true; }
            if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
            if (!wall)
                d[a] = (T)RawBits<S>::template load<0>(ra, (uint32_t)(((Q * (sy + ny * sz) + a) * nx + sx) * es));
            else
                d[a] = wall_value<T>(own(a), p, a, in_lid);
        }
    }
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    if constexpr (std::is_same<S, __half>::value) {
        if (p.sr) {
            const uint32_t base = sr_base(l + (uint32_t)g.nxy * (uint32_t)z, step);
#pragma unroll
            for (int a = 0; a < Q; ++a)
                RawBits<S>::template store_sr<StAux>(rb, (uint32_t)((lane_el + a * nx) * es), d[a],
                                                     base + (uint32_t)a * kWeyl);
            return;
        }
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) RawBits<S>::template store<StAux>(rb, (uint32_t)((lane_el + a * nx) * es), d[a]);
}

template <typename S, typename T, int Route, int StAux, bool AnyForced>
__global__ void __launch_bounds__(MaxThreads<T>::value)
batch_packed_kernel(const S *__restrict__ A, S *__restrict__ B, const BatchInst<T> *__restrict__ inst,
                    const int32_t *__restrict__ tile_inst, uint32_t ntiles, uint32_t passes,
                    const uint32_t *__restrict__ step_base, uint32_t step_off) {
    const uint32_t step = __builtin_amdgcn_readfirstlane(*step_base + step_off);
    const uint32_t waves = blockDim.x >> 6;
    const uint32_t w0 = blockIdx.x * waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t t = w0; t < ntiles; t += gridDim.x * waves) {
        const int i = __builtin_amdgcn_readfirstlane(tile_inst[t]);
        const Geom g = inst[i].g;
        const int64_t base = inst[i].base;
        const uint32_t local = t - inst[i].tile0;
        const uint32_t chunks = inst[i].chunks;
        const int z = (int)(local / chunks);
        const uint32_t l0 = (local - (uint32_t)z * chunks) * passes * 64u;
        const Relax<T> p = inst[i].p;       // a copy: read once per item, not at each use
        const uint32_t bytes = inst[i].bytes;
        const float inv_nx = inst[i].inv_nx;
        for (uint32_t j = 0; j < passes; ++j) {
            const uint32_t l = l0 + j * 64u;
            if (l >= (uint32_t)g.nxy) break;
            if (AnyForced && inst[i].forced)
                packed_pass<S, T, true, Route, StAux>(A + base, B + base, g, p, bytes, inv_nx, l + lane, z, step);
            else
                packed_pass<S, T, false, Route, StAux>(A + base, B + base, g, p, bytes, inv_nx, l + lane, z, step);
        }
    }
}

template <typename S, typename T, int StAux, bool AF>
static hipError_t launch_batch_h(const void *A, void *B, const void *inst, const int32_t *tiles, uint32_t ntiles,
                                 int route, bool rows, uint32_t passes, dim3 grid, dim3 block, BatchStep s,
                                 hipStream_t st) {
    const S *a = (const S *)A;
    S *b = (S *)B;
    const BatchInst<T> *d = (const BatchInst<T> *)inst;
    if (rows && passes > 0) {
        if (route == 0)
            hipLaunchKernelGGL((batch_packed_kernel<S, T, 0, StAux, AF>), grid, block, 0, st, a, b, d, tiles, ntiles,
                               passes, s.base, s.off);
        else
            hipLaunchKernelGGL((batch_packed_kernel<S, T, 1, StAux, AF>), grid, block, 0, st, a, b, d, tiles, ntiles,
                               passes, s.base, s.off);
        return hipGetLastError();
    }
    if (rows) {
        if (route == 0)
            hipLaunchKernelGGL((batch_rows_kernel<S, T, 0, StAux, AF>), grid, block, 0, st, a, b, d,
                               (const RowItem *)tiles, ntiles, s.base, s.off);
        else
            hipLaunchKernelGGL((batch_rows_kernel<S, T, 1, StAux, AF>), grid, block, 0, st, a, b, d,
                               (const RowItem *)tiles, ntiles, s.base, s.off);
        return hipGetLastError();
    }
    if (route == 0)
        hipLaunchKernelGGL((batch_step_kernel<S, T, 0, StAux, AF>), grid, block, 0, st, a, b, d, tiles, ntiles, s.base,
                           s.off);
    else
        hipLaunchKernelGGL((batch_step_kernel<S, T, 1, StAux, AF>), grid, block, 0, st, a, b, d, tiles, ntiles, s.base,
                           s.off);
    return hipGetLastError();
}

template <typename S, typename T>
static hipError_t launch_batch_t(const void *A, void *B, const void *inst, const int32_t *tiles, uint32_t ntiles,
                                 int route, bool rows, uint32_t passes, bool nt, bool any_forced, dim3 grid, dim3 block,
                                 BatchStep s, hipStream_t st) {
    // batches without a body force get kernels without the forced collision (half the code)
    if (any_forced)
        return nt ? launch_batch_h<S, T, 2, true>(A, B, inst, tiles, ntiles, route, rows, passes, grid, block, s, st)
                  : launch_batch_h<S, T, 0, true>(A, B, inst, tiles, ntiles, route, rows, passes, grid, block, s, st);
    return nt ? launch_batch_h<S, T, 2, false>(A, B, inst, tiles, ntiles, route, rows, passes, grid, block, s, st)
              : launch_batch_h<S, T, 0, false>(A, B, inst, tiles, ntiles, route, rows, passes, grid, block, s, st);
}

static hipError_t launch_batch(int storage, const void *A, void *B, const void *inst, const int32_t *tiles,
                               uint32_t ntiles, int route, bool rows, uint32_t passes, bool nt, bool any_forced,
                               dim3 grid, dim3 block, BatchStep s, hipStream_t st) {
    switch (storage) {
    case 0:
        return launch_batch_t<double, double>(A, B, inst, tiles, ntiles, route, rows, passes, nt, any_forced, grid,
                                              block, s, st);
    case 1:
        return launch_batch_t<float, float>(A, B, inst, tiles, ntiles, route, rows, passes, nt, any_forced, grid, block,
                                            s, st);
    default:
        return launch_batch_t<__half, float>(A, B, inst, tiles, ntiles, route, rows, passes, nt, any_forced, grid,
                                             block, s, st);
    }
}

__global__ void __launch_bounds__(64) set_step_kernel(uint32_t *__restrict__ p, uint32_t v) {
    if (threadIdx.x == 0) *p = v;
}

static uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
    const unsigned char *c = (const unsigned char *)data;
    for (size_t k = 0; k < n; ++k) { h ^= c[k]; h *= 1099511628211ull; }
    return h;
}

}  // namespace clbm

using namespace clbm;

struct clbm_batch {
    int count;
    int storage;
    int route;
    bool rows;              // row layout
    std::vector<clbm_params> prm;
    std::vector<Geom> geom;
    std::vector<Relax<double>> rd;
    std::vector<Relax<float>> rf;
    std::vector<int64_t> base;      // element offsets
    std::vector<int> forced;
    void *pool[2];
    size_t bytes_each;
    int cur;
    bool initialized;
    int64_t steps_done;
    clbm_batch_config cfg;
    int num_cus;
    // device tables
    uint32_t *d_step;       // collision index before the current run of launches
    void *d_inst;
    int32_t *d_tiles;       // tile list: instance per tile, or RowItem (4 values) per row item
    size_t tile_cap;        // int32 values
    uint32_t ntiles;
    // reductions
    double *partials;
    int nblocks_max;
    double *results;
    double *host_results;
    std::vector<double *> snapshot;
    std::vector<char> have_snapshot;
    // graphs
    hipStream_t cap_stream;
    hipGraphExec_t exec[2];
    int exec_steps[2];
    std::string cache_path;
    std::string cache_key;
};

namespace {

// each instance's state starts 256-byte aligned in the pools
size_t instance_bytes(const clbm_params *p) {
    return (state_bytes_of(p) + 255) / 256 * 256;
}

void drop_graphs(clbm_batch *b) {
    for (int k = 0; k < 2; ++k) {
        if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
        b->exec[k] = nullptr;
        b->exec_steps[k] = 0;
    }
}

int max_threads(const clbm_batch *b) { return b->storage == CLBM_F64 ? 256 : 512; }

clbm_status check_config(const clbm_batch *b, const clbm_batch_config *c) {
    const int mt = max_threads(b);
    if (c->bx < 64 || c->by != 1 || c->bx > mt || c->bx % 64 != 0)
        return fail(CLBM_EINVAL, "batch tile %d x %d: need by = 1 and bx a multiple of 64, <= %d", c->bx, c->by, mt);
    if (c->blocks_per_cu < 1 || c->blocks_per_cu > 1024) return fail(CLBM_EINVAL, "blocks_per_cu must lie in 1..1024");
    if (c->graph_steps < 0 || c->graph_steps > 4096) return fail(CLBM_EINVAL, "graph_steps must lie in 0..4096");
    if (c->nt_stores != 0 && c->nt_stores != 1) return fail(CLBM_EINVAL, "nt_stores must be 0 or 1");
    if (c->passes < 0 || c->passes > 256) return fail(CLBM_EINVAL, "passes must lie in 0..256");
    if (c->passes > 0 && !b->rows) return fail(CLBM_EINVAL, "packed items (passes > 0) need the row layout");
    return CLBM_OK;
}

// Rebuild the flattened tile list and the instance descriptors for a tile shape.
template <typename T>
clbm_status upload_tables_t(clbm_batch *b, const std::vector<Relax<T>> &relax) {
    std::vector<BatchInst<T>> inst(b->count);
    std::vector<int32_t> tiles;
    uint64_t total = 0;
    for (int i = 0; i < b->count; ++i) {
        const Geom &g = b->geom[i];
        BatchInst<T> &d = inst[i];
        memset(&d, 0, sizeof(d));
        d.g = g;
        d.p = relax[i];
        d.base = b->base[i];
        d.inv_nx = 1.0f / (float)g.nx;
        d.tile0 = (uint32_t)total;
        d.forced = b->forced[i];
        d.bytes = (uint32_t)state_bytes_of(&b->prm[i]);
        if (b->rows && b->cfg.passes > 0) {
            const uint64_t per = 64ull * (uint64_t)b->cfg.passes;
            d.chunks = (uint32_t)(((uint64_t)g.nxy + per - 1) / per);
            total += (uint64_t)d.chunks * (uint64_t)g.nz;
        } else if (b->rows) {
            d.chunks = (uint32_t)((g.nx + 63) / 64);
        } else {
            d.chunks = (uint32_t)((g.nxy + b->cfg.bx - 1) / b->cfg.bx);
            total += (uint64_t)d.chunks * (uint64_t)g.nz;
        }
    }
    const bool per_row = b->rows && b->cfg.passes == 0;
    if (per_row) {
        // row items in row order; the short tails (at most 32 values) of two
        // consecutive inner rows share a wave, one per half
        for (int i = 0; i < b->count; ++i) {
            const Geom &g = b->geom[i];
            const int32_t chunks = (int32_t)inst[i].chunks, tail = g.nx % 64;
            const bool short_tail = tail != 0 && tail <= 32;
            const int32_t x_tail = 64 * (chunks - 1);
            int32_t pending = -1;
            inst[i].tile0 = (uint32_t)(tiles.size() / 4);
            auto push = [&](int32_t row, int32_t x0, int32_t pair) {
                tiles.push_back(i);
                tiles.push_back(row);
                tiles.push_back(x0);
                tiles.push_back(pair);
            };
            for (int32_t z = 0; z < g.nz; ++z)
                for (int32_t y = 0; y < g.ny; ++y) {
                    const int32_t row = y + g.ny * z;
                    for (int32_t c = 0; c < (short_tail ? chunks - 1 : chunks); ++c) push(row, 64 * c, 0);
                    if (!short_tail) continue;
                    const bool inner = y > 0 && y < g.ny - 1 && z > 0 && z < g.nz - 1;
                    if (!inner) {
                        push(row, x_tail, 0);
                    } else if (pending < 0) {
                        pending = row;
                    } else {
                        push(pending, x_tail, row - pending);
                        pending = -1;
                    }
                }
            if (pending >= 0) push(pending, x_tail, 0);
            if (tiles.size() / 4 > 0x1fffffffull) return fail(CLBM_EINVAL, "batch has more than 2^29 row items");
        }
        total = tiles.size() / 4;
    } else {
        if (total > 0x7fffffffull) return fail(CLBM_EINVAL, "batch has more than 2^31 tiles");
        tiles.resize(total);
        for (int i = 0; i < b->count; ++i) {
            const uint64_t n = (uint64_t)inst[i].chunks * (uint64_t)b->geom[i].nz;
            std::fill(tiles.begin() + inst[i].tile0, tiles.begin() + inst[i].tile0 + n, i);
        }
    }
    const size_t vals = tiles.size();
    if (vals > b->tile_cap) {
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        b->d_tiles = nullptr;
        HIP_TRY(hipMalloc((void **)&b->d_tiles, sizeof(int32_t) * vals), "batch: tile table");
        b->tile_cap = vals;
    }
    HIP_TRY(hipMemcpy(b->d_tiles, tiles.data(), sizeof(int32_t) * vals, hipMemcpyHostToDevice), "batch: tiles");
    HIP_TRY(hipMemcpy(b->d_inst, inst.data(), sizeof(BatchInst<T>) * b->count, hipMemcpyHostToDevice),
            "batch: descriptors");
    b->ntiles = (uint32_t)total;
    drop_graphs(b);
    return CLBM_OK;
}

clbm_status upload_tables(clbm_batch *b) {
    return b->storage == CLBM_F64 ? upload_tables_t<double>(b, b->rd) : upload_tables_t<float>(b, b->rf);
}

// Sets the device step base to the steps taken so far (before a run of
// launches; a kernel, not a copy, so it can precede graph replays).
hipError_t set_step_base(clbm_batch *b, hipStream_t st) {
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, b->d_step, (uint32_t)b->steps_done);
    return hipGetLastError();
}

hipError_t launch_one_step(clbm_batch *b, int from, uint32_t off, hipStream_t st) {
    // rows: a tile is one wave's item, bx / 64 of them per workgroup
    const uint64_t per_block = b->rows ? (uint64_t)(b->cfg.bx / 64) : 1u;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)b->cfg.blocks_per_cu * b->num_cus,
                                                       std::max<uint64_t>((b->ntiles + per_block - 1) / per_block, 1u));
    return launch_batch(b->storage, b->pool[from], b->pool[1 - from], b->d_inst, b->d_tiles, b->ntiles, b->route,
                        b->rows, (uint32_t)b->cfg.passes, b->cfg.nt_stores != 0,
                        std::any_of(b->forced.begin(), b->forced.end(), [](int f) { return f != 0; }), dim3(grid),
                        dim3(b->cfg.bx), BatchStep{b->d_step, off}, st);
}

clbm_status build_graph(clbm_batch *b, int parity) {
    const int k = b->cfg.graph_steps;
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "batch: begin capture");
    int c = parity;
    hipError_t e = hipSuccess;
    for (int s = 0; s < k && e == hipSuccess; ++s) {
        e = launch_one_step(b, c, (uint32_t)s + 1u, b->cap_stream);
        c = 1 - c;
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e, "batch: capture launch");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "batch: end capture");
    e = hipGraphInstantiate(&b->exec[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "batch: instantiate graph");
    b->exec_steps[parity] = k;
    return CLBM_OK;
}

std::string make_cache_key(const clbm_batch *b) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &b->storage, sizeof(b->storage));
    h = fnv1a(h, &b->route, sizeof(b->route));
    h = fnv1a(h, &b->count, sizeof(b->count));
    for (int i = 0; i < b->count; ++i) {
        const int32_t dims[3] = {b->prm[i].nx, b->prm[i].ny, b->prm[i].nz};
        h = fnv1a(h, dims, sizeof(dims));
    }
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    char buf[64];
    snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return arch + "-" + buf;
}

bool read_cache(clbm_batch *b, clbm_batch_config *out) {
    if (b->cache_path.empty()) return false;
    FILE *fh = fopen(b->cache_path.c_str(), "r");
    if (!fh) return false;
    char key[256];
    clbm_batch_config c;
    bool found = false;
    while (fscanf(fh, "%255s %d %d %d %d %d %d", key, &c.bx, &c.by, &c.blocks_per_cu, &c.graph_steps, &c.nt_stores,
                  &c.passes) == 7) {
        if (b->cache_key == key && check_config(b, &c) == CLBM_OK) {
            *out = c;
            found = true;       // the last entry for a key wins
        }
    }
    fclose(fh);
    return found;
}

void append_cache(clbm_batch *b, const clbm_batch_config &c, double ms) {
    if (b->cache_path.empty()) return;
    FILE *fh = fopen(b->cache_path.c_str(), "a");
    if (!fh) return;
    fprintf(fh, "%s %d %d %d %d %d %d\n", b->cache_key.c_str(), c.bx, c.by, c.blocks_per_cu, c.graph_steps,
            c.nt_stores, c.passes);
    (void)ms;
    fclose(fh);
}

clbm_status check_index(clbm_batch *b, int32_t i) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (i < 0 || i >= b->count) return fail(CLBM_EINVAL, "instance %d out of range 0..%d", i, b->count - 1);
    return CLBM_OK;
}

const char *storage_ptr(clbm_batch *b, int buf, int32_t i) {
    return (const char *)b->pool[buf] + (size_t)b->base[i] * elem_bytes(b->storage);
}

}  // namespace

extern "C" {

clbm_status clbm_batch_size(const clbm_params *inst, int32_t count, size_t *bytes_each) {
    if (!inst || count < 1) return fail(CLBM_EINVAL, "need at least one instance");
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        clbm_status st = validate(&inst[i]);
        if (st != CLBM_OK) return fail(st, "instance %d: %s", i, g_err.c_str());
        if (inst[i].storage != inst[0].storage) return fail(CLBM_EINVAL, "instance %d: storage differs", i);
        if (inst[i].collision == CLBM_COLLIDE_SRT)
            return fail(CLBM_EINVAL, "instance %d: batches run the cascaded scheme only", i);
        if (inst[i].layout != inst[0].layout) return fail(CLBM_EINVAL, "instance %d: layout differs", i);
        // the row of a node within its layer comes from a float estimate with
        // one correction, exact while a layer has at most 2^22 nodes
        if ((int64_t)inst[i].nx * inst[i].ny > ((int64_t)1 << 22))
            return fail(CLBM_EINVAL, "instance %d: a z layer of more than 2^22 nodes", i);
        // row layout: packed items address an instance's state with 32-bit signed byte offsets
        if (inst[i].layout == CLBM_LAYOUT_ROWS && state_bytes_of(&inst[i]) >= ((size_t)1 << 31) - ((size_t)1 << 24))
            return fail(CLBM_EINVAL, "instance %d: a state of 2 GiB or more in a row-layout batch", i);
        total += instance_bytes(&inst[i]);
    }
    if (bytes_each) *bytes_each = total;
    return CLBM_OK;
}

clbm_status clbm_batch_create(const clbm_params *inst, int32_t count, void *pool_a, void *pool_b,
                              size_t bytes_each, const char *tune_cache_path, clbm_batch **out) {
    if (!out) return fail(CLBM_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    clbm_status st = clbm_batch_size(inst, count, &need);
    if (st != CLBM_OK) return st;
    if (!pool_a || !pool_b || pool_a == pool_b) return fail(CLBM_EINVAL, "need two distinct pools");
    if (!aligned256(pool_a) || !aligned256(pool_b)) return fail(CLBM_EINVAL, "pools must be 256-byte aligned");
    if (bytes_each < need) return fail(CLBM_EINVAL, "pools hold %zu bytes, need %zu", bytes_each, need);

    clbm_batch *b = new clbm_batch();
    b->count = count;
    b->storage = inst[0].storage;
    b->rows = inst[0].layout == CLBM_LAYOUT_ROWS;
    b->route = 0;
    for (int i = 0; i < count; ++i)
        if (route_of(&inst[i]) == 1) b->route = 1;   // one form for the whole batch
    if (b->route == 0)
        for (int i = 0; i < count; ++i)
            if (inst[i].collision == CLBM_COLLIDE_GHAT) b->route = 1;
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
        b->prm.push_back(inst[i]);
        b->geom.push_back(make_geom(&inst[i]));
        b->rd.push_back(make_relax<double>(&inst[i]));
        b->rf.push_back(make_relax<float>(&inst[i]));
        b->base.push_back(off);
        b->forced.push_back(inst[i].force[0] != 0.0 || inst[i].force[1] != 0.0 || inst[i].force[2] != 0.0);
        off += (int64_t)(instance_bytes(&inst[i]) / elem_bytes(inst[i].storage));
    }
    b->pool[0] = pool_a;
    b->pool[1] = pool_b;
    b->bytes_each = bytes_each;
    b->cfg.bx = max_threads(b);
    b->cfg.by = 1;
    b->cfg.blocks_per_cu = 1024;    // capped at one item per wave (row layout) or one tile per workgroup
    b->cfg.graph_steps = 20;
    b->cfg.nt_stores = 0;
    b->cfg.passes = 0;          // one row run per wave item: faster than packed items on the 64-cavity mix
    b->num_cus = 256;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->num_cus = cus;
    b->cache_path = tune_cache_path ? tune_cache_path : "";
    b->cache_key = make_cache_key(b);
    clbm_batch_config cached;
    if (read_cache(b, &cached)) b->cfg = cached;

    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    const size_t inst_size = b->storage == CLBM_F64 ? sizeof(BatchInst<double>) : sizeof(BatchInst<float>);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_step, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(b->d_step, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&b->d_inst, inst_size * count);
    int64_t maxn = 0;
    for (int i = 0; i < count; ++i) maxn = std::max<int64_t>(maxn, (int64_t)b->geom[i].n);
    b->nblocks_max = (int)std::min<int64_t>(1024, (maxn + kReduceThreads - 1) / kReduceThreads);
    if (e == hipSuccess) e = hipMalloc((void **)&b->partials, sizeof(double) * kReduceSlots * b->nblocks_max);
    if (e == hipSuccess) e = hipMalloc((void **)&b->results, sizeof(double) * kReduceSlots * count);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&b->host_results, sizeof(double) * kReduceSlots * count, hipHostMallocDefault);
    b->snapshot.assign(count, nullptr);
    b->have_snapshot.assign(count, 0);
    for (int i = 0; i < count && e == hipSuccess; ++i)
        if (inst[i].track_residual) e = hipMalloc((void **)&b->snapshot[i], sizeof(double) * 3 * b->geom[i].n);
    if (e != hipSuccess) {
        clbm_batch_destroy(b);
        return hip_fail(e, "clbm_batch_create: allocation");
    }
    st = upload_tables(b);
    if (st != CLBM_OK) {
        clbm_batch_destroy(b);
        return st;
    }
    *out = b;
    return CLBM_OK;
}

clbm_status clbm_batch_destroy(clbm_batch *b) {
    if (!b) return CLBM_OK;
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_step) (void)hipFree(b->d_step);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->partials) (void)hipFree(b->partials);
    if (b->results) (void)hipFree(b->results);
    if (b->host_results) (void)hipHostFree(b->host_results);
    for (double *s : b->snapshot)
        if (s) (void)hipFree(s);
    delete b;
    return CLBM_OK;
}

clbm_status clbm_batch_init_rest(clbm_batch *b, void *stream) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    for (int i = 0; i < b->count; ++i)
        HIP_TRY(launch_init(b->storage, nullptr, (void *)storage_ptr(b, 0, i), nullptr, b->geom[i], b->rd[i],
                            b->rf[i],
                            b->forced[i], b->route, (hipStream_t)stream),
                "clbm_batch_init_rest");
    b->cur = 0;
    b->initialized = true;
    b->steps_done = 0;
    std::fill(b->have_snapshot.begin(), b->have_snapshot.end(), 0);
    return CLBM_OK;
}

clbm_status clbm_batch_init_populations(clbm_batch *b, int32_t i, const double *f0, int on_device, void *stream) {
    clbm_status st = check_index(b, i);
    if (st != CLBM_OK) return st;
    if (!f0) return fail(CLBM_EINVAL, "f0 is NULL");
    if (on_device != 0 && on_device != 1) return fail(CLBM_EINVAL, "on_device must be 0 or 1");
    if (!b->initialized) return fail(CLBM_ESTATE, "initialise the batch with clbm_batch_init_rest first");
    hipStream_t s = (hipStream_t)stream;
    const double *src = f0;
    double *staged = nullptr;
    if (!on_device) {
        const size_t bytes = sizeof(double) * Q * (size_t)b->geom[i].n;
        HIP_TRY(hipMalloc((void **)&staged, bytes), "clbm_batch_init_populations: staging allocation");
        hipError_t e = hipMemcpyAsync(staged, f0, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipFree(staged);
            return hip_fail(e, "clbm_batch_init_populations: copy");
        }
        src = staged;
    }
    hipError_t e = launch_init(b->storage, src, (void *)storage_ptr(b, b->cur, i), nullptr, b->geom[i], b->rd[i],
                               b->rf[i], b->forced[i], b->route, s);
    if (staged) {
        hipError_t e2 = hipStreamSynchronize(s);
        (void)hipFree(staged);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "clbm_batch_init_populations");
    b->have_snapshot[i] = 0;
    return CLBM_OK;
}

clbm_status clbm_batch_step(clbm_batch *b, int64_t nsteps, void *stream) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (nsteps < 0) return fail(CLBM_EINVAL, "nsteps must be >= 0");
    if (!b->initialized) return fail(CLBM_ESTATE, "clbm_batch_step before an init call");
    hipStream_t st = (hipStream_t)stream;
    const int k = b->cfg.graph_steps;
    while (k > 0 && nsteps >= k) {
        if (!b->exec[b->cur] || b->exec_steps[b->cur] != k) {
            clbm_status s = build_graph(b, b->cur);
            if (s != CLBM_OK) return s;
        }
        HIP_TRY(set_step_base(b, st), "clbm_batch_step: step base");
        HIP_TRY(hipGraphLaunch(b->exec[b->cur], st), "clbm_batch_step: graph launch");
        if (k & 1) b->cur = 1 - b->cur;
        b->steps_done += k;
        nsteps -= k;
    }
    if (nsteps > 0) HIP_TRY(set_step_base(b, st), "clbm_batch_step: step base");
    for (uint32_t off = 1; nsteps > 0; --nsteps, ++off) {
        HIP_TRY(launch_one_step(b, b->cur, off, st), "clbm_batch_step");
        b->cur = 1 - b->cur;
        b->steps_done++;
    }
    return CLBM_OK;
}

clbm_status clbm_batch_step_each(clbm_batch *b, int64_t nsteps, void *stream) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (nsteps < 0) return fail(CLBM_EINVAL, "nsteps must be >= 0");
    if (!b->initialized) return fail(CLBM_ESTATE, "clbm_batch_step_each before an init call");
    hipStream_t st = (hipStream_t)stream;
    for (; nsteps > 0; --nsteps) {
        for (int i = 0; i < b->count; ++i) {
            StepLaunch c;
            const int nx = b->geom[i].nx;
            c.bx = nx >= 256 ? 256 : (nx >= 64 ? 64 * (nx / 64) : nx);
            if (c.bx > 256) c.bx = 256;
            c.by = 1;
            while (c.bx * c.by * 2 <= 256 && c.by * 2 <= b->geom[i].ny) c.by *= 2;
            c.xcd_remap = 0;
            c.nt_loads = 0;
            c.nt_stores = 1;
            c.fuse_steps = 1;
            c.fuse_rows = 8;
            c.fuse_planes = 1;
            Relax<double> pd = b->rd[i];
            Relax<float> pf = b->rf[i];
            pd.step = pf.step = (uint32_t)(b->steps_done + 1);
            if (b->rows) {
                if (nx >= 64) c.by = 1;         // one lattice row per block, as for a single lattice
                HIP_TRY(launch_step_rows(b->storage, storage_ptr(b, b->cur, i), (void *)storage_ptr(b, 1 - b->cur, i),
                                         b->geom[i], pd, pf, b->forced[i], b->route, c, st),
                        "clbm_batch_step_each");
            } else {
                HIP_TRY(launch_step(b->storage, storage_ptr(b, b->cur, i), (void *)storage_ptr(b, 1 - b->cur, i),
                                    b->geom[i], pd, pf, b->forced[i], b->route, c, st),
                        "clbm_batch_step_each");
            }
        }
        b->cur = 1 - b->cur;
        b->steps_done++;
    }
    return CLBM_OK;
}

clbm_status clbm_batch_macroscopic(clbm_batch *b, int32_t i, void *rho, void *u, int32_t out_prec, void *stream) {
    clbm_status st = check_index(b, i);
    if (st != CLBM_OK) return st;
    if (out_prec != CLBM_F64 && out_prec != CLBM_F32)
        return fail(CLBM_EINVAL, "out_prec must be CLBM_F64 or CLBM_F32 (got %d)", out_prec);
    if (!b->initialized) return fail(CLBM_ESTATE, "clbm_batch_macroscopic before an init call");
    if (!rho && !u) return CLBM_OK;
    HIP_TRY(launch_macroscopic(b->storage, storage_ptr(b, b->cur, i), nullptr, rho, u, out_prec == CLBM_F32,
                               b->geom[i], b->prm[i].force, (hipStream_t)stream),
            "clbm_batch_macroscopic");
    return CLBM_OK;
}

clbm_status clbm_batch_populations(clbm_batch *b, int32_t i, double *f, void *stream) {
    clbm_status st = check_index(b, i);
    if (st != CLBM_OK) return st;
    if (!f) return fail(CLBM_EINVAL, "output is NULL");
    if (!b->initialized) return fail(CLBM_ESTATE, "clbm_batch_populations before an init call");
    HIP_TRY(launch_export(b->storage, storage_ptr(b, b->cur, i), f, b->geom[i], (hipStream_t)stream),
            "clbm_batch_populations");
    return CLBM_OK;
}

clbm_status clbm_batch_reduce(clbm_batch *b, double *out, void *stream) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (!out) return fail(CLBM_EINVAL, "out is NULL");
    if (!b->initialized) return fail(CLBM_ESTATE, "clbm_batch_reduce before an init call");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < b->count; ++i) {
        const int nb = (int)std::min<int64_t>(b->nblocks_max, ((int64_t)b->geom[i].n + kReduceThreads - 1) /
                                                                   kReduceThreads);
        HIP_TRY(launch_reduce(b->storage, storage_ptr(b, b->cur, i), nullptr, b->snapshot[i],
                              b->have_snapshot[i] ? 1 : 0,
                              b->geom[i], b->prm[i].force, b->partials, nb, b->results + (size_t)kReduceSlots * i,
                              st),
                "clbm_batch_reduce");
    }
    HIP_TRY(hipMemcpyAsync(b->host_results, b->results, sizeof(double) * kReduceSlots * b->count,
                           hipMemcpyDeviceToHost, st),
            "clbm_batch_reduce: copy");
    HIP_TRY(hipStreamSynchronize(st), "clbm_batch_reduce: sync");
    double bad = 0.0;
    for (int i = 0; i < b->count; ++i) {
        const double *r = b->host_results + (size_t)kReduceSlots * i;
        double *o = out + 8 * (size_t)i;
        o[0] = r[9] + r[0];
        o[1] = r[1]; o[2] = r[2]; o[3] = r[3];
        o[4] = (b->snapshot[i] && b->have_snapshot[i] && r[5] > 0.0) ? sqrt(r[4] / r[5]) : 0.0;
        o[5] = r[6];
        o[6] = r[7];
        o[7] = r[8];
        if (b->snapshot[i]) b->have_snapshot[i] = 1;
        bad += r[6];
    }
    if (bad > 0.0) return fail(CLBM_EUNSTABLE, "%.0f nodes hold non-finite populations", bad);
    return CLBM_OK;
}

clbm_status clbm_batch_set_config(clbm_batch *b, const clbm_batch_config *c) {
    if (!b || !c) return fail(CLBM_EINVAL, "NULL argument");
    clbm_status st = check_config(b, c);
    if (st != CLBM_OK) return st;
    const bool tiles_change = c->bx != b->cfg.bx || c->by != b->cfg.by || c->passes != b->cfg.passes;
    b->cfg = *c;
    drop_graphs(b);
    return tiles_change ? upload_tables(b) : CLBM_OK;
}

clbm_status clbm_batch_get_config(clbm_batch *b, clbm_batch_config *c) {
    if (!b || !c) return fail(CLBM_EINVAL, "NULL argument");
    *c = b->cfg;
    return CLBM_OK;
}

clbm_status clbm_batch_state(clbm_batch *b, int *buffer_index, int64_t *steps_done) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (buffer_index) *buffer_index = b->cur;
    if (steps_done) *steps_done = b->steps_done;
    return CLBM_OK;
}

clbm_status clbm_batch_autotune(clbm_batch *b, void *stream, clbm_batch_config *best, double *best_ms) {
    if (!b) return fail(CLBM_EINVAL, "batch handle is NULL");
    if (!b->initialized) return fail(CLBM_ESTATE, "autotune needs an initialised state");
    hipStream_t st = (hipStream_t)stream;
    static const int shapes[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}};
    static const int bpcs[] = {8, 32, 128, 1024};      // 1024: one item per wave up to 2^21 items (2^20 at bx 256)
    const clbm_batch_config keep = b->cfg;
    clbm_batch_config win = keep;
    double win_ms = 1e300;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "autotune: event");
    HIP_TRY(hipEventCreate(&e1), "autotune: event");
    clbm_status result = CLBM_OK;
    static const int packings[] = {0, 2, 4, 8};     // row layout: one row run per item, or packed passes
    for (const auto &sh : shapes)
    for (int pk : packings) {
        clbm_batch_config c = keep;
        c.bx = sh[0];
        c.by = sh[1];
        c.passes = pk;
        if (check_config(b, &c) != CLBM_OK) continue;
        for (int k = 0; k < 8; ++k) {
            c.blocks_per_cu = bpcs[k % 4];
            c.nt_stores = k / 4;
            if ((result = clbm_batch_set_config(b, &c)) != CLBM_OK) break;
            // trials read the state and write the spare pool: the state is unchanged
            hipError_t e = launch_one_step(b, b->cur, 1u, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch_one_step(b, b->cur, 1u, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { result = hip_fail(e, "autotune: trial"); break; }
            if (ms / 5.0 < win_ms) { win_ms = ms / 5.0; win = c; }
        }
        if (result != CLBM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != CLBM_OK) {
        clbm_batch_set_config(b, &keep);
        return result;
    }
    result = clbm_batch_set_config(b, &win);
    if (result != CLBM_OK) return result;
    append_cache(b, win, win_ms);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return CLBM_OK;
}

}  // extern "C"
