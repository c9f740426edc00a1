// Row layout helpers shared by the two-buffer and in-place row kernels.
//
// Row layout: the 19 populations of lattice row r = y + ny z are 19
// consecutive runs of nx values, population a of node x at element
// (19 r + a) nx + x (Geom::plane = nx, Geom::row = 19 nx).  A row kernel
// runs waves of 64 consecutive x of one row (blockDim.x a multiple of 64),
// so every direction's source or target run has a uniform (scalar) base and
// one lane offset serves all of them.  Rows off the y and z faces and rows on
// them go to separate launches: the inner-row kernels then carry no face
// logic.
#pragma once

#include "clbm_internal.hpp"

namespace clbm {

__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}

struct RowGrid {
    uint32_t gx;            // tiles along x
    uint32_t rows;          // rows handled by the launch
    uint32_t aligned;       // largest multiple of 8 <= number of workgroups
    int32_t remap;          // XCD-contiguous tile order
    int32_t zf, yf;         // face rows: z faces (1 or 2) and y faces (1 or 2)
};

// Row index of the wave and tile of the workgroup (blockDim.x a multiple of 64).
__device__ inline bool row_of(const RowGrid &R, int &x, uint32_t &ri) {
    uint32_t b = blockIdx.x;
    if (R.remap && b < R.aligned) b = (b & 7u) * (R.aligned >> 3) + (b >> 3);
    const uint32_t tx = b % R.gx;
    ri = __builtin_amdgcn_readfirstlane((b / R.gx) * blockDim.y + threadIdx.y);
    x = (int)(tx * blockDim.x + threadIdx.x);
    return ri < R.rows;
}

// inner rows: y in [1, ny - 2], z in [1, nz - 2]
__device__ inline void inner_row(const Geom &g, uint32_t ri, int &y, int &z) {
    const uint32_t w = (uint32_t)g.ny - 2u;
    y = 1 + (int)(ri % w);
    z = 1 + (int)(ri / w);
}

// face rows: every row of the z faces, then the y-face rows of the inner z layers
__device__ inline void face_row(const Geom &g, const RowGrid &R, uint32_t ri, int &y, int &z) {
    const uint32_t nzr = (uint32_t)R.zf * (uint32_t)g.ny;
    if (ri < nzr) {
        y = (int)(ri % (uint32_t)g.ny);
        z = ri < (uint32_t)g.ny ? 0 : g.nz - 1;
    } else {
        const uint32_t k = ri - nzr;
        z = 1 + (int)(k / (uint32_t)R.yf);
        y = (k % (uint32_t)R.yf) == 0 ? 0 : g.ny - 1;
    }
}

// Launch shapes of the inner-row and face-row kernels for blocks of bx x by
// (bx a multiple of 64); inner rows may be none (ny or nz below 3).
struct RowLaunch {
    RowGrid inner, face;
    uint32_t inner_blocks, face_blocks;
};

inline RowLaunch row_launch(const Geom &g, int bx, int by, int remap) {
    RowLaunch L;
    RowGrid R;
    R.gx = (uint32_t)((g.nx + bx - 1) / bx);
    R.zf = g.nz > 1 ? 2 : 1;
    R.yf = g.ny > 1 ? 2 : 1;
    R.remap = remap;
    R.rows = (g.ny > 2 && g.nz > 2) ? (uint32_t)(g.ny - 2) * (uint32_t)(g.nz - 2) : 0u;
    L.inner_blocks = R.gx * ((R.rows + by - 1) / by);
    R.aligned = L.inner_blocks & ~7u;
    L.inner = R;
    R.rows = (uint32_t)R.zf * (uint32_t)g.ny + (g.nz > 2 ? (uint32_t)(g.nz - 2) * (uint32_t)R.yf : 0u);
    L.face_blocks = R.gx * ((R.rows + by - 1) / by);
    R.aligned = L.face_blocks & ~7u;
    R.remap = 0;
    L.face = R;
    return L;
}

// Row kernels group the x-face bounce-back loads of a wave (row_gather's
// XGroup) with FP32 storage: at 512^3 the one-step launch runs 1.3% and the
// two-step one 2.9% faster, the 64-cavity batch 2.8% (its waves all hold face
// lanes; compiled at seven waves per SIMD, since the grouped loads need more
// than the 64 VGPRs of eight).  FP16 storage, bound by its arithmetic, ran 3%
// slower that way and keeps the per-direction path.
template <typename S> struct XGroupRows { static constexpr bool value = std::is_same<S, float>::value; };

// A wave may serve two rows r and r + k of one lattice as two halves (the
// short tails of two rows in a batch): every run the second half reads or
// writes lies k row groups after the first half's, the same byte distance D
// for all 19 directions, so its lanes add D to their offsets (`Shift::lane`)
// and every descriptor's range grows by D (`Shift::range`).
struct Shift {
    uint32_t lane;      // bytes added to this lane's offsets (0 or D)
    uint32_t range;     // D: added to every descriptor's range (uniform)
};

// Pull of node x of row (y, z) with the wall rules into d; y and z uniform
// over the wave (or over each half, Pair); Face: the row lies on a y or z face;
// XGroup: the x-face bounce-back loads of a wave issued together (below).
template <typename S, typename T, int LdAux, bool Face, bool Pair = false, bool XGroup = false>
__device__ inline void row_gather(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z,
                                  T (&d)[Q], Shift sh = Shift{0u, 0u}) {
    static_assert(!(Pair && Face), "paired rows lie off the y and z faces");
    constexpr uint32_t es = sizeof(S);
    const int64_t r = (int64_t)z * g.ny + y;
    // Each direction reads a run of its source row through a base one value
    // before the run; the lane offset selects x - cx(a) + 1, wrapped on a
    // periodic x axis.  Offsets stay within nx + 2 values of the base.  On a
    // non-periodic x face the source column x - cx(a) = -1 or nx is a ghost,
    // whose value the x-face rule below supplies: those lanes take an offset
    // beyond the descriptor's range, so the load returns 0 without touching
    // memory (and the cache line past the run is not fetched for them).
    // (the ranges pass through readfirstlane so that the compiler keeps the
    // descriptors in scalar registers)
    // (a second half's offsets, past D, stay outside too: D + (nx + 2) values < 2^31 bytes)
    const uint32_t run_range = __builtin_amdgcn_readfirstlane((uint32_t)(g.nx + 2) * es);
    const uint32_t range = Pair ? run_range + sh.range : run_range;
    const uint32_t add = Pair ? sh.lane : 0u;
    constexpr uint32_t outside = 0x80000000u;
    const uint32_t o0 = (uint32_t)(x + 1) * es + add;
    const uint32_t op = (x == 0 ? (g.px ? run_range - 2 * es : outside) : (uint32_t)x * es) + add;     // cx = +1
    const uint32_t om = (x == g.nx - 1 ? (g.px ? es : outside) : (uint32_t)(x + 2) * es) + add;      // cx = -1
    auto lane_off = [&](int a) { return cx(a) == 1 ? op : (cx(a) == -1 ? om : o0); };
    auto run = [&](int a, int64_t row) {
        return row_rsrc(A + row * g.row + (int64_t)a * g.nx - 1, range);
    };
    // the node's own row group, for the bounce-back values (slot in the lane offset)
    const uint32_t own_range = __builtin_amdgcn_readfirstlane((uint32_t)Q * (uint32_t)g.nx * es);
    const __amdgpu_buffer_rsrc_t own_rsrc = row_rsrc(A + r * g.row, Pair ? own_range + sh.range : own_range);
    auto own = [&](int a) {
        return (T)RawBits<S>::template load<LdAux>(own_rsrc, (uint32_t)(opp(a) * g.nx + x) * es + add);
    };
    if constexpr (!Face) {
#pragma unroll
        for (int a = 0; a < Q; ++a)
            d[a] = (T)RawBits<S>::template load<LdAux>(run(a, r - cy(a) - (int64_t)cz(a) * g.ny), lane_off(a));
    } else {
        // rows on a y or z face: per direction (uniformly) the source row is
        // inside, wrapped on a periodic axis, or a ghost: half-way bounce-back
        // returns the node's own population opposite to a, plus the
        // moving-wall term for a ghost in the lid plane
        const int m = g.lid_mask;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            int sy = y - cy(a), sz = z - cz(a);
            bool wall = false;
            if (sy < 0 || sy >= g.ny) { if (g.py) sy = sy < 0 ? sy + g.ny : sy - g.ny; else wall = true; }
            if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
            if (!wall) {
                d[a] = (T)RawBits<S>::template load<LdAux>(run(a, (int64_t)sz * g.ny + sy), lane_off(a));
            } else {
                const int sx = x - cx(a);
                const bool in_lid = ((m & 4) && sy == -1) || ((m & 8) && sy == g.ny) || ((m & 16) && sz == -1) ||
                                    ((m & 32) && sz == g.nz) || ((m & 1) && sx == -1) || ((m & 2) && sx == g.nx);
                d[a] = wall_value<T>(own(a), p, a, in_lid);
            }
        }
    }
    // lanes on a non-periodic x face: directions whose source row is inside
    // the lattice but whose source column is a ghost take the bounce-back of
    // the node's own opposite population (XGroup: the wave issues these loads
    // all together, the lanes without such a ghost taking an out-of-range
    // offset, i.e. no memory access, and selects the wall values afterwards,
    // so that it waits for memory once instead of once per direction)
    if constexpr (!XGroup) {
        if (!g.px && (x == 0 || x == g.nx - 1)) {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                if (cx(a) == 0 || !((x == 0 && cx(a) == 1) || (x == g.nx - 1 && cx(a) == -1))) continue;
                const int sy = y - cy(a), sz = z - cz(a);
                const bool row_wall = (!g.py && (sy < 0 || sy >= g.ny)) || (!g.pz && (sz < 0 || sz >= g.nz));
                if (row_wall) continue;     // bounced back above, with the lid term of every ghost coordinate
                d[a] = wall_value<T>(own(a), p, a, (g.lid_mask & (cx(a) == 1 ? 1 : 2)) != 0);
            }
        }
    } else if (!g.px) {
        const bool lo = x == 0, hi = x == g.nx - 1;
        if (__builtin_amdgcn_ballot_w64(lo || hi) != 0) {       // uniform over the wave
            T o[Q];
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                if (cx(a) == 0) continue;
                const bool ghost = cx(a) == 1 ? lo : hi;
                o[a] = (T)RawBits<S>::template load<LdAux>(
                    own_rsrc, ghost ? (uint32_t)(opp(a) * g.nx + x) * es + add : outside);
            }
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                if (cx(a) == 0) continue;
                const int sy = y - cy(a), sz = z - cz(a);
                const bool row_wall = (!g.py && (sy < 0 || sy >= g.ny)) || (!g.pz && (sz < 0 || sz >= g.nz));
                if (row_wall) continue;     // bounced back above, with the lid term of every ghost coordinate
                const bool ghost = cx(a) == 1 ? lo : hi;
                const T w = wall_value<T>(o[a], p, a, (g.lid_mask & (cx(a) == 1 ? 1 : 2)) != 0);
                d[a] = ghost ? w : d[a];
            }
        }
    }
}

// Store of the 19 populations of node x of row (y, z) (y, z uniform; Pair:
// the second half's lanes shifted as in row_gather).  FP16 with stochastic
// rounding (sr): rounded in the store itself with the seeds of round_state
// (sr_base = sr_base(node, step)).
template <typename S, typename T, int StAux, bool Pair = false>
__device__ inline void row_store(S *__restrict__ B, const Geom &g, int x, int y, int z, const T (&d)[Q],
                                 bool sr = false, uint32_t seed_base = 0, Shift sh = Shift{0u, 0u}) {
    constexpr uint32_t es = sizeof(S);
    const uint32_t run_range = __builtin_amdgcn_readfirstlane((uint32_t)g.nx * es);
    const uint32_t srange = Pair ? run_range + sh.range : run_range;
    S *out = B + ((int64_t)z * g.ny + y) * g.row;
    const uint32_t lane = (uint32_t)x * es + (Pair ? sh.lane : 0u);
    if constexpr (std::is_same<S, __half>::value) {
        if (sr) {
            // each conversion keeps the high half of its first operand: the
            // previous direction's result (stored already) serves, so no
            // register is cleared per value; the stored low halves are those
            // of sr_to_f16_bits
            typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
            half2_t h = __builtin_bit_cast(half2_t, (float)d[0]);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                h = __builtin_amdgcn_cvt_sr_f16_f32(h, (float)d[a], seed_base + (uint32_t)a * kWeyl, false);
                __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, h[0]),
                                                      row_rsrc(out + (int64_t)a * g.nx, srange), (int)lane, 0, StAux);
            }
            return;
        }
    }
#pragma unroll
    for (int a = 0; a < Q; ++a)
        RawBits<S>::template store<StAux>(row_rsrc(out + (int64_t)a * g.nx, srange), lane, d[a]);
}

// One step of node x of row (y, z): gather, collide, store; `step` is the
// index of the collision (keys the stochastic rounding of FP16 storage).
template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route, bool Face, bool XGroup = false>
__device__ inline void row_step(const S *__restrict__ A, S *__restrict__ B, const Geom &g, const Relax<T> &p, int x,
                                int y, int z, uint32_t step) {
    T d[Q];
    row_gather<S, T, LdAux, Face, false, XGroup>(A, g, p, x, y, z, d);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    const uint32_t node = (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
    row_store<S, T, StAux>(B, g, x, y, z, d, p.sr != 0, sr_base(node, step));
}

// The same step for a wave serving two inner rows r = y + ny z (lanes with
// hi false) and r + k (lanes with hi true), each lane at column x of its row.
template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route>
__device__ inline void row_step_pair(const S *__restrict__ A, S *__restrict__ B, const Geom &g, const Relax<T> &p,
                                     int x, int y, int z, uint32_t k, bool hi, uint32_t step) {
    constexpr uint32_t es = sizeof(S);
    const uint32_t D = k * (uint32_t)g.row * es;
    const Shift sh{hi ? D : 0u, D};
    T d[Q];
    row_gather<S, T, LdAux, false, true, XGroupRows<S>::value>(A, g, p, x, y, z, d, sh);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    const uint32_t node = (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z + (hi ? k : 0u));
    row_store<S, T, StAux, true>(B, g, x, y, z, d, p.sr != 0, sr_base(node, step), sh);
}

}  // namespace clbm
