// Two time steps per launch: temporal blocking of the pull stream-collide.
//
// A workgroup is ROWS waves.  Wave w works on lattice row y0 - 1 + w and lane
// l on column x0 - 1 + l, so the workgroup covers a 64 x ROWS patch of
// columns whose inner 62 x (ROWS - 2) columns are its output.  It marches
// along z through its chunk of output planes [z0, z1).  For plane m it first
// computes the state after the first step, I(m), at every column of the patch
// (the ring of halo columns included) exactly as the one-step kernel does
// (same gather with the wall rules, same collision, rounded to the storage
// type), and keeps it on chip.  Output plane z = m - 1 then pulls its
// second-step inputs from I(z - 1), I(z) and I(z + 1) instead of memory,
// collides and is written.  The result is the state that two one-step
// launches leave; memory sees one read of the patch (with its halo) and one
// write per node per two steps.
//
// On-chip placement of I(m), by the direction's (e_y, e_z):
//   e_y = 0   registers of the column's own lane, passed to the x neighbours
//             by lane shuffles: e_z = 0 {0, 1, 2}, +1 {5, 11, 12}, -1 {6, 13, 14};
//   e_y != 0  LDS rings indexed by plane: e_z = 0 {3, 4, 7, 8, 9, 10} three
//             slots, e_z = +1 {15, 16} four slots, e_z = -1 {17, 18} three.
// A plane's e_z = +1 values are read by the output plane above it, its
// e_z = -1 values by the plane below, and all of its own-node values serve
// the bounce-back of the output plane at its own height.  With one barrier per
// plane, a slot read while producing output z is rewritten no earlier than
// while producing z + 2, which the ring sizes guarantee.
//
// Either state layout: in the row layout a wave's first-step row and output
// row are lattice rows, so its loads and stores go through the one-step row
// kernel's gather and store (scalar row bases, one lane offset); in the planes
// layout through the per-plane gather.
#include "clbm_rows.hpp"

namespace clbm {

namespace {

constexpr int kLanes = 64;
constexpr int kOut = kLanes - 2;    // output columns per wave

// position of an e_y != 0 direction inside its LDS group
__host__ __device__ constexpr int lds_index(int a) {
    return a == 3 ? 0 : a == 4 ? 1 : a == 7 ? 2 : a == 8 ? 3 : a == 9 ? 4 : a == 10 ? 5
         : a == 15 || a == 17 ? 0 : 1;
}
// register slot of an e_y = 0 direction inside its e_z class
__host__ __device__ constexpr int reg_index(int a) { return cx(a) == 0 ? 0 : (cx(a) == 1 ? 1 : 2); }

template <typename S, int ROWS> struct FusedShared {
    S e0[3][6][ROWS][kLanes];
    S up[4][2][ROWS][kLanes];
    S dn[3][2][ROWS][kLanes];
};

// prefetched first-step inputs of the next plane: one row per wave, each
// lane's 19 values at its own position (written by direct-to-LDS loads); a
// separate LDS object, so that reads of the rings need not wait for them
template <typename S, int ROWS, bool PF> struct FusedInput {
    S in[PF ? Q : 1][PF ? ROWS : 1][PF ? kLanes : 1];
};

// s_waitcnt lgkmcnt(0) with vmcnt and expcnt left free (gfx9 encoding)
constexpr int kWaitLgkmcnt0 = 0xC07F;

// element size of a direct-to-LDS load (allowed: 1, 2, 4, 12, 16 bytes)
template <typename S, bool PF> struct LdsBytes { static constexpr int value = PF ? (int)sizeof(S) : 4; };

// s_waitcnt vmcnt(0) with the other counters left free (gfx9 encoding)
constexpr int kWaitVmcnt0 = 0x0F70;

// DPP controls of the whole-wave shifts by one lane (gfx9 encoding): lane l
// reads lane l - 1 (shift right) or lane l + 1 (shift left)
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

// x neighbours of the e_y = 0 values held in registers: lane l takes lane
// l - 1's value (from_left) or lane l + 1's (from_right); the end lanes get
// values no output uses.  FP32 by a whole-wave DPP shift (one VALU move,
// no LDS round trip), FP64 through the LDS permute.
template <typename T> __device__ inline T from_left(T v) { return __shfl_up(v, 1, kLanes); }
template <typename T> __device__ inline T from_right(T v) { return __shfl_down(v, 1, kLanes); }
template <> __device__ inline float from_left<float>(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kDppWaveShr1, 0xF, 0xF,
                                                                 false));
}
template <> __device__ inline float from_right<float>(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kDppWaveShl1, 0xF, 0xF,
                                                                 false));
}

template <typename S, typename T> __device__ inline T round_trip(T v) {
    return Conv<S, T>::load(Conv<S, T>::store(v));
}

}  // namespace

struct FusedGrid {
    uint32_t gx, gy, gz;    // patches along x and y, z chunks
    int32_t cz;             // output planes per z chunk
    uint32_t aligned;       // largest multiple of 8 <= number of workgroups
    int32_t remap;          // XCD-contiguous patch order
};

// StAux: cache hint of the population stores (0 plain, 2 non-temporal);
// Rows: row layout (else planes)
template <typename S, typename T, bool Forced, int Route, int ROWS, bool PF, int StAux, bool Rows>
__global__ void __launch_bounds__(kLanes * ROWS)
stream_collide2_kernel(const S *__restrict__ A, S *__restrict__ B, Geom g, Relax<T> p, FusedGrid L) {
    static_assert(!(Rows && PF), "the direct-to-LDS prefetch reads the planes layout");
    __shared__ FusedShared<S, ROWS> sh;
    __shared__ FusedInput<S, ROWS, PF> pf;
    const int l = (int)(threadIdx.x & (kLanes - 1));
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kLanes));
    uint32_t b = blockIdx.x;
    // XCD-contiguous order: workgroups b, b + 8, ... share an XCD (and its L2),
    // so they take neighbouring patches, whose halos and partly written cache
    // lines then meet in the same cache
    if (L.remap && b < L.aligned) b = (b & 7u) * (L.aligned >> 3) + (b >> 3);
    const int tx = (int)(b % L.gx);
    b /= L.gx;
    const int ty = (int)(b % L.gy);
    const int tz = (int)(b / L.gy);
    const int gx = tx * kOut - 1 + l;             // this lane's column (unwrapped)
    const int gy = ty * (ROWS - 2) - 1 + w;       // this wave's row (unwrapped)
    const int z0 = tz * L.cz;
    const int z1 = min(z0 + L.cz, g.nz);
    const bool out = l >= 1 && l <= kOut && gx < g.nx && w >= 1 && w <= ROWS - 2 && gy < g.ny;

    // First-step column of this lane: needed up to one past the last output
    // column/row; wrapped on periodic axes; none (a ghost) beyond a wall.
    int wx = gx, wy = gy;
    bool col = gx <= min(g.nx, tx * kOut + kOut) && gy <= min(g.ny, ty * (ROWS - 2) + ROWS - 2);
    if (wx < 0 || wx >= g.nx) { if (g.px) wx = wx < 0 ? wx + g.nx : wx - g.nx; else col = false; }
    if (wy < 0 || wy >= g.ny) { if (g.py) wy = wy < 0 ? wy + g.ny : wy - g.ny; else col = false; }

    T r0c[3], r0n[3];              // e_z = 0,  e_y = 0 of I(z), I(z + 1)
    T rpp[3], rpc[3], rpn[3];      // e_z = +1, e_y = 0 of I(z - 1), I(z), I(z + 1)
    T rmc[3], rmn[3];              // e_z = -1, e_y = 0 of I(z), I(z + 1)

    // Issue the interior pull loads of plane m straight into this wave's row
    // of sh.in (no registers held while they are in flight).
    auto prefetch = [&](int m) {
        if constexpr (PF) {
            const S *Am = A;
            asm volatile("" : "+s"(Am));
            int wz = m;
            bool v = col;
            if (wz < 0 || wz >= g.nz) { if (g.pz) wz = wz < 0 ? wz + g.nz : wz - g.nz; else v = false; }
            if (v) {
                const uint32_t self = (uint32_t)wx + (uint32_t)g.nx * (uint32_t)wy + (uint32_t)g.nxy * (uint32_t)wz;
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                        (void *)(Am + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * sizeof(S)), kBufferFlags);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        r, (__attribute__((address_space(3))) void *)&pf.in[a][w][0], LdsBytes<S, PF>::value,
                        (int)(pull_offset(g, a, self) * sizeof(S)), 0, 0, 0);
                }
            }
        }
    };

    // I(m) into LDS ring slots (index jm = m - z0 + 1) and the given registers
    auto first_step = [&](int m, int jm, T (&o0)[3], T (&op)[3], T (&om)[3]) {
        // The buffer descriptors of the 19 planes are rebuilt from the base
        // pointer on every plane instead of being kept (and spilled) across
        // the loop: the empty asm hides the pointer's loop invariance.
        const S *Am = A;
        asm volatile("" : "+s"(Am));
        int wz = m;
        bool v = col;
        if (wz < 0 || wz >= g.nz) { if (g.pz) wz = wz < 0 ? wz + g.nz : wz - g.nz; else v = false; }
        T d[Q];
        if constexpr (PF) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // this wave's prefetch has landed
        if (v) {
            const uint32_t self = (uint32_t)wx + (uint32_t)g.nx * (uint32_t)wy + (uint32_t)g.nxy * (uint32_t)wz;
            if constexpr (Rows) {
                // the wave's row (wy, wz) is uniform: off the y and z faces, or on one
                if (wy >= 1 && wy <= g.ny - 2 && wz >= 1 && wz <= g.nz - 2)
                    row_gather<S, T, 0, false, false, XGroupRows<S>::value>(A, g, p, wx, wy, wz, d);
                else
                    row_gather<S, T, 0, true, false, XGroupRows<S>::value>(A, g, p, wx, wy, wz, d);
            } else if constexpr (PF) {
#pragma unroll
                for (int a = 0; a < Q; ++a) d[a] = Conv<S, T>::load(pf.in[a][w][l]);
                fix_edges<S, T>(Am, g, p, wx, wy, wz, self, d);
            } else {
                gather<S, T, 0>(Am, g, p, wx, wy, wz, self, d);
            }
            collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
            round_state<S, T>(d, p, self, p.step);
        } else {
#pragma unroll
            for (int a = 0; a < Q; ++a) d[a] = T(0);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if (cy(a) == 0) {
                const T r = round_trip<S, T>(d[a]);
                if (cz(a) == 0) o0[reg_index(a)] = r;
                else if (cz(a) == 1) op[reg_index(a)] = r;
                else om[reg_index(a)] = r;
            } else if (cz(a) == 0) {
                sh.e0[jm % 3][lds_index(a)][w][l] = Conv<S, T>::store(d[a]);
            } else if (cz(a) == 1) {
                sh.up[jm % 4][lds_index(a)][w][l] = Conv<S, T>::store(d[a]);
            } else {
                sh.dn[jm % 3][lds_index(a)][w][l] = Conv<S, T>::store(d[a]);
            }
        }
    };

    // second step at output plane z (jz = z - z0 + 1 indexes I(z))
    auto second_step = [&](int z, int jz) {
        // every lane takes part in the shuffles; lanes 1..62 use them
        const T n1 = from_left(r0c[1]), n2 = from_right(r0c[2]);
        const T n11 = from_left(rpp[1]), n12 = from_right(rpp[2]);
        const T n13 = from_left(rmn[1]), n14 = from_right(rmn[2]);
        if (!out) return;
        T d[Q];
        d[0] = r0c[0]; d[1] = n1; d[2] = n2;
        d[5] = rpp[0]; d[11] = n11; d[12] = n12;
        d[6] = rmn[0]; d[13] = n13; d[14] = n14;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if (cy(a) == 0) continue;
            const int r = w - cy(a), c = l - cx(a);
            if (cz(a) == 0) d[a] = Conv<S, T>::load(sh.e0[jz % 3][lds_index(a)][r][c]);
            else if (cz(a) == 1) d[a] = Conv<S, T>::load(sh.up[(jz + 3) % 4][lds_index(a)][r][c]);
            else d[a] = Conv<S, T>::load(sh.dn[(jz + 1) % 3][lds_index(a)][r][c]);
        }
        const bool xw = !g.px && (gx == 0 || gx == g.nx - 1);
        const bool yw = !g.py && (gy == 0 || gy == g.ny - 1);
        const bool zw = !g.pz && (z == 0 || z == g.nz - 1);
        if (xw || yw || zw) {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const int sx = gx - cx(a), sy = gy - cy(a), sz = z - cz(a);
                const bool ghost = (!g.px && (sx < 0 || sx >= g.nx)) || (!g.py && (sy < 0 || sy >= g.ny)) ||
                                   (!g.pz && (sz < 0 || sz >= g.nz));
                if (!ghost) continue;
                const int o = opp(a);
                T own;
                if (cy(o) == 0)
                    own = cz(o) == 0 ? r0c[reg_index(o)] : (cz(o) == 1 ? rpc[reg_index(o)] : rmc[reg_index(o)]);
                else if (cz(o) == 0)
                    own = Conv<S, T>::load(sh.e0[jz % 3][lds_index(o)][w][l]);
                else if (cz(o) == 1)
                    own = Conv<S, T>::load(sh.up[jz % 4][lds_index(o)][w][l]);
                else
                    own = Conv<S, T>::load(sh.dn[jz % 3][lds_index(o)][w][l]);
                d[a] = wall_value<T>(own, p, a, ghost_in_lid(g, sx, sy, sz));
            }
        }
        collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
        round_state<S, T>(d, p, (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy + (uint32_t)g.nxy * (uint32_t)z, p.step + 1u);
        if constexpr (Rows) {
            row_store<S, T, StAux>(B, g, gx, gy, z, d);
        } else {
            S *Bz = B;
            asm volatile("" : "+s"(Bz));
            const uint32_t self = (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy + (uint32_t)g.nxy * (uint32_t)z;
#pragma unroll
            for (int a = 0; a < Q; ++a) Plane<S, StAux>::store(Bz, g, a, self, d[a]);
        }
    };

    // plane m = z0 - 1 .. z1: first step of I(m), then the output plane m - 1
    prefetch(z0 - 1);
    for (int m = z0 - 1; m <= z1; ++m) {
        first_step(m, m - z0 + 1, r0n, rpn, rmn);
        if (m < z1) prefetch(m + 1);
        if constexpr (PF) {
            // only the LDS ring writes must be visible to the other waves; the
            // prefetch stays in flight across the barrier
            __builtin_amdgcn_s_waitcnt(kWaitLgkmcnt0);
            __builtin_amdgcn_s_barrier();
        } else {
            __syncthreads();
        }
        if (m > z0) second_step(m - 1, m - z0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            r0c[k] = r0n[k];
            rpp[k] = rpc[k];
            rpc[k] = rpn[k];
            rmc[k] = rmn[k];
        }
    }
}

template <typename S, typename T, bool Forced, int Route, int ROWS, bool PF, bool Rows>
static hipError_t launch2_f(const void *A, void *B, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                            hipStream_t st) {
    FusedGrid L;
    L.gx = (uint32_t)((g.nx + kOut - 1) / kOut);
    L.gy = (uint32_t)((g.ny + ROWS - 3) / (ROWS - 2));
    L.cz = c.fuse_planes;
    L.gz = (uint32_t)((g.nz + c.fuse_planes - 1) / c.fuse_planes);
    const uint64_t nb = (uint64_t)L.gx * L.gy * L.gz;
    if (nb == 0 || nb > 0x7fffffffull) return hipErrorInvalidValue;
    L.aligned = (uint32_t)nb & ~7u;
    L.remap = c.xcd_remap;
    if (c.nt_stores)
        hipLaunchKernelGGL((stream_collide2_kernel<S, T, Forced, Route, ROWS, PF, 2, Rows>), dim3((uint32_t)nb),
                           dim3(kLanes * ROWS), 0, st, (const S *)A, (S *)B, g, p, L);
    else
        hipLaunchKernelGGL((stream_collide2_kernel<S, T, Forced, Route, ROWS, PF, 0, Rows>), dim3((uint32_t)nb),
                           dim3(kLanes * ROWS), 0, st, (const S *)A, (S *)B, g, p, L);
    return hipGetLastError();
}

template <typename S, typename T, int ROWS, bool PF, bool Rows>
static hipError_t launch2_l(const void *A, void *B, const Geom &g, const Relax<T> &p, bool forced, int route,
                            const StepLaunch &c, hipStream_t st) {
    if (route == 0)
        return forced ? launch2_f<S, T, true, 0, ROWS, PF, Rows>(A, B, g, p, c, st)
                      : launch2_f<S, T, false, 0, ROWS, PF, Rows>(A, B, g, p, c, st);
    return forced ? launch2_f<S, T, true, 1, ROWS, PF, Rows>(A, B, g, p, c, st)
                  : launch2_f<S, T, false, 1, ROWS, PF, Rows>(A, B, g, p, c, st);
}

// row layout: no direct-to-LDS prefetch (ROWS 12 runs without it)
template <typename S, typename T, int ROWS, bool PF = false>
static hipError_t launch2_r(const void *A, void *B, const Geom &g, const Relax<T> &p, bool forced, int route,
                            const StepLaunch &c, hipStream_t st) {
    return g.rows ? launch2_l<S, T, ROWS, false, true>(A, B, g, p, forced, route, c, st)
                  : launch2_l<S, T, ROWS, PF, false>(A, B, g, p, forced, route, c, st);
}

hipError_t launch_step2(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                        const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st) {
    if (c.fuse_planes < 1 || route == 2) return hipErrorInvalidValue;   // no two-step form of the BGK model
    const int rows = c.fuse_rows;
    switch (storage) {
    case 0:
        if (rows != 8) return hipErrorInvalidValue;
        return launch2_r<double, double, 8>(A, B, g, pd, forced, route, c, st);
    case 1:
        // rows 12: the next plane's loads go straight to LDS (153 KiB in all)
        return rows == 16 ? launch2_r<float, float, 16>(A, B, g, pf, forced, route, c, st)
             : rows == 12 ? launch2_r<float, float, 12, true>(A, B, g, pf, forced, route, c, st)
                          : launch2_r<float, float, 8>(A, B, g, pf, forced, route, c, st);
    default:
        return rows == 16 ? launch2_r<__half, float, 16>(A, B, g, pf, forced, route, c, st)
                          : launch2_r<__half, float, 8>(A, B, g, pf, forced, route, c, st);
    }
}

}  // namespace clbm
