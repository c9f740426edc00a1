// One time step on the row layout: the 19 populations of lattice row
// r = y + ny z are stored as 19 consecutive runs of nx values, population a
// of node x at element (19 r + a) nx + x.
//
// A step then reads, for every row, parts of the 9 row groups r - e_y - ny e_z
// and writes one row group: a few compact regions instead of 38 planes spread
// over the whole buffer, which keeps the DRAM page and bank traffic of
// neighbouring waves together.
//
//   stream_collide_rows       rows off the y and z faces.  Each wave covers
//                             64 consecutive x of one row (blockDim.x a
//                             multiple of 64), so the source of direction a
//                             is a uniform address plus the lane's x: one
//                             scalar base per load and store, one shared
//                             lane offset; only the lanes on an x face take a
//                             wall rule.
//   stream_collide_rows_face  the rows on a y or z face (about 6/L of an L^3
//                             lattice), launched after the first kernel: per
//                             direction, uniformly, a source row inside,
//                             wrapped, or a ghost (bounce-back).  Keeping them
//                             apart keeps the first kernel's scalar registers
//                             low enough for eight waves per SIMD.
//   stream_collide_any        any block shape: the full rule on every lane
//                             (narrow lattices).
#include "clbm_rows.hpp"

namespace clbm {

namespace {

// Pull along e_a with the full wall logic (Eq. cascaded streaming with the
// rules of Sec. 4), in either layout: periodic wrap, half-way bounce-back,
// moving lid.  a = 0 returns the node's own rest population.
template <typename S, typename T>
__device__ inline T pull_any(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int a, int x, int y, int z) {
    int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
    const bool in_lid = ghost_in_lid(g, sx, sy, sz);
    bool wall = false;
    if (sx < 0 || sx >= g.nx) { if (g.px) sx = sx < 0 ? sx + g.nx : sx - g.nx; else wall = true; }
    if (sy < 0 || sy >= g.ny) { if (g.py) sy = sy < 0 ? sy + g.ny : sy - g.ny; else wall = true; }
    if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
    if (!wall) return (T)Conv<S, T>::load(A[elem(g, a, sx, sy, sz)]);
    return wall_value<T>((T)Conv<S, T>::load(A[elem(g, opp(a), x, y, z)]), p, a, in_lid);
}

__device__ inline void tile_of(const LaunchGrid &L, uint32_t &tx, uint32_t &ty, int &z) {
    uint32_t b = blockIdx.x;
    if (L.remap && b < L.aligned) b = (b & 7u) * (L.aligned >> 3) + (b >> 3);
    tx = b % L.gx;
    b /= L.gx;
    ty = b % L.gy;
    z = (int)(b / L.gy);
}

}  // namespace

template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
stream_collide_rows_kernel(const S *__restrict__ A, S *__restrict__ B, Geom g, Relax<T> p, RowGrid R) {
    int x;
    uint32_t ri;
    if (!row_of(R, x, ri) || x >= g.nx) return;
    int y, z;
    inner_row(g, ri, y, z);
    row_step<S, T, Forced, LdAux, StAux, Route, false, XGroupRows<S>::value>(A, B, g, p, x, y, z, p.step);
}

template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
stream_collide_rows_face_kernel(const S *__restrict__ A, S *__restrict__ B, Geom g, Relax<T> p, RowGrid R) {
    int x;
    uint32_t ri;
    if (!row_of(R, x, ri) || x >= g.nx) return;
    int y, z;
    face_row(g, R, ri, y, z);
    row_step<S, T, Forced, LdAux, StAux, Route, true, XGroupRows<S>::value>(A, B, g, p, x, y, z, p.step);
}

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
stream_collide_any_kernel(const S *__restrict__ A, S *__restrict__ B, Geom g, Relax<T> p, LaunchGrid L) {
    uint32_t tx, ty;
    int z;
    tile_of(L, tx, ty, z);
    const int x = (int)(tx * blockDim.x + threadIdx.x);
    const int y = (int)(ty * blockDim.y + threadIdx.y);
    if (y >= g.ny || x >= g.nx) return;
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = pull_any<S, T>(A, g, p, a, x, y, z);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z), p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) B[elem(g, a, x, y, z)] = Conv<S, T>::store(d[a]);
}

template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route>
static hipError_t launch_rows_k(const S *a, S *b, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                                hipStream_t st) {
    // inner rows, then the face rows
    const RowLaunch L = row_launch(g, c.bx, c.by, c.xcd_remap);
    const dim3 block(c.bx, c.by);
    if (L.inner.rows > 0) {
        hipLaunchKernelGGL((stream_collide_rows_kernel<S, T, Forced, LdAux, StAux, Route>), dim3(L.inner_blocks),
                           block, 0, st, a, b, g, p, L.inner);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((stream_collide_rows_face_kernel<S, T, Forced, LdAux, StAux, Route>), dim3(L.face_blocks),
                       block, 0, st, a, b, g, p, L.face);
    return hipGetLastError();
}

template <typename S, typename T, bool Forced, int Route>
static hipError_t launch_rows_f(const void *A, void *B, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                                hipStream_t st) {
    const S *a = (const S *)A;
    S *b = (S *)B;
    if (c.bx % 64 != 0) {
        LaunchGrid L;
        L.gx = (g.nx + c.bx - 1) / c.bx;
        L.gy = (g.ny + c.by - 1) / c.by;
        L.gz = g.nz;
        const uint32_t nb = L.gx * L.gy * L.gz;
        L.aligned = nb & ~7u;
        L.remap = c.xcd_remap;
        hipLaunchKernelGGL((stream_collide_any_kernel<S, T, Forced, Route>), dim3(nb), dim3(c.bx, c.by), 0, st, a, b,
                           g, p, L);
        return hipGetLastError();
    }
    if (Route != 0)     // the printed form and the comparison model: only the store hint is tunable
        return c.nt_stores ? launch_rows_k<S, T, Forced, 0, 2, Route>(a, b, g, p, c, st)
                           : launch_rows_k<S, T, Forced, 0, 0, Route>(a, b, g, p, c, st);
    switch ((c.nt_loads ? 1 : 0) | (c.nt_stores ? 2 : 0)) {
    case 0: return launch_rows_k<S, T, Forced, 0, 0, Route>(a, b, g, p, c, st);
    case 1: return launch_rows_k<S, T, Forced, 2, 0, Route>(a, b, g, p, c, st);
    case 2: return launch_rows_k<S, T, Forced, 0, 2, Route>(a, b, g, p, c, st);
    default: return launch_rows_k<S, T, Forced, 2, 2, Route>(a, b, g, p, c, st);
    }
}

template <typename S, typename T>
static hipError_t launch_rows_t(const void *A, void *B, const Geom &g, const Relax<T> &p, bool forced, int route,
                                const StepLaunch &c, hipStream_t st) {
    if (route == 2) return forced ? hipErrorInvalidValue : launch_rows_f<S, T, false, 2>(A, B, g, p, c, st);
    if (route == 0)
        return forced ? launch_rows_f<S, T, true, 0>(A, B, g, p, c, st) : launch_rows_f<S, T, false, 0>(A, B, g, p, c, st);
    return forced ? launch_rows_f<S, T, true, 1>(A, B, g, p, c, st) : launch_rows_f<S, T, false, 1>(A, B, g, p, c, st);
}

hipError_t launch_step_rows(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                            const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st) {
    switch (storage) {
    case 0: return launch_rows_t<double, double>(A, B, g, pd, forced, route, c, st);
    case 1: return launch_rows_t<float, float>(A, B, g, pf, forced, route, c, st);
    default: return launch_rows_t<__half, float>(A, B, g, pf, forced, route, c, st);
    }
}

}  // namespace clbm
