// In-place stepping with one state buffer: the AA access pattern.
//
// The buffer holds pre-collision populations in their natural slots (slot a
// of node x holds f_a(x)) before an even step.
//   even step: every node collides its own populations and stores f~_a into
//              its own slot opp(a);
//   odd step:  node x pulls f~_a(x - e_a) from slot opp(a) of x - e_a (where
//              the even step left it), collides, and pushes f~_a(x) to slot a
//              of x + e_a, its natural slot for the next even step.
// A pair of launches advances two time steps (collide, stream, collide,
// stream) with the same memory traffic per node update as the two-buffer
// pull, in half the memory.  Within a launch each node reads and then
// overwrites exactly the locations no other node touches: the odd step's read
// set {(opp(a), x - e_a)} equals its write set {(a, x + e_a)}.  Walls: a
// ghost source returns the node's own f~_opp(a), which the even step left in
// slot a of x, plus the lid term; a ghost target sends f~_a back into slot
// opp(a) of x with the lid term of direction opp(a) — the value the pull rule
// gives at the next step.  Periodic axes wrap.
#include "clbm_rows.hpp"

namespace clbm {

namespace {

__device__ inline bool wrap(int &c, int n, int periodic) {
    if (c >= 0 && c < n) return true;
    if (!periodic) return false;
    c = c < 0 ? c + n : c - n;
    return true;
}

__device__ inline void locate(const LaunchGrid &L, int &x, int &y, int &z) {
    uint32_t b = blockIdx.x;
    if (L.remap && b < L.aligned) b = (b & 7u) * (L.aligned >> 3) + (b >> 3);
    const uint32_t tx = b % L.gx;
    b /= L.gx;
    const uint32_t ty = b % L.gy;
    z = (int)(b / L.gy);
    x = (int)(tx * blockDim.x + threadIdx.x);
    y = (int)(ty * blockDim.y + threadIdx.y);
}

}  // namespace

// The even step writes back into the lines it has just read.
constexpr int EvenStAux = 0;

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_even_kernel(S *__restrict__ A, Geom g, Relax<T> p, LaunchGrid L) {
    int x, y, z;
    locate(L, x, y, z);
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t self = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y + (uint32_t)g.nxy * (uint32_t)z;
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = (T)Plane<S>::load(A, g, a, self);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, self, p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) Plane<S, EvenStAux>::store(A, g, opp(a), self, d[a]);
}

// The odd step's pushes land one element off the wave's alignment along x:
// ordinary (cached) stores let L2 merge the partial lines of neighbouring waves.
constexpr int OddStAux = 0;

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_odd_kernel(S *__restrict__ A, Geom g, Relax<T> p, LaunchGrid L) {
    int x, y, z;
    locate(L, x, y, z);
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t self = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y + (uint32_t)g.nxy * (uint32_t)z;
    const bool edge = x == 0 || x == g.nx - 1 || y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = (T)Plane<S>::load(A, g, opp(a), pull_offset(g, a, self));
    if (edge) {
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
            const bool in_lid = ghost_in_lid(g, sx, sy, sz);
            const bool ok = wrap(sx, g.nx, g.px) & wrap(sy, g.ny, g.py) & wrap(sz, g.nz, g.pz);
            if (ok)
                d[a] = (T)Plane<S>::load(A, g, opp(a), (uint32_t)(sx + g.nx * sy + g.nxy * sz));
            else
                d[a] = wall_value<T>((T)Plane<S>::load(A, g, a, self), p, a, in_lid);
        }
    }
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, self, p.step);
    if (!edge) {
#pragma unroll
        for (int a = 0; a < Q; ++a)
            Plane<S, OddStAux>::store(A, g, a, self + (uint32_t)(cx(a) + cy(a) * g.nx + cz(a) * g.nxy), d[a]);
        return;
    }
    Plane<S, 2>::store(A, g, 0, self, d[0]);
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        int tx = x + cx(a), ty = y + cy(a), tz = z + cz(a);
        const bool in_lid = ghost_in_lid(g, tx, ty, tz);
        const bool ok = wrap(tx, g.nx, g.px) & wrap(ty, g.ny, g.py) & wrap(tz, g.nz, g.pz);
        if (ok)
            Plane<S, 2>::store(A, g, a, (uint32_t)(tx + g.nx * ty + g.nxy * tz), d[a]);
        else
            Plane<S, 2>::store(A, g, opp(a), self, wall_value<T>(d[a], p, opp(a), in_lid));
    }
}

// f0 (FP64, unpadded planes; NULL: the rest state) written as deviations
// into the natural slots, without a collision.
template <typename S>
__global__ void __launch_bounds__(256) store_plain_kernel(const double *__restrict__ f0, S *__restrict__ A, Geom g) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    using T = typename StoreCompute<S>::T;
#pragma unroll
    for (int a = 0; a < Q; ++a)
        A[elem_i(g, a, i)] = Conv<S, T>::store(f0 ? (T)(f0[(int64_t)a * N + i] - weight(a)) : T(0));
}

// ---------------------------------------------------------------------------
// The same pair of steps on the row layout (waves of 64 x of one row; scalar
// bases per direction as in the two-buffer row kernels).
// ---------------------------------------------------------------------------
// Even step: the node's own 19 runs, collided, each value stored in the run
// of the opposite direction.
template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_even_rows_kernel(S *__restrict__ A, Geom g, Relax<T> p, RowGrid R) {
    constexpr uint32_t es = sizeof(S);
    int x;
    uint32_t ri;
    if (!row_of(R, x, ri) || x >= g.nx) return;
    // one descriptor for the row group; the run of direction a at scalar offset a nx
    const uint32_t run = __builtin_amdgcn_readfirstlane((uint32_t)g.nx * es);
    const __amdgpu_buffer_rsrc_t own = row_rsrc(A + (int64_t)ri * g.row, (uint32_t)Q * run);
    const uint32_t lane = (uint32_t)x * es;
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = (T)RawBits<S>::template load<0>(own, lane, (uint32_t)a * run);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)x + (uint32_t)g.nx * ri, p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) RawBits<S>::template store<EvenStAux>(own, lane, d[a], (uint32_t)opp(a) * run);
}

// Odd step at node x of an inner row (y, z off the y and z faces): every
// source and target row lies inside the lattice.  Pull: f~_a(x - e_a) from
// run opp(a) of the source row (base one value before the run, lane offset
// x - cx(a) + 1, wrapped on a periodic x axis; the lanes of a non-periodic x
// face read a neighbouring run there and are redone).  Push: f~_a(x) to run a
// of the target row at x + cx(a); on a non-periodic x face the lanes whose
// target column is a ghost skip that store and the bounce-back below stores
// into the node's own row group instead.
template <typename S, typename T, bool Forced, int Route>
__device__ inline void aa_odd_row(S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z) {
    constexpr uint32_t es = sizeof(S);
    const int64_t r = (int64_t)z * g.ny + y;
    const uint32_t prange = __builtin_amdgcn_readfirstlane((uint32_t)(g.nx + 2) * es);
    const uint32_t srange = __builtin_amdgcn_readfirstlane((uint32_t)g.nx * es);
    const bool xl = x == 0, xr = x == g.nx - 1;
    // pull offsets from the base one value before the run; a ghost source
    // column of a non-periodic x face (replaced below) takes an offset beyond
    // the descriptor's range, so its load touches no memory
    constexpr uint32_t outside = 0x80000000u;
    const uint32_t o0 = (uint32_t)(x + 1) * es;
    const uint32_t op = xl ? (g.px ? prange - 2 * es : outside) : (uint32_t)x * es;       // cx = +1: source x - 1
    const uint32_t om = xr ? (g.px ? es : outside) : (uint32_t)(x + 2) * es;              // cx = -1: source x + 1
    // push offsets from the run start (kept inside the run on the lanes that skip the store)
    const uint32_t t0 = (uint32_t)x * es;
    const uint32_t tp = xr ? (g.px ? 0u : t0) : (uint32_t)(x + 1) * es;          // cx = +1: target x + 1
    const uint32_t tm = xl ? (g.px ? srange - es : t0) : (uint32_t)(x - 1) * es; // cx = -1: target x - 1
    auto pull_off = [&](int a) { return cx(a) == 1 ? op : (cx(a) == -1 ? om : o0); };
    auto push_off = [&](int a) { return cx(a) == 1 ? tp : (cx(a) == -1 ? tm : t0); };
    // pulls: one descriptor per source row group (from one value before it),
    // the run opp(a) at a scalar offset; every address lies inside the group
    const uint32_t run = __builtin_amdgcn_readfirstlane((uint32_t)g.nx * es);
    const uint32_t grange = (uint32_t)Q * run + 2 * es;
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const S *base = A + (r - cy(a) - (int64_t)cz(a) * g.ny) * g.row - 1;
        d[a] = (T)RawBits<S>::template load<0>(row_rsrc(base, grange), pull_off(a), (uint32_t)opp(a) * run);
    }
    const bool xwall = !g.px && (xl || xr);
    if (xwall) {
        // source column is a ghost: the node's own f~_opp(a), left in run a by the even step
#pragma unroll
        for (int a = 1; a < Q; ++a)
            if ((xl && cx(a) == 1) || (xr && cx(a) == -1))
                d[a] = wall_value<T>((T)Conv<S, T>::load(A[elem(g, a, x, y, z)]), p, a,
                                     (g.lid_mask & (cx(a) == 1 ? 1 : 2)) != 0);
    }
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)x + (uint32_t)g.nx * (uint32_t)r, p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        if (xwall && ((xl && cx(a) == -1) || (xr && cx(a) == 1))) continue;
        S *base = A + (r + cy(a) + (int64_t)cz(a) * g.ny) * g.row + (int64_t)a * g.nx;
        RawBits<S>::template store<OddStAux>(row_rsrc(base, srange), push_off(a), d[a]);
    }
    if (xwall) {
        // target column is a ghost: back into the node's own run opp(a), with
        // the lid term of direction opp(a): the value the pull rule gives next step
#pragma unroll
        for (int a = 1; a < Q; ++a)
            if ((xl && cx(a) == -1) || (xr && cx(a) == 1))
                A[elem(g, opp(a), x, y, z)] =
                    Conv<S, T>::store(wall_value<T>(d[a], p, opp(a), (g.lid_mask & (cx(a) == -1 ? 1 : 2)) != 0));
    }
}

// Even and odd steps at one node with the full wall rule per lane, in either
// layout (face rows of the row kernels, and narrow lattices).
template <typename S, typename T, bool Forced, int Route>
__device__ inline void aa_even_any(S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z) {
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = (T)Conv<S, T>::load(A[elem(g, a, x, y, z)]);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z), p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) A[elem(g, opp(a), x, y, z)] = Conv<S, T>::store(d[a]);
}

template <typename S, typename T, bool Forced, int Route>
__device__ inline void aa_odd_any(S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z) {
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
        const bool in_lid = ghost_in_lid(g, sx, sy, sz);
        const bool ok = wrap(sx, g.nx, g.px) & wrap(sy, g.ny, g.py) & wrap(sz, g.nz, g.pz);
        d[a] = ok ? (T)Conv<S, T>::load(A[elem(g, opp(a), sx, sy, sz)])
                  : wall_value<T>((T)Conv<S, T>::load(A[elem(g, a, x, y, z)]), p, a, in_lid);
    }
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z), p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        int tx = x + cx(a), ty = y + cy(a), tz = z + cz(a);
        const bool in_lid = ghost_in_lid(g, tx, ty, tz);
        const bool ok = wrap(tx, g.nx, g.px) & wrap(ty, g.ny, g.py) & wrap(tz, g.nz, g.pz);
        if (ok)
            A[elem(g, a, tx, ty, tz)] = Conv<S, T>::store(d[a]);
        else
            A[elem(g, opp(a), x, y, z)] = Conv<S, T>::store(wall_value<T>(d[a], p, opp(a), in_lid));
    }
}

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_odd_rows_kernel(S *__restrict__ A, Geom g, Relax<T> p, RowGrid R) {
    int x;
    uint32_t ri;
    if (!row_of(R, x, ri) || x >= g.nx) return;
    int y, z;
    inner_row(g, ri, y, z);
    aa_odd_row<S, T, Forced, Route>(A, g, p, x, y, z);
}

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_odd_rows_face_kernel(S *__restrict__ A, Geom g, Relax<T> p, RowGrid R) {
    int x;
    uint32_t ri;
    if (!row_of(R, x, ri) || x >= g.nx) return;
    int y, z;
    face_row(g, R, ri, y, z);
    aa_odd_any<S, T, Forced, Route>(A, g, p, x, y, z);
}

// any block shape, row layout: every node with the full rule
template <typename S, typename T, bool Forced, int Route, bool Odd>
__global__ void __launch_bounds__(MaxThreads<T>::value)
aa_any_kernel(S *__restrict__ A, Geom g, Relax<T> p, LaunchGrid L) {
    int x, y, z;
    locate(L, x, y, z);
    if (x >= g.nx || y >= g.ny) return;
    if (Odd)
        aa_odd_any<S, T, Forced, Route>(A, g, p, x, y, z);
    else
        aa_even_any<S, T, Forced, Route>(A, g, p, x, y, z);
}

template <typename S, typename T, bool Forced, int Route>
static hipError_t aa_pair_rows_f(void *A, const Geom &g, const Relax<T> &p, const StepLaunch &c, hipStream_t st) {
    const RowLaunch L = row_launch(g, c.bx, c.by, c.xcd_remap);
    const dim3 block(c.bx, c.by);
    RowGrid all = L.inner;      // the even step: every row, r = ri
    all.rows = (uint32_t)g.ny * (uint32_t)g.nz;
    const uint32_t nb = all.gx * ((all.rows + c.by - 1) / c.by);
    all.aligned = nb & ~7u;
    Relax<T> q = p;             // the odd step is the next collision
    q.step = p.step + 1u;
    hipLaunchKernelGGL((aa_even_rows_kernel<S, T, Forced, Route>), dim3(nb), block, 0, st, (S *)A, g, p, all);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.inner.rows > 0) {
        hipLaunchKernelGGL((aa_odd_rows_kernel<S, T, Forced, Route>), dim3(L.inner_blocks), block, 0, st, (S *)A, g,
                           q, L.inner);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((aa_odd_rows_face_kernel<S, T, Forced, Route>), dim3(L.face_blocks), block, 0, st, (S *)A, g,
                       q, L.face);
    return hipGetLastError();
}

template <typename S, typename T, bool Forced, int Route>
static hipError_t aa_pair_f(void *A, const Geom &g, const Relax<T> &p, const StepLaunch &c, hipStream_t st) {
    if (g.rows && c.bx % 64 == 0) return aa_pair_rows_f<S, T, Forced, Route>(A, g, p, c, st);
    LaunchGrid L;
    L.gx = (g.nx + c.bx - 1) / c.bx;
    L.gy = (g.ny + c.by - 1) / c.by;
    L.gz = g.nz;
    const uint32_t nb = (uint32_t)L.gx * L.gy * L.gz;
    L.aligned = nb & ~7u;
    L.remap = c.xcd_remap;
    dim3 grid(nb), block(c.bx, c.by);
    Relax<T> q = p;             // the odd step is the next collision
    q.step = p.step + 1u;
    if (g.rows) {
        hipLaunchKernelGGL((aa_any_kernel<S, T, Forced, Route, false>), grid, block, 0, st, (S *)A, g, p, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((aa_any_kernel<S, T, Forced, Route, true>), grid, block, 0, st, (S *)A, g, q, L);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((aa_even_kernel<S, T, Forced, Route>), grid, block, 0, st, (S *)A, g, p, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((aa_odd_kernel<S, T, Forced, Route>), grid, block, 0, st, (S *)A, g, q, L);
    return hipGetLastError();
}

template <typename S, typename T>
static hipError_t aa_pair_t(void *A, const Geom &g, const Relax<T> &p, bool forced, int route, const StepLaunch &c,
                            hipStream_t st) {
    if (route == 2) return forced ? hipErrorInvalidValue : aa_pair_f<S, T, false, 2>(A, g, p, c, st);
    if (route == 1) return forced ? aa_pair_f<S, T, true, 1>(A, g, p, c, st) : aa_pair_f<S, T, false, 1>(A, g, p, c, st);
    return forced ? aa_pair_f<S, T, true, 0>(A, g, p, c, st) : aa_pair_f<S, T, false, 0>(A, g, p, c, st);
}

hipError_t launch_aa_pair(int storage, void *A, const Geom &g, const Relax<double> &pd, const Relax<float> &pf,
                          bool forced, int route, const StepLaunch &c, hipStream_t st) {
    switch (storage) {
    case 0: return aa_pair_t<double, double>(A, g, pd, forced, route, c, st);
    case 1: return aa_pair_t<float, float>(A, g, pf, forced, route, c, st);
    default: return aa_pair_t<__half, float>(A, g, pf, forced, route, c, st);
    }
}

hipError_t launch_store_plain(int storage, const double *f0, void *A, const Geom &g, hipStream_t st) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    dim3 grid((unsigned)((N + 255) / 256)), block(256);
    switch (storage) {
    case 0: hipLaunchKernelGGL(store_plain_kernel<double>, grid, block, 0, st, f0, (double *)A, g); break;
    case 1: hipLaunchKernelGGL(store_plain_kernel<float>, grid, block, 0, st, f0, (float *)A, g); break;
    default: hipLaunchKernelGGL(store_plain_kernel<__half>, grid, block, 0, st, f0, (__half *)A, g); break;
    }
    return hipGetLastError();
}

}  // namespace clbm
