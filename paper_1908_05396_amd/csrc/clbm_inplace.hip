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
#include "clbm_internal.hpp"

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
        Plane<S>::store(A, g, a, (uint32_t)i, f0 ? (T)(f0[(int64_t)a * N + i] - weight(a)) : T(0));
}

template <typename S, typename T, bool Forced, int Route>
static hipError_t aa_pair_f(void *A, const Geom &g, const Relax<T> &p, const StepLaunch &c, hipStream_t st) {
    LaunchGrid L;
    L.gx = (g.nx + c.bx - 1) / c.bx;
    L.gy = (g.ny + c.by - 1) / c.by;
    L.gz = g.nz;
    const uint32_t nb = (uint32_t)L.gx * L.gy * L.gz;
    L.aligned = nb & ~7u;
    L.remap = c.xcd_remap;
    dim3 grid(nb), block(c.bx, c.by);
    hipLaunchKernelGGL((aa_even_kernel<S, T, Forced, Route>), grid, block, 0, st, (S *)A, g, p, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((aa_odd_kernel<S, T, Forced, Route>), grid, block, 0, st, (S *)A, g, p, L);
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
