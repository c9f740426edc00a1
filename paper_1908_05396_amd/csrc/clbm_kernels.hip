// Kernels of the D3Q19 cascaded power-law LBM for gfx950 and their launchers.
//
//   stream_collide        one time step in the planes layout: pull gather +
//                         collision + store (Sec. 3); the row layout's step is in
//                         clbm_rows.hip
//   stream_collide_flags  one time step of a lattice with per-node solid flags
//                         (either layout, one thread per node)
//   init_collide          collide a caller-supplied FP64 state once (time 0), either layout
//   macroscopic           rho and u from the stored post-collision state
//   export                f = w + stored deviation, as FP64
//   reduce                FP64 block partials of mass, momentum, residual, NaNs
//   reduce_final          fixed-order sum of the partials
#include <mutex>

#include "clbm_internal.hpp"

namespace clbm {

// ---------------------------------------------------------------------------
// Fused stream-collide
// ---------------------------------------------------------------------------
// One thread per node, blocks of (blockDim.x, blockDim.y) nodes in the
// x-y plane of one z layer, launched as a 1-D grid.  Consecutive workgroups
// are dispatched round-robin to the eight XCDs; with `remap` set, workgroup b
// takes the tile (b mod 8) * (B/8) + b / 8, so each XCD sweeps a contiguous
// slab and the neighbour rows a node pulls from sit in the same L2.
// G > 1: the interior loads and the stores go through descriptors shared by G
// planes (PlaneGroup), when G planes span less than 4 GiB.
template <typename S, typename T, bool Forced, int LdAux, int StAux, int Route, int G>
__global__ void __launch_bounds__(MaxThreads<T>::value)
stream_collide_kernel(const S *__restrict__ A, S *__restrict__ B, Geom g, Relax<T> p, LaunchGrid L) {
    uint32_t b = blockIdx.x;
    if (L.remap && b < L.aligned) b = (b & 7u) * (L.aligned >> 3) + (b >> 3);
    const uint32_t tx = b % L.gx;
    b /= L.gx;
    const uint32_t ty = b % L.gy;
    const int z = (int)(b / L.gy);
    const int x = (int)(tx * blockDim.x + threadIdx.x);
    const int y = (int)(ty * blockDim.y + threadIdx.y);
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t self = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y + (uint32_t)g.nxy * (uint32_t)z;
    T d[Q];
    if constexpr (G == 1) {
        gather<S, T, LdAux>(A, g, p, x, y, z, self, d);
        collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
        round_state<S, T>(d, p, self, p.step);
#pragma unroll
        for (int a = 0; a < Q; ++a) Plane<S, StAux>::store(B, g, a, self, d[a]);
    } else {
        gather_grouped<S, T, LdAux, G>(A, g, p, x, y, z, self, d);
        collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
        round_state<S, T>(d, p, self, p.step);
        const uint32_t sb = self * (uint32_t)sizeof(S);
#pragma unroll
        for (int a = 0; a < Q; ++a)
            RawBits<S>::template store<StAux>(PlaneGroup<S, G>::rsrc(B, g, a), sb + PlaneGroup<S, G>::offset(g, a),
                                              d[a]);
    }
}

// ---------------------------------------------------------------------------
// Lattices with per-node solid flags (0 fluid, 1 wall, 2 wall moving with the
// lid velocity).  A fluid node pulls along e_a from x - e_a; when that source
// is a solid node, or a ghost beyond a wall of the box, half-way bounce-back
// (Sec. 4.1) returns the node's own post-collision population opposite to a,
// plus the moving-wall term (Sec. 4.3) for a moving solid node or a ghost in
// the lid plane.  Solid nodes are not part of the fluid and hold the rest
// state (zero deviations).  One thread per node in either layout; plain
// loads (the flags of the 18 neighbours come from cache).
// ---------------------------------------------------------------------------
template <typename S, typename T>
__device__ inline T pull_flagged(const S *__restrict__ A, const uint8_t *__restrict__ flags, const Geom &g,
                                 const Relax<T> &p, int a, int x, int y, int z) {
    int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
    bool in_lid = ghost_in_lid(g, sx, sy, sz);
    bool wall = false;
    if (sx < 0 || sx >= g.nx) { if (g.px) sx = sx < 0 ? sx + g.nx : sx - g.nx; else wall = true; }
    if (sy < 0 || sy >= g.ny) { if (g.py) sy = sy < 0 ? sy + g.ny : sy - g.ny; else wall = true; }
    if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
    if (!wall) {
        const uint8_t fs = flags[(int64_t)sx + (int64_t)g.nx * ((int64_t)sy + (int64_t)g.ny * sz)];
        if (fs == 0) return (T)Conv<S, T>::load(A[elem(g, a, sx, sy, sz)]);
        in_lid = fs == 2;
    }
    return wall_value<T>((T)Conv<S, T>::load(A[elem(g, opp(a), x, y, z)]), p, a, in_lid);
}

template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(256)
stream_collide_flags_kernel(const S *__restrict__ A, S *__restrict__ B, const uint8_t *__restrict__ flags, Geom g,
                            Relax<T> p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)g.n) return;
    const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / g.nxy);
    T d[Q];
    if (flags[i] != 0) {
#pragma unroll
        for (int a = 0; a < Q; ++a) d[a] = T(0);
    } else {
#pragma unroll
        for (int a = 0; a < Q; ++a)
            d[a] = a == 0 ? (T)Conv<S, T>::load(A[elem(g, 0, x, y, z)]) : pull_flagged<S, T>(A, flags, g, p, a, x, y, z);
        collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
        round_state<S, T>(d, p, (uint32_t)i, p.step);
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) B[elem(g, a, x, y, z)] = Conv<S, T>::store(d[a]);
}

// Any flag other than fluid (0), wall (1) or moving wall (2) sets *bad.
__global__ void __launch_bounds__(256)
check_flags_kernel(const uint8_t *__restrict__ flags, int64_t n, double *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i] > 2) *bad = 1.0;
}

__global__ void __launch_bounds__(64) fill_kernel(double *__restrict__ out, int n, double v) {
    if ((int)threadIdx.x < n) out[threadIdx.x] = v;
}

// ---------------------------------------------------------------------------
// Collide-only initialisation from FP64 populations (unpadded planes); a
// NULL source means the rest state f = w.  Solid nodes (flags) hold the rest
// state.
// ---------------------------------------------------------------------------
template <typename S, typename T, bool Forced, int Route>
__global__ void __launch_bounds__(256)
init_collide_kernel(const double *__restrict__ f0, S *__restrict__ B, const uint8_t *__restrict__ flags, Geom g,
                    Relax<T> p) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (flags && flags[i] != 0) {
#pragma unroll
        for (int a = 0; a < Q; ++a) B[elem_i(g, a, i)] = Conv<S, T>::store(T(0));
        return;
    }
    T d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = f0 ? (T)(f0[(int64_t)a * N + i] - weight(a)) : T(0);
    collide<T, Forced, Route, NewtonSteps<S>::value>(d, p, nullptr);
    round_state<S, T>(d, p, (uint32_t)i, p.step);
#pragma unroll
    for (int a = 0; a < Q; ++a) B[elem_i(g, a, i)] = Conv<S, T>::store(d[a]);
}

// ---------------------------------------------------------------------------
// Moments of the stored state
// ---------------------------------------------------------------------------
template <typename S>
__device__ inline void node_moments(const S *__restrict__ A, const Geom &g, int64_t i, double &D,
                                    double &jx, double &jy, double &jz, bool &finite) {
    D = jx = jy = jz = 0.0;
    finite = true;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        double v = (double)Conv<S, typename StoreCompute<S>::T>::load(A[elem_i(g, a, i)]);
        finite = finite && isfinite(v);
        D += v;
        jx += cx(a) * v;
        jy += cy(a) * v;
        jz += cz(a) * v;
    }
}

// Density and velocity in FP64, written as O (double or float); solid nodes
// report rho = 1, u = 0.
template <typename S, typename O>
__global__ void __launch_bounds__(256)
macroscopic_kernel(const S *__restrict__ A, const uint8_t *__restrict__ flags, O *__restrict__ rho,
                   O *__restrict__ u, Geom g, double fx, double fy, double fz) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double r = 1.0, ux = 0.0, uy = 0.0, uz = 0.0;
    if (!(flags && flags[i] != 0)) {
        double D, jx, jy, jz;
        bool finite;
        node_moments(A, g, i, D, jx, jy, jz, finite);
        r = 1.0 + D;
        ux = (jx - 0.5 * fx) / r;
        uy = (jy - 0.5 * fy) / r;
        uz = (jz - 0.5 * fz) / r;
    }
    if (rho) rho[i] = (O)r;
    if (u) {
        u[i] = (O)ux;
        u[N + i] = (O)uy;
        u[2 * N + i] = (O)uz;
    }
}

template <typename S>
__global__ void __launch_bounds__(256)
export_kernel(const S *__restrict__ A, double *__restrict__ f, Geom g) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int a = 0; a < Q; ++a)
        f[(int64_t)a * N + i] =
            weight(a) + (double)Conv<S, typename StoreCompute<S>::T>::load(A[elem_i(g, a, i)]);
}

// ---------------------------------------------------------------------------
// FP64 reductions: per-block partials, then a single-block fixed-order sum.
// Slots: 0 sum(rho - 1), 1..3 momentum, 4 sum |u - u_prev|^2, 5 sum |u|^2,
// 6 non-finite nodes, 7 max |u|, 8 kinetic energy, 9 fluid nodes.  Solid
// nodes (flags) are left out.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

template <typename S>
__global__ void __launch_bounds__(kReduceThreads)
reduce_kernel(const S *__restrict__ A, const uint8_t *__restrict__ flags, double *__restrict__ snap, int have_prev,
              Geom g, double fx, double fy, double fz, double *__restrict__ partials) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    double acc[kReduceSlots];
#pragma unroll
    for (int k = 0; k < kReduceSlots; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (flags && flags[i] != 0) continue;
        double D, jx, jy, jz;
        bool finite;
        node_moments(A, g, i, D, jx, jy, jz, finite);
        const double r = 1.0 + D;
        const double mx = jx - 0.5 * fx, my = jy - 0.5 * fy, mz = jz - 0.5 * fz;
        const double ux = mx / r, uy = my / r, uz = mz / r;
        const double u2 = ux * ux + uy * uy + uz * uz;
        acc[0] += D;
        acc[1] += mx;
        acc[2] += my;
        acc[3] += mz;
        if (snap) {
            if (have_prev) {
                const double dx = ux - snap[i], dy = uy - snap[N + i], dz = uz - snap[2 * N + i];
                acc[4] += dx * dx + dy * dy + dz * dz;
            }
            snap[i] = ux;
            snap[N + i] = uy;
            snap[2 * N + i] = uz;
        }
        acc[5] += u2;
        acc[6] += finite ? 0.0 : 1.0;
        acc[7] = fmax(acc[7], finite ? sqrt(u2) : 0.0);
        acc[8] += 0.5 * r * u2;
        acc[9] += 1.0;
    }
    __shared__ double sm[kReduceSlots][kReduceThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kReduceSlots; ++k) {
        const double v = (k == 7) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) sm[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < kReduceSlots) {
        const int k = threadIdx.x;
        double v = sm[k][0];
        for (int w = 1; w < kReduceThreads / 64; ++w) v = (k == 7) ? fmax(v, sm[k][w]) : v + sm[k][w];
        partials[(int64_t)blockIdx.x * kReduceSlots + k] = v;
    }
}

__global__ void __launch_bounds__(64)
reduce_final_kernel(const double *__restrict__ partials, int nblocks, double *__restrict__ out) {
    const int k = threadIdx.x;
    if (k >= kReduceSlots) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double x = partials[(int64_t)b * kReduceSlots + k];
        v = (k == 7) ? fmax(v, x) : v + x;
    }
    out[k] = v;
}

// ---------------------------------------------------------------------------
// Reduction without allocation: the block partials and the final sums live in
// a file-scope device array, one copy per GPU, which the host reaches only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name in host code is not a device address).  Every call on a
// GPU shares that GPU's copy: calls that overlap on one GPU race.  The final
// kernel writes the eight outputs of clbm_reduce to the caller's device
// memory; nothing is copied to the host.
// ---------------------------------------------------------------------------
constexpr int kScratchDoubles = (kNoAllocMaxBlocks + 1) * kReduceSlots;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Device address of this GPU's scratch (looked up once per device, with that
// device current).
static hipError_t scratch_address(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Fixed-order sums of the partials (as reduce_final_kernel), then the eight
// outputs of clbm_reduce: fluid mass, momentum, residual, non-finite count,
// max |u|, kinetic energy.
__global__ void __launch_bounds__(64)
reduce_finish_kernel(const double *__restrict__ partials, int nblocks, int have_prev, double *__restrict__ sums,
                     double *__restrict__ out) {
    const int k = threadIdx.x;
    if (k < kReduceSlots) {
        double v = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            const double x = partials[(int64_t)b * kReduceSlots + k];
            v = (k == 7) ? fmax(v, x) : v + x;
        }
        sums[k] = v;
    }
    __syncthreads();
    if (k == 0) {
        out[0] = sums[9] + sums[0];
        out[1] = sums[1];
        out[2] = sums[2];
        out[3] = sums[3];
        out[4] = (have_prev && sums[5] > 0.0) ? sqrt(sums[4] / sums[5]) : 0.0;
        out[5] = sums[6];
        out[6] = sums[7];
        out[7] = sums[8];
    }
}

template <typename S>
static hipError_t launch_reduce_noalloc_t(const void *A, const uint8_t *flags, double *snap, int have_prev,
                                          const Geom &g, const double *F, int nblocks, double *out,
                                          hipStream_t st) {
    double *ptr = nullptr;
    hipError_t e = scratch_address(&ptr);
    if (e != hipSuccess) return e;
    double *sums = ptr + (size_t)kNoAllocMaxBlocks * kReduceSlots;
    hipLaunchKernelGGL((reduce_kernel<S>), dim3(nblocks), dim3(kReduceThreads), 0, st, (const S *)A, flags, snap,
                       have_prev, g, F[0], F[1], F[2], ptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_finish_kernel, dim3(1), dim3(64), 0, st, (const double *)ptr, nblocks,
                       snap && have_prev ? 1 : 0, sums, out);
    return hipGetLastError();
}

hipError_t launch_reduce_noalloc(int storage, const void *A, const uint8_t *flags, double *snap, int have_prev,
                                 const Geom &g, const double *F, int nblocks, double *out, hipStream_t st) {
    if (nblocks < 1 || nblocks > kNoAllocMaxBlocks) return hipErrorInvalidValue;
    switch (storage) {
    case 0: return launch_reduce_noalloc_t<double>(A, flags, snap, have_prev, g, F, nblocks, out, st);
    case 1: return launch_reduce_noalloc_t<float>(A, flags, snap, have_prev, g, F, nblocks, out, st);
    default: return launch_reduce_noalloc_t<__half>(A, flags, snap, have_prev, g, F, nblocks, out, st);
    }
}

// ---------------------------------------------------------------------------
// The FP16 rounding of the state on its own (test utility): stochastic with
// the given seeds (the hardware conversion the step kernels use), or nearest
// even.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
f16_round_kernel(const float *__restrict__ in, const uint32_t *__restrict__ seeds, uint16_t *__restrict__ out,
                 int64_t n, int stochastic) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = stochastic ? sr_to_f16_grid(in[i], seeds[i]) : in[i];
    out[i] = __builtin_bit_cast(uint16_t, __float2half_rn(v));
}

hipError_t launch_f16_round(const float *in, const uint32_t *seeds, uint16_t *out, int64_t n, int stochastic,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f16_round_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, seeds, out, n, stochastic);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain streaming copy (bandwidth reference)
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
copy_probe_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const f32x4 *)src,
                       (f32x4 *)dst, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename S, typename T, bool Forced, int Route, int G>
static hipError_t launch_step_g(const void *A, void *B, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                                hipStream_t st);

// planes per shared descriptor: 4 when four planes span less than 4 GiB
template <typename S>
static int plane_group(const Geom &g) {
    return (uint64_t)g.plane * sizeof(S) * 4u <= 0xFFFFFFFFull ? 4 : 1;
}

template <typename S, typename T, bool Forced, int Route>
static hipError_t launch_step_f(const void *A, void *B, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                                hipStream_t st) {
    return plane_group<S>(g) == 4 ? launch_step_g<S, T, Forced, Route, 4>(A, B, g, p, c, st)
                                  : launch_step_g<S, T, Forced, Route, 1>(A, B, g, p, c, st);
}

template <typename S, typename T, bool Forced, int Route, int G>
static hipError_t launch_step_g(const void *A, void *B, const Geom &g, const Relax<T> &p, const StepLaunch &c,
                                hipStream_t st) {
    LaunchGrid L;
    L.gx = (g.nx + c.bx - 1) / c.bx;
    L.gy = (g.ny + c.by - 1) / c.by;
    L.gz = g.nz;
    const uint32_t nb = (uint32_t)L.gx * L.gy * L.gz;
    L.aligned = nb & ~7u;
    L.remap = c.xcd_remap;
    dim3 grid(nb), block(c.bx, c.by);
    const S *a = (const S *)A;
    S *b = (S *)B;
    if (Route == 1) {   // the printed form: only the store hint is tunable
        if (c.nt_stores)
            hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 0, 2, Route, G>), grid, block, 0, st, a, b, g, p, L);
        else
            hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 0, 0, Route, G>), grid, block, 0, st, a, b, g, p, L);
        return hipGetLastError();
    }
    const int mode = (c.nt_loads ? 1 : 0) | (c.nt_stores ? 2 : 0);
    switch (mode) {
    case 0: hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 0, 0, Route, G>), grid, block, 0, st, a, b, g, p, L); break;
    case 1: hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 2, 0, Route, G>), grid, block, 0, st, a, b, g, p, L); break;
    case 2: hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 0, 2, Route, G>), grid, block, 0, st, a, b, g, p, L); break;
    default: hipLaunchKernelGGL((stream_collide_kernel<S, T, Forced, 2, 2, Route, G>), grid, block, 0, st, a, b, g, p, L); break;
    }
    return hipGetLastError();
}

template <typename S, typename T>
static hipError_t launch_step_t(const void *A, void *B, const Geom &g, const Relax<T> &p, bool forced, int route,
                                const StepLaunch &c, hipStream_t st) {
    if (route == 2) return forced ? hipErrorInvalidValue : launch_step_f<S, T, false, 2>(A, B, g, p, c, st);
    if (route == 0)
        return forced ? launch_step_f<S, T, true, 0>(A, B, g, p, c, st) : launch_step_f<S, T, false, 0>(A, B, g, p, c, st);
    return forced ? launch_step_f<S, T, true, 1>(A, B, g, p, c, st) : launch_step_f<S, T, false, 1>(A, B, g, p, c, st);
}

hipError_t launch_step(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                       const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st) {
    switch (storage) {
    case 0: return launch_step_t<double, double>(A, B, g, pd, forced, route, c, st);
    case 1: return launch_step_t<float, float>(A, B, g, pf, forced, route, c, st);
    default: return launch_step_t<__half, float>(A, B, g, pf, forced, route, c, st);
    }
}

template <typename S, typename T, bool Forced, int Route>
static void launch_init_k(const double *f0, void *B, const uint8_t *flags, const Geom &g, const Relax<T> &p,
                          hipStream_t st) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((init_collide_kernel<S, T, Forced, Route>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       st, f0, (S *)B, flags, g, p);
}

template <typename S, typename T>
static hipError_t launch_init_t(const double *f0, void *B, const uint8_t *flags, const Geom &g, const Relax<T> &p,
                                bool forced, int route, hipStream_t st) {
    if (route == 2) {
        if (forced) return hipErrorInvalidValue;
        launch_init_k<S, T, false, 2>(f0, B, flags, g, p, st);
    } else if (route == 0) {
        if (forced) launch_init_k<S, T, true, 0>(f0, B, flags, g, p, st);
        else launch_init_k<S, T, false, 0>(f0, B, flags, g, p, st);
    } else {
        if (forced) launch_init_k<S, T, true, 1>(f0, B, flags, g, p, st);
        else launch_init_k<S, T, false, 1>(f0, B, flags, g, p, st);
    }
    return hipGetLastError();
}

hipError_t launch_init(int storage, const double *f0, void *B, const uint8_t *flags, const Geom &g,
                       const Relax<double> &pd, const Relax<float> &pf, bool forced, int route, hipStream_t st) {
    switch (storage) {
    case 0: return launch_init_t<double, double>(f0, B, flags, g, pd, forced, route, st);
    case 1: return launch_init_t<float, float>(f0, B, flags, g, pf, forced, route, st);
    default: return launch_init_t<__half, float>(f0, B, flags, g, pf, forced, route, st);
    }
}

template <typename S, typename T, bool Forced, int Route>
static void launch_flags_k(const void *A, void *B, const uint8_t *flags, const Geom &g, const Relax<T> &p,
                           hipStream_t st) {
    hipLaunchKernelGGL((stream_collide_flags_kernel<S, T, Forced, Route>), dim3((unsigned)((g.n + 255) / 256)),
                       dim3(256), 0, st, (const S *)A, (S *)B, flags, g, p);
}

template <typename S, typename T>
static hipError_t launch_flags_t(const void *A, void *B, const uint8_t *flags, const Geom &g, const Relax<T> &p,
                                 bool forced, int route, hipStream_t st) {
    if (route == 2) {
        if (forced) return hipErrorInvalidValue;
        launch_flags_k<S, T, false, 2>(A, B, flags, g, p, st);
    } else if (route == 0) {
        if (forced) launch_flags_k<S, T, true, 0>(A, B, flags, g, p, st);
        else launch_flags_k<S, T, false, 0>(A, B, flags, g, p, st);
    } else {
        if (forced) launch_flags_k<S, T, true, 1>(A, B, flags, g, p, st);
        else launch_flags_k<S, T, false, 1>(A, B, flags, g, p, st);
    }
    return hipGetLastError();
}

hipError_t launch_step_flags(int storage, const void *A, void *B, const uint8_t *flags, const Geom &g,
                             const Relax<double> &pd, const Relax<float> &pf, bool forced, int route, hipStream_t st) {
    switch (storage) {
    case 0: return launch_flags_t<double, double>(A, B, flags, g, pd, forced, route, st);
    case 1: return launch_flags_t<float, float>(A, B, flags, g, pf, forced, route, st);
    default: return launch_flags_t<__half, float>(A, B, flags, g, pf, forced, route, st);
    }
}

hipError_t launch_check_flags(const uint8_t *flags, int64_t n, double *bad, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, bad, 1, 0.0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(check_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, flags, n, bad);
    return hipGetLastError();
}

template <typename S, typename O>
static hipError_t launch_macro_t(const void *A, const uint8_t *flags, void *rho, void *u, const Geom &g,
                                 const double *F, hipStream_t st) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((macroscopic_kernel<S, O>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       (const S *)A, flags, (O *)rho, (O *)u, g, F[0], F[1], F[2]);
    return hipGetLastError();
}

template <typename O>
static hipError_t launch_macro_o(int storage, const void *A, const uint8_t *flags, void *rho, void *u,
                                 const Geom &g, const double *F, hipStream_t st) {
    switch (storage) {
    case 0: return launch_macro_t<double, O>(A, flags, rho, u, g, F, st);
    case 1: return launch_macro_t<float, O>(A, flags, rho, u, g, F, st);
    default: return launch_macro_t<__half, O>(A, flags, rho, u, g, F, st);
    }
}

hipError_t launch_macroscopic(int storage, const void *A, const uint8_t *flags, void *rho, void *u, bool out_f32,
                              const Geom &g, const double *F, hipStream_t st) {
    return out_f32 ? launch_macro_o<float>(storage, A, flags, rho, u, g, F, st)
                   : launch_macro_o<double>(storage, A, flags, rho, u, g, F, st);
}

template <typename S>
static hipError_t launch_export_t(const void *A, double *f, const Geom &g, hipStream_t st) {
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((export_kernel<S>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       (const S *)A, f, g);
    return hipGetLastError();
}

hipError_t launch_export(int storage, const void *A, double *f, const Geom &g, hipStream_t st) {
    switch (storage) {
    case 0: return launch_export_t<double>(A, f, g, st);
    case 1: return launch_export_t<float>(A, f, g, st);
    default: return launch_export_t<__half>(A, f, g, st);
    }
}

template <typename S>
static hipError_t launch_reduce_t(const void *A, const uint8_t *flags, double *snap, int have_prev, const Geom &g,
                                  const double *F, double *partials, int nblocks, double *out, hipStream_t st) {
    hipLaunchKernelGGL((reduce_kernel<S>), dim3(nblocks), dim3(kReduceThreads), 0, st, (const S *)A, flags, snap,
                       have_prev, g, F[0], F[1], F[2], partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(64), 0, st, (const double *)partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_reduce(int storage, const void *A, const uint8_t *flags, double *snap, int have_prev,
                         const Geom &g, const double *F, double *partials, int nblocks, double *out, hipStream_t st) {
    switch (storage) {
    case 0: return launch_reduce_t<double>(A, flags, snap, have_prev, g, F, partials, nblocks, out, st);
    case 1: return launch_reduce_t<float>(A, flags, snap, have_prev, g, F, partials, nblocks, out, st);
    default: return launch_reduce_t<__half>(A, flags, snap, have_prev, g, F, partials, nblocks, out, st);
    }
}

}  // namespace clbm
