// Device side of the D3Q19 cascaded power-law LBM (arXiv:1908.05396) for
// gfx950: lattice constants, the pull gather with the wall rules, and the
// central-moment collision with the locally solved power-law relaxation rate.
//
// Everything works on deviations d = f - w from the rest weights, which keeps
// the small, physically relevant parts of the moments representable in FP32
// and FP16 (the rest values 1, 1/3, 1/9 cancel analytically).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clbm {

constexpr int Q = 19;

// Particle velocities in the order of Sec. 3.
__host__ __device__ constexpr int cx(int a) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[a];
}
__host__ __device__ constexpr int cy(int a) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[a];
}
__host__ __device__ constexpr int cz(int a) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[a];
}
__host__ __device__ constexpr int opp(int a) {
    constexpr int v[Q] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[a];
}
__host__ __device__ constexpr double weight(int a) {
    return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------------------
// Storage conversions
// ---------------------------------------------------------------------------
template <typename S, typename T> struct Conv;
template <> struct Conv<double, double> {
    __device__ static double load(double v) { return v; }
    __device__ static double store(double v) { return v; }
};
template <> struct Conv<float, float> {
    __device__ static float load(float v) { return v; }
    __device__ static float store(float v) { return v; }
};
template <> struct Conv<__half, float> {
    __device__ static float load(__half v) { return __half2float(v); }
    __device__ static __half store(float v) { return __float2half_rn(v); }
};

// ---------------------------------------------------------------------------
// Parameters (by value in kernel arguments)
// ---------------------------------------------------------------------------
struct Geom {
    int32_t nx, ny, nz;
    int32_t nxy;            // nx * ny
    int32_t n;              // nx * ny * nz (< 2^31)
    int32_t px, py, pz;     // periodic flags
    int32_t lid_axis;       // 0, 1, 2, or -1 for no lid
    int32_t lid_side;       // +1: the ghost plane beyond n-1; -1: the one before 0
    int32_t lid_mask;       // bit f-1 set for lid face f (1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z)
    int32_t rows;           // 1: row layout, 0: planes
    int64_t plane;          // element stride between populations a and a + 1 of a node
    int64_t row;            // element stride between rows y and y + 1 (planes: nx, rows: 19 nx)
};

// Element index of population a of node (x, y, z) in either layout: planes
// (plane = padded plane, row = nx) or rows (plane = nx, row = 19 nx).
__host__ __device__ inline int64_t elem(const Geom &g, int a, int x, int y, int z) {
    return (int64_t)a * g.plane + x + g.row * ((int64_t)z * g.ny + y);
}
// The same for node index i = x + nx (y + ny z) (i < 2^31).
__device__ inline int64_t elem_i(const Geom &g, int a, int64_t i) {
    const uint32_t r = (uint32_t)i / (uint32_t)g.nx;
    const uint32_t x = (uint32_t)i - r * (uint32_t)g.nx;
    return (int64_t)a * g.plane + x + g.row * (int64_t)r;
}

// ---------------------------------------------------------------------------
// Planes layout: access through raw buffer descriptors, one descriptor per
// population plane (base = plane start, range = n elements), 32-bit byte
// offsets from a VGPR.  Offsets outside the range return 0 without touching
// memory, so the interior pull can run unguarded and edge lanes are patched
// afterwards.
// ---------------------------------------------------------------------------
constexpr int kBufferFlags = 0x00020000;   // raw (untyped) buffer, gfx9 family

template <typename S, int Aux = 0> struct Plane;
template <int Aux> struct Plane<float, Aux> {
    __device__ static float load(const float *A, const Geom &g, int a, uint32_t i) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 4u), kBufferFlags);
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(i * 4u), 0, Aux));
    }
    __device__ static void store(float *B, const Geom &g, int a, uint32_t i, float v) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 4u), kBufferFlags);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)(i * 4u), 0, Aux);
    }
};
template <int Aux> struct Plane<double, Aux> {
    __device__ static double load(const double *A, const Geom &g, int a, uint32_t i) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 8u), kBufferFlags);
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 8u), 0, Aux));
    }
    __device__ static void store(double *B, const Geom &g, int a, uint32_t i, double v) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 8u), kBufferFlags);
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)(i * 8u), 0, Aux);
    }
};
template <int Aux> struct Plane<__half, Aux> {
    __device__ static float load(const __half *A, const Geom &g, int a, uint32_t i) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 2u), kBufferFlags);
        return __half2float(
            __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)(i * 2u), 0, Aux)));
    }
    __device__ static void store(__half *B, const Geom &g, int a, uint32_t i, float v) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(B + (int64_t)a * g.plane), (short)0, (int)((uint32_t)g.n * 2u), kBufferFlags);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, __float2half_rn(v)), r,
                                              (int)(i * 2u), 0, Aux);
    }
};

// Grouped access for the hot loop: G consecutive planes share one descriptor
// whose range spans the G planes; the plane is selected by a uniform byte
// offset added to the lane's offset, so the per-plane descriptors (four SGPRs
// each) need not all be live.  Every address stays inside the group: offsets
// past it return 0 (loads) or are dropped (stores), and a wrapped negative
// offset lands in an earlier plane of the same group, whose value the edge
// rule then replaces.  Valid when G planes span less than 4 GiB.
template <typename S, int G> struct PlaneGroup {
    __device__ static __amdgpu_buffer_rsrc_t rsrc(const S *A, const Geom &g, int a) {
        const int k = a / G;
        const int cnt = (Q - k * G) < G ? (Q - k * G) : G;
        return __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + (int64_t)(k * G) * g.plane), (short)0,
            (int)((uint32_t)cnt * (uint32_t)g.plane * (uint32_t)sizeof(S)), kBufferFlags);
    }
    // byte offset of plane a inside its group
    __device__ static uint32_t offset(const Geom &g, int a) {
        return (uint32_t)(a % G) * (uint32_t)g.plane * (uint32_t)sizeof(S);
    }
};

// ---------------------------------------------------------------------------
// Stochastic rounding of the FP16 state
// ---------------------------------------------------------------------------
// Round-to-nearest of slowly varying FP16 values repeats the same rounding
// error step after step, which acts on the flow like a spurious source term.
// Rounding each stored value up or down at random, with the probability that
// makes the expected result equal to the FP32 value, turns that bias into
// zero-mean noise.  gfx950 converts with a seed in hardware; the conversion
// compares the upper 19 bits of the seed with the discarded part of the
// mantissa (measured: the lower 13 bits do not change the result).
//
// Seeds: a word per (node, collision index) from a bijective integer mixer
// (xor-shift / odd-multiply rounds) of the node index and a key of the
// collision index, plus a Weyl increment (golden ratio) per direction, in
// 32-bit wrap-around arithmetic: fresh bits for every value at every step.
// (A low-discrepancy sequence along the steps of each value, the per-step
// part a fixed increment instead of a hash, was measured and rejected: its
// FP16 field error was 3-40x larger, e.g. 7e-2 instead of 1.8e-3 on the 256^3
// cavity after 50000 steps.)  Every launch form and layout draws the same
// seeds for the same value, so results do not depend on the launch
// configuration.
__host__ __device__ constexpr uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
constexpr uint32_t kWeyl = 0x9E3779B9u;      // 2^32 (golden ratio - 1): per direction

// key of a collision index (uniform over a launch)
__host__ __device__ constexpr uint32_t step_key(uint32_t step) { return mix32(step * 0x85EBCA77u + 0x27D4EB2Fu); }

// seed of direction 0 of a node at a collision index
__device__ inline uint32_t sr_base(uint32_t node, uint32_t step) { return mix32(node ^ step_key(step)); }

__device__ inline uint16_t sr_to_f16_bits(float v, uint32_t seed) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t h = __builtin_amdgcn_cvt_sr_f16_f32(half2_t{0, 0}, v, seed, false);
    return __builtin_bit_cast(uint16_t, h[0]);
}

__device__ inline float sr_to_f16_grid(float v, uint32_t seed) {
    return (float)__builtin_bit_cast(_Float16, sr_to_f16_bits(v, seed));
}

// Raw buffer access at a lane byte offset `byte` plus a uniform byte offset
// `so` (the instruction's scalar offset operand).  Callers that pass so != 0
// keep byte + so inside the descriptor's range, so the result does not
// depend on whether the range check counts the scalar offset.
template <typename S> struct RawBits;
template <> struct RawBits<float> {
    template <int Aux> __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t byte, uint32_t so = 0) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte, (int)so, Aux));
    }
    template <int Aux> __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t byte, float v, uint32_t so = 0) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)byte, (int)so, Aux);
    }
};
template <> struct RawBits<__half> {
    template <int Aux> __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t byte, uint32_t so = 0) {
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)byte, (int)so, Aux)));
    }
    // store with stochastic rounding (seed as for sr_to_f16_bits)
    template <int Aux> __device__ static void store_sr(__amdgpu_buffer_rsrc_t r, uint32_t byte, float v, uint32_t seed,
                                                       uint32_t so = 0) {
        __builtin_amdgcn_raw_buffer_store_b16(sr_to_f16_bits(v, seed), r, (int)byte, (int)so, Aux);
    }
    template <int Aux> __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t byte, float v, uint32_t so = 0) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, __float2half_rn(v)), r, (int)byte, (int)so,
                                              Aux);
    }
};
template <> struct RawBits<double> {
    template <int Aux> __device__ static double load(__amdgpu_buffer_rsrc_t r, uint32_t byte, uint32_t so = 0) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte, (int)so, Aux));
    }
    template <int Aux> __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t byte, double v, uint32_t so = 0) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)byte, (int)so, Aux);
    }
};

template <typename T> struct Relax {
    T lid6[3];              // 6 rho_w U_w: the moving-wall term is w_a (e_a . lid6)
    T log2_3K;              // log2(3 K)
    T three_K;              // 3 K
    T n;                    // power-law index
    T k;                    // (n - 1) / 2
    T tau_min, tau_max;     // 3 nu_min + 1/2, 3 nu_max + 1/2
    T s_lo, s_hi;           // log2(tau_min - 1/2) - 1, log2(tau_max - 1/2) + 1
    T omega_bulk;
    T omega_high[9];
    T force[3];
    int32_t newtonian;      // n == 1
    int32_t literal;        // fourth-order attractor without 1/rho
    int32_t sr;             // FP16 storage: stochastic rounding of the stored values (else nearest even)
    uint32_t step;          // index of the collision a launch performs (0: the initial one); keys the rounding
};

// ---------------------------------------------------------------------------
// Local relaxation rate omega^nu (Sec. 3.2)
// ---------------------------------------------------------------------------
// With the non-equilibrium second-order moments m4..m9, the strain-rate
// tensor of Eq. (strain rate tensor) is S = omega P + q I with P traceless,
// so |gamma|^2 = 2 S:S = (a / tau^2 + b) / rho^2 where
//   a = 3 (m7^2 - m7 m8 + m8^2) + 9 (m4^2 + m5^2 + m6^2),
//   b = 3/2 omega_9^2 m9^2,
// and tau = 1/omega^nu must satisfy tau - 1/2 = 3 nu(|gamma|(tau)) with
// nu = K |gamma|^(n-1) / rho clipped to [nu_min, nu_max].  Writing
// s = log2(tau - 1/2), the unclipped equation is
//   phi(s) = s - log2(3K) + n log2(rho) - k log2(a/tau^2 + b) = 0,
// k = (n-1)/2, whose slope 1 + 2k a (tau-1/2) / (tau (a + b tau^2)) lies
// between min(1, n) and max(1, n): phi has exactly one root and is nearly
// linear in s, so Newton from the tau = 1 estimate converges in a few steps.
// The clipped solution is the unclipped root clamped to [tau_min, tau_max].
template <typename T> struct NewtonTol;
// FP32: four iterations from the tau = 1 estimate reach full precision over
// n in [0.4, 1.6], K over five decades and a over twelve (checked against a
// bisection reference); they start the FP64 solve, which then iterates to
// convergence.  The FP32 and FP16 storage kernels take three (NewtonSteps),
// which already leave only the solve's own FP32 rounding.
template <> struct NewtonTol<float> {
    static constexpr bool fixed = true;
    static constexpr int maxit = 4;
    static constexpr float tol = 0.0f;
};
template <> struct NewtonTol<double> {
    static constexpr bool fixed = false;
    static constexpr int maxit = 16;
    static constexpr double tol = 1e-9;     // the step that is this small lands exact to FP64
};

// FP32: the hardware log2/exp2/reciprocal (about 1 ulp); the arguments stay
// in the normal range (tau - 1/2 in [2^-10, 2^5], q handled by the window).
// FP64: library log2/exp2, reciprocal refined to full precision.
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double fast_log2(double x) { return log2(x); }
__device__ inline double fast_exp2(double x) { return exp2(x); }
__device__ inline double fast_rcp(double x) { return 1.0 / x; }

template <typename T>
__device__ inline T clampv(T v, T lo, T hi) { return fmin(fmax(v, lo), hi); }

// s is confined to [s_lo, s_hi] (one octave beyond log2 of the clip bounds of
// tau - 1/2): if the root lies outside, the iterates stop at the window edge
// and the final clamp of tau gives the clipped viscosity, as required.
// NI: fixed Newton steps of the FP32 iteration (FP64 iterates to convergence).
template <typename T, int NI = NewtonTol<T>::maxit>
__device__ inline T solve_tau(const Relax<T> &p, T rho, T a, T b) {
    if (p.newtonian) return clampv(T(0.5) + p.three_K * fast_rcp(rho), p.tau_min, p.tau_max);
    const T q0 = a + b;
    if (q0 == T(0)) {
        // no shear: the power law gives nu -> infinity (n < 1) or 0 (n > 1)
        return p.k < T(0) ? p.tau_max : p.tau_min;
    }
    const T c = p.log2_3K - p.n * fast_log2(rho);
    T s;
    if constexpr (NewtonTol<T>::fixed) {
        s = clampv(c + p.k * fast_log2(q0), p.s_lo, p.s_hi);   // exact if tau were 1
    } else {
        // FP64: the FP32 iteration (hardware transcendentals) gives the root
        // to ~1e-6; the FP64 steps below then converge in two or three.
        const float cf = (float)c, kf = (float)p.k, af = (float)a, bf = (float)b;
        const float lo = (float)p.s_lo, hi = (float)p.s_hi, two_kf = 2.0f * kf;
        float sf = clampv(cf + kf * fast_log2((float)q0), lo, hi);
        for (int it = 0; it < NewtonTol<float>::maxit; ++it) {
            const float e = fast_exp2(sf);
            const float it1 = fast_rcp(0.5f + e);
            const float u = af * (it1 * it1);
            const float q = u + bf;
            const float phi = sf - cf - kf * fast_log2(q);
            sf = clampv(sf - phi * q * fast_rcp(q + two_kf * u * (e * it1)), lo, hi);
        }
        s = (T)sf;
        if (!(s == s)) s = clampv(c + p.k * fast_log2(q0), p.s_lo, p.s_hi);   // FP32 range trouble
    }
    const T two_k = T(2) * p.k;
    for (int it = 0; it < (NewtonTol<T>::fixed ? NI : NewtonTol<T>::maxit); ++it) {
        const T e = fast_exp2(s);                 // tau - 1/2
        const T it1 = fast_rcp(T(0.5) + e);       // 1/tau
        const T u = a * (it1 * it1);              // a / tau^2
        const T q = u + b;
        const T phi = s - c - p.k * fast_log2(q);
        // slope 1 + 2k (u/q) (tau - 1/2)/tau = (q + 2k u (tau - 1/2)/tau) / q, so the
        // Newton step phi/slope takes one reciprocal; the denominator is at
        // least (1 - |2k|) q > 0 for n in (0, 2) and at least q for n >= 1
        const T sn = clampv(s - phi * q * fast_rcp(q + two_k * u * (e * it1)), p.s_lo, p.s_hi);
        if (NewtonTol<T>::fixed) {
            s = sn;
            continue;
        }
        const T ds = sn - s;
        s = sn;
        // quadratic convergence (phi is nearly linear in s, |phi''/phi'| = O(1)):
        // after a step of size |ds| < tol the error is O(ds^2) < 1e-18
        if (fabs(ds) < NewtonTol<T>::tol) break;
    }
    return clampv(T(0.5) + fast_exp2(s), p.tau_min, p.tau_max);
}

// ---------------------------------------------------------------------------
// d += M0^{-1} dR: populations whose raw moments (monomials 1, x, y, z, xy,
// xz, yz, xx, yy, zz, xyy, xzz, xxy, yzz, xxz, yyz, xxyy, xxzz, yyzz) are dR.
// Each edge population is fixed by the four moments of its plane, each face
// pair by its axis moments minus the edge contributions, and the rest
// population by mass.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void add_raw_moment_change(T d[Q], T dR0, T dRx, T dRy, T dRz, T dRxy, T dRxz, T dRyz, T dRxx,
                                             T dRyy, T dRzz, T dRxyy, T dRxzz, T dRxxy, T dRyzz, T dRxxz,
                                             T dRyyz, T dRxxyy, T dRxxzz, T dRyyzz) {
    const T q = T(0.25), h = T(0.5);
    {
        const T s0 = dRxxyy + dRxy, s1 = dRxyy + dRxxy, s2 = dRxxyy - dRxy, s3 = dRxyy - dRxxy;
        d[7] += q * (s0 + s1);
        d[10] += q * (s0 - s1);
        d[8] += q * (s2 - s3);
        d[9] += q * (s2 + s3);
    }
    {
        const T s0 = dRxxzz + dRxz, s1 = dRxzz + dRxxz, s2 = dRxxzz - dRxz, s3 = dRxzz - dRxxz;
        d[11] += q * (s0 + s1);
        d[14] += q * (s0 - s1);
        d[12] += q * (s2 - s3);
        d[13] += q * (s2 + s3);
    }
    {
        const T s0 = dRyyzz + dRyz, s1 = dRyzz + dRyyz, s2 = dRyyzz - dRyz, s3 = dRyzz - dRyyz;
        d[15] += q * (s0 + s1);
        d[18] += q * (s0 - s1);
        d[16] += q * (s2 - s3);
        d[17] += q * (s2 + s3);
    }
    {
        const T ex = dRxx - dRxxyy - dRxxzz, ox = dRx - dRxyy - dRxzz;
        const T ey = dRyy - dRxxyy - dRyyzz, oy = dRy - dRxxy - dRyzz;
        const T ez = dRzz - dRxxzz - dRyyzz, oz = dRz - dRxxz - dRyyz;
        d[1] += h * (ex + ox); d[2] += h * (ex - ox);
        d[3] += h * (ey + oy); d[4] += h * (ey - oy);
        d[5] += h * (ez + oz); d[6] += h * (ez - oz);
    }
    d[0] += dR0 + (dRxxyy + dRxxzz + dRyyzz) - (dRxx + dRyy + dRzz);
}

// ---------------------------------------------------------------------------
// Collision (Sec. 3): central moments about u, relaxation to the factorized
// attractors, back to populations.  d[] holds deviations f - w on entry
// (pre-collision) and on exit (post-collision).  `omega_out` receives
// omega^nu.  This is the form for the paper's parameter choice
// omega_9 = omega_10..18 = 1: the third-order central moments go to zero and
// the fourth-order ones to their attractors, so only moments up to second
// order of the incoming state are needed.
// ---------------------------------------------------------------------------
template <typename T, bool Forced, int NI = NewtonTol<T>::maxit>
__device__ inline void collide_unit_high(T d[Q], const Relax<T> &p, T *omega_out) {
    const T third = T(1) / T(3);
    // raw moments of the deviations (the rest part contributes 1, 0, 1/3, 0)
    const T exy_p = d[7] + d[10], exy_m = d[8] + d[9];
    const T exz_p = d[11] + d[14], exz_m = d[12] + d[13];
    const T eyz_p = d[15] + d[18], eyz_m = d[16] + d[17];
    const T Exy = exy_p + exy_m, Exz = exz_p + exz_m, Eyz = eyz_p + eyz_m;
    const T Fx = d[1] + d[2], Fy = d[3] + d[4], Fz = d[5] + d[6];
    const T D = d[0] + (Fx + Fy + Fz) + (Exy + Exz + Eyz);          // rho - 1
    T Jx = (d[1] - d[2]) + ((d[7] - d[10]) + (d[9] - d[8])) + ((d[11] - d[14]) + (d[13] - d[12]));
    T Jy = (d[3] - d[4]) + ((d[7] - d[10]) + (d[8] - d[9])) + ((d[15] - d[18]) + (d[17] - d[16]));
    T Jz = (d[5] - d[6]) + ((d[11] - d[14]) + (d[12] - d[13])) + ((d[15] - d[18]) + (d[16] - d[17]));
    T Mxy = exy_p - exy_m, Mxz = exz_p - exz_m, Myz = eyz_p - eyz_m;
    T Mxx = Fx + Exy + Exz, Myy = Fy + Exy + Eyz, Mzz = Fz + Exz + Eyz;   // minus 1/3

    const T rho = T(1) + D;
    const T irho = fast_rcp(rho);
    T fx = T(0), fy = T(0), fz = T(0);
    if (Forced) {
        fx = p.force[0]; fy = p.force[1]; fz = p.force[2];
        Jx += T(0.5) * fx; Jy += T(0.5) * fy; Jz += T(0.5) * fz;
    }
    const T ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
    if (Forced) {
        // first half of the source: raw moments F . grad_u (u^mnp) / 2
        Mxy += T(0.5) * (fx * uy + fy * ux);
        Mxz += T(0.5) * (fx * uz + fz * ux);
        Myz += T(0.5) * (fy * uz + fz * uy);
        Mxx += fx * ux; Myy += fy * uy; Mzz += fz * uz;
    }
    // second-order central moments (diagonal ones minus 1/3)
    const T kxy = Mxy - Jx * uy, kxz = Mxz - Jx * uz, kyz = Myz - Jy * uz;
    const T cxx = Mxx - Jx * ux, cyy = Myy - Jy * uy, czz = Mzz - Jz * uz;

    // non-equilibrium moments m4..m9 and the local omega^nu
    const T m7 = cxx - cyy, m8 = cxx - czz, m9 = (cxx + cyy + czz) - D;
    const T a = T(3) * (m7 * m7 - m7 * m8 + m8 * m8) + T(9) * (kxy * kxy + kxz * kxz + kyz * kyz);
    const T b = T(1.5) * m9 * m9;   // omega_9 = 1
    const T tau = solve_tau<T, NI>(p, rho, a, b);
    const T om = fast_rcp(tau);
    if (omega_out) *omega_out = om;
    const T r = T(1) - om;

    // relaxation: off-diagonal and deviatoric parts by (1 - omega), the trace
    // to its attractor rho (omega_9 = 1)
    const T txy = r * kxy, txz = r * kxz, tyz = r * kyz;
    const T p7 = r * (cxx - cyy);
    const T p8 = r * (cxx + cyy - T(2) * czz);
    const T txx = (T(2) * D + p8 + T(3) * p7) * (T(1) / T(6));
    const T tyy = (T(2) * D + p8 - T(3) * p7) * (T(1) / T(6));
    const T tzz = (D - p8) * third;
    const T Kxx = third + txx, Kyy = third + tyy, Kzz = third + tzz;
    // fourth-order attractors kxx*kyy/rho (minus the rest value 1/9)
    T a_xy = (txx + tyy) * third + txx * tyy;
    T a_xz = (txx + tzz) * third + txx * tzz;
    T a_yz = (tyy + tzz) * third + tyy * tzz;
    if (!p.literal) {
        const T d9 = D * (T(1) / T(9));
        a_xy = (a_xy - d9) * irho;
        a_xz = (a_xz - d9) * irho;
        a_yz = (a_yz - d9) * irho;
    }

    // post-collision raw moments (binomial shift back by u); third-order
    // central moments are zero.  The collision is applied as an increment,
    // f~ = f + Omega (Eq. cascaded collision): Omega is mapped from the
    // changes of the raw moments, which are exact for the conserved ones (0
    // and F) and small for the others, so FP32/FP16 rounding does not build
    // up in mass and momentum.
    T dRx = T(0), dRy = T(0), dRz = T(0);
    T dRxy = txy - kxy, dRxz = txz - kxz, dRyz = tyz - kyz;
    T dRxx = txx - cxx, dRyy = tyy - cyy, dRzz = tzz - czz;
    T Rxyy = T(2) * uy * txy + ux * Kyy + Jx * uy * uy;
    T Rxxy = T(2) * ux * txy + uy * Kxx + Jx * ux * uy;
    T Rxzz = T(2) * uz * txz + ux * Kzz + Jx * uz * uz;
    T Rxxz = T(2) * ux * txz + uz * Kxx + Jx * ux * uz;
    T Ryzz = T(2) * uz * tyz + uy * Kzz + Jy * uz * uz;
    T Ryyz = T(2) * uy * tyz + uz * Kyy + Jy * uy * uz;
    T Rxxyy = a_xy + uy * uy * Kxx + ux * ux * Kyy + T(4) * ux * uy * txy + Jx * ux * uy * uy;
    T Rxxzz = a_xz + uz * uz * Kxx + ux * ux * Kzz + T(4) * ux * uz * txz + Jx * ux * uz * uz;
    T Ryyzz = a_yz + uz * uz * Kyy + uy * uy * Kzz + T(4) * uy * uz * tyz + Jy * uy * uz * uz;
    if (Forced) {
        // both halves of the source on conserved and second-order moments,
        // the second half on the higher ones
        dRx = fx; dRy = fy; dRz = fz;
        dRxy += fx * uy + fy * ux;
        dRxz += fx * uz + fz * ux;
        dRyz += fy * uz + fz * uy;
        dRxx += T(2) * fx * ux; dRyy += T(2) * fy * uy; dRzz += T(2) * fz * uz;
        Rxyy += T(0.5) * (fx * uy * uy) + fy * ux * uy;
        Rxxy += fx * ux * uy + T(0.5) * (fy * ux * ux);
        Rxzz += T(0.5) * (fx * uz * uz) + fz * ux * uz;
        Rxxz += fx * ux * uz + T(0.5) * (fz * ux * ux);
        Ryzz += T(0.5) * (fy * uz * uz) + fz * uy * uz;
        Ryyz += fy * uy * uz + T(0.5) * (fz * uy * uy);
        Rxxyy += fx * ux * uy * uy + fy * ux * ux * uy;
        Rxxzz += fx * ux * uz * uz + fz * ux * ux * uz;
        Ryyzz += fy * uy * uz * uz + fz * uy * uy * uz;
    }
    // incoming third- and fourth-order raw moments (partial sums from above)
    const T dRxyy = Rxyy - ((d[7] - d[10]) + (d[9] - d[8]));
    const T dRxxy = Rxxy - ((d[7] - d[10]) + (d[8] - d[9]));
    const T dRxzz = Rxzz - ((d[11] - d[14]) + (d[13] - d[12]));
    const T dRxxz = Rxxz - ((d[11] - d[14]) + (d[12] - d[13]));
    const T dRyzz = Ryzz - ((d[15] - d[18]) + (d[17] - d[16]));
    const T dRyyz = Ryyz - ((d[15] - d[18]) + (d[16] - d[17]));
    const T dRxxyy = Rxxyy - Exy, dRxxzz = Rxxzz - Exz, dRyyzz = Ryyzz - Eyz;

    add_raw_moment_change<T>(d, T(0), dRx, dRy, dRz, dRxy, dRxz, dRyz, dRxx, dRyy, dRzz, dRxyy, dRxzz, dRxxy,
                             dRyzz, dRxxz, dRyyz, dRxxyy, dRxxzz, dRyyzz);
}

// ---------------------------------------------------------------------------
// Collision in the paper's own form (Sec. 3.1, 3.3): raw moments, the changes
// of moments g4..g18 of the cascade (Eqs. collision kernel g4 - g18), then
// f~ = f + K.g with the orthogonal matrix K.  Three corrections to the
// printed text: K_14 of alpha = 15 is +1 and f~_15 carries +g6 (both from
// the definitions of K_14 and K_6), the brackets of g15 - g17 close as the
// relaxation principle requires, and the fourth-order attractor products
// are divided by rho (unless `literal`).  Any omega_9 and omega_10..18 are
// allowed.  With a body force the raw moments are those of the half-forced
// state and the full source (central moments (0, F, 0, ...)) is added.
// ---------------------------------------------------------------------------
template <typename T, bool Forced, int NI = NewtonTol<T>::maxit>
__device__ inline void collide_ghat(T d[Q], const Relax<T> &p, T *omega_out) {
    const T third = T(1) / T(3);
    // raw moments of the deviations (rest parts: 1, 1/3 on the diagonal, 1/9
    // on xxyy, xxzz, yyzz, zero elsewhere)
    const T Exy = (d[7] + d[10]) + (d[8] + d[9]);
    const T Exz = (d[11] + d[14]) + (d[12] + d[13]);
    const T Eyz = (d[15] + d[18]) + (d[16] + d[17]);
    const T D = d[0] + ((d[1] + d[2]) + (d[3] + d[4]) + (d[5] + d[6])) + (Exy + Exz + Eyz);
    T Jx = (d[1] - d[2]) + ((d[7] - d[10]) + (d[9] - d[8])) + ((d[11] - d[14]) + (d[13] - d[12]));
    T Jy = (d[3] - d[4]) + ((d[7] - d[10]) + (d[8] - d[9])) + ((d[15] - d[18]) + (d[17] - d[16]));
    T Jz = (d[5] - d[6]) + ((d[11] - d[14]) + (d[12] - d[13])) + ((d[15] - d[18]) + (d[16] - d[17]));
    T kxy = (d[7] + d[10]) - (d[8] + d[9]);
    T kxz = (d[11] + d[14]) - (d[12] + d[13]);
    T kyz = (d[15] + d[18]) - (d[16] + d[17]);
    T kxx = (d[1] + d[2]) + Exy + Exz, kyy = (d[3] + d[4]) + Exy + Eyz, kzz = (d[5] + d[6]) + Exz + Eyz;
    T kxyy = (d[7] - d[10]) + (d[9] - d[8]), kxxy = (d[7] - d[10]) + (d[8] - d[9]);
    T kxzz = (d[11] - d[14]) + (d[13] - d[12]), kxxz = (d[11] - d[14]) + (d[12] - d[13]);
    T kyzz = (d[15] - d[18]) + (d[17] - d[16]), kyyz = (d[15] - d[18]) + (d[16] - d[17]);
    T kxxyy = Exy, kxxzz = Exz, kyyzz = Eyz;

    const T rho = T(1) + D;
    const T irho = fast_rcp(rho);
    T fx = T(0), fy = T(0), fz = T(0);
    if (Forced) {
        fx = p.force[0]; fy = p.force[1]; fz = p.force[2];
        Jx += T(0.5) * fx; Jy += T(0.5) * fy; Jz += T(0.5) * fz;
    }
    const T ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
    const T ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    // source raw moments F . grad_u(u^mnp) (zero unless forced)
    T sxy = T(0), sxz = T(0), syz = T(0), sxx = T(0), syy = T(0), szz = T(0);
    T sxyy = T(0), sxzz = T(0), sxxy = T(0), syzz = T(0), sxxz = T(0), syyz = T(0);
    T sxxyy = T(0), sxxzz = T(0), syyzz = T(0);
    if (Forced) {
        sxy = fx * uy + fy * ux; sxz = fx * uz + fz * ux; syz = fy * uz + fz * uy;
        sxx = T(2) * fx * ux; syy = T(2) * fy * uy; szz = T(2) * fz * uz;
        sxyy = fx * uy2 + T(2) * fy * ux * uy; sxxy = T(2) * fx * ux * uy + fy * ux2;
        sxzz = fx * uz2 + T(2) * fz * ux * uz; sxxz = T(2) * fx * ux * uz + fz * ux2;
        syzz = fy * uz2 + T(2) * fz * uy * uz; syyz = T(2) * fy * uy * uz + fz * uy2;
        sxxyy = T(2) * (fx * ux * uy2 + fy * ux2 * uy);
        sxxzz = T(2) * (fx * ux * uz2 + fz * ux2 * uz);
        syyzz = T(2) * (fy * uy * uz2 + fz * uy2 * uz);
        kxy += T(0.5) * sxy; kxz += T(0.5) * sxz; kyz += T(0.5) * syz;
        kxx += T(0.5) * sxx; kyy += T(0.5) * syy; kzz += T(0.5) * szz;
        kxyy += T(0.5) * sxyy; kxxy += T(0.5) * sxxy; kxzz += T(0.5) * sxzz;
        kxxz += T(0.5) * sxxz; kyzz += T(0.5) * syzz; kyyz += T(0.5) * syyz;
        kxxyy += T(0.5) * sxxyy; kxxzz += T(0.5) * sxxzz; kyyzz += T(0.5) * syyzz;
    }
    // full raw second moments kxx + 1/3, ...
    const T Kxx = third + kxx, Kyy = third + kyy, Kzz = third + kzz;

    // non-equilibrium moments (Sec. 3.2) and the local omega^nu
    const T m4 = kxy - rho * ux * uy, m5 = kxz - rho * ux * uz, m6 = kyz - rho * uy * uz;
    const T m7 = (kxx - kyy) - rho * (ux2 - uy2), m8 = (kxx - kzz) - rho * (ux2 - uz2);
    const T m9 = (kxx + kyy + kzz) - (rho * (ux2 + uy2 + uz2) + D);
    const T a = T(3) * (m7 * m7 - m7 * m8 + m8 * m8) + T(9) * (m4 * m4 + m5 * m5 + m6 * m6);
    const T b = T(1.5) * p.omega_bulk * p.omega_bulk * m9 * m9;
    const T om = fast_rcp(solve_tau<T, NI>(p, rho, a, b));
    if (omega_out) *omega_out = om;
    const T w9 = p.omega_bulk;
    const T w10 = p.omega_high[0], w11 = p.omega_high[1], w12 = p.omega_high[2], w13 = p.omega_high[3];
    const T w14 = p.omega_high[4], w15 = p.omega_high[5], w16 = p.omega_high[6], w17 = p.omega_high[7];
    const T w18 = p.omega_high[8];

    // second order (Eqs. g4 - g9)
    const T g4 = om * T(0.25) * (-kxy + rho * ux * uy);
    const T g5 = om * T(0.25) * (-kxz + rho * ux * uz);
    const T g6 = om * T(0.25) * (-kyz + rho * uy * uz);
    const T g7 = om * (T(1) / T(12)) * (-(kxx - kyy) + rho * (ux2 - uy2));
    const T g8 = om * (T(1) / T(36)) * (-(kxx + kyy - T(2) * kzz) + rho * (ux2 + uy2 - T(2) * uz2));
    const T g9 = w9 * (T(1) / T(126)) * (-(kxx + kyy + kzz) + rho * (ux2 + uy2 + uz2) + D);
    // third order (Eqs. g10 - g15)
    const T q8 = T(0.125), q34 = T(0.75);
    const T g10 = w10 * q8 * (-(kxyy + kxzz) + T(2) * (uy * kxy + uz * kxz) + ux * (Kyy + Kzz) -
                              T(2) * rho * ux * (uy2 + uz2)) +
                  (uy * g4 + uz * g5) + q34 * ux * (-(g7 + g8) + T(14) * g9);
    const T g11 = w11 * q8 * (-(kyzz + kxxy) + T(2) * (ux * kxy + uz * kyz) + uy * (Kxx + Kzz) -
                              T(2) * rho * uy * (ux2 + uz2)) +
                  (ux * g4 + uz * g6) + q34 * uy * (g7 - g8 + T(14) * g9);
    const T g12 = w12 * q8 * (-(kxxz + kyyz) + T(2) * (ux * kxz + uy * kyz) + uz * (Kxx + Kyy) -
                              T(2) * rho * uz * (ux2 + uy2)) +
                  (ux * g5 + uy * g6) + T(1.5) * uz * (g8 + T(7) * g9);
    const T g13 = w13 * q8 * (-(kxyy - kxzz) + T(2) * (uy * kxy - uz * kxz) + ux * (kyy - kzz) -
                              T(2) * rho * ux * (uy2 - uz2)) +
                  (uy * g4 - uz * g5) + q34 * ux * (-g7 + T(3) * g8);
    const T g14 = w14 * q8 * (-(kyzz - kxxy) + T(2) * (uz * kyz - ux * kxy) + uy * (kzz - kxx) -
                              T(2) * rho * uy * (uz2 - ux2)) +
                  (-ux * g4 + uz * g6) + q34 * uy * (-g7 - T(3) * g8);
    const T g15 = w15 * q8 * (-(kxxz - kyyz) + T(2) * (ux * kxz - uy * kyz) + uz * (kxx - kyy) -
                              T(2) * rho * uz * (ux2 - uy2)) +
                  (ux * g5 - uy * g6) + T(1.5) * uz * g7;
    // post-collision second-order central moments (moments of K.g)
    const T txx = (kxx - rho * ux2) + T(6) * g7 + T(6) * g8 + T(42) * g9;
    const T tyy = (kyy - rho * uy2) - T(6) * g7 + T(6) * g8 + T(42) * g9;
    const T tzz = (kzz - rho * uz2) - T(12) * g8 + T(42) * g9;
    // attractor products minus their rest values
    const T pxy = (txx + tyy) * third + txx * tyy;
    const T pxz = (txx + tzz) * third + txx * tzz;
    const T pyz = (tyy + tzz) * third + tyy * tzz;
    T A16, A17, A18;
    if (p.literal) {
        A16 = pxy + pxz + pyz;
        A17 = pxy + pxz - T(2) * pyz;
        A18 = pxy - pxz;
    } else {
        A16 = (pxy + pxz + pyz - D * third) * irho;
        A17 = (pxy + pxz - T(2) * pyz) * irho;
        A18 = (pxy - pxz) * irho;
    }
    // fourth order (Eqs. g16 - g18); raw fourth moments enter as deviations
    const T uxuy = ux * uy, uxuz = ux * uz, uyuz = uy * uz;
    const T g16 = w16 * (T(1) / T(12)) *
                      (-(kxxyy + kxxzz + kyyzz) + T(2) * ux * (kxyy + kxzz) + T(2) * uy * (kxxy + kyzz) +
                       T(2) * uz * (kxxz + kyyz) - ux2 * (Kyy + Kzz) - uy2 * (Kzz + Kxx) - uz2 * (Kxx + Kyy) -
                       T(4) * (uxuy * kxy + uxuz * kxz + uyuz * kyz) +
                       T(3) * rho * (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) + A16) -
                  (T(4) / T(3)) * (uxuy * g4 + uxuz * g5 + uyuz * g6) + T(0.5) * (ux2 - uy2) * g7 +
                  T(0.5) * (ux2 + uy2 - T(2) * uz2) * g8 + (-T(7) * (ux2 + uy2 + uz2) - T(8)) * g9 +
                  (T(4) / T(3)) * (ux * g10 + uy * g11 + uz * g12);
    const T g17 = w17 * (T(1) / T(24)) *
                      (-(kxxyy + kxxzz - T(2) * kyyzz) +
                       T(2) * (ux * kxyy + ux * kxzz + uy * kxxy + uz * kxxz - T(2) * (uy * kyzz + uz * kyyz)) -
                       ux2 * (Kyy + Kzz) - uy2 * (Kxx - T(2) * Kzz) - uz2 * (Kxx - T(2) * Kyy) -
                       T(4) * (uxuy * kxy + uxuz * kxz - T(2) * uyuz * kyz) + A17 +
                       T(3) * rho * (ux2 * uy2 + ux2 * uz2 - T(2) * uy2 * uz2)) -
                  (T(2) / T(3)) * (uxuy * g4 + uxuz * g5) + (T(4) / T(3)) * uyuz * g6 +
                  T(0.25) * (ux2 - uy2 - T(3) * uz2 - T(2)) * g7 + T(0.25) * (ux2 - T(5) * uy2 + uz2 - T(2)) * g8 +
                  T(1.75) * (-T(2) * ux2 + uy2 + uz2) * g9 + (T(2) / T(3)) * ux * g10 -
                  third * (uy * g11 + uz * g12) - uy * g14 + uz * g15;
    const T g18 = w18 * q8 *
                      (-(kxxyy - kxxzz) + T(2) * (ux * kxyy - ux * kxzz + uy * kxxy - uz * kxxz) -
                       ux2 * (Kyy - Kzz) - uy2 * Kxx + uz2 * Kxx - T(4) * (uxuy * kxy - uxuz * kxz) + A18 +
                       T(3) * rho * (ux2 * uy2 - ux2 * uz2)) -
                  T(2) * uxuy * g4 + T(2) * uxuz * g5 + q34 * (ux2 - uy2 + uz2 + T(2) / T(3)) * g7 +
                  q34 * (-T(3) * ux2 - uy2 + uz2 - T(2)) * g8 + T(5.25) * (-uy2 + uz2) * g9 + uy * g11 -
                  uz * g12 + T(2) * ux * g13 - uy * g14 - uz * g15;

    // f~ = f + K.g (Eq. post-collision distribution functions)
    const T c9 = T(8) * g9 + g16;
    d[0] += T(12) * g16 - T(30) * g9;
    {
        const T s = g7 + g8 - T(11) * g9 - T(4) * (g16 + g17);
        d[1] += s - T(4) * g10;
        d[2] += s + T(4) * g10;
    }
    {
        const T s = -g7 + g8 - T(11) * g9 - T(4) * g16 + T(2) * (g17 - g18);
        d[3] += s - T(4) * g11;
        d[4] += s + T(4) * g11;
    }
    {
        const T s = -T(2) * g8 - T(11) * g9 - T(4) * g16 + T(2) * (g17 + g18);
        d[5] += s - T(4) * g12;
        d[6] += s + T(4) * g12;
    }
    {
        const T s = T(2) * g8 + c9 + g17 + g18;
        d[7] += s + g4 + g10 + g11 + g13 - g14;
        d[8] += s - g4 - g10 + g11 - g13 - g14;
        d[9] += s - g4 + g10 - g11 + g13 + g14;
        d[10] += s + g4 - g10 - g11 - g13 + g14;
    }
    {
        const T s = g7 - g8 + c9 + g17 - g18;
        d[11] += s + g5 + g10 + g12 - g13 + g15;
        d[12] += s - g5 - g10 + g12 + g13 + g15;
        d[13] += s - g5 + g10 - g12 - g13 - g15;
        d[14] += s + g5 - g10 - g12 + g13 - g15;
    }
    {
        const T s = -g7 - g8 + c9 - T(2) * g17;
        d[15] += s + g6 + g11 + g12 + g14 - g15;
        d[16] += s - g6 - g11 + g12 - g14 - g15;
        d[17] += s - g6 + g11 - g12 + g14 + g15;
        d[18] += s + g6 - g11 - g12 - g14 + g15;
    }
    if (Forced)
        add_raw_moment_change<T>(d, T(0), fx, fy, fz, sxy, sxz, syz, sxx, syy, szz, sxyy, sxzz, sxxy, syzz,
                                 sxxz, syyz, sxxyy, sxxzz, syyzz);
}

// ---------------------------------------------------------------------------
// Single-relaxation-time (BGK) collision with the power-law relaxation time:
// the comparison model of Sec. 5, where every population relaxes at the one
// rate 1/tau towards the second-order polynomial equilibrium (textbook D3Q19
// form).  The strain rate of this model is S = -Pi_neq / (2 rho c_s^2 tau), so
// |gamma|^2 = 4.5 Pi_neq:Pi_neq / (rho tau)^2 and tau solves the same local
// equation as the cascaded rate with a = 4.5 Pi_neq:Pi_neq and b = 0.  On
// deviations d = f - w: f_eq - w = w (D + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u))
// and Pi_neq = M(d) - J u - D/3 I, with M(d) the second moments of d.
// Unforced only.
// ---------------------------------------------------------------------------
template <typename T, int NI = NewtonTol<T>::maxit>
__device__ inline void collide_srt(T d[Q], const Relax<T> &p, T *omega_out) {
    const T third = T(1) / T(3);
    const T exy_p = d[7] + d[10], exy_m = d[8] + d[9];
    const T exz_p = d[11] + d[14], exz_m = d[12] + d[13];
    const T eyz_p = d[15] + d[18], eyz_m = d[16] + d[17];
    const T Exy = exy_p + exy_m, Exz = exz_p + exz_m, Eyz = eyz_p + eyz_m;
    const T Fx = d[1] + d[2], Fy = d[3] + d[4], Fz = d[5] + d[6];
    const T D = d[0] + (Fx + Fy + Fz) + (Exy + Exz + Eyz);          // rho - 1
    const T Jx = (d[1] - d[2]) + ((d[7] - d[10]) + (d[9] - d[8])) + ((d[11] - d[14]) + (d[13] - d[12]));
    const T Jy = (d[3] - d[4]) + ((d[7] - d[10]) + (d[8] - d[9])) + ((d[15] - d[18]) + (d[17] - d[16]));
    const T Jz = (d[5] - d[6]) + ((d[11] - d[14]) + (d[12] - d[13])) + ((d[15] - d[18]) + (d[16] - d[17]));
    const T Mxy = exy_p - exy_m, Mxz = exz_p - exz_m, Myz = eyz_p - eyz_m;
    const T Mxx = Fx + Exy + Exz, Myy = Fy + Exy + Eyz, Mzz = Fz + Exz + Eyz;
    const T rho = T(1) + D;
    const T irho = fast_rcp(rho);
    const T ux = Jx * irho, uy = Jy * irho, uz = Jz * irho;
    const T d3 = D * third;
    const T pxx = Mxx - Jx * ux - d3, pyy = Myy - Jy * uy - d3, pzz = Mzz - Jz * uz - d3;
    const T pxy = Mxy - Jx * uy, pxz = Mxz - Jx * uz, pyz = Myz - Jy * uz;
    const T a = T(4.5) * ((pxx * pxx + pyy * pyy + pzz * pzz) + T(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
    const T om = fast_rcp(solve_tau<T, NI>(p, rho, a, T(0)));
    if (omega_out) *omega_out = om;
    const T usq = T(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T eu = T(cx(q)) * ux + T(cy(q)) * uy + T(cz(q)) * uz;
        const T deq = (T)weight(q) * (D + rho * (T(3) * eu + T(4.5) * eu * eu - usq));
        d[q] += om * (deq - d[q]);
    }
}

// ---------------------------------------------------------------------------
// Wall rules.  A ghost (source outside the lattice on a non-periodic axis)
// lies in the lid plane when its coordinate along the lid axis is just beyond
// the lid face; edges and corners of that plane included.
__device__ inline bool ghost_in_lid(const Geom &g, int sx, int sy, int sz) {
    const int m = g.lid_mask;
    return ((m & 1) && sx == -1) || ((m & 2) && sx == g.nx) || ((m & 4) && sy == -1) ||
           ((m & 8) && sy == g.ny) || ((m & 16) && sz == -1) || ((m & 32) && sz == g.nz);
}

// Half-way bounce-back along e_a: the node's own post-collision population
// opposite to a (w_a = w_opp(a), so the deviation carries over), plus the
// moving-wall term w_a 6 rho_w (e_a . U_w) for a ghost in the lid plane.
template <typename T>
__device__ inline T wall_value(T own_opposite, const Relax<T> &p, int a, bool in_lid) {
    T v = own_opposite;
    if (in_lid) v += (T)weight(a) * (T(cx(a)) * p.lid6[0] + T(cy(a)) * p.lid6[1] + T(cz(a)) * p.lid6[2]);
    return v;
}

// Pull along one direction with the full wall logic (used for lanes on the
// lattice edge): periodic wrap, half-way bounce-back, moving lid.
template <typename S, typename T>
__device__ inline T pull_edge(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int a, int x, int y,
                              int z, uint32_t self) {
    int sx = x - cx(a), sy = y - cy(a), sz = z - cz(a);
    const bool in_lid = ghost_in_lid(g, sx, sy, sz);
    bool wall = false;
    if (sx < 0 || sx >= g.nx) { if (g.px) sx = sx < 0 ? sx + g.nx : sx - g.nx; else wall = true; }
    if (sy < 0 || sy >= g.ny) { if (g.py) sy = sy < 0 ? sy + g.ny : sy - g.ny; else wall = true; }
    if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
    if (!wall) return (T)Plane<S>::load(A, g, a, (uint32_t)(sx + g.nx * sy + g.nxy * sz));
    return wall_value<T>((T)Plane<S>::load(A, g, opp(a), self), p, a, in_lid);
}

// Element index within plane a of the interior pull source of node `self`
// (outside the plane for lanes on the lattice edge, which get the full rule).
__device__ inline uint32_t pull_offset(const Geom &g, int a, uint32_t self) {
    return self + (uint32_t)(-(cx(a) + cy(a) * g.nx + cz(a) * g.nxy));
}

// Lanes on the lattice edge: redo the directions that cross it with the full
// rule (half-way bounce-back returns d_opp(a)(x) since w_a = w_opp(a), plus
// the moving-wall term in the lid plane; periodic axes wrap).
template <typename S, typename T>
__device__ inline void fix_edges(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z,
                                 uint32_t self, T d[Q]) {
    const bool yz_edge = y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
    if (yz_edge) {
#pragma unroll
        for (int a = 1; a < Q; ++a) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
    } else {
        if (x == 0) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == 1) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
        }
        if (x == g.nx - 1) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == -1) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
        }
    }
}

// Pull along a direction that leaves the lattice through an x face only (the
// node is off the y and z faces): periodic x takes the far column, otherwise
// half-way bounce-back, with the lid term when the lid is that x face.  The
// same values as pull_edge, with the x face known.
template <typename S, typename T>
__device__ inline T pull_x_face(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int a, uint32_t self) {
    if (g.px) {
        const int jump = cx(a) == 1 ? g.nx - 1 : 1 - g.nx;
        return (T)Plane<S>::load(A, g, a, self + (uint32_t)(jump - cy(a) * g.nx - cz(a) * g.nxy));
    }
    const bool in_lid = (g.lid_mask & (cx(a) == 1 ? 1 : 2)) != 0;
    return wall_value<T>((T)Plane<S>::load(A, g, opp(a), self), p, a, in_lid);
}

// Pull gather (Eq. cascaded streaming with the wall rules of Sec. 4).  Node
// (x, y, z) receives along e_a the post-collision population that left
// (x, y, z) - e_a.  Interior lanes read at a uniform offset per direction;
// lanes on the lattice edge redo the directions that cross it (fix_edges).
// (The edge logic is written out here again rather than calling fix_edges:
// the one-step kernels compile measurably faster code this way.)
template <typename S, typename T, int LdAux = 0>
__device__ inline void gather(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z,
                              uint32_t self, T d[Q]) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int off = -(cx(a) + cy(a) * g.nx + cz(a) * g.nxy);
        d[a] = (T)Plane<S, LdAux>::load(A, g, a, self + (uint32_t)off);
    }
    const bool yz_edge = y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
    if (yz_edge) {
#pragma unroll
        for (int a = 1; a < Q; ++a) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
    } else {
        if (x == 0) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == 1) d[a] = pull_x_face<S, T>(A, g, p, a, self);
        }
        if (x == g.nx - 1) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == -1) d[a] = pull_x_face<S, T>(A, g, p, a, self);
        }
    }
}

// gather() with the interior loads through grouped descriptors (PlaneGroup).
template <typename S, typename T, int LdAux, int G>
__device__ inline void gather_grouped(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int x, int y, int z,
                                      uint32_t self, T d[Q]) {
    const uint32_t sb = self * (uint32_t)sizeof(S);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const uint32_t c = PlaneGroup<S, G>::offset(g, a) -
                           (uint32_t)(cx(a) + cy(a) * g.nx + cz(a) * g.nxy) * (uint32_t)sizeof(S);
        d[a] = (T)RawBits<S>::template load<LdAux>(PlaneGroup<S, G>::rsrc(A, g, a), sb + c);
    }
    const bool yz_edge = y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
    if (yz_edge) {
#pragma unroll
        for (int a = 1; a < Q; ++a) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
    } else {
        if (x == 0) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == 1) d[a] = pull_x_face<S, T>(A, g, p, a, self);
        }
        if (x == g.nx - 1) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == -1) d[a] = pull_x_face<S, T>(A, g, p, a, self);
        }
    }
}

}  // namespace clbm
