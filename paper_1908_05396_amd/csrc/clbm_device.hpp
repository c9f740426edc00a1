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
    int64_t plane;          // elements per population plane
};

// ---------------------------------------------------------------------------
// Plane access through raw buffer descriptors: one descriptor per population
// plane (base = plane start, range = n elements), 32-bit byte offsets from a
// VGPR.  Offsets outside the range return 0 without touching memory, so the
// interior pull can run unguarded and edge lanes are patched afterwards.
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

template <typename T> struct Relax {
    T lidc[Q];              // moving-wall term 2 w_a rho_w (e_a . U_w) / c_s^2 per direction
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
// bisection reference); FP64 iterates to convergence.
template <> struct NewtonTol<float> {
    static constexpr bool fixed = true;
    static constexpr int maxit = 4;
    static constexpr float tol = 0.0f;
};
template <> struct NewtonTol<double> {
    static constexpr bool fixed = false;
    static constexpr int maxit = 16;
    static constexpr double tol = 1e-9;     // one more step after this is exact to FP64
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
template <typename T>
__device__ inline T solve_tau(const Relax<T> &p, T rho, T a, T b) {
    if (p.newtonian) return clampv(T(0.5) + p.three_K * fast_rcp(rho), p.tau_min, p.tau_max);
    const T q0 = a + b;
    if (q0 == T(0)) {
        // no shear: the power law gives nu -> infinity (n < 1) or 0 (n > 1)
        return p.k < T(0) ? p.tau_max : p.tau_min;
    }
    const T c = p.log2_3K - p.n * fast_log2(rho);
    T s = clampv(c + p.k * fast_log2(q0), p.s_lo, p.s_hi);   // exact if tau were 1
    const T two_k = T(2) * p.k;
    bool last = false;
    for (int it = 0; it < NewtonTol<T>::maxit; ++it) {
        const T e = fast_exp2(s);                 // tau - 1/2
        const T it1 = fast_rcp(T(0.5) + e);       // 1/tau
        const T q = a * (it1 * it1) + b;
        const T phi = s - c - p.k * fast_log2(q);
        // slope 1 + 2k (a / (tau^2 q)) (tau - 1/2) / tau, with a/(tau^2 q) = 1 - b/q
        const T dphi = T(1) + two_k * (T(1) - b * fast_rcp(q)) * (e * it1);
        const T sn = clampv(s - phi * fast_rcp(dphi), p.s_lo, p.s_hi);
        if (NewtonTol<T>::fixed) {
            s = sn;
            continue;
        }
        const T ds = sn - s;
        s = sn;
        if (last) break;
        if (fabs(ds) < NewtonTol<T>::tol) last = true;   // quadratic convergence: one more step
    }
    return clampv(T(0.5) + fast_exp2(s), p.tau_min, p.tau_max);
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
template <typename T, bool Forced>
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
    const T tau = solve_tau(p, rho, a, b);
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

    // Omega from the raw-moment changes (inverse of the monomial moment map)
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
    d[0] += (dRxxyy + dRxxzz + dRyyzz) - (dRxx + dRyy + dRzz);
}

// ---------------------------------------------------------------------------
// Pull gather (Eq. cascaded streaming with the wall rules of Sec. 4).
// ---------------------------------------------------------------------------
// Node (x, y, z) receives along e_a the post-collision population that left
// (x, y, z) - e_a.  If that source lies beyond a bounce-back wall, half-way
// bounce-back returns the population this node sent toward the wall,
// d_opp(a)(x) (deviations: w_a = w_opp(a)), plus the moving-wall term when the
// ghost belongs to the lid plane.
// Pull along one direction with the full wall logic (used for lanes on the
// lattice edge): periodic wrap, half-way bounce-back, moving lid.
template <typename S, typename T>
__device__ inline T pull_edge(const S *__restrict__ A, const Geom &g, const Relax<T> &p, int a, int x, int y,
                              int z, uint32_t self) {
    const int ex = cx(a), ey = cy(a), ez = cz(a);
    int sx = x - ex, sy = y - ey, sz = z - ez;
    bool wall = false;
    if (sx < 0 || sx >= g.nx) { if (g.px) sx = sx < 0 ? sx + g.nx : sx - g.nx; else wall = true; }
    if (sy < 0 || sy >= g.ny) { if (g.py) sy = sy < 0 ? sy + g.ny : sy - g.ny; else wall = true; }
    if (sz < 0 || sz >= g.nz) { if (g.pz) sz = sz < 0 ? sz + g.nz : sz - g.nz; else wall = true; }
    if (!wall) return (T)Plane<S>::load(A, g, a, (uint32_t)(sx + g.nx * sy + g.nxy * sz));
    T v = (T)Plane<S>::load(A, g, opp(a), self);
    if (g.lid_axis >= 0) {
        // the ghost lies in the lid plane when the source coordinate along the
        // lid axis is just beyond the lid face
        const int sc = g.lid_axis == 0 ? x - ex : (g.lid_axis == 1 ? y - ey : z - ez);
        const int nmax = g.lid_axis == 0 ? g.nx : (g.lid_axis == 1 ? g.ny : g.nz);
        if ((g.lid_side > 0 && sc == nmax) || (g.lid_side < 0 && sc == -1)) v += p.lidc[a];
    }
    return v;
}

// Pull gather (Eq. cascaded streaming with the wall rules of Sec. 4).  Node
// (x, y, z) receives along e_a the post-collision population that left
// (x, y, z) - e_a.  Interior lanes read at a uniform offset per direction;
// lanes on the lattice edge redo the directions that cross it with the full
// rule (half-way bounce-back returns d_opp(a)(x) since w_a = w_opp(a), plus
// the moving-wall term in the lid plane; periodic axes wrap).
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
                if (cx(a) == 1) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
        }
        if (x == g.nx - 1) {
#pragma unroll
            for (int a = 1; a < Q; ++a)
                if (cx(a) == -1) d[a] = pull_edge<S, T>(A, g, p, a, x, y, z, self);
        }
    }
}

}  // namespace clbm
