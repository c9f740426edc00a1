// Internal declarations shared by the kernel and runtime translation units.
#pragma once

#include <type_traits>

#include "clbm_device.hpp"

namespace clbm {

template <typename S> struct StoreCompute;
template <> struct StoreCompute<double> { using T = double; };
template <> struct StoreCompute<float> { using T = float; };
template <> struct StoreCompute<__half> { using T = float; };

constexpr int kReduceThreads = 256;
// threads per stream-collide block: FP32 arithmetic needs < 128 VGPRs, FP64
// about 160, which allows four waves per block
template <typename T> struct MaxThreads { static constexpr int value = 512; };
template <> struct MaxThreads<double> { static constexpr int value = 256; };

struct LaunchGrid {
    uint32_t gx, gy, gz;    // tiles along x, y and z layers
    uint32_t aligned;       // largest multiple of 8 <= number of workgroups
    int32_t remap;          // XCD-contiguous tile order
};

struct StepLaunch {
    int32_t bx, by;         // threads per block along x and y
    int32_t xcd_remap;
    int32_t nt_loads, nt_stores;
    int32_t fuse_steps;     // 1: one step per launch; 2: two (temporal blocking)
    int32_t fuse_rows;      // rows per two-step workgroup, halo rows included (8 or 16)
    int32_t fuse_planes;    // output z planes per two-step workgroup
};
constexpr int kReduceSlots = 10;
// reduction blocks of a lattice: at most this many (grid-stride loop beyond)
constexpr int kReduceMaxBlocks = 1024;
// block partials the no-allocation reduction holds in its static scratch
constexpr int kNoAllocMaxBlocks = 1024;

hipError_t launch_step(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                       const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st);
hipError_t launch_step_rows(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                            const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st);
hipError_t launch_step2(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                        const Relax<float> &pf, bool forced, int route, const StepLaunch &c, hipStream_t st);
hipError_t launch_aa_pair(int storage, void *A, const Geom &g, const Relax<double> &pd, const Relax<float> &pf,
                          bool forced, int route, const StepLaunch &c, hipStream_t st);
hipError_t launch_store_plain(int storage, const double *f0, void *A, const Geom &g, hipStream_t st);
hipError_t launch_init(int storage, const double *f0, void *B, const uint8_t *flags, const Geom &g,
                       const Relax<double> &pd, const Relax<float> &pf, bool forced, int route, hipStream_t st);
hipError_t launch_step_flags(int storage, const void *A, void *B, const uint8_t *flags, const Geom &g,
                             const Relax<double> &pd, const Relax<float> &pf, bool forced, int route, hipStream_t st);
hipError_t launch_check_flags(const uint8_t *flags, int64_t n, double *bad, hipStream_t st);

// Collision forms: 0 = central-moment form for omega_9..18 = 1, 1 = the
// paper's printed changes of moments g4..g18 with f~ = f + K.g.
// Route 2: the single-relaxation-time comparison model (unforced only).
template <typename T, bool Forced, int Route, int NI = NewtonTol<T>::maxit>
__device__ inline void collide(T d[Q], const Relax<T> &p, T *omega_out) {
    if constexpr (Route == 0) {
        collide_unit_high<T, Forced, NI>(d, p, omega_out);
    } else if constexpr (Route == 1) {
        collide_ghat<T, Forced, NI>(d, p, omega_out);
    } else {
        static_assert(!Forced, "the single-relaxation-time model is unforced");
        collide_srt<T, NI>(d, p, omega_out);
    }
}

// FP16 storage with stochastic rounding: replace the post-collision values of
// node `node` by FP16 values drawn up or down (exactly representable, so the
// stores that follow convert them without further rounding).  No-op for the
// other storage types and for round-to-nearest.
template <typename S, typename T>
__device__ inline void round_state(T d[Q], const Relax<T> &p, uint32_t node, uint32_t step) {
    if constexpr (std::is_same<S, __half>::value) {
        if (p.sr) {
            const uint32_t base = sr_base(node, step);
            // the conversion keeps the high half of its first operand: the
            // previous direction's result serves (values as sr_to_f16_grid)
            typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
            half2_t h = __builtin_bit_cast(half2_t, (float)d[0]);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                h = __builtin_amdgcn_cvt_sr_f16_f32(h, (float)d[a], base + (uint32_t)a * kWeyl, false);
                d[a] = (T)(float)h[0];
            }
        }
    }
}

// Newton steps of the FP32 relaxation-rate solve (FP32 and FP16 storage; FP64
// storage iterates to convergence).  Three steps from the tau = 1 estimate
// leave a relative tau error <= 1.4e-6 in exact arithmetic over n in
// [0.4, 1.6], K over five decades and a over twelve, and in FP32 arithmetic
// the solve's own rounding is as large: a fourth step changes tau only at
// that level (emulated in FP32: max |dtau| 2.6e-5 vs 2.2e-5 at n = 0.4, the
// same at n >= 0.9).
template <typename S> struct NewtonSteps { static constexpr int value = 3; };
hipError_t launch_macroscopic(int storage, const void *A, const uint8_t *flags, void *rho, void *u, bool out_f32,
                              const Geom &g, const double *F, hipStream_t st);
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t st);
hipError_t launch_f16_round(const float *in, const uint32_t *seeds, uint16_t *out, int64_t n, int stochastic,
                            hipStream_t st);
hipError_t launch_export(int storage, const void *A, double *f, const Geom &g, hipStream_t st);
hipError_t launch_reduce(int storage, const void *A, const uint8_t *flags, double *snap, int have_prev,
                         const Geom &g, const double *F, double *partials, int nblocks, double *out, hipStream_t st);
hipError_t launch_reduce_noalloc(int storage, const void *A, const uint8_t *flags, double *snap, int have_prev,
                                 const Geom &g, const double *F, int nblocks, double *out, hipStream_t st);

}  // namespace clbm
