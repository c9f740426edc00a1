// Internal declarations shared by the kernel and runtime translation units.
#pragma once

#include "clbm_device.hpp"

namespace clbm {

template <typename S> struct StoreCompute;
template <> struct StoreCompute<double> { using T = double; };
template <> struct StoreCompute<float> { using T = float; };
template <> struct StoreCompute<__half> { using T = float; };

constexpr int kReduceThreads = 256;
constexpr int kMaxBlock = 256;      // threads per stream-collide block
constexpr int kReduceSlots = 9;

hipError_t launch_step(int storage, const void *A, void *B, const Geom &g, const Relax<double> &pd,
                       const Relax<float> &pf, bool forced, dim3 block, hipStream_t st);
hipError_t launch_init(int storage, const double *f0, void *B, const Geom &g, const Relax<double> &pd,
                       const Relax<float> &pf, bool forced, hipStream_t st);
hipError_t launch_macroscopic(int storage, const void *A, double *rho, double *u, const Geom &g,
                              const double *F, hipStream_t st);
hipError_t launch_export(int storage, const void *A, double *f, const Geom &g, hipStream_t st);
hipError_t launch_reduce(int storage, const void *A, float *snap, int have_prev, const Geom &g,
                         const double *F, double *partials, int nblocks, double *out, hipStream_t st);

}  // namespace clbm
