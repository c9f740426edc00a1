// Host-side helpers shared by the single-lattice and batch runtimes:
// error reporting, parameter validation and kernel parameter set-up.
#pragma once

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "../../include/clbm.h"
#include "clbm_internal.hpp"

namespace clbm {

extern thread_local std::string g_err;



inline clbm_status fail(clbm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
inline clbm_status fail(clbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

inline clbm_status hip_fail(hipError_t e, const char *what) {
    return fail(CLBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                          \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

inline size_t elem_bytes(int storage) { return storage == CLBM_F64 ? 8 : (storage == CLBM_F32 ? 4 : 2); }

// Element stride between populations a and a + 1 of a node: the padded plane
// (planes layout) or nx (rows layout).
inline int64_t plane_stride_of(const clbm_params *p) {
    if (p->layout == CLBM_LAYOUT_ROWS) return p->nx;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int64_t align = 256 / (int64_t)elem_bytes(p->storage);   // elements per 256 B
    int64_t plane = (N + align - 1) / align * align;
    if (p->plane_pad >= 0) {
        plane += (p->plane_pad + align - 1) / align * align;
    } else if ((plane * (int64_t)elem_bytes(p->storage)) % 65536 == 0) {
        plane += align;
    }
    return plane;
}

// Bytes of one state buffer: 19 planes, or 19 values per node in rows.
inline size_t state_bytes_of(const clbm_params *p) {
    const int64_t per_pop = p->layout == CLBM_LAYOUT_ROWS ? (int64_t)p->nx * p->ny * p->nz : plane_stride_of(p);
    return (size_t)per_pop * Q * elem_bytes(p->storage);
}

inline bool unit_high_omegas(const clbm_params *p) {
    if (p->omega_bulk != 1.0) return false;
    for (int k = 0; k < 9; ++k)
        if (p->omega_high[k] != 1.0) return false;
    return true;
}

inline int route_of(const clbm_params *p) {
    if (p->collision == CLBM_COLLIDE_SRT) return 2;
    if (p->collision == CLBM_COLLIDE_GHAT) return 1;
    if (p->collision == CLBM_COLLIDE_CENTRAL) return 0;
    return unit_high_omegas(p) ? 0 : 1;
}

inline clbm_status validate(const clbm_params *p) {
    if (!p) return fail(CLBM_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(CLBM_EINVAL, "dimensions must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (p->storage < CLBM_F64 || p->storage > CLBM_F16_DEV)
        return fail(CLBM_EINVAL, "unknown storage %d", p->storage);
    if (p->layout != CLBM_LAYOUT_PLANES && p->layout != CLBM_LAYOUT_ROWS)
        return fail(CLBM_EINVAL, "unknown layout %d", p->layout);
    if (p->f16_rounding != CLBM_F16_STOCHASTIC && p->f16_rounding != CLBM_F16_NEAREST_EVEN)
        return fail(CLBM_EINVAL, "unknown f16_rounding %d", p->f16_rounding);
    // one population plane is addressed through a buffer descriptor with a
    // 32-bit byte range; node indices are 32-bit in either layout
    if (p->layout == CLBM_LAYOUT_PLANES && N * (int64_t)elem_bytes(p->storage) > ((int64_t)1 << 32) - 256)
        return fail(CLBM_EINVAL, "lattice of %lld nodes: one population plane exceeds 4 GiB", (long long)N);
    if (N >= ((int64_t)1 << 31))
        return fail(CLBM_EINVAL, "lattice of %lld nodes: at most 2^31 - 1 nodes", (long long)N);
    // rows: the descriptors of a wave span at most 20 runs of nx + 64 values
    if (p->layout == CLBM_LAYOUT_ROWS &&
        (int64_t)(Q + 1) * (p->nx + 64) * (int64_t)elem_bytes(p->storage) >= ((int64_t)1 << 31))
        return fail(CLBM_EINVAL, "row of %d values too long for the row layout", p->nx);
    if (!(p->K > 0.0) || !isfinite(p->K)) return fail(CLBM_EINVAL, "K must be finite and > 0");
    if (!(p->n > 0.0) || !isfinite(p->n)) return fail(CLBM_EINVAL, "n must be finite and > 0");
    if (!(p->nu_min > 0.0) || !(p->nu_max > p->nu_min) || !isfinite(p->nu_max))
        return fail(CLBM_EINVAL, "need 0 < nu_min < nu_max < inf");
    if (!(p->omega_bulk > 0.0 && p->omega_bulk < 2.0)) return fail(CLBM_EINVAL, "omega_bulk must lie in (0, 2)");
    for (int k = 0; k < 9; ++k)
        if (!(p->omega_high[k] > 0.0 && p->omega_high[k] < 2.0))
            return fail(CLBM_EINVAL, "omega_high[%d] must lie in (0, 2)", k);
    if (p->collision < CLBM_COLLIDE_AUTO || p->collision > CLBM_COLLIDE_SRT)
        return fail(CLBM_EINVAL, "unknown collision form %d", p->collision);
    if (p->collision == CLBM_COLLIDE_SRT && (p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0))
        return fail(CLBM_EINVAL, "the single-relaxation-time model is unforced");
    if (p->collision == CLBM_COLLIDE_CENTRAL && !unit_high_omegas(p))
        return fail(CLBM_EINVAL, "the central-moment form needs omega_bulk = omega_high = 1");
    for (int d = 0; d < 3; ++d) {
        if (p->periodic[d] != 0 && p->periodic[d] != 1) return fail(CLBM_EINVAL, "periodic flags must be 0 or 1");
        if (!isfinite(p->force[d]) || !isfinite(p->lid_velocity[d]))
            return fail(CLBM_EINVAL, "force and lid velocity must be finite");
    }
    if (p->lid_face < CLBM_LID_NONE || p->lid_face > CLBM_LID_PZ)
        return fail(CLBM_EINVAL, "unknown lid face %d", p->lid_face);
    if (p->lid_face != CLBM_LID_NONE && p->periodic[(p->lid_face - 1) / 2])
        return fail(CLBM_EINVAL, "the lid face lies on a periodic axis");
    if (!(p->rho_wall > 0.0) || !isfinite(p->rho_wall)) return fail(CLBM_EINVAL, "rho_wall must be > 0");
    if (p->attractor_literal != 0 && p->attractor_literal != 1)
        return fail(CLBM_EINVAL, "attractor_literal must be 0 or 1");
    if (p->plane_pad < -1 || p->plane_pad > (1 << 24)) return fail(CLBM_EINVAL, "plane_pad out of range");
    return CLBM_OK;
}

template <typename T>
inline Relax<T> make_relax(const clbm_params *p) {
    Relax<T> r;
    memset(&r, 0, sizeof(r));
    for (int d = 0; d < 3; ++d) r.lid6[d] = (T)(6.0 * p->rho_wall * p->lid_velocity[d]);
    r.log2_3K = (T)log2(3.0 * p->K);
    r.three_K = (T)(3.0 * p->K);
    r.n = (T)p->n;
    r.k = (T)(0.5 * (p->n - 1.0));
    r.tau_min = (T)(3.0 * p->nu_min + 0.5);
    r.tau_max = (T)(3.0 * p->nu_max + 0.5);
    r.s_lo = (T)(log2(3.0 * p->nu_min) - 1.0);
    r.s_hi = (T)(log2(3.0 * p->nu_max) + 1.0);
    r.omega_bulk = (T)p->omega_bulk;
    for (int k = 0; k < 9; ++k) r.omega_high[k] = (T)p->omega_high[k];
    for (int d = 0; d < 3; ++d) r.force[d] = (T)p->force[d];
    r.newtonian = p->n == 1.0;
    r.literal = p->attractor_literal;
    r.sr = p->storage == CLBM_F16_DEV && p->f16_rounding == CLBM_F16_STOCHASTIC;
    r.step = 0;
    return r;
}

inline Geom make_geom(const clbm_params *p) {
    Geom g;
    g.nx = p->nx; g.ny = p->ny; g.nz = p->nz;
    g.nxy = p->nx * p->ny;
    g.n = p->nx * p->ny * p->nz;
    g.px = p->periodic[0]; g.py = p->periodic[1]; g.pz = p->periodic[2];
    if (p->lid_face == CLBM_LID_NONE) {
        g.lid_axis = -1; g.lid_side = 0; g.lid_mask = 0;
    } else {
        g.lid_axis = (p->lid_face - 1) / 2;
        g.lid_side = ((p->lid_face - 1) % 2) ? 1 : -1;
        g.lid_mask = 1 << (p->lid_face - 1);
    }
    g.plane = plane_stride_of(p);
    g.rows = p->layout == CLBM_LAYOUT_ROWS;
    g.row = g.rows ? (int64_t)Q * p->nx : (int64_t)p->nx;
    return g;
}

inline bool aligned256(const void *ptr) { return ((uintptr_t)ptr & 255u) == 0; }


}  // namespace clbm
