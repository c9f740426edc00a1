// C-ABI of the D3Q19 cascaded power-law LBM library (declared in clbm.h):
// parameter validation, handles, kernel parameter set-up and launches.
#include <array>
#include <vector>

#include "clbm_host.hpp"

using namespace clbm;

namespace clbm {
thread_local std::string g_err;
}  // namespace clbm

struct clbm_lattice {
    clbm_params prm;
    Geom geom;
    Relax<double> rd;
    Relax<float> rf;
    bool forced;
    int route;
    bool in_place;          // one buffer, AA access pattern; stores pre-collision populations
    const uint8_t *flags;   // caller's per-node solid flags (NULL: the box of the parameters)
    void *buf[2];
    size_t bytes_each;
    int cur;
    bool initialized;
    int64_t steps_done;
    StepLaunch launch;
    // reduction scratch (library-owned)
    double *partials;
    double *result;
    double *host_result;
    int nblocks;
    double *snapshot;       // FP64 velocity of the previous reduction (residual)
    bool have_snapshot;
};

// Default launch form (measured on the 512^3 cavity, MI355X, in the developed
// flow): one step per launch for every storage type.  Two steps per launch
// halve the state traffic but recompute the first step on the patch ring
// (18-37% more collisions); FP32 comes out even, FP16 (bound by arithmetic)
// and FP64 (whose Newton solve dominates once the whole cavity moves) lose.
// The two-step defaults below are the best measured shapes.
// Velocity output subtracts F/2 from the momentum of the stored state: right
// for post-collision populations (two-buffer form); the in-place form stores
// pre-collision populations, whose momentum needs + F/2.
static std::array<double, 3> output_force(const clbm_lattice *h, const double F[3]) {
    const double s = h->in_place ? -1.0 : 1.0;
    return {s * F[0], s * F[1], s * F[2]};
}

// Index of the next collision (0: the initial one), which keys the stochastic
// rounding of FP16 storage.
static void set_step(clbm_lattice *h, int64_t step) {
    h->rd.step = h->rf.step = (uint32_t)step;
}

static void default_fusion(const clbm_params *p, StepLaunch *c) {
    const bool f64 = p->storage == CLBM_F64;
    c->fuse_steps = 1;
    c->fuse_rows = f64 ? 8 : 16;
    int planes = f64 ? 32 : 8;
    if (planes > p->nz) planes = p->nz;
    c->fuse_planes = planes < 1 ? 1 : planes;
}

extern "C" {

const char *clbm_last_error(void) { return g_err.c_str(); }

#ifndef CLBM_SOURCE_HASH
#define CLBM_SOURCE_HASH "unknown"
#endif
const char *clbm_version(void) { return "clbm 0.2 (gfx950, D3Q19 cascaded power-law) src " CLBM_SOURCE_HASH; }

clbm_status clbm_lattice_tables(int32_t *e, int32_t *o, double *w) {
    for (int a = 0; a < Q; ++a) {
        if (e) { e[3 * a] = cx(a); e[3 * a + 1] = cy(a); e[3 * a + 2] = cz(a); }
        if (o) o[a] = opp(a);
        if (w) w[a] = weight(a);
    }
    return CLBM_OK;
}

clbm_status clbm_copy_probe(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(CLBM_EINVAL, "copy probe: NULL pointer");
    if (bytes % 16 != 0 || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return fail(CLBM_EINVAL, "copy probe: bytes and pointers must be multiples of 16");
    HIP_TRY(launch_copy_probe(src, dst, bytes, (hipStream_t)stream), "clbm_copy_probe");
    return CLBM_OK;
}

clbm_status clbm_f16_round(const float *in, const uint32_t *seeds, uint16_t *out, int64_t n, int32_t mode,
                           void *stream) {
    if (n < 0) return fail(CLBM_EINVAL, "f16 round: n must be >= 0");
    if (mode != CLBM_F16_STOCHASTIC && mode != CLBM_F16_NEAREST_EVEN)
        return fail(CLBM_EINVAL, "f16 round: unknown mode %d", mode);
    if (n > 0 && (!in || !out || (mode == CLBM_F16_STOCHASTIC && !seeds)))
        return fail(CLBM_EINVAL, "f16 round: NULL pointer");
    HIP_TRY(launch_f16_round(in, seeds, out, n, mode == CLBM_F16_STOCHASTIC, (hipStream_t)stream), "clbm_f16_round");
    return CLBM_OK;
}

clbm_status clbm_params_default(clbm_params *p) {
    if (!p) return fail(CLBM_EINVAL, "params is NULL");
    memset(p, 0, sizeof(*p));
    p->nx = p->ny = p->nz = 1;
    p->storage = CLBM_F32;
    p->track_residual = 1;
    p->plane_pad = -1;
    p->layout = CLBM_LAYOUT_ROWS;
    p->K = 0.01;
    p->n = 1.0;
    p->nu_min = (1.0 / 1.95 - 0.5) / 3.0;
    p->nu_max = (1.0 / 0.1 - 0.5) / 3.0;
    p->omega_bulk = 1.0;
    for (int k = 0; k < 9; ++k) p->omega_high[k] = 1.0;
    p->rho_wall = 1.0;
    return CLBM_OK;
}

clbm_status clbm_buffer_size(const clbm_params *p, int64_t *plane, size_t *bytes) {
    clbm_status st = validate(p);
    if (st != CLBM_OK) return st;
    const int64_t ps = plane_stride_of(p);
    if (plane) *plane = ps;
    if (bytes) *bytes = state_bytes_of(p);
    return CLBM_OK;
}

static clbm_status create_common(const clbm_params *p, void *pop_a, void *pop_b, size_t bytes_each, bool in_place,
                                 const uint8_t *flags, clbm_lattice **out) {
    if (!out) return fail(CLBM_EINVAL, "out is NULL");
    *out = nullptr;
    clbm_status st = validate(p);
    if (st != CLBM_OK) return st;
    size_t need = 0;
    clbm_buffer_size(p, nullptr, &need);
    if (!pop_a || !pop_b) return fail(CLBM_EINVAL, "state buffers must not be NULL");
    if (pop_a == pop_b && !in_place) return fail(CLBM_EINVAL, "the two state buffers must differ");
    if (!aligned256(pop_a) || !aligned256(pop_b)) return fail(CLBM_EINVAL, "state buffers must be 256-byte aligned");
    if (bytes_each < need)
        return fail(CLBM_EINVAL, "state buffers hold %zu bytes, need %zu", bytes_each, need);

    clbm_lattice *h = (clbm_lattice *)calloc(1, sizeof(clbm_lattice));
    if (!h) return fail(CLBM_ENOMEM, "host allocation failed");
    h->prm = *p;
    h->geom = make_geom(p);
    h->rd = make_relax<double>(p);
    h->rf = make_relax<float>(p);
    h->forced = p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0;
    h->route = route_of(p);
    h->in_place = in_place;
    h->flags = flags;
    h->buf[0] = pop_a;
    h->buf[1] = pop_b;
    h->bytes_each = bytes_each;
    h->cur = 0;
    // default launch: up to 256 threads along x (whole 64-wide waves), rows
    // stacked along y when the lattice is narrow
    int bx = p->nx >= 256 ? 256 : (p->nx >= 64 ? 64 * (p->nx / 64) : p->nx);
    if (bx > 256) bx = 256;
    // row layout (512^3 cavity, MI355X): 256-wide blocks (FP64: 128) in
    // XCD-contiguous order run 1-6% faster than the dispatch order
    const bool rows = p->layout == CLBM_LAYOUT_ROWS;
    if (rows && p->storage == CLBM_F64 && bx > 128) bx = 128;
    int by = 1;
    const int threads = (rows && p->nx >= 64) ? bx : 256;   // rows: one lattice row per block
    while (bx * by * 2 <= threads && by * 2 <= p->ny) by *= 2;
    h->launch.bx = bx;
    h->launch.by = by;
    h->launch.xcd_remap = rows ? 1 : 0;
    h->launch.nt_loads = 0;
    h->launch.nt_stores = 1;    // streaming stores: the new state is not re-read this step
    default_fusion(p, &h->launch);

    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    int64_t nb = (N + kReduceThreads - 1) / kReduceThreads;
    h->nblocks = (int)(nb < kReduceMaxBlocks ? nb : kReduceMaxBlocks);
    hipError_t e = hipMalloc((void **)&h->partials, sizeof(double) * kReduceSlots * (h->nblocks + 1));
    if (e == hipSuccess) {
        h->result = h->partials + (size_t)kReduceSlots * h->nblocks;
        e = hipHostMalloc((void **)&h->host_result, sizeof(double) * kReduceSlots, hipHostMallocDefault);
    }
    if (e == hipSuccess && p->track_residual) e = hipMalloc((void **)&h->snapshot, sizeof(double) * 3 * N);
    if (e != hipSuccess) {
        clbm_destroy(h);
        return hip_fail(e, "clbm_create: scratch allocation");
    }
    if (flags) {
        // every flag must be fluid, wall or moving wall (checked once, here)
        e = launch_check_flags(flags, N, h->result, nullptr);
        if (e == hipSuccess) e = hipMemcpy(h->host_result, h->result, sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            clbm_destroy(h);
            return hip_fail(e, "clbm_create: flag check");
        }
        if (h->host_result[0] != 0.0) {
            clbm_destroy(h);
            return fail(CLBM_EINVAL, "flags hold values other than 0 (fluid), 1 (wall) and 2 (moving wall)");
        }
    }
    *out = h;
    return CLBM_OK;
}

clbm_status clbm_create(const clbm_params *p, void *pop_a, void *pop_b, size_t bytes_each, const uint8_t *flags,
                        clbm_lattice **out) {
    return create_common(p, pop_a, pop_b, bytes_each, false, flags, out);
}

clbm_status clbm_create_in_place(const clbm_params *p, void *pop, size_t bytes, clbm_lattice **out) {
    return create_common(p, pop, pop, bytes, true, nullptr, out);
}

clbm_status clbm_destroy(clbm_lattice *h) {
    if (!h) return CLBM_OK;
    if (h->partials) (void)hipFree(h->partials);
    if (h->host_result) (void)hipHostFree(h->host_result);
    if (h->snapshot) (void)hipFree(h->snapshot);
    free(h);
    return CLBM_OK;
}

// A temporary device copy of host populations (19 N doubles), released by
// the caller after the stream has consumed it.
static clbm_status stage_host_populations(const double *f0_host, int64_t N, hipStream_t st, double **dev) {
    *dev = nullptr;
    HIP_TRY(hipMalloc((void **)dev, sizeof(double) * Q * (size_t)N), "init: staging allocation");
    hipError_t e = hipMemcpyAsync(*dev, f0_host, sizeof(double) * Q * (size_t)N, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return hip_fail(e, "init: copy of the host populations");
    }
    return CLBM_OK;
}

clbm_status clbm_init_populations(clbm_lattice *h, const double *f0, int on_device, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (!f0) return fail(CLBM_EINVAL, "f0 is NULL");
    if (on_device != 0 && on_device != 1) return fail(CLBM_EINVAL, "on_device must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    const double *src = f0;
    double *staged = nullptr;
    if (!on_device) {
        clbm_status s = stage_host_populations(f0, (int64_t)h->geom.n, st, &staged);
        if (s != CLBM_OK) return s;
        src = staged;
    }
    h->cur = 0;
    set_step(h, 0);
    hipError_t e = h->in_place ? launch_store_plain(h->prm.storage, src, h->buf[0], h->geom, st)
                               : launch_init(h->prm.storage, src, h->buf[0], h->flags, h->geom, h->rd, h->rf,
                                             h->forced, h->route, st);
    if (staged) {
        hipError_t e2 = hipStreamSynchronize(st);
        (void)hipFree(staged);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "clbm_init_populations");
    h->initialized = true;
    h->steps_done = 0;
    h->have_snapshot = false;
    return CLBM_OK;
}

clbm_status clbm_init_rest(clbm_lattice *h, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    h->cur = 0;
    set_step(h, 0);
    // f = w: every deviation is zero; the two-buffer form collides that state once
    if (h->in_place)
        HIP_TRY(launch_store_plain(h->prm.storage, nullptr, h->buf[0], h->geom, (hipStream_t)stream),
                "clbm_init_rest");
    else
        HIP_TRY(launch_init(h->prm.storage, nullptr, h->buf[0], h->flags, h->geom, h->rd, h->rf, h->forced,
                            h->route, (hipStream_t)stream),
                "clbm_init_rest");
    h->initialized = true;
    h->steps_done = 0;
    h->have_snapshot = false;
    return CLBM_OK;
}

clbm_status clbm_step(clbm_lattice *h, int64_t nsteps, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(CLBM_EINVAL, "nsteps must be >= 0");
    if (!h->initialized) return fail(CLBM_ESTATE, "clbm_step before an init call");
    hipStream_t st = (hipStream_t)stream;
    if (h->in_place) {
        if (nsteps % 2) return fail(CLBM_EINVAL, "in-place lattices advance by even step counts (got %lld)",
                                    (long long)nsteps);
        for (int64_t t = 0; t < nsteps; t += 2) {
            set_step(h, h->steps_done + 1);
            HIP_TRY(launch_aa_pair(h->prm.storage, h->buf[0], h->geom, h->rd, h->rf, h->forced, h->route,
                                   h->launch, st),
                    "clbm_step (in place)");
            h->steps_done += 2;
        }
        return CLBM_OK;
    }
    if (h->flags) {
        for (int64_t t = 0; t < nsteps; ++t) {
            set_step(h, h->steps_done + 1);
            HIP_TRY(launch_step_flags(h->prm.storage, h->buf[h->cur], h->buf[1 - h->cur], h->flags, h->geom, h->rd,
                                      h->rf, h->forced, h->route, st),
                    "clbm_step (flagged lattice)");
            h->cur = 1 - h->cur;
            h->steps_done++;
        }
        return CLBM_OK;
    }
    int64_t t = 0;
    if (h->launch.fuse_steps == 2) {
        for (; t + 2 <= nsteps; t += 2) {
            set_step(h, h->steps_done + 1);
            HIP_TRY(launch_step2(h->prm.storage, h->buf[h->cur], h->buf[1 - h->cur], h->geom, h->rd, h->rf,
                                 h->forced, h->route, h->launch, st),
                    "clbm_step (two-step launch)");
            h->cur = 1 - h->cur;
            h->steps_done += 2;
        }
    }
    for (; t < nsteps; ++t) {
        set_step(h, h->steps_done + 1);
        if (h->geom.rows)
            HIP_TRY(launch_step_rows(h->prm.storage, h->buf[h->cur], h->buf[1 - h->cur], h->geom, h->rd, h->rf,
                                     h->forced, h->route, h->launch, st),
                    "clbm_step");
        else
            HIP_TRY(launch_step(h->prm.storage, h->buf[h->cur], h->buf[1 - h->cur], h->geom, h->rd, h->rf,
                                h->forced, h->route, h->launch, st),
                    "clbm_step");
        h->cur = 1 - h->cur;
        h->steps_done++;
    }
    return CLBM_OK;
}

clbm_status clbm_macroscopic(clbm_lattice *h, void *rho, void *u, int32_t out_prec, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (out_prec != CLBM_F64 && out_prec != CLBM_F32)
        return fail(CLBM_EINVAL, "out_prec must be CLBM_F64 or CLBM_F32 (got %d)", out_prec);
    if (!h->initialized) return fail(CLBM_ESTATE, "clbm_macroscopic before an init call");
    if (!rho && !u) return CLBM_OK;
    const double F[3] = {h->prm.force[0], h->prm.force[1], h->prm.force[2]};
    HIP_TRY(launch_macroscopic(h->prm.storage, h->buf[h->cur], h->flags, rho, u, out_prec == CLBM_F32, h->geom,
                               output_force(h, F).data(), (hipStream_t)stream),
            "clbm_macroscopic");
    return CLBM_OK;
}

clbm_status clbm_populations(clbm_lattice *h, double *f, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (!f) return fail(CLBM_EINVAL, "output is NULL");
    if (!h->initialized) return fail(CLBM_ESTATE, "clbm_populations before an init call");
    HIP_TRY(launch_export(h->prm.storage, h->buf[h->cur], f, h->geom, (hipStream_t)stream), "clbm_populations");
    return CLBM_OK;
}

clbm_status clbm_reduce(clbm_lattice *h, double out[8], void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (!out) return fail(CLBM_EINVAL, "out is NULL");
    if (!h->initialized) return fail(CLBM_ESTATE, "clbm_reduce before an init call");
    hipStream_t st = (hipStream_t)stream;
    const double F[3] = {h->prm.force[0], h->prm.force[1], h->prm.force[2]};
    HIP_TRY(launch_reduce(h->prm.storage, h->buf[h->cur], h->flags, h->snapshot, h->have_snapshot ? 1 : 0,
                          h->geom, output_force(h, F).data(), h->partials, h->nblocks, h->result, st),
            "clbm_reduce");
    HIP_TRY(hipMemcpyAsync(h->host_result, h->result, sizeof(double) * kReduceSlots, hipMemcpyDeviceToHost, st),
            "clbm_reduce: copy");
    HIP_TRY(hipStreamSynchronize(st), "clbm_reduce: sync");
    const double *r = h->host_result;
    out[0] = r[9] + r[0];      // fluid nodes + sum of (rho - 1)
    out[1] = r[1]; out[2] = r[2]; out[3] = r[3];
    out[4] = (h->snapshot && h->have_snapshot && r[5] > 0.0) ? sqrt(r[4] / r[5]) : 0.0;
    out[5] = r[6];
    out[6] = r[7];
    out[7] = r[8];
    if (h->snapshot) h->have_snapshot = true;
    if (r[6] > 0.0) return fail(CLBM_EUNSTABLE, "%.0f nodes hold non-finite populations", r[6]);
    return CLBM_OK;
}

clbm_status clbm_reduce_noalloc(clbm_lattice *h, double *out_dev, void *stream) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (!out_dev) return fail(CLBM_EINVAL, "out_dev is NULL");
    if (!h->initialized) return fail(CLBM_ESTATE, "clbm_reduce_noalloc before an init call");
    if (h->nblocks > kNoAllocMaxBlocks)
        return fail(CLBM_EINVAL, "clbm_reduce_noalloc: %d reduction blocks exceed the static scratch of %d",
                    h->nblocks, kNoAllocMaxBlocks);
    const double F[3] = {h->prm.force[0], h->prm.force[1], h->prm.force[2]};
    HIP_TRY(launch_reduce_noalloc(h->prm.storage, h->buf[h->cur], h->flags, h->snapshot, h->have_snapshot ? 1 : 0,
                                  h->geom, output_force(h, F).data(), h->nblocks, out_dev, (hipStream_t)stream),
            "clbm_reduce_noalloc");
    if (h->snapshot) h->have_snapshot = true;
    return CLBM_OK;
}

clbm_status clbm_state(clbm_lattice *h, int *buffer_index, int64_t *steps_done) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (buffer_index) *buffer_index = h->cur;
    if (steps_done) *steps_done = h->steps_done;
    return CLBM_OK;
}

clbm_status clbm_set_launch(clbm_lattice *h, const clbm_launch *c) {
    if (!h || !c) return fail(CLBM_EINVAL, "NULL argument");
    const int maxt = h->prm.storage == CLBM_F64 ? 256 : 512;
    if (c->bx < 1 || c->by < 1 || c->bx * c->by > maxt)
        return fail(CLBM_EINVAL, "block %d x %d: need 1 <= bx*by <= %d", c->bx, c->by, maxt);
    if ((c->xcd_remap | c->nt_loads | c->nt_stores) & ~1) return fail(CLBM_EINVAL, "launch flags must be 0 or 1");
    if (c->fuse_steps != 1 && c->fuse_steps != 2) return fail(CLBM_EINVAL, "fuse_steps must be 1 or 2");
    const bool rows_ok = c->fuse_rows == 8 || (c->fuse_rows == 16 && h->prm.storage != CLBM_F64) ||
                         (c->fuse_rows == 12 && h->prm.storage == CLBM_F32);
    if (!rows_ok) return fail(CLBM_EINVAL, "fuse_rows must be 8, 16 (not FP64) or 12 (FP32 only)");
    if (c->fuse_planes < 1) return fail(CLBM_EINVAL, "fuse_planes must be >= 1");
    if (c->fuse_steps == 2 && h->in_place) return fail(CLBM_EINVAL, "in-place lattices run one step per launch");
    if (c->fuse_steps == 2 && h->route == 2)
        return fail(CLBM_EINVAL, "the single-relaxation-time model runs one step per launch");
    if (c->fuse_steps == 2 && h->flags) return fail(CLBM_EINVAL, "flagged lattices run one step per launch");
    if (c->reserved != 0) return fail(CLBM_EINVAL, "reserved field must be 0");
    h->launch.bx = c->bx;
    h->launch.by = c->by;
    h->launch.xcd_remap = c->xcd_remap;
    h->launch.nt_loads = c->nt_loads;
    h->launch.nt_stores = c->nt_stores;
    h->launch.fuse_steps = c->fuse_steps;
    h->launch.fuse_rows = c->fuse_rows;
    h->launch.fuse_planes = c->fuse_planes;
    return CLBM_OK;
}

clbm_status clbm_get_launch(clbm_lattice *h, clbm_launch *c) {
    if (!h || !c) return fail(CLBM_EINVAL, "NULL argument");
    c->bx = h->launch.bx;
    c->by = h->launch.by;
    c->xcd_remap = h->launch.xcd_remap;
    c->nt_loads = h->launch.nt_loads;
    c->nt_stores = h->launch.nt_stores;
    c->fuse_steps = h->launch.fuse_steps;
    c->fuse_rows = h->launch.fuse_rows;
    c->fuse_planes = h->launch.fuse_planes;
    c->reserved = 0;
    return CLBM_OK;
}

clbm_status clbm_set_block(clbm_lattice *h, int32_t bx, int32_t by) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    clbm_launch c;
    clbm_get_launch(h, &c);
    c.bx = bx;
    c.by = by;
    return clbm_set_launch(h, &c);
}

clbm_status clbm_autotune(clbm_lattice *h, void *stream, clbm_launch *best, double *best_ms) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (h->in_place) return fail(CLBM_EINVAL, "autotune: the one-buffer form overwrites its state");
    if (h->flags) return fail(CLBM_EINVAL, "autotune: flagged lattices run one generic kernel");
    if (!h->initialized) return fail(CLBM_ESTATE, "autotune needs an initialised state");
    hipStream_t st = (hipStream_t)stream;
    const int maxt = h->prm.storage == CLBM_F64 ? 256 : 512;
    const int wmax = (h->prm.nx + 63) / 64 * 64;
    // candidates: one step per launch over block shapes, tile orders and cache
    // hints, plus the two-step configuration in place if there is one
    std::vector<StepLaunch> cands;
    for (int bx = 64; bx <= 512 && (bx <= wmax || bx == 64); bx *= 2)
        for (int by = 1; by <= 4; by *= 2) {
            if (bx * by > maxt || (by > 1 && by > h->prm.ny)) continue;
            for (int mode = 0; mode < 8; ++mode) {
                StepLaunch c = h->launch;
                c.fuse_steps = 1;
                c.bx = bx;
                c.by = by;
                c.xcd_remap = mode & 1;
                c.nt_loads = (mode >> 1) & 1;
                c.nt_stores = (mode >> 2) & 1;
                cands.push_back(c);
            }
        }
    // two steps per launch (not for the comparison model): patch heights 8 and 16 (not FP64), z chunks of 16
    // and 32 planes, both patch orders and store hints
    if (h->route != 2)
        for (int rows = 8; rows <= 16; rows += 8) {
            if (rows == 16 && h->prm.storage == CLBM_F64) continue;
            for (int planes = 16; planes <= 32; planes *= 2)
                for (int mode = 0; mode < 4; ++mode) {
                    StepLaunch c = h->launch;
                    c.fuse_steps = 2;
                    c.fuse_rows = rows;
                    c.fuse_planes = planes;
                    c.xcd_remap = mode & 1;
                    c.nt_stores = mode >> 1;
                    cands.push_back(c);
                }
        }
    if (h->launch.fuse_steps == 2)      // the two-step configuration in place
        cands.push_back(h->launch);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "autotune: event");
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "autotune: event");
    }
    // a trial launch reads the current buffer and writes the other one
    auto trial = [&](const StepLaunch &c) -> hipError_t {
        const void *A = h->buf[h->cur];
        void *B = h->buf[1 - h->cur];
        if (c.fuse_steps == 2)
            return launch_step2(h->prm.storage, A, B, h->geom, h->rd, h->rf, h->forced, h->route, c, st);
        if (h->geom.rows)
            return launch_step_rows(h->prm.storage, A, B, h->geom, h->rd, h->rf, h->forced, h->route, c, st);
        return launch_step(h->prm.storage, A, B, h->geom, h->rd, h->rf, h->forced, h->route, c, st);
    };
    const int reps = 3;
    StepLaunch win = h->launch;
    double win_ms = 1e300;
    for (const StepLaunch &c : cands) {
        e = trial(c);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = trial(c);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        const double per_step = ms / reps / (c.fuse_steps == 2 ? 2.0 : 1.0);
        if (per_step < win_ms) {
            win_ms = per_step;
            win = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "autotune: trial launch");
    h->launch = win;
    if (best) clbm_get_launch(h, best);
    if (best_ms) *best_ms = win_ms;
    return CLBM_OK;
}

clbm_status clbm_get_block(clbm_lattice *h, int32_t *bx, int32_t *by) {
    if (!h) return fail(CLBM_EINVAL, "handle is NULL");
    if (bx) *bx = h->launch.bx;
    if (by) *by = h->launch.by;
    return CLBM_OK;
}

}  // extern "C"
