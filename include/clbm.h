/*
 * clbm.h — D3Q19 cascaded (central-moment, multiple-relaxation-time) lattice
 * Boltzmann method for power-law fluids on AMD Instinct MI355X (gfx950).
 *
 * Method: Adam, Hajabdollahi & Premnath, "Cascaded lattice Boltzmann modeling
 * and simulations of three-dimensional non-Newtonian fluid flows",
 * arXiv:1908.05396.  Section numbers below refer to that paper.
 *
 * One time step (Sec. 3) is: collide every node (central moments about the
 * local velocity, second-order rates set from the local shear rate through
 * the power-law viscosity, higher orders relaxed to factorized attractors),
 * then stream (Eq. cascaded streaming).  The library fuses both into one pull
 * kernel: each node gathers the post-collision populations of its upwind
 * neighbours, applies the wall rules, collides and writes its own
 * post-collision populations to the other of two buffers.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3, rest density 1.
 *   - Particle velocities e_alpha, alpha = 0..18, in the order of Sec. 3:
 *     rest; +x -x +y -y +z -z; (+1,+1,0) (-1,+1,0) (+1,-1,0) (-1,-1,0);
 *     (+1,0,+1) (-1,0,+1) (+1,0,-1) (-1,0,-1); (0,+1,+1) (0,-1,+1) (0,+1,-1)
 *     (0,-1,-1).
 *   - Node index i = x + nx*(y + ny*z) (x fastest).  Walls are not stored:
 *     they sit half-way between the outermost fluid node and a virtual ghost
 *     layer (half-way bounce-back, Sec. 4.1).
 *   - State buffers hold one value per (alpha, node) in one of two layouts
 *     (clbm_layout).  Planes: for each alpha a plane of `plane_stride`
 *     values (>= nx*ny*nz, padded), value(alpha, i) at element
 *     alpha*plane_stride + i.  Rows: the 19 values of a lattice row (fixed
 *     y, z) stored as 19 consecutive runs of nx, value(alpha, x, y, z) at
 *     element ((y + ny*z)*19 + alpha)*nx + x.  Each value is the deviation
 *     f_alpha - w_alpha of the post-collision population (pre-collision in
 *     the one-buffer form of clbm_create_in_place) from the rest
 *     weight w = (1/3, 1/18 x 6, 1/36 x 12), stored as double (CLBM_F64),
 *     float (CLBM_F32) or IEEE half (CLBM_F16_DEV, rounded as
 *     clbm_params.f16_rounding says).
 *     Arithmetic is double for CLBM_F64 and float otherwise.
 *   - State buffers and pools must be 256-byte aligned device memory owned
 *     by the caller.  The library never frees caller memory.  It allocates a
 *     small amount of its own device memory in clbm_create (reduction
 *     partials, an optional FP64 velocity snapshot) and none in clbm_step.
 *   - Streams are hipStream_t values passed as void* (0 = null stream).
 *     clbm_step and the other launches are asynchronous; clbm_reduce
 *     synchronizes its stream.
 *   - Every function returns clbm_status; on failure clbm_last_error()
 *     returns a message (thread-local).  A handle must be used from one host
 *     thread at a time.
 */
#ifndef CLBM_H
#define CLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CLBM_OK = 0,
    CLBM_EINVAL = -1,    /* bad argument or parameter */
    CLBM_ENOMEM = -2,    /* library-side allocation failed */
    CLBM_EHIP = -3,      /* a HIP runtime call failed */
    CLBM_EUNSTABLE = -4, /* clbm_reduce found NaN/Inf in the state */
    CLBM_ESTATE = -5     /* call out of order (e.g. step before init) */
} clbm_status;

typedef enum {
    CLBM_F64 = 0,     /* FP64 storage, FP64 arithmetic */
    CLBM_F32 = 1,     /* FP32 storage of f - w, FP32 arithmetic */
    CLBM_F16_DEV = 2  /* FP16 storage of f - w, FP32 arithmetic */
} clbm_storage;

/* Two algebraically equivalent forms of the cascaded collision (they agree
 * to rounding; see tests): the central-moment form relaxes each central-moment
 * combination and maps the raw-moment changes back to populations, and is
 * specialised to omega_9 = omega_10..18 = 1 (the paper's choice); the printed
 * form evaluates the changes of moments g4..g18 and f~ = f + K.g (Sec. 3.1,
 * 3.3) for any omega_9, omega_10..18.  A third value selects the paper's
 * single-relaxation-time comparison model instead of its scheme. */
typedef enum {
    CLBM_COLLIDE_AUTO = 0,     /* central-moment form when omega_9..18 are all 1, else printed form */
    CLBM_COLLIDE_CENTRAL = 1,  /* requires omega_9..18 = 1 */
    CLBM_COLLIDE_GHAT = 2,
    CLBM_COLLIDE_SRT = 3       /* not the paper's scheme: its single-relaxation-time (BGK) comparison
                                  model (Sec. 5) with the same power-law relaxation time, for cost and
                                  stability comparisons; unforced, one step per launch, no batches */
} clbm_collision;

/* Layout of the state buffers (see Conventions).  Both hold the same values
 * and give the same results; the row layout keeps the 19 populations of a row
 * within 19*nx consecutive values, so one step reads 9 and writes 1 compact
 * region per row instead of touching 38 planes far apart in memory, which
 * DRAM serves faster.  Both run one or two steps per launch. */
typedef enum {
    CLBM_LAYOUT_PLANES = 0,
    CLBM_LAYOUT_ROWS = 1
} clbm_layout;

typedef enum {
    CLBM_LID_NONE = 0, CLBM_LID_MX = 1, CLBM_LID_PX = 2, CLBM_LID_MY = 3,
    CLBM_LID_PY = 4, CLBM_LID_MZ = 5, CLBM_LID_PZ = 6
} clbm_lid_face;

/* Rounding of the FP16 state.  Stochastic (default): each stored collision
 * result is rounded up or down at random, with the probability that makes
 * the expected stored value equal to the FP32 result, so rounding errors do
 * not repeat from step to step (round-to-nearest of a slowly changing value
 * repeats the same error every step, a bias that accumulates in the flow).
 * The random bits are a counter-based hash of the node and the collision
 * index, offset per direction: results are reproducible and do not depend on
 * the launch form, layout or block shape.  Nearest even: IEEE
 * round-to-nearest-even. */
typedef enum { CLBM_F16_STOCHASTIC = 0, CLBM_F16_NEAREST_EVEN = 1 } clbm_f16_rounding;

/* Per-node flag values of the optional flag array of clbm_create: a fluid
 * node is updated by the scheme; a link from a fluid node to a wall node is
 * closed by half-way bounce-back (Sec. 4.1), and to a moving-wall node by
 * bounce-back with the moving-wall momentum term of lid_velocity (Sec. 4.3). */
enum { CLBM_FLUID = 0, CLBM_WALL = 1, CLBM_MOVING_WALL = 2 };

/* Problem description (Sec. 2 constitutive law, Sec. 3 scheme, Sec. 4 set-ups).
 * Fill with clbm_params_default() and override. */
typedef struct {
    int32_t nx, ny, nz;        /* fluid nodes per axis (each >= 1) */
    int32_t periodic[3];       /* 1: periodic axis; 0: half-way bounce-back walls at both ends */
    int32_t lid_face;          /* clbm_lid_face: the wall whose ghost plane moves with lid_velocity
                                  (edge and corner ghosts of that plane included) */
    int32_t storage;           /* clbm_storage */
    int32_t attractor_literal; /* 0: fourth-order attractors kxx*kyy/rho (default);
                                  1: kxx*kyy as printed (linearly unstable, for study only) */
    int32_t track_residual;    /* 1: keep an FP64 velocity snapshot (24 bytes per node) for the
                                  steady-state residual of clbm_reduce; 0: no residual */
    int32_t plane_pad;         /* planes layout: extra elements between population planes (>= 0), on
                                  top of the 256-byte rounding; -1: library default (see
                                  clbm_buffer_size); unused in the row layout */
    int32_t collision;         /* clbm_collision: which algebraic form of the collision runs */
    int32_t layout;            /* clbm_layout of the state buffers */
    int32_t f16_rounding;      /* CLBM_F16_DEV storage: how collision results are rounded to FP16
                                  (clbm_f16_rounding); ignored for the other storage types */
    double K;                  /* consistency coefficient mu_p > 0 (Eq. 5) */
    double n;                  /* power-law index n > 0 (Eq. 5; n = 1 Newtonian) */
    double nu_min, nu_max;     /* clip of the apparent kinematic viscosity mu/rho,
                                  0 < nu_min < nu_max; the relaxation rate is then
                                  1/(3 nu_max + 1/2) <= omega <= 1/(3 nu_min + 1/2).  Rates
                                  near 2 at the lid corners of shear-thinning cavities at
                                  Re ~ 10^3 make the scheme diverge; the default caps omega
                                  at 1.95 */
    double omega_bulk;         /* omega_9 in (0, 2); the paper uses 1 */
    double omega_high[9];      /* omega_10 .. omega_18 in (0, 2); the paper uses 1 */
    double force[3];           /* body force per unit volume (0: unforced kernel) */
    double lid_velocity[3];    /* velocity U_w of the moving wall */
    double rho_wall;           /* density in the moving-wall term 2 w rho_w (e.U_w)/c_s^2, > 0 */
} clbm_params;

typedef struct clbm_lattice clbm_lattice;

/* Defaults: 1x1x1, no periodic axis, no lid, FP32 storage, normalized
 * attractors, residual tracking on, default plane padding, automatic
 * collision form, row layout, K = 0.01, n = 1, viscosity clip for omega in [0.1, 1.95],
 * omega_bulk = omega_high = 1 (the paper's choice, Sec. 3.2), no force,
 * rho_wall = 1.  EINVAL if p is NULL. */
clbm_status clbm_params_default(clbm_params *p);

/* Element stride between the values of populations alpha and alpha + 1 of
 * a node, and the bytes one state buffer needs.  Planes: the stride is the
 * plane, nx*ny*nz rounded up to 256 bytes, plus plane_pad elements (default:
 * 256 bytes more when the rounded plane is a multiple of 64 KiB, so the 19
 * planes do not all start on the same HBM channel); the buffer holds 19
 * planes.  Rows: the stride is nx and the buffer holds 19*nx*ny*nz values
 * (plane_pad unused).  Either output pointer may be NULL.  Validates the
 * parameters (EINVAL). */
clbm_status clbm_buffer_size(const clbm_params *p, int64_t *plane_stride, size_t *bytes);

/* Create a lattice (the problem statement of Sec. 4: dimensions, power law
 * K and n of Eq. 5, body force or lid velocity, wall kinds) over two
 * caller-owned state buffers of `bytes_each` bytes (>= clbm_buffer_size),
 * 256-byte aligned device memory.
 *
 * flags: NULL, or a device array of nx*ny*nz bytes (node index
 * x + nx*(y + ny*z)) of CLBM_FLUID / CLBM_WALL / CLBM_MOVING_WALL, owned by
 * the caller, read by every step and left unchanged for the lifetime of the
 * lattice.  NULL gives the box of the parameters (walls, lid and periodic
 * axes on its faces, the geometry of every set-up of Sec. 4) and the tuned
 * kernels.  With flags, solid nodes are inside the lattice (the box faces
 * still follow the parameters), hold the rest state, report rho = 1 and
 * u = 0, and are left out of clbm_reduce; such lattices run one generic
 * kernel, one step per launch (fuse_steps = 2 and clbm_autotune are refused).
 *
 * Validates every parameter and flag value (EINVAL, with the reason in
 * clbm_last_error), allocates reduction scratch (ENOMEM/EHIP).  With flags
 * the call synchronizes the null stream once (flag check).  The state is
 * undefined until an init call. */
clbm_status clbm_create(const clbm_params *p, void *pop_a, void *pop_b, size_t bytes_each,
                        const uint8_t *flags, clbm_lattice **out);

/* Create a lattice over ONE caller-owned state buffer (half the memory of
 * clbm_create), stepped in place with the AA access pattern: an even step
 * collides every node and stores each post-collision population in the
 * node's slot of the opposite direction; an odd step pulls those from the
 * neighbours, collides and pushes the results into the neighbours' natural
 * slots.  Same bytes per node update and same results (to rounding) as the
 * two-buffer form.  Differences: the buffer holds PRE-collision populations
 * (time t, before its collision), so clbm_populations returns those;
 * clbm_init_* store the initial populations without colliding them;
 * clbm_step accepts even step counts only (EINVAL otherwise); one step per
 * launch (fuse_steps = 2 is refused); either layout; no per-node flags.
 * Velocities from clbm_macroscopic and clbm_reduce are the same physical
 * quantities as in the two-buffer form.  The streaming and collision are
 * those of clbm_step (Sec. 3); the access pattern is the published "AA"
 * scheme for single-buffer lattice Boltzmann updates (Bailey et al., ICPP
 * 2009). */
clbm_status clbm_create_in_place(const clbm_params *p, void *pop, size_t bytes, clbm_lattice **out);

/* Rest initial state f = w (rho = 1, u = 0; the rest state of the
 * attractors of Sec. 3), collided once so the buffer holds post-collision
 * populations (time 0; stored as is in the in-place form).  Asynchronous. */
clbm_status clbm_init_rest(clbm_lattice *h, void *stream);

/* Initial state from caller populations f0 (double, 19 planes of
 * nx*ny*nz values, unpadded, alpha-major, in the velocity order of Sec. 3):
 * collided once (Eq. cascaded collision) and stored in the state's format
 * (the in-place form stores f0 itself).  f0 is only read.  on_device = 1:
 * f0 is device memory and the call is asynchronous (f0 must stay valid until
 * `stream` has run it); on_device = 0: f0 is host memory, which the call
 * copies through a temporary device buffer (ENOMEM/EHIP if that allocation
 * fails) and then synchronizes `stream`.  Other values: EINVAL. */
clbm_status clbm_init_populations(clbm_lattice *h, const double *f0, int on_device, void *stream);

/* Advance nsteps time steps (>= 0; Sec. 3: collision, Eq. cascaded
 * collision with the local relaxation rate of Sec. 3.2, then streaming,
 * Eq. cascaded streaming, with the wall rules of Sec. 4): one fused pull
 * stream-collide launch per step (two steps per launch with fuse_steps = 2;
 * in the in-place form one launch per step and nsteps even).  Asynchronous;
 * no host synchronization, no allocation, no NaN check (clbm_reduce does
 * that).  EINVAL for nsteps < 0, ESTATE before an init call. */
clbm_status clbm_step(clbm_lattice *h, int64_t nsteps, void *stream);

/* Density and velocity at the current time (the hydrodynamic fields of
 * Sec. 3, Eq. hydrodynamic fields), computed in FP64 and written to device
 * outputs in out_prec (CLBM_F64: double, CLBM_F32: float; CLBM_F16_DEV is
 * refused with EINVAL), unpadded: rho[i], u[c*N + i] for c = x, y, z.
 * Collision conserves mass and momentum, so they are read from the stored
 * post-collision populations: rho = sum f, u = (sum e f - F/2)/rho (in-place
 * form, pre-collision populations: u = (sum e f + F/2)/rho).  Solid nodes of
 * a flagged lattice report rho = 1, u = 0.  Either pointer may be NULL.
 * Asynchronous. */
clbm_status clbm_macroscopic(clbm_lattice *h, void *rho_dev, void *u_dev, int32_t out_prec, void *stream);

/* The stored populations f = w + stored deviation (Sec. 3 velocity order),
 * as double, 19 unpadded planes (device output, 19 N doubles):
 * post-collision, or pre-collision in the in-place form.  Asynchronous. */
clbm_status clbm_populations(clbm_lattice *h, double *f_dev, void *stream);

/* FP64 reductions over the fluid nodes (the conserved mass and momentum of
 * the collision, Sec. 3; the steady-state criterion of the cavity runs,
 * Sec. 4.3), synchronizes `stream`:
 *   out[0] total mass sum rho          out[4] residual |u - u_prev|_2 / |u|_2
 *   out[1..3] total momentum sum rho u     against the previous clbm_reduce
 *                                          (0 on the first call or if untracked;
 *                                          the previous velocity is kept in FP64)
 *   out[5] number of nodes with non-finite populations
 *   out[6] max |u|                     out[7] kinetic energy sum rho |u|^2 / 2
 * Returns CLBM_EUNSTABLE (after filling out) if out[5] > 0. */
clbm_status clbm_reduce(clbm_lattice *h, double out[8], void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * reductions of clbm_reduce with no allocation, no host synchronization and
 * no host copy: the eight values are written to out_dev (8 doubles of device
 * memory owned by the caller) on `stream`, asynchronously; non-finite
 * populations show in out_dev[5] (the call cannot return CLBM_EUNSTABLE).
 * The residual uses and updates the same FP64 snapshot as clbm_reduce, and
 * whether a previous velocity exists is decided when the call is made.  The
 * block partials go to a static scratch array of the library (1024 blocks of
 * 10 doubles plus 10, one copy per GPU, held until the process ends); a
 * lattice needing more blocks is refused with EINVAL (none does: lattices
 * are reduced with at most 1024 blocks).  Every call on one GPU shares that
 * scratch, so calls that overlap on one GPU (two streams, or two threads)
 * race; serialize them. */
clbm_status clbm_reduce_noalloc(clbm_lattice *h, double *out_dev, void *stream);

/* Index (0 = pop_a, 1 = pop_b; always 0 in the in-place form) of the buffer
 * holding the current state, and the number of steps taken since the last
 * init.  Either output may be NULL. */
clbm_status clbm_state(clbm_lattice *h, int *buffer_index, int64_t *steps_done);

/* Launch configuration of the stream-collide kernel (results do not depend
 * on it; only speed does). */
typedef struct {
    int32_t bx, by;      /* threads per block along x and y: bx*by at most 512 (FP32/FP16
                            storage) or 256 (FP64); whole 64-lane waves run fastest (row
                            layout: bx a multiple of 64 takes the fast kernel, other widths a
                            kernel that applies the full wall rule on every lane) */
    int32_t xcd_remap;   /* 1: workgroup b takes tile (b mod 8)*(B/8) + b/8, so each of the
                            eight XCDs sweeps a contiguous slab of the lattice (both launch
                            forms) */
    int32_t nt_loads;    /* 1: non-temporal hint on population loads (one-step launch) */
    int32_t nt_stores;   /* 1: non-temporal hint on population stores (both launch forms) */
    int32_t fuse_steps;  /* time steps per launch: 1, or 2 (temporal blocking: a workgroup
                            computes the first step on a 64 x fuse_rows patch of columns plus
                            its one-node ring, keeps it on chip and writes the second step of
                            the inner 62 x (fuse_rows - 2) columns, marching along z; the
                            result equals two one-step launches).  clbm_step runs an odd
                            remainder as one one-step launch.  Either layout (not the
                            one-buffer form) */
    int32_t fuse_rows;   /* rows of a two-step workgroup, ring included: 8, 16 (not FP64), or
                            12 (FP32; planes layout: the next plane's loads go straight to LDS) */
    int32_t fuse_planes; /* output z planes per two-step workgroup, >= 1 */
    int32_t reserved;    /* must be 0 */
} clbm_launch;

clbm_status clbm_set_launch(clbm_lattice *h, const clbm_launch *cfg);
clbm_status clbm_get_launch(clbm_lattice *h, clbm_launch *cfg);

/* Shorthands for the block shape alone. */
clbm_status clbm_set_block(clbm_lattice *h, int32_t bx, int32_t by);
clbm_status clbm_get_block(clbm_lattice *h, int32_t *bx, int32_t *by);

/* Time one step per launch over block widths 64..512 (multiples of 64, up
 * to the lattice width rounded up to 64), 1, 2 or 4 rows per block, both tile
 * orders and both cache hints, and two steps per launch over patch heights 8
 * and 16 (8 only for FP64), z chunks of 16 and 32 planes, both patch orders
 * and both store hints (not for the single-relaxation-time model), plus the
 * two-step configuration in place if fuse_steps = 2, on the current state; keep the fastest and report it and its
 * time per step in ms (either output may be NULL).  The trial launches read
 * the current buffer and write the other one, so the state is unchanged; the
 * call synchronizes its stream.  Refused (EINVAL) for the one-buffer form,
 * whose steps overwrite the state, and before an init call (ESTATE). */
clbm_status clbm_autotune(clbm_lattice *h, void *stream, clbm_launch *best, double *best_ms);

/* Release the handle and the library's own memory (never the caller's
 * buffers or flags).  NULL is accepted.  Work already queued on a stream must
 * not be outstanding. */
clbm_status clbm_destroy(clbm_lattice *h);

/* Message for the last failing call on this thread ("" if none). */
const char *clbm_last_error(void);

/* ------------------------------------------------------------------------
 * Batches: many independent lattices (uneven sizes, Re, n, lids, forces)
 * advanced together, one launch per time step whose workgroups stride over
 * the tiles of all instances (a persistent grid of a few workgroups per CU,
 * or up to one tile per wave: blocks_per_cu); k steps are captured into a
 * hipGraph and replayed.  All instances share the storage type and the
 * layout (EINVAL otherwise).  Instance i occupies clbm_buffer_size bytes of
 * its params, rounded up to 256, at a 256-byte-aligned offset of each pool, in
 * instance order.  Row layout: each wave takes (instance, z layer, k passes
 * of 64 consecutive nodes) items, or (instance, row, run of 64 x) items, the
 * short tails (at most 32 values) of two inner rows of an instance sharing
 * one wave, a 32-lane half each; planes: each workgroup takes (instance,
 * z layer, run of bx nodes) tiles.
 * Row-layout instances hold less than 2 GiB of state each.
 * ------------------------------------------------------------------------ */
typedef struct clbm_batch clbm_batch;

typedef struct {
    int32_t bx, by;            /* threads per workgroup, a multiple of 64, <= 512 (<= 256 for FP64;
                                  default: that maximum);
                                  planes: the tile is bx consecutive nodes of one z layer (x fastest);
                                  rows: bx / 64 waves, each on its own items; by must be 1 */
    int32_t blocks_per_cu;     /* grid = blocks_per_cu x CUs workgroups (1..1024), at most one item
                                  per wave; the workgroups stride over the item list (default 1024:
                                  one item per wave up to 1024 x CUs x bx/64 items, 2^21 on 256 CUs
                                  at bx 512, so that the dispatcher balances the uneven item costs) */
    int32_t graph_steps;       /* steps per captured graph (0: plain launches) */
    int32_t nt_stores;         /* 1: non-temporal (streaming) stores, 0: plain stores (default: the
                                  short runs of small lattices leave partial cache lines, which plain
                                  stores let the cache merge) */
    int32_t passes;            /* row layout: 0 = each wave item is one row's run of 64 x, or the short
                                  tails of two inner rows (default);
                                  k > 0 = each item is k passes of 64 consecutive nodes of a z layer
                                  (rows packed into whole waves: fewer idle lanes for narrow lattices,
                                  per-lane row addressing); planes layout: must be 0 */
} clbm_batch_config;

/* Bytes each of the two pools must hold for these instances. */
clbm_status clbm_batch_size(const clbm_params *inst, int32_t count, size_t *bytes_each);

/* Create a batch of independent instances, each a problem statement as for
 * clbm_create (Sec. 4: dimensions, K and n of Eq. 5, lid or force), over two
 * caller-owned pools of bytes_each >= clbm_batch_size bytes (256-byte
 * aligned device memory).  Validates every instance (EINVAL, with the
 * instance index in the message); allocates the instance descriptors, the
 * tile table and reduction scratch; reads the tuned launch configuration
 * from tune_cache_path (nullable) when it holds an entry for exactly this set
 * of instances. */
clbm_status clbm_batch_create(const clbm_params *inst, int32_t count, void *pool_a, void *pool_b,
                              size_t bytes_each, const char *tune_cache_path, clbm_batch **out);

/* Rest state for every instance, or caller populations for instance i, as
 * clbm_init_rest and clbm_init_populations (on_device as there). */
clbm_status clbm_batch_init_rest(clbm_batch *b, void *stream);
clbm_status clbm_batch_init_populations(clbm_batch *b, int32_t i, const double *f0, int on_device, void *stream);

/* Advance every instance by nsteps (the time step of clbm_step, Sec. 3):
 * one launch per step over all tiles, replayed from captured
 * graphs in chunks of graph_steps.  Asynchronous; the first call for a
 * graph length and buffer parity instantiates its graph. */
clbm_status clbm_batch_step(clbm_batch *b, int64_t nsteps, void *stream);

/* Reference path with the same results: one single-lattice launch per
 * instance per step. */
clbm_status clbm_batch_step_each(clbm_batch *b, int64_t nsteps, void *stream);

/* Outputs of instance i, as clbm_macroscopic and clbm_populations. */
clbm_status clbm_batch_macroscopic(clbm_batch *b, int32_t i, void *rho_dev, void *u_dev, int32_t out_prec,
                                   void *stream);
clbm_status clbm_batch_populations(clbm_batch *b, int32_t i, double *f_dev, void *stream);

/* FP64 reductions of clbm_reduce for every instance: out[8*i + k]
 * (synchronizes; EUNSTABLE if any instance holds non-finite values). */
clbm_status clbm_batch_reduce(clbm_batch *b, double *out, void *stream);

/* Time candidate launch configurations (bx, blocks_per_cu, nt_stores) on the
 * current state (each trial writes only the spare pool, so the state is
 * unchanged), keep the fastest, and append it to the tune cache when one was
 * given.  `best` (nullable)
 * receives it; `best_ms` (nullable) its time per step. */
clbm_status clbm_batch_autotune(clbm_batch *b, void *stream, clbm_batch_config *best, double *best_ms);

clbm_status clbm_batch_set_config(clbm_batch *b, const clbm_batch_config *cfg);
clbm_status clbm_batch_get_config(clbm_batch *b, clbm_batch_config *cfg);
clbm_status clbm_batch_state(clbm_batch *b, int *buffer_index, int64_t *steps_done);
clbm_status clbm_batch_destroy(clbm_batch *b);

/* Measurement utility: copy `bytes` (a multiple of 16) from src to dst
 * (device memory, 16-byte aligned, not overlapping) with a plain streaming
 * kernel.  Gives the achievable HBM bandwidth of the device and the
 * calibration of hardware byte counters against a kernel of known traffic.
 * Asynchronous on `stream`. */
clbm_status clbm_copy_probe(const void *src, void *dst, size_t bytes, void *stream);

/* Test utility: the rounding of FP32 values to the FP16 state on its own.
 * in: n floats, seeds: n random words (stochastic mode), out: n IEEE half
 * bit patterns; device memory; mode: clbm_f16_rounding.  Asynchronous.
 * The step kernels apply exactly this conversion to every stored collision
 * result, with seeds from the hash described at clbm_f16_rounding. */
clbm_status clbm_f16_round(const float *in, const uint32_t *seeds, uint16_t *out, int64_t n, int32_t mode,
                           void *stream);

/* Version string and the lattice tables compiled into the kernels (for
 * tests): e[3*alpha + c], opposite[alpha], w[alpha]. */
const char *clbm_version(void);
clbm_status clbm_lattice_tables(int32_t *e, int32_t *opposite, double *w);

#ifdef __cplusplus
}
#endif
#endif /* CLBM_H */
