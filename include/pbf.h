/*
 * libpbf — adaptive position-based fluids (APBF) time steps on one AMD
 * Instinct MI355X (gfx950), behind a plain C ABI.
 *
 * Method: Koester & Krueger, "Adaptive Position-Based Fluids" (IJCGA 6(3),
 * 2016).  One step follows the simulation loop of Section 5 (Fig. 7):
 *   1. apply external forces and predict positions for every particle,
 *   2. find neighbours of every particle (uniform grid built by a counting
 *      sort of cell keys, particles reordered by cell, Section 6),
 *   3. for iterations l = 1..N_l, for the active set P_l (Eqs. 9-10):
 *      lambda_i (Eqs. 4-6), Delta p_i with contact response (Eq. 7),
 *      position update; finished particles (Eq. 11) keep their position,
 *   4. update velocity and position of every particle.
 * Each particle's level N_i (Eq. 8), which is also its iteration count,
 * comes from an explicit array, a uniform value, or the distance to a
 * camera (DTC adaption model, Section 4.1).
 *
 * Readings taken where the paper leaves details open (identical in the FP64
 * oracle that the test suite checks this library against):
 *   - density kernel: poly6 W = 315/(64 pi h^9) (h^2 - r^2)^3, self term
 *     included; gradient: spiky, -45/(pi h^6) (h - r)^2 d/r;
 *   - uniform mass m: lambda_i = -C_i / ((m/rho0^2)(|sum_j gW|^2 +
 *     sum_j |gW|^2) + eps), C_i = rho_i/rho0 - 1;
 *     Delta p_i = (1/rho0) sum_j (lambda_i + lambda_j) gW_ij;
 *   - neighbour sets N_i = { j != i : |x*_i - x*_j|^2 < h^2 } are found once
 *     per step from the predicted positions and kept for every iteration;
 *   - a finished particle keeps its last lambda, and active neighbours use it;
 *   - contacts are the box walls: positions are clamped to [lo, hi] after
 *     prediction and after every update; optional solid obstacles add the
 *     contact finding, pre-stabilisation and contact response of Fig. 7
 *     (pbf_batch_set_obstacles);
 *   - optional force-based cohesion (pbf_batch_set_cohesion);
 *   - iteration k = 0..n_max-1 corrects particle i only while k < N_i.
 *
 * Conventions (every entry point):
 *   - returns a pbf_status; nothing aborts or exits;
 *   - argument checks run on the host before any HIP call; a failed check
 *     leaves the context unchanged;
 *   - positions/velocities cross the boundary as float[3*n], x/y/z
 *     interleaved, in particle-ID order (batch: scenes concatenated in
 *     scene order, particle IDs local to each scene);
 *   - "on_device" flags say whether a caller pointer is device memory
 *     (hipMalloc / torch) or host memory; caller buffers are borrowed only
 *     for the duration of the call; the library owns all its device state;
 *   - one context = one HIP stream; work is enqueued asynchronously on it;
 *     calls that return data to host memory synchronise that stream;
 *   - faults detected on the device (neighbour capacity, non-finite
 *     positions) are latched and reported by the next synchronising call;
 *   - a context is not thread-safe; distinct contexts are independent.
 */
#ifndef PBF_H
#define PBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbf_ctx pbf_ctx; /* opaque; owns every device buffer it uses */

typedef enum {
    PBF_OK = 0,
    PBF_ERR_INVALID_ARG = -1,   /* bad argument or parameter; nothing changed */
    PBF_ERR_NONFINITE = -2,     /* NaN/Inf in inputs, or positions became non-finite */
    PBF_ERR_OUT_OF_MEMORY = -3, /* device or host allocation failed */
    PBF_ERR_DEVICE = -4,        /* a HIP call failed (message in pbf_last_error) */
    PBF_ERR_CAPACITY = -5       /* a particle exceeded the neighbour capacity, a grid
                                   cell held more than PBF_MAX_CELL particles, or a
                                   tile too dense for on-chip staging held more than
                                   1024 particles in six cells of a grid row */
} pbf_status;

#define PBF_MAX_ITERS 32          /* largest iteration count / level */
#define PBF_MAX_CELL 4096         /* largest particle count of one grid cell */
#define PBF_DEFAULT_NEIGHBOURS 96 /* per-particle neighbour capacity if 0 is given */
#define PBF_MAX_SCENES 65535

/* LOD (level) modes, Section 4.1 / Eq. 8 */
#define PBF_LOD_UNIFORM 0  /* N_i = n_max for every particle: plain PBF */
#define PBF_LOD_EXPLICIT 1 /* N_i from a caller array (particle-ID order) */
#define PBF_LOD_DTC 2      /* distance to camera, recomputed each step from the
                              positions at the start of the step */
#define PBF_LOD_DTVS 3     /* distance to the visible surface along the camera
                              ray, recomputed each step likewise */
#define PBF_MAX_SPLAT 16   /* largest splat radius in pixels (DTVS) */
#define PBF_MAX_IMAGE 8192 /* largest DTVS image side in pixels */
#define PBF_MAX_CAMERAS 4  /* DTC: `camera` and up to 3 further cameras */

/* pbf_params.flags */
#define PBF_FLAG_UNILATERAL 1u /* unilateral density constraint C_i = max(rho_i/rho0 - 1, 0):
                                  resists compression only (the variant named in the
                                  paper's evaluation setup, Section 7) */

/* Per-scene parameters.  All lengths in the same unit as positions. */
typedef struct pbf_params {
    int32_t n;              /* particles, >= 0 */
    int32_t n_min, n_max;   /* level range, 1 <= n_min <= n_max <= PBF_MAX_ITERS */
    int32_t grid_dims[3];   /* cells per axis (edge h from box_lo); 0 => ceil(extent/h) */
    float box_lo[3], box_hi[3]; /* walls; box_hi >= box_lo per axis */
    float h;                /* smoothing length = cell edge, > 0 */
    float rho0;             /* rest density, > 0 */
    float mass;             /* particle mass, > 0 */
    float eps;              /* relaxation added to lambda's denominator, >= 0 */
    float dt;               /* time step, > 0 */
    float gravity[3];       /* external acceleration */
    int32_t max_neighbours; /* neighbour capacity; 0 => PBF_DEFAULT_NEIGHBOURS; the
                               context uses the largest value over its scenes */
    uint32_t flags;         /* PBF_FLAG_* bits; others must be 0 */
} pbf_params;

/* Level source (Section 4.1).  A distance d is mapped to a level by
 * t = clamp((d - d_near) / (d_far - d_near), 0, 1),
 * N = clamp(n_max - floor(t (n_max - n_min + 1)), n_min, n_max): near
 * particles iterate n_max times, far ones n_min.  Both distance models are
 * evaluated in float32 with one rounding per operation.
 *
 * DTC: d = |x - camera|.
 *
 * DTVS: the camera is a pinhole at `camera` with unit vectors `forward` and
 * `up` (right = forward x up), `focal` pixels per unit of depth and a
 * width x height image.  With q = x - camera, z = q.forward: a particle with
 * z > splat projects to pixel (floor(focal (q.right) / z + width / 2),
 * floor(focal (q.up) / z + height / 2)) and is splatted as a square of
 * (2 r + 1)^2 pixels, r = min(ceil(focal splat / z), PBF_MAX_SPLAT), keeping
 * per pixel the smallest |q|.  d = |q| minus that depth at the particle's
 * own pixel (the particles seen there are the surface); particles behind
 * the camera or outside the image get the lowest level.
 *
 * Several cameras (DTC, Section 4.1): each of `camera` and the
 * n_extra_cameras further ones maps its own distance through its own range;
 * the particle takes the highest of these levels.  Automatic range
 * (auto_range = 1, DTC and DTVS): every step, each camera's d_near and d_far
 * are the smallest and largest of its distances over the scene's particles
 * at the start of the step (DTVS: over the particles seen; [0, 0] when none
 * is); the given ranges are then ignored.  A t that is not a number (a range
 * of zero width) counts as 0. */
typedef struct pbf_lod_desc {
    int32_t mode;            /* PBF_LOD_* */
    const uint8_t *levels;   /* EXPLICIT: n levels in [n_min, n_max], particle-ID order */
    int32_t levels_on_device;
    float camera[3];         /* DTC, DTVS */
    float d_near, d_far;     /* DTC, DTVS: d_far > d_near */
    float forward[3], up[3]; /* DTVS: camera frame, unit length, orthogonal */
    float focal;             /* DTVS: > 0 */
    int32_t width, height;   /* DTVS: image in pixels, 1 .. PBF_MAX_IMAGE */
    float splat;             /* DTVS: splat radius of a particle, >= 0 */
    int32_t n_extra_cameras; /* DTC: 0 .. PBF_MAX_CAMERAS - 1 */
    float extra_camera[PBF_MAX_CAMERAS - 1][3];
    float extra_range[PBF_MAX_CAMERAS - 1][2]; /* d_near, d_far of each (d_far > d_near) */
    int32_t auto_range;      /* DTC, DTVS: 0 or 1 */
} pbf_lod_desc;

/* Solid obstacles (signed-distance shapes, Section 6) and pre-stabilisation
 * (Section 4.3, Fig. 6; the contact lines of Fig. 7).  Each step:
 *   - contact finding, from the predicted positions x* of every particle:
 *     obstacle o is a contact of particle i when the obstacle grown by h
 *     holds x*_i (sphere: the ball of radius r + h; cone: its slant moved
 *     out by h; box: the box grown by h per axis), decided in float32;
 *   - pre-stabilisation, stab_iters times: a particle with N_i < stab_s lying
 *     inside a contact obstacle has x*_i moved to the closest point of the
 *     obstacle's surface (then clamped to the walls), and x_i moved by the
 *     same amount, so that the push-out adds no velocity;
 *   - contact response in every update of an active particle:
 *     x*_i + Delta p_i is moved out of each contact obstacle it lies in, in
 *     obstacle order, before the wall clamp.
 * Closest surface points: sphere, radially from the centre (straight up from
 * the centre itself); box, through the face of least penetration (first axis
 * on ties); cone (apex H above the centre, radius R at the centre's height,
 * the slant continued below that circle: a cone standing on the floor, which
 * fluid never leaves through its base), in the plane of the axis and the
 * point, to the foot of the perpendicular on the slant line (on the axis the
 * plane through +x). */
#define PBF_MAX_OBSTACLES 4
#define PBF_OBSTACLE_SPHERE 1 /* centre; a[0] radius */
#define PBF_OBSTACLE_CONE 2   /* centre of the base circle; a[0] base radius, a[1] height (+y) */
#define PBF_OBSTACLE_BOX 3    /* centre; a[0..2] half extents (axis-aligned) */

typedef struct pbf_obstacle {
    int32_t kind;      /* PBF_OBSTACLE_* */
    float centre[3];
    float a[3];        /* sizes as listed for the kind, > 0 where used */
} pbf_obstacle;

typedef struct pbf_contact_desc {
    int32_t count;                              /* 0..PBF_MAX_OBSTACLES */
    pbf_obstacle obstacles[PBF_MAX_OBSTACLES];  /* first `count` used */
    int32_t stab_iters;                         /* pre-stabilisation iterations, 0..PBF_MAX_ITERS */
    int32_t stab_set;                           /* S: particles with N_i < S are pre-stabilised,
                                                   1 (none) .. the scene's n_max */
} pbf_contact_desc;

/* Statistics of the most recent step (read with pbf_stats; synchronises). */
typedef struct pbf_step_stats {
    int32_t n_iters;                     /* loop bound: largest n_max over scenes */
    int64_t active[PBF_MAX_ITERS];       /* |P_k| for k = 0..n_iters-1 */
    int64_t particle_iterations;         /* sum_i N_i = sum_k |P_k| */
    int64_t neighbour_pairs;             /* sum_i |N_i| */
    int32_t max_neighbours;              /* largest |N_i| */
    int64_t total_particle_iterations;   /* sum over every step since create or
                                            pbf_set_state, counted on the device */
    int64_t total_steps;                 /* steps counted in the same span */
    int32_t max_stage;                   /* largest neighbourhood staged by one tile
                                            (particles in its 6^3 cells) */
    int32_t tiles_unstaged;              /* tiles whose neighbourhood exceeded the
                                            on-chip stage and was read from HBM */
} pbf_step_stats;

/* ---------------- core entry points ---------------- */

/* One scene.  x0, v0: float[3n] in ID order, copied.  hip_stream: a
 * hipStream_t (NULL => the library creates its own non-blocking stream).
 * The new context starts with PBF_LOD_UNIFORM. */
pbf_status pbf_create(const pbf_params *params, const float *x0, const float *v0,
                      int32_t inputs_on_device, void *hip_stream, pbf_ctx **out);

/* Set the level source (scene 0 of a context); applies from the next step.
 * EXPLICIT levels are copied. */
pbf_status pbf_set_lod(pbf_ctx *ctx, const pbf_lod_desc *lod);

/* Advance every scene of the context by n_steps >= 0 steps; asynchronous. */
pbf_status pbf_step(pbf_ctx *ctx, int32_t n_steps);

/* Positions float[3 * n_total] in ID order (scenes concatenated) into a
 * caller buffer.  Host buffers synchronise the stream first. */
pbf_status pbf_read_positions(pbf_ctx *ctx, float *out, int32_t out_on_device);

/* Velocities, same layout and rules as pbf_read_positions. */
pbf_status pbf_read_velocities(pbf_ctx *ctx, float *out, int32_t out_on_device);

/* Wait for the stream; report latched device faults (CAPACITY, NONFINITE). */
pbf_status pbf_sync(pbf_ctx *ctx);

void pbf_destroy(pbf_ctx *ctx);
const char *pbf_last_error(const pbf_ctx *ctx);  /* never NULL */
const char *pbf_status_string(pbf_status s);     /* never NULL */

/* ---------------- batched scenes ---------------- */

/* n_scenes independent scenes in one context, advanced together: every
 * kernel of a step covers all scenes at once (one launch per pass).
 * params: n_scenes entries; x0, v0: float[3 * sum n] with scenes
 * concatenated in order. */
pbf_status pbf_batch_create(int32_t n_scenes, const pbf_params *params, const float *x0,
                            const float *v0, int32_t inputs_on_device, void *hip_stream,
                            pbf_ctx **out);
pbf_status pbf_batch_set_lod(pbf_ctx *ctx, int32_t scene, const pbf_lod_desc *lod);
/* Obstacles and pre-stabilisation of one scene (0-based), copied; applies
 * from the next step.  count = 0 and stab_iters = 0 remove them.  Invalid
 * descriptors (kind, non-finite or non-positive sizes, counts out of range)
 * give PBF_ERR_INVALID_ARG and change nothing.  A context with obstacles in
 * any scene adds one per-particle pass after the neighbour search and keeps
 * a byte per particle (the contact set of the last step). */
pbf_status pbf_batch_set_obstacles(pbf_ctx *ctx, int32_t scene, const pbf_contact_desc *desc);
/* Force-based cohesion of one scene (0-based): the option the paper names
 * beside the unilateral density constraint at the end of Section 7's setup,
 * by reference to the works it cites there.  Reading (the same in the test
 * suite's FP64 oracle): particle i gets the acceleration
 *   a_i = -gamma m sum_{j in N_i} C(|x_i - x_j|) (x_i - x_j) / |x_i - x_j|,
 *   C(r) = 32/(pi h^9) (h - r)^3 r^3          for h/2 < r <= h,
 *          32/(pi h^9) (2 (h - r)^3 r^3 - h^6/64) for 0 < r <= h/2, else 0
 * (the cohesion kernel of Akinci et al. 2013), an external force of Fig. 7's
 * first loop evaluated at the positions x at the start of the step over the
 * neighbour sets N_i found at the predicted positions; once the sets are
 * known it is applied to the prediction, x*_i += dt^2 a_i, clamped into the
 * box (what adding dt a_i to v_i in the first loop gives).  gamma >= 0 and
 * finite (0 removes it), in units of m^3 / (kg s^2) with m the particle mass;
 * applies from the next step.  Anything else, or a bad scene index, gives
 * PBF_ERR_INVALID_ARG and changes nothing.  A context with cohesion in any
 * scene adds one tile pass after the neighbour search; rollouts reject such
 * contexts (the reverse mode does not differentiate it). */
pbf_status pbf_batch_set_cohesion(pbf_ctx *ctx, int32_t scene, float gamma);
/* Positions of one scene, float[3 * n_scene] in its ID order. */
pbf_status pbf_batch_read_positions(pbf_ctx *ctx, int32_t scene, float *out,
                                    int32_t out_on_device);
pbf_status pbf_get_counts(const pbf_ctx *ctx, int32_t *n_scenes, int64_t *n_total);

/* ---------------- device memory ---------------- */

/* Bound on the device memory the library holds, for callers that share the
 * GPU and must cap it: once set, any device allocation the library would
 * make beyond `bytes` in total (all contexts of the process) fails, and the
 * entry point that needed it returns PBF_ERR_OUT_OF_MEMORY with the
 * context unchanged (pbf_create and pbf_batch_create return no context).
 * 0 removes the bound (the default); memory already held is unaffected.
 * PBF_ERR_INVALID_ARG if bytes < 0.  Process-wide; safe to call from any
 * thread. */
pbf_status pbf_set_memory_limit(int64_t bytes);

/* Device bytes held by the library now, all contexts of the process. */
int64_t pbf_device_bytes(void);

/* ---------------- execution control ---------------- */

/* enable != 0: each step is captured once into a hipGraph (one per buffer
 * parity) and replayed; 0: kernels are launched one by one. */
pbf_status pbf_set_graph(pbf_ctx *ctx, int32_t enable);

/* Launch shape of one kernel class (threads per block, a multiple of 64 in
 * [64, 1024], at most 512 for the neighbour, lambda and update tile kernels;
 * some classes have a fixed shape and accept only their default); 0 restores
 * the default.  Kernel classes are numbered
 * 0..pbf_kernel_count()-1 and named by pbf_kernel_name(). */
int32_t pbf_kernel_count(void);
const char *pbf_kernel_name(int32_t kernel);  /* NULL if out of range */
pbf_status pbf_set_block_size(pbf_ctx *ctx, int32_t kernel, int32_t threads);

/* Per-kernel timing with HIP events recorded on the context stream around
 * every launch (direct launches only; graph mode is switched off while
 * enabled).  pbf_profile_read synchronises and returns, per kernel class,
 * total milliseconds and launch counts accumulated since enabling. */
pbf_status pbf_profile_enable(pbf_ctx *ctx, int32_t enable);
pbf_status pbf_profile_read(pbf_ctx *ctx, double *total_ms, int64_t *launches, int32_t count);

/* ---------------- state, statistics, debug (ID order, synchronising) --- */

pbf_status pbf_stats(pbf_ctx *ctx, pbf_step_stats *out);
/* Cell key of each particle's predicted position in the last step (key local
 * to its scene's grid: (cz * dims_y + cy) * dims_x + cx). */
pbf_status pbf_debug_keys(pbf_ctx *ctx, uint32_t *keys);
/* Storage order after the last step's counting sort, as particle IDs
 * (batch: global IDs = scene offset + local ID). */
pbf_status pbf_debug_permutation(pbf_ctx *ctx, int32_t *ids);
/* Neighbour sets of the last step: counts[n_total] and, if ids != NULL and
 * cap >= total, ids of each particle's neighbours (global IDs, ascending),
 * particle after particle.  *total receives the number of entries. */
pbf_status pbf_debug_neighbours(pbf_ctx *ctx, int32_t *counts, int32_t *ids, int64_t cap,
                                int64_t *total);
/* Last lambda of every particle (from its last active iteration). */
pbf_status pbf_debug_lambda(pbf_ctx *ctx, float *lambda);
/* Levels N_i used in the last step. */
pbf_status pbf_debug_levels(pbf_ctx *ctx, uint8_t *levels);
/* Contacts found in the last step (bit o set: obstacle o of the particle's
 * scene); zeros where no scene has obstacles. */
pbf_status pbf_debug_contacts(pbf_ctx *ctx, uint8_t *mask);
/* Debug poisoning (enable 0 or 1): from the next step on, every step first
 * fills the float buffers it writes before reading them (the predicted
 * positions, both x* buffers with their lambda lanes, and the free halves of
 * the position and velocity buffers) with quiet NaNs; the scene-index lane
 * of the position buffer gets scene 0, so a stray read yields a NaN position,
 * never an out-of-range scene.  A correct step is bit-identical with and
 * without it; a read of a value the step did not write surfaces as
 * PBF_ERR_NONFINITE from the commit's check or as NaN results.  Integer
 * buffers (indices, codes, tables) are not poisoned, since a stray index
 * would address memory out of bounds.  Changing it drops the captured step
 * graphs.  Costs five fills of n float4 per step. */
pbf_status pbf_debug_poison(pbf_ctx *ctx, int32_t enable);
/* Save / restore the dynamic state (positions and velocities, ID order,
 * host buffers float[3 * n_total] each, plus the step counter).  A restored
 * context continues bit-identically to one that never stopped. */
pbf_status pbf_get_state(pbf_ctx *ctx, float *x, float *v, int64_t *step);
pbf_status pbf_set_state(pbf_ctx *ctx, const float *x, const float *v, int64_t step);

/* ---------------- quality measure ---------------- */

/* Average density, the quality measure of the paper's evaluation (Section 7,
 * Fig. 9): rho_i / rho0 (Eqs. 5-6 with the poly6 kernel, the particle itself
 * included) of every particle of every scene at the positions after the
 * last step, over neighbour sets found afresh at those positions (a counting
 * sort and grid search of their own; the state, the last step's debug views
 * and the running totals are unchanged).  out (host, double[2]): out[0] =
 * mean over all particles, out[1] = maximum.  rho_rel (optional, NULL to
 * skip): float[n_total] in ID order, host memory (on_device = 0) or device
 * memory (1).  Synchronises.  PBF_ERR_INVALID_ARG if no step has run since
 * the context was created or its state set; PBF_ERR_CAPACITY if the fresh
 * search overflows the neighbour or staging capacity.  Its buffers (about
 * the size of one step's neighbour structure) are allocated by the first
 * call and kept until pbf_destroy. */
pbf_status pbf_density(pbf_ctx *ctx, double *out, float *rho_rel, int32_t on_device);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * measure as pbf_density, same arguments, results bit-identical to it, but
 * nothing is allocated.  Its work buffers live in one fixed device array
 * of PBF_STATIC_SCRATCH_BYTES per GPU, part of the library's code object,
 * held from the first use on that GPU until the process ends.  Needs
 * n_total * (2 * nbr_stride + 36) + n_tiles * 1197 bytes plus at most 8 KiB
 * (nbr_stride = neighbour capacity rounded up to 8; n_tiles = tiles of
 * 4x4x4 cells over all scenes); a context that needs more gets
 * PBF_ERR_INVALID_ARG and nothing is enqueued.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (two
 * streams, two threads) race and give wrong results; the library itself
 * orders nothing between them.  The array keeps the last call's contents;
 * each call clears what must start at zero. */
#define PBF_STATIC_SCRATCH_BYTES (64ll << 20)
pbf_status pbf_density_noalloc(pbf_ctx *ctx, double *out, float *rho_rel, int32_t on_device);

/* ---------------- differentiable rollout (training form) ---------------- */

/* Advance every scene by n_steps >= 1 steps like pbf_step, keeping a device
 * copy of the state (x, v) before steps 0, ckpt_every, 2 ckpt_every, ...
 * (ckpt_every >= 1), for a later pbf_rollout_backward.  Direct launches. */
pbf_status pbf_rollout_forward(pbf_ctx *ctx, int32_t n_steps, int32_t ckpt_every);

/* Reverse mode of the last pbf_rollout_forward (no step or state change in
 * between): dl_dx, dl_dv = dL/dx_T and dL/dv_T of the final state, float[3
 * n_total] in ID order; dl_dx0, dl_dv0 receive dL/dx_0 and dL/dv_0 of the
 * state at the start of the rollout.  Each step is differentiated with its
 * levels, neighbour sets and wall contacts held fixed (the adjoint of
 * Eqs. 4-7 and of Fig. 7's prediction and update); every segment between
 * checkpoints is recomputed from its checkpoint.  All four buffers are host
 * memory (on_device = 0, synchronises) or device memory (1).  Scenes with
 * obstacles or the unilateral constraint are not differentiated
 * (pbf_rollout_forward gives PBF_ERR_INVALID_ARG).  The context is left at the final state of the rollout, stored in ID order (after an
 * error its state is unspecified).  The checkpoints and the reverse pass's
 * work buffers (per recorded step: n (K+1) 16 B of positions plus the
 * neighbour codes) stay allocated in the context for the next call of the
 * same shape, until pbf_destroy. */
pbf_status pbf_rollout_backward(pbf_ctx *ctx, const float *dl_dx, const float *dl_dv,
                                float *dl_dx0, float *dl_dv0, int32_t on_device);

#ifdef __cplusplus
}
#endif
#endif /* PBF_H */
