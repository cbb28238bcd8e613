/*
 * mr.h -- C ABI of the multiresolution block-octree hot path on one MI355X.
 *
 * Method: Gillis & van Rees, "MURPHY -- a scalable multiresolution framework
 * for scientific computing on 3D block-structured collocated grids"
 * (arXiv 2112.07537).  A periodic unit cube is covered by a 2:1-balanced
 * octree of cubic blocks of nb^3 points; a scalar phi obeys
 * d(phi)/dt + div(u phi) = 0 (transport problem of section 5, divergence-free
 * u).  Ghost points across resolution jumps, block refinement / coarsening and
 * the refinement criterion all use interpolating wavelets N.Nt with
 * N in {2,4,6}, Nt in {0,2} (section 2, filter tables of the supplementary
 * filter-bank section).
 *
 * Conventions
 *  - Every call returns an mr_status; MR_OK is 0, errors are negative.  On an
 *    error, mr_last_error() returns a thread-local message.  Invalid
 *    arguments give MR_EINVAL and change no state.
 *  - Geometry: block (L, i, j, k) has spacing h_L = 2^-L / nb; its local point
 *    (x, y, z) sits at ((i*nb + x), (j*nb + y), (k*nb + z)) * h_L (node-based,
 *    left-aligned).  Field data are block-major: block b occupies nb^3
 *    consecutive values with x fastest, then y, then z.  Blocks are ordered
 *    by Morton key of (L, i, j, k); the order changes at every adaptation.
 *  - Precision: bulk arrays are FP64 (MR_F64) or FP32 (MR_F32); the detail
 *    transform, its norms, threshold comparisons and moment sums are FP64.
 *  - Host pointers passed in are caller-owned and only read/written during
 *    the call.  Device memory is owned by the library (hipMalloc) and freed
 *    by mr_grid_destroy, except the field buffers when the caller passes a
 *    pool to mr_grid_create (they are then slices of that caller-owned
 *    pool, never freed or grown by the library).
 *  - Streams: device work is issued on the hipStream_t given at creation;
 *    with NULL the library creates a private non-blocking stream.  mr_ghost,
 *    mr_rk3_step and mr_details with on_device = 1 are asynchronous; every
 *    other call synchronises the stream.
 *  - A grid handle is not thread-safe.
 */
#ifndef MR_H
#define MR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mr_grid mr_grid; /* opaque, owned by the library */

typedef enum {
  MR_OK = 0,
  MR_EINVAL = -1,     /* invalid argument or configuration                */
  MR_ENOMEM = -2,     /* device or host allocation failed                 */
  MR_ECAPACITY = -3,  /* block capacity (max_blocks) would be exceeded    */
  MR_EHIP = -4,       /* a HIP runtime call failed                        */
  MR_ESTATE = -5,     /* call not valid in the grid's current state       */
  MR_ENONFINITE = -6  /* a detail norm came out NaN or infinite           */
} mr_status;

typedef enum { MR_F64 = 0, MR_F32 = 1 } mr_prec;

/* Grid configuration (section 2.2 and the adaptation supplement). */
typedef struct {
  int32_t nb;          /* points per block edge: 8, 16 or 24.  The samples
                          of a ghost reconstruction must stay within half a
                          block around the block: nb = 8 takes N = 2 only,
                          nb = 16 takes N <= 4, nb = 24 every wavelet
                          (else MR_EINVAL at creation)                      */
  int32_t wavelet_N;   /* interpolation order N: 2, 4 or 6                  */
  int32_t wavelet_Nt;  /* vanishing moments Nt: 0 (Donoho) or 2 (lifted)    */
  int32_t fd_order;    /* right-hand side: 2, 4 or 6 = central finite
                          differences of that order on -(u . grad) phi
                          (or on the Laplacian, MR_VEL_DIFFUSION);
                          3 or 5 = the conservative CONS-3 / CONS-5
                          fixed-weight WENO fluxes of the finite-difference
                          supplement (f^+ / f^- by the velocity's sign)     */
  int32_t level_min;   /* 0 <= level_min <= level_max <= 12                 */
  int32_t level_max;
  int32_t prec;        /* mr_prec of field arrays                           */
  int32_t detail_ext;  /* 1: criterion includes the extension band of the
                          "coarse region extension" column of Table 3 taken
                          in same-level neighbours; 0: block interior only  */
  int32_t n_fields;    /* scalar fields carried by the grid (>= 1)          */
  int32_t exec_mode;   /* 0: batched launches (default); 1: plain, one
                          launch per block per operation; 2: batched with
                          the whole RK3 step captured in a hipGraph         */
  double eps_refine;   /* refine if ||gamma||_inf >= eps_refine (absolute)  */
  double eps_coarsen;  /* coarsen if all 8 siblings <= eps_coarsen          */
  int64_t max_blocks;  /* capacity of the block pool                        */
} mr_config;

/* Velocity fields; each component does not depend on its own coordinate,
 * so the advective and conservative forms coincide. */
enum { MR_VEL_CONST = 0,    /* u = (p0, p1, p2)                             */
       MR_VEL_ROTATING = 1, /* u = (-(y - p1), x - p0, p2)                  */
       MR_VEL_SHEAR = 2,    /* u = (sin 2pi z, sin 2pi x, sin 2pi y)        */
       MR_VEL_DIFFUSION = 3 /* not a velocity: the right-hand side is
                               p0 * laplacian(phi) with central second
                               differences of order fd_order (2 = DIFF-2,
                               4 = DIFF-4, 6) of the finite-difference
                               supplement; fd_order 3 / 5 give MR_EINVAL;
                               mr_cfl_dt gives cfl h^2 / (6 p0)            */
};
typedef struct {
  int32_t kind;
  int32_t reserved;
  double p[8];
} mr_velocity;

/* Analytic initial conditions (evaluated in FP64). */
enum { MR_IC_GAUSS_SUM = 0,  /* n terms, params[5*g..5*g+4] = cx, cy, cz,
                                sigma, a: a*exp(-|x-c|^2/sigma^2) with the
                                minimum-image periodic distance              */
       MR_IC_TANH_SHELL = 1 }; /* params = ax, ay, az, w:
                                0.5*(1 - tanh(d/w)), d = (rho-1)*min(a),
                                rho = |(x - 1/2)/a| (component-wise)         */
typedef struct {
  int32_t kind;
  int32_t n;
  const double* params;
} mr_ic;

typedef struct {
  int32_t iters;      /* adaptation iterations that changed the tree     */
  int32_t refined;    /* blocks refined (each into 8)                     */
  int32_t coarsened;  /* sibling sets coarsened (each 8 into 1)           */
  int32_t in_band;    /* blocks whose norm is within 1e-4 relative of a
                         threshold at the last flag evaluation            */
  int64_t n_blocks;   /* leaves after adaptation                          */
} mr_adapt_stats;

/* Launch-shape knobs of the ghost kernels (no effect on results beyond
 * the rounding order of restriction tiles): the LDS budget in bytes that a
 * c->f, f->c or substitution work item is tiled to (each item's box is
 * halved along its longest axis until its LDS fits; a launch reserves its
 * largest item's LDS per workgroup, so smaller tiles let more workgroups
 * share a CU), and the substitution workgroup size (256 or 512 threads).
 * 0 in a field of mr_set_tuning keeps the current value.  Budgets must lie
 * in [4096, 65536]. */
typedef struct {
  int32_t lds_refine;     /* c->f items, default 20480                       */
  int32_t lds_restrict;   /* f->c items, default 24576                       */
  int32_t lds_subst;      /* substitution items, default 37888               */
  int32_t subst_threads;  /* 256 or 512, default 512                         */
  int32_t reserved[4];
} mr_tuning;

/* Create a grid (the block-structured grid of section 2.2 with the
 * adaptation parameters of section 2.2.5).  hip_stream: a hipStream_t, or
 * NULL for a private stream owned by the grid.  dev_pool: NULL (the library
 * allocates the field buffers with hipMalloc), or device memory owned by the
 * caller, 256-byte aligned, of pool_bytes >= mr_pool_bytes(cfg) bytes, e.g.
 * a torch uint8 tensor that the caller keeps alive until mr_grid_destroy;
 * the library then takes the fixed-capacity buffers (fields, their
 * adaptation alternates, two work buffers: max_blocks blocks each) from it
 * and never frees it.  Buffers that follow the tree (ghost patches, work
 * lists, metadata, adaptation scratch) are always the library's.  A pool
 * that is misaligned or too small gives MR_EINVAL.  The tree starts as the
 * uniform tree at level_min with zero fields.  Warns (mr_last_error) but
 * succeeds when eps_refine/eps_coarsen <= 2^N (section 2.2.5: flip-flops). */
mr_status mr_grid_create(const mr_config* cfg, void* hip_stream, void* dev_pool,
                         size_t pool_bytes, mr_grid** out);

/* Bytes a caller pool must hold for cfg: (2 n_fields + 2) buffers of
 * max_blocks * nb^3 values of the field precision, each rounded up to a
 * multiple of 256.  No device call. */
mr_status mr_pool_bytes(const mr_config* cfg, size_t* bytes);
mr_status mr_grid_destroy(mr_grid* g);

/* Replace the tree by the n leaves (level[i], ijk[3*i..3*i+2]); the set must
 * tile the unit cube and be 2:1 balanced over the 26-neighbourhood with the
 * periodic wrap, else MR_EINVAL.  Fields are set to zero. */
mr_status mr_set_tree(mr_grid* g, int64_t n, const int32_t* level, const int32_t* ijk);

/* Evaluate the initial condition on every current leaf of field `field`. */
mr_status mr_sample_ic(mr_grid* g, int32_t field, const mr_ic* ic);

/* Initial grid: uniform at level_min, then {sample the IC, criterion,
 * refine only} until stable, then one adaptation (mr_adapt).  */
mr_status mr_init_ic(mr_grid* g, int32_t field, const mr_ic* ic, int32_t max_iter,
                     mr_adapt_stats* stats);

/* Ghost reconstruction of `field` (sections 2.2.2, 2.2.4, 2.3 and the
 * ghosting algorithms Part 1 / Part 2), in this order: ghost patches of
 * every fine block in its coarser regions (zero-detail refinement of the
 * samples as they stand); the substitution of the slab points of every fine
 * block next to a coarser leaf, degree 1, 2 then 3 over the whole level
 * (section 2.3), written into the field; the patches of every coarse block
 * inside its finer regions (restriction of the substituted finer data).
 * Patches are `depth` points deep (0 = the stencil depth: 1 for fd_order
 * 2, 2 for 3 and 4, 3 for 5 and 6).
 * Asynchronous. */
mr_status mr_ghost(mr_grid* g, int32_t field, int32_t depth);

/* Copy blocks [b0, b0+nblk) of `field` with their ghost layer of `depth`
 * points, as filled by the last mr_ghost of that depth, to host memory:
 * (nb+2*depth)^3 values per block in field precision.  Synchronises. */
mr_status mr_ghost_get(mr_grid* g, int32_t field, int32_t depth, int64_t b0,
                       int64_t nblk, void* host, size_t bytes);

/* Block criterion of section 2.2.5: ghost reconstruction, one-level forward
 * transform (x, y, z), per-block max |gamma| (FP64).  norms: n_blocks
 * doubles, host (on_device = 0, synchronises) or device (on_device = 1);
 * with on_device = 1, norms may be NULL: the norms stay in the library's
 * device buffer (asynchronous).  With on_device = 0 a NaN or infinite norm
 * (non-finite field values) returns MR_ENONFINITE after the norms are
 * written; mr_adapt returns the same before changing the tree. */
mr_status mr_details(mr_grid* g, int32_t field, double* norms, int32_t on_device);

/* mr_details without any allocation, for callers that cannot allocate
 * (code under graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same ghost reconstruction and detail pass, with the
 * per-block band maxima in a static device array of 27 * 65536 doubles
 * (one per GPU, resident until the process ends) instead of the grid's
 * buffer, and the n_blocks FP64 norms written to dev_norms (caller-owned
 * device memory).  Asynchronous on the grid's stream.  Grids of more than
 * 65536 blocks give MR_ECAPACITY.  Every call on one GPU shares the static
 * array: calls that overlap on one GPU (two grids' streams, two threads)
 * race and must be ordered by the caller.  Every value the pass reads from
 * the array it has written in the same call. */
mr_status mr_details_noalloc(mr_grid* g, int32_t field, double* dev_norms);

/* Iterative adaptation (adaptation supplement): criterion, flags, policy
 * (refinement priority and propagation, 2:1, no coarsening of blocks refined
 * in this call, level bounds), refine / coarsen all fields, update step, until
 * no block changes or max_iter iterations.  Transactional over the call:
 * when an iteration's new tree would exceed max_blocks (MR_ECAPACITY) or a
 * norm is not finite (MR_ENONFINITE), the tree and every field come back
 * exactly as they were before the call (the substitution of the criterion's
 * ghost reconstructions included).  The call copies every field once into a
 * library-owned buffer of the current tree's size for this.  Synchronises. */
mr_status mr_adapt(mr_grid* g, int32_t field, int32_t max_iter, mr_adapt_stats* stats);

/* One adaptation iteration with block statuses given by the caller instead
 * of the criterion (a prescribed adaptation, e.g. the static two-level grids
 * of the convergence test of section 4.3): flags[b] for block b in the order
 * of mr_block_meta is +1 (refine, below level_max), -1 (coarsen, above
 * level_min) or 0 (keep).  The policy of the adaptation supplement applies:
 * refinement propagates to coarser neighbours, and a sibling set coarsens
 * only when all eight are flagged and no neighbour is finer or refining.
 * Every field is refined / coarsened / updated as in mr_adapt.  flags is
 * host memory of mr_grid_n_blocks entries; other values give MR_EINVAL.
 * Transactional like mr_adapt.  Synchronises. */
mr_status mr_adapt_flags(mr_grid* g, const int8_t* flags, mr_adapt_stats* stats);

/* One SSP-RK3 step of `field` (time-integration supplement) with the
 * configured right-hand side (central FD or CONS-3 / CONS-5); each stage
 * reconstructs the ghosts first.  Asynchronous. */
mr_status mr_rk3_step(mr_grid* g, int32_t field, double dt, const mr_velocity* vel);

/* One explicit stage (time-integration supplement; a building block for
 * other explicit schemes and for a pure right-hand side): ghost
 * reconstruction of field y (its substitution changes y in place), then
 * out = a_un * un + b * (c_y * y + dt * L(y)) with L the configured
 * right-hand side (-(u . grad) phi, or the CONS flux difference).  With
 * a_un = 0, b = 1, c_y = 0, dt = 1, out = L(y).  y, un, out are field
 * indices; out must differ from y (un may equal either).  Asynchronous. */
mr_status mr_stage(mr_grid* g, int32_t y, int32_t un, int32_t out, double a_un, double b,
                   double c_y, double dt, const mr_velocity* vel);

/* Replace the refinement and coarsening thresholds of section 2.2.5 (used
 * by the next mr_adapt / mr_details flag evaluation); needs
 * eps_refine > eps_coarsen >= 0, else MR_EINVAL. */
mr_status mr_set_thresholds(mr_grid* g, double eps_refine, double eps_coarsen);

/* Fused step: the block criterion of `field` (as mr_details), then one
 * SSP-RK3 step of it (as mr_rk3_step), whose first stage uses the ghosts
 * that the criterion's wide reconstruction (section 2.2.5, Table 3) has
 * just made for the same values; only stages 2 and 3 reconstruct theirs.
 * The norms are those of the field before the step.  Results equal
 * mr_details followed by mr_rk3_step up to the rounding order of the f->c
 * ghost values (the restriction tiles differ with the ghost depth).
 * norms, on_device: as in mr_details; with on_device = 0 the call
 * synchronises, and MR_ENONFINITE is returned after the step has been
 * applied.  Asynchronous with on_device = 1; captured into a graph of its
 * own in graph execution mode.  The detail pass runs on a second,
 * library-owned stream beside the step and is joined back into the grid's
 * stream before the call's work ends there.  The first call (and the first
 * after a tree grows) allocates a second ghost-patch buffer of the same size
 * as the first; it is freed by mr_grid_destroy. */
mr_status mr_details_rk3_step(mr_grid* g, int32_t field, double dt, const mr_velocity* vel,
                              double* norms, int32_t on_device);

/* dt = cfl * h_min / max_x sum_d |u_d(x)| for the current tree. */
mr_status mr_cfl_dt(const mr_grid* g, const mr_velocity* vel, double cfl, double* dt);

/* Leaf metadata in block order: *n receives the leaf count; level and ijk
 * (3 per leaf) are written when non-NULL and must hold *n_cap entries. */
mr_status mr_block_meta(const mr_grid* g, int64_t n_cap, int64_t* n, int32_t* level,
                        int32_t* ijk);

/* Copy the field to/from host memory, block-major, field precision.
 * bytes must equal n_blocks*nb^3*sizeof(value).  Synchronises. */
mr_status mr_field_get(mr_grid* g, int32_t field, void* host, size_t bytes);
mr_status mr_field_set(mr_grid* g, int32_t field, const void* host, size_t bytes);

/* Device pointer of a field (valid until the next mr_adapt / mr_set_tree /
 * mr_init_ic / mr_grid_destroy). */
mr_status mr_field_ptr(mr_grid* g, int32_t field, void** dev_ptr);

/* FP64 discrete moments (section 2.1.4, per axis): out[0] = sum h^3 phi,
 * out[1..3] = sum h^3 phi x_d, x_d the point coordinates in [0, 1).  Block
 * partials are added on the host with a compensated sum, so the result is
 * reproducible bit for bit.  Synchronises. */
mr_status mr_moments(mr_grid* g, int32_t field, double out[4]);

/* Distance of a field to an analytic initial condition evaluated in FP64 at
 * the leaves' points (the error norms of the validation experiments of
 * section 4: the epsilon test compares the compressed-and-refined field with
 * the field sampled on the finest level): out[0] = max |phi - f|,
 * out[1] = sqrt(sum h^3 (phi - f)^2).  Synchronises. */
mr_status mr_ic_error(mr_grid* g, int32_t field, const mr_ic* ic, double out[2]);

/* Set the launch-shape knobs (see mr_tuning) and rebuild the work lists of
 * the current tree; MR_EINVAL for values out of range (nothing changes).
 * An autotuner times them per configuration; results do not depend on them
 * except for the rounding order of f->c sums.  Synchronises. */
mr_status mr_set_tuning(mr_grid* g, const mr_tuning* t);

/* The knobs in effect. */
mr_status mr_get_tuning(mr_grid* g, mr_tuning* t);

/* Architecture name of the current HIP device (e.g. "gfx950"), the key
 * under which tuned knobs are cached; written NUL-terminated into out
 * (host memory of n bytes). */
mr_status mr_device_arch(char* out, size_t n);

/* Kernel timing with HIP events recorded on the grid's stream around each
 * launch of the named kernel family ("rhs", "details", "ghost_refine",
 * "ghost_subst", "ghost_restrict").  mr_prof_enable(g, 1) clears and starts recording;
 * mr_prof_read synchronises and returns the summed milliseconds, the number
 * of launches and the points processed per launch.  The names
 * "adapt_criterion", "adapt_plan", "adapt_apply" and "tree_commit" return
 * the host wall-clock time of those phases of mr_adapt / tree changes and
 * their count (always recorded; cleared by mr_prof_enable). */
mr_status mr_prof_enable(mr_grid* g, int32_t on);
mr_status mr_prof_read(mr_grid* g, const char* kernel, double* total_ms, int64_t* launches,
                       int64_t* points_per_launch);

/* Counts describing the current tree: out[0] = leaves, out[1] = ghost values
 * produced per stencil-depth reconstruction, out[2] = substitution work
 * items, out[3] = finest level, out[4] = coarsest level, out[5] = refinement
 * work items, out[6] = restriction work items, out[7] / out[8] = their LDS
 * bytes, out[9] = allocated patch values; per stencil-depth reconstruction,
 * the values each launch must write and read: out[10] / out[11] = c->f patch
 * values / coarse samples, out[12] / out[13] = substituted points / staged
 * points, out[14] / out[15] = f->c patch values / fine window points;
 * out[16..21] = the same six counts for the wide reconstruction of the
 * detail pass. */
mr_status mr_tree_stats(const mr_grid* g, int64_t out[22]);

/* Wait until all work issued on the grid's stream has finished. */
mr_status mr_sync(mr_grid* g);

const char* mr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MR_H */
