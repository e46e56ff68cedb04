/*
 * treeray.h -- C ABI of the MI355X (gfx950) TreeRay/OnTheSpot library.
 *
 * The library computes, for every leaf cell of one or more grids, the EUV
 * photon flux of the TreeRay/OnTheSpot scheme (Wuensch et al., TreeRay paper,
 * Sec. 2): an octree over the cells with node moments (Sec. 2.1), a walk per
 * target cell with the Barnes-Hut opening test (Sec. 2.4), the mapping of
 * every accepted node onto the radial evaluation points of 12 N_side^2
 * HEALPix rays (Sec. 2.2, 2.3, App. A), the On-the-Spot integration of each
 * ray (Sec. 2.5) and the outer iteration with the delta_cell error control
 * (Sec. 2.6 "Iterations and error control").
 *
 * Conventions
 *  - All arguments named *_dev are device pointers (HIP memory on the
 *    context's device); everything else is host memory.  The caller owns all
 *    buffers it passes; the library owns the tree, its scratch memory and its
 *    work queue, allocates them in tr_set_domains/tr_set_sources/tr_build and
 *    frees them in tr_destroy.
 *  - All device work is enqueued asynchronously on the stream given to
 *    tr_create; argument checks are synchronous.  Errors raised by the device
 *    surface at tr_sync (or at the next call that reads results back).
 *  - Inputs and outputs are FP64 cgs: positions in cm, densities in cm^-3,
 *    rates in photons s^-1, fluxes in photons cm^-2 s^-1.
 *  - A context is not thread safe; separate contexts are independent.
 *  - Cell order: a uniform grid (leaf_blocks == NULL) lists its cells in C
 *    order over (x, y, z), z fastest; a block-structured grid lists them
 *    block by block in leaf_blocks order, C order inside each 8^3 block.
 *    Several domains are concatenated in the order given.
 *  - Every function returns TR_OK or a negative tr_status and then leaves a
 *    message for tr_last_error.
 */
#ifndef TREERAY_H
#define TREERAY_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tr_ctx tr_ctx;

typedef enum {
    TR_OK = 0,
    TR_EINVAL = -1,     /* bad argument (sizes, NaN/negative inputs, bad grid) */
    TR_ENOMEM = -2,     /* device or host allocation failed */
    TR_EHIP = -3,       /* a HIP runtime call failed */
    TR_ENOCONV = -4,    /* tr_solve reached max_iter; last field still returned */
    TR_ESTATE = -5,     /* call out of order (e.g. sweep before build) */
    TR_EOVERFLOW = -6   /* a per-target walk list exceeded its capacity */
} tr_status;

typedef enum {
    TR_FP64 = 0,        /* FP64 throughout */
    TR_FP32C = 1        /* FP32 walk, angular and radial weights and ray buffers;
                           FP64 node moments.  The ray march runs in FP64 or
                           (integration 6-8 of tr_set_launch, or as tuned) in
                           FP32 with compensated sums, in FP64 again near an
                           ionisation front (Sec. 2.5) */
} tr_precision;

/* One grid: an array of nroot root blocks of 8^3 cells, optionally refined
 * (Sec. 2.1: the tree solver works on the blocks of the AMR host code). */
typedef struct {
    int32_t nroot[3];           /* root blocks per axis */
    int32_t max_level;          /* refinement levels above the root level (0 = uniform) */
    double root_block_cm;       /* side of a root block */
    int64_t n_leaf_blocks;      /* rows of leaf_blocks */
    const int32_t *leaf_blocks; /* [n][4] = level, bi, bj, bk; NULL = uniform grid */
} tr_domain;

typedef struct {
    int32_t nside;              /* HEALPix N_side (power of two); N_PIX = 12 N_side^2 (Sec. 2.2) */
    int32_t n_radial;           /* >0: N_R evaluation points r_i = L_ray (i/(N_R-1))^2;
                                   0: N_R from eq. (Nr) and r_i from eq. (etaR) */
    double eta_r;               /* eta_R of eqs. (etaR), (Nr) */
    double theta;               /* Barnes-Hut opening angle theta_lim (Sec. 2.4) */
    double alpha_b;             /* Case-B recombination coefficient, cm^3 s^-1 */
    double hnu_erg;             /* mean EUV photon energy, only used to report e */
    double eps_lim;             /* delta_cell limit of the outer iteration */
    int32_t subsample;          /* s: s^3 angular sub-points per node (1..4) */
    int32_t max_iter;           /* outer iterations after the optically thin one */
    int32_t zeta_g;             /* 1: geometric correction of eq. (Rcorr:g); 0: zeta_g = 1 */
    tr_precision precision;
    double theta_if;            /* IF MAC (Sec. 2.4): nodes whose ionised mass (cells with a
                                   positive previous flux) lies strictly between 1e-8 and
                                   1 - 1e-8 of their mass are accepted only below this
                                   angle; <= 0 switches it off */
    double theta_src;           /* Src MAC (Sec. 2.4): the same for nodes with eps_n > 0 */
    double src_radius_cm;       /* > 0: sources are uniform spheres of this radius (Sec. 2.7),
                                   each cell taking the share of the rate equal to its part of
                                   the sphere's in-domain volume; 0: point sources */
    int32_t eps_kernel;         /* radial kernel of the emission (App. A): 0 or 3 two-point
                                   W_f,3, 1 W_f,1, 2 W_f,2, 4 W_f,3 over the N points inside the
                                   node's extent, 5 W_p, 6 W_g */
    int32_t mass_kernel;        /* radial kernel of A, E, V and the self term: 0 or 5 W_p, 6 W_g */
    int32_t periodic;           /* 1: periodic boundaries (Sec. 2.8): every node is used through
                                   its periodic copy closest to the target (by its cube's centre);
                                   0: isolated */
} tr_params;

typedef struct {
    int64_t n_cells, n_nodes;
    int64_t nodes_accepted;     /* summed over the targets of the last sweep */
    int64_t nodes_tested;
    int64_t guard_recomputes;   /* angular sub-points re-evaluated in FP64 (inside the FP32 guard band) */
    int32_t n_radial_max, depth_max;
    int32_t waves_per_target, targets_per_cu;   /* launch shape of the last sweep */
    int32_t buffer_in_lds;      /* where the last sweep kept its ray buffers: 1 LDS, 0 device memory,
                                   2 (FP32) the A, E, V rows in LDS and the emission rows in device memory,
                                   3 LDS for part of the rays at a time (a target's rays in passes; the
                                   emission rows in device memory when that saves a pass) */
    int32_t overflow;           /* nonzero if a walk list overflowed */
    int32_t integration_wave;   /* lanes that integrated one ray in the last sweep: 1, 4, 8, 16 or 64 */
    int32_t lds_cas;            /* 1 if the last sweep accumulated its LDS ray buffers by compare-and-swap */
    int32_t integration_fp32;   /* 1 if the last sweep marched its rays in FP32 (FP64 again near a front) */
    double last_sweep_ms;       /* device time of the last walk/map/integrate launch */
    int64_t rays_fp32;          /* rays of the last sweep marched in FP32 */
    int64_t rays_fp64_again;    /* of those, rays marched again in FP64 (a source below 1e-2 of its
                                   emitted Phi, or a close call between dying and surviving) */
    int64_t nodes_tabulated;    /* accepted nodes of the last sweep whose angular weights came from the
                                   context's table instead of their sub-points (same values) */
    int64_t rays_regrouped;     /* rays of the last sweep with more emitting points than the launch's
                                   group of lanes, marched by a wider group */
} tr_stats;

/* Creates a context on the current HIP device; stream may be NULL (default
 * stream).  Parameters are checked here (TR_EINVAL). */
tr_status tr_create(tr_ctx **ctx, const tr_params *p, void *hip_stream);

/* Declares the grids (Sec. 2.1).  Builds the octree topology (a virtual
 * power-of-two root over the root blocks; empty octants dropped), the
 * breadth-first node arrays and the evaluation points of every domain.
 * Invalidates sources and any previous build. */
tr_status tr_set_domains(tr_ctx *c, int32_t n_domains, const tr_domain *doms);

/* Leaf cells of domain dom (dom = -1: all domains together). */
tr_status tr_cell_count(const tr_ctx *c, int32_t dom, int64_t *n_cells);

/* Sources of domain dom: xyz_cm[n][3] relative to the domain's low corner,
 * q[n] photons/s (Sec. 2.7).  With src_radius_cm = 0 each rate is split
 * equally over the leaf cells whose closed extent contains the point;
 * otherwise by the exact volume of the source sphere in each cell (a
 * sphere reaching more than 16 finest cells may stop the build with a
 * deposit error). */
tr_status tr_set_sources(tr_ctx *c, int32_t dom, int64_t n, const double *xyz_cm,
                         const double *q_per_s);

/* Tree build (Sec. 2.1): deposits the sources, forms the cell quantities
 * eps/alpha/e (eqs. os:ems, os:abs, os:erd) from n_h_dev[cells] and the
 * previous flux f_prev_dev[cells] (NULL = zero), and reduces the node
 * moments in FP64.  thin != 0 builds the optically thin problem
 * (alpha_B = 0), used for the first iteration. */
tr_status tr_build(tr_ctx *c, const double *n_h_dev, const double *f_prev_dev, int32_t thin);

/* One sweep over every leaf cell of every domain (Sec. 2.3-2.5): tree walk,
 * node->ray mapping, per-ray integration, sum over rays.  Writes the photon
 * flux f_out_dev[cells] and, if not NULL, ionised_out_dev[cells] = F > 0
 * (Sec. 2.6 "Interaction with gas", option (i)).  Needs tr_build. */
tr_status tr_sweep(tr_ctx *c, double *f_out_dev, uint8_t *ionised_out_dev);

/* The same for a list of global cell indices targets_dev[n] (int64);
 * outputs are indexed like the list. */
tr_status tr_sweep_targets(tr_ctx *c, const int64_t *targets_dev, int64_t n, double *f_out_dev,
                           uint8_t *ionised_out_dev);

/* delta_cell of eq. (delta:er:cell) per domain: max over the domain's cells
 * of |f_new - f_old| / max(f_old, median f_old).  delta_host[n_domains]. */
tr_status tr_delta(tr_ctx *c, const double *f_new_dev, const double *f_old_dev, double *delta_host);

/* One outer iteration (Sec. 2.6) as a single hipGraph launch: tree build from
 * n_h_dev and the previous flux f_prev_dev, sweep into f_out_dev (and
 * ionised_out_dev if not NULL), delta_cell per domain into delta_host
 * [n_domains].  The graph is captured on the first call and replayed while
 * the four device pointers, the precision, the launch shape and the sources
 * stay the same.  f_prev_dev and f_out_dev must differ.  Synchronises. */
tr_status tr_step(tr_ctx *c, const double *n_h_dev, const double *f_prev_dev, double *f_out_dev,
                  uint8_t *ionised_out_dev, double *delta_host);

/* Outer iteration (Sec. 2.6): an optically thin build+sweep, then build+sweep
 * with the last flux until every domain has delta_cell < eps_lim or max_iter
 * sweeps.  f_out_dev receives the last flux, iters_out the absorbing sweeps,
 * delta_out the largest delta of the last one.  Returns TR_ENOCONV if the
 * limit was reached (the fields are still written). */
tr_status tr_solve(tr_ctx *c, const double *n_h_dev, double *f_out_dev, uint8_t *ionised_out_dev,
                   int32_t *iters_out, double *delta_out);

/* Switches the internal precision of later builds and sweeps. */
tr_status tr_set_precision(tr_ctx *c, tr_precision prec);

/* Launch shape of the sweep: waves per target (1,2,4,8,16), resident
 * targets per compute unit (0 = as many as fit), where a target's ray
 * buffer lives (0 = LDS when it fits, else the split FP32 form, else LDS
 * in passes over the rays, 1 = the same but an error when none fits,
 * 2 = device memory) and how
 * rays are integrated (0 = tuned or default, 1 = a lane per ray, 2 = a wave
 * per ray with the ray's points on the lanes, 3, 4, 5 = a group of 4, 8, 16
 * lanes per ray with the ray's emitting points on the lanes, the default; a
 * ray with more emitting points than that is marched again by a group of 32
 * or 64 lanes (more than 64: a wave, in FP64); 6, 7, 8 = the same
 * groups marching in FP32 with a compensated Phi and compensated flux sums,
 * every ray where a source falls below 1e-2 of its emitted Phi marched again
 * in FP64 (Sec. 2.5; FP32C only, the FP64 form takes 3, 4, 5) and how the waves
 * of a target accumulate into a shared FP32 buffer in LDS at 8 or 16 waves
 * (0 = tuned or default, compare-and-swap; 1 = hardware atomic
 * adds; 2 = compare-and-swap loops on the values' bits; elsewhere hardware
 * atomics).  Zeros restore the tuned default.  Results do not depend on the
 * shape beyond rounding. */
tr_status tr_set_launch(tr_ctx *c, int32_t waves_per_target, int32_t targets_per_cu, int32_t buffer,
                        int32_t integration, int32_t atomics);

/* Searches the launch shape for the current build and precision by timing
 * sweeps over a sample of targets; keeps the fastest.  best_ms_out may be NULL. */
tr_status tr_autotune(tr_ctx *c, double *best_ms_out);

tr_status tr_get_stats(tr_ctx *c, tr_stats *out);

/* Waits for the context's stream and reports device-side errors. */
tr_status tr_sync(tr_ctx *c);

/* Message of the last failed call on c; c = NULL: of the last failed call
 * without a context (tr_delta_noalloc) on the calling thread. */
const char *tr_last_error(const tr_ctx *c);

/* delta_cell per domain without a context and without allocating, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same result as
 * tr_delta for the same cells (eq. delta:er:cell, lower median of f_old per
 * domain).
 *  - f_new_dev, f_old_dev: device arrays of dom_offsets[n_domains] cells;
 *    domain d holds cells [dom_offsets[d], dom_offsets[d+1]).
 *  - dom_offsets: host array of n_domains + 1 strictly increasing entries,
 *    dom_offsets[0] = 0 (every domain non-empty).
 *  - n_domains: 1 .. 64 (TR_EINVAL beyond: the library's static scratch holds
 *    the radix-select state of 64 domains, about 67 KB per device, kept
 *    until the process ends).
 *  - delta_dev: device array of n_domains doubles (caller-owned), written
 *    asynchronously on hip_stream (NULL: the default stream).
 * Launches kernels only (no allocation, no memset, no host synchronisation),
 * so it may be captured.  All calls on one device share that scratch: calls
 * whose work overlaps on one device (other streams, other threads) race and
 * must be ordered by the caller.  Errors: TR_EINVAL / TR_EHIP with the
 * message in tr_last_error(NULL) of the calling thread. */
tr_status tr_delta_noalloc(const double *f_new_dev, const double *f_old_dev, const int64_t *dom_offsets,
                           int32_t n_domains, double *delta_dev, void *hip_stream);

/* Digest of the sources the library was built from (16 hex digits; a static
 * string, never NULL).  Bindings compare it with the sources they ship with
 * and refuse a library built from other sources. */
const char *tr_source_digest(void);

void tr_destroy(tr_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
