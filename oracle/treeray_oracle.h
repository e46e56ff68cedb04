/*
 * FP64 CPU oracle for the TreeRay/OnTheSpot sweep (Wuensch et al., TreeRay
 * paper, Sec. 2).  TEST INFRASTRUCTURE ONLY: the tests, the package smoke
 * check and the CPU-baseline leg of the benchmark call it; the HIP library
 * never does.  It shares no code with the HIP library.
 *
 * Everything is in cgs, FP64.  Geometry (cell and node positions, the
 * opening-angle test, angular sub-points) is done in units of the finest cell
 * so that it is exact; physical distances are those times the finest cell size.
 */
#ifndef TREERAY_ORACLE_H
#define TREERAY_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nroot[3];          /* root blocks per axis, 8^3 cells each */
    int32_t max_level;         /* refinement levels above the root level */
    double root_block_cm;      /* side of a root block */
    int64_t n_leaf_blocks;     /* rows of leaf_blocks (ignored if NULL) */
    const int32_t *leaf_blocks;/* [n][4] = level, bi, bj, bk; NULL = uniform */
} orc_domain;

typedef struct {
    int32_t nside;             /* HEALPix N_side; N_PIX = 12 N_side^2 */
    int32_t n_radial;          /* >0: N_R points at L_ray (i/(N_R-1))^2; 0: eq. (Nr) */
    double eta_r;              /* radial resolution parameter of eq. (etaR) */
    double theta;              /* Barnes-Hut opening angle */
    double alpha_b;            /* Case-B recombination coefficient; 0 = optically thin */
    int32_t subsample;         /* s: s^3 angular sub-points per node */
    int32_t zeta_g;            /* 1: geometric correction as printed; 0: zeta_g = 1 */
    double theta_if;           /* IF MAC opening angle (Sec. 2.4); <= 0: off */
    double theta_src;          /* Src MAC opening angle (Sec. 2.4); <= 0: off */
    double src_radius_cm;      /* > 0: sources are uniform spheres of this radius (Sec. 2.7) */
    int32_t eps_kernel;        /* emission kernel, ORC_K_* (0: two-point W_f,3) */
    int32_t mass_kernel;       /* kernel of A, E, V: ORC_K_P (0 too) or ORC_K_G */
    int32_t periodic;          /* 1: periodic boundaries, nearest copy of every node (Sec. 2.8) */
} orc_params;

enum { ORC_K_DEFAULT = 0, ORC_K_F1 = 1, ORC_K_F2 = 2, ORC_K_F3 = 3, ORC_K_F3N = 4, ORC_K_P = 5, ORC_K_G = 6 };

typedef struct {
    int64_t nodes_accepted;    /* summed over the swept targets */
    int64_t nodes_tested;
    int64_t n_nodes;           /* size of the tree */
    int32_t n_radial;          /* evaluation points actually used */
    int32_t depth;             /* deepest node level */
} orc_stats;

/* status codes: 0 ok, -1 bad argument, -2 out of memory, -3 bad grid */

int64_t orc_cell_count(const orc_domain *d);
/* lo (finest-cell units) and size of every leaf cell, in input order */
int orc_cell_geometry(const orc_domain *d, int64_t *lo3, int64_t *size);

int orc_radial_points(const orc_domain *d, const orc_params *p, int32_t max_n, double *r_out);

/* One sweep: tree of the current gas, walk + map + per-ray integration for the
 * listed targets (all cells if targets == NULL).  f_prev = photon flux of the
 * previous iteration per cell (NULL -> zero).  f_out/ion_out are indexed like
 * the target list (or all cells). */
int orc_sweep(const orc_domain *d, const orc_params *p, const double *n_h,
              int64_t n_src, const double *src_xyz_cm, const double *src_q,
              const double *f_prev, int64_t n_targets, const int64_t *targets,
              double *f_out, uint8_t *ion_out, orc_stats *st);

/* The same with the target loop on `threads` OpenMP threads (0: the default)
 * and its wall time (tree build excluded) in *seconds if not NULL. */
int orc_sweep_timed(const orc_domain *d, const orc_params *p, const double *n_h,
                    int64_t n_src, const double *src_xyz_cm, const double *src_q,
                    const double *f_prev, int64_t n_targets, const int64_t *targets,
                    double *f_out, uint8_t *ion_out, orc_stats *st, int32_t threads, double *seconds);

/* Outer iteration: a thin sweep, then sweeps fed with the last flux until
 * delta_cell < eps_lim or max_iter sweeps; returns the number of sweeps after
 * the thin one in *iters and the last delta in *delta. */
int orc_solve(const orc_domain *d, const orc_params *p, const double *n_h,
              int64_t n_src, const double *src_xyz_cm, const double *src_q,
              double eps_lim, int32_t max_iter, double *f_out, uint8_t *ion_out,
              int32_t *iters, double *delta);

double orc_delta_cell(int64_t n, const double *f_new, const double *f_old);
double orc_delta_tot(int64_t n, const double *f_new, const double *f_old, const double *dv);

/* point-source rates per cell */
int orc_deposit(const orc_domain *d, int64_t n_src, const double *src_xyz_cm,
                const double *src_q, double *ndot_out);

/* sources as uniform spheres of radius_cm: rates split by the sphere volume in each cell */
int orc_deposit_spheres(const orc_domain *d, int64_t n_src, const double *src_xyz_cm,
                        const double *src_q, double radius_cm, double *ndot_out);
/* volume of the ball (centre, R) inside the box [lo, hi] */
double orc_ball_box_volume(double cx, double cy, double cz, double R, const double *lo, const double *hi);

/* radial kernels of App. A: W_g, smoothing weights (P or G), emission weights */
double orc_wg(double x);
void orc_mass_weights(int32_t kind, int32_t n, const double *r, double d, double h, double *v_out);
void orc_eps_weights(int32_t kind, int32_t n, const double *r, double d, double h, double *u_out);

/* OpenMP threads a sweep uses, and setting them (n >= 1) */
int32_t orc_num_threads(void);
void orc_set_num_threads(int32_t n);

/* ---- pieces exposed for the pin tests ---- */
int64_t orc_ang2pix(int32_t nside, double x, double y, double z);
void orc_ang2pix_many(int32_t nside, int64_t n, const double *xyz, int64_t *out);
void orc_pix2vec(int32_t nside, int64_t pix, double *v3);
double orc_wp(double x);
/* normalised W_p weights over the points (radial mapping of A, E, V) */
void orc_wp_weights(int32_t n, const double *r, double d, double h, double *v_out);
/* two-point flux-conserving W_f,3 weights (radial mapping of emission) */
void orc_wf3_weights(int32_t n, const double *r, double d, double *u_out);
/* OTS integration of one ray; eps/A/E/V are the mapped totals */
double orc_integrate_ray(int32_t n, const double *r, const double *eps, const double *A,
                         const double *E, const double *V, int32_t nside, int32_t zeta_g);
/* accepted nodes of one target: lo3, size, moments (eps, alpha, E, V,
 * mass, com3, ionised mass); returns count or <0 */
int64_t orc_accepted(const orc_domain *d, const orc_params *p, const double *n_h,
                     int64_t n_src, const double *src_xyz_cm, const double *src_q,
                     const double *f_prev, int64_t target, int64_t max_out,
                     int64_t *lo_size_out /* [max][4] */, double *mom_out /* [max][9] */);

/* angular weights of one node box [olo, ohi) (finest units) seen from xt:
 * the distinct pixels of its s^3 sub-box midpoints and their counts (arrays of
 * s^3 entries); returns the number of distinct pixels or <0 */
int32_t orc_node_pixels(int32_t nside, int32_t s, const int64_t *olo, const int64_t *ohi, const double *xt,
                        int64_t *pix_out, int32_t *count_out);
/* mapped ray buffers of one target before the integration, [N_PIX][N_R]
 * each (self term included); returns N_R or <0 */
int32_t orc_target_rays(const orc_domain *d, const orc_params *p, const double *n_h, int64_t n_src,
                        const double *src_xyz_cm, const double *src_q, const double *f_prev, int64_t target,
                        int32_t max_nr, double *eps_out, double *a_out, double *e_out, double *v_out);

#ifdef __cplusplus
}
#endif
#endif
