/*
 * impact_oracle.h -- reference CPU implementation of the IMDP abstraction and
 * interval iteration (IMPaCT, arXiv 2401.03555).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, FP64, single-threaded
 * oracle that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the GPU library, and never reads any
 * value produced by it.
 *
 * Every function follows a definition or algorithm of the paper; the citation
 * is given at each function.  Where the paper is silent the reading used is
 * stated at the function (and listed in the design notes of the repository).
 */
#ifndef IMPACT_ORACLE_H
#define IMPACT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_DIM 8

/* Entry targets that are not grid cells. */
#define ORC_T_OUT (-1)  /* leaving the bounded state set (Remark 4.1) */
#define ORC_T_TAIL (-2) /* in-domain mass outside the +-k sigma window */

/* Cell classes (Section 3.1 relabelling). */
#define ORC_SAFE 0
#define ORC_TARGET 1
#define ORC_AVOID 2

/* Specification kinds (Definition of specifications, Section 3.1). */
#define ORC_SAFETY 0
#define ORC_REACH 1
#define ORC_REACH_AVOID 2

/* System kinds: x+ = f(x,u) + w with w ~ N(0, diag(sigma^2)). */
#define ORC_SYS_AFFINE 0   /* f = A x + B u + c                              */
#define ORC_SYS_UNICYCLE 1 /* f = (x0 + dt v cos x2, x1 + dt v sin x2, x2 + dt om) */

typedef struct {
  int32_t kind, dim_x, dim_u;
  const double *A; /* dim_x * dim_x, row-major (affine only)  */
  const double *B; /* dim_x * dim_u, row-major (affine only)  */
  const double *c; /* dim_x (affine only)                      */
  double dt;       /* unicycle sampling time                   */
} orc_system;

typedef struct {
  int32_t dim;
  const double *lb, *ub; /* dim each */
  const int32_t *n;      /* cells per dimension */
} orc_grid;

typedef struct {
  int32_t count, dim_u;
  const double *values; /* count * dim_u, row-major */
} orc_inputs;

/* A built abstraction, in host memory, rows indexed by position. */
typedef struct {
  int64_t n_states, n_rows, n_entries;
  int32_t n_inputs, dim, windowed;
  int32_t *win;     /* n_rows * 2 * dim : klo[0..dim) then W[0..dim) */
  double *ot;       /* n_rows * 4 : OUT lo, OUT hi, TAIL lo, TAIL hi  */
  int64_t *row_ptr; /* n_rows + 1                                     */
  int32_t *target;  /* n_entries : cell index, ORC_T_OUT or ORC_T_TAIL */
  double *lo, *hi;  /* n_entries                                      */
} orc_imdp;

typedef struct {
  int64_t sweeps[2];
  double gap[2];
  int32_t converged[2];
  int64_t n_safe;
} orc_iter_info;

/* ---- grid and dynamics ---- */
double orc_cell_edge(const orc_grid *g, int i, int64_t k);
void orc_interval_cos(double lo, double hi, double *cmin, double *cmax);
void orc_interval_sin(double lo, double hi, double *smin, double *smax);
int orc_mean_box(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
                 int64_t state, int32_t input, double *mlo, double *mhi);

/* ---- per-dimension Gaussian masses ---- */
double orc_gauss_cell_mass(double a, double b, double m, double sigma);
void orc_factor_bounds(double a, double b, double mlo, double mhi, double sigma,
                       double *flo, double *fhi);
double orc_exit_prob(double lb, double ub, double m, double sigma);

/* ---- abstraction ---- */
int orc_build(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
              const double *sigma, double k_sigma, const int64_t *rows,
              int64_t n_rows, orc_imdp *out);
void orc_imdp_free(orc_imdp *m);

/* ---- correlated noise by Monte Carlo integration (Section 4.1) ---- */
/* Full covariance given as its inverse P and det(Cov); cell masses by plain
   Monte Carlo over the caller's points of [0,1)^dim (shared by every cell);
   min / max over the source cell from a G^dim lattice of candidate means,
   each widened by a bound on the mass moved by the lattice spacing; kappa
   standard errors of each estimate added on each side. */
typedef struct {
  const double *inv_cov; /* dim * dim, row-major, symmetric positive definite */
  double det_cov;        /* determinant of the covariance (not of its inverse) */
  int64_t n_samples;     /* >= 1 */
  const double *samples; /* n_samples * dim points of [0, 1)^dim             */
  int32_t grid_pts;      /* G >= 1 candidate means per dimension             */
  double kappa;          /* >= 0 standard errors added on each side          */
} orc_mc_noise;

int orc_marginal_sigma(int d, const double *inv_cov, double *sigma);
double orc_mc_cover_radius(int d, const double *inv_cov, const double *mlo, const double *mhi,
                           int G);
double orc_mc_shift_bound(int d, const double *sigma, double norm, double rho, double vol,
                          const double *zlo, const double *zhi);
void orc_mc_cell_estimate(int d, const double *inv_cov, double norm, const double *a,
                          const double *b, const double *m, int64_t n, const double *samples,
                          double *p, double *se);
int orc_build_mc(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
                 const orc_mc_noise *mc, double k_sigma, const int64_t *rows,
                 int64_t n_rows, orc_imdp *out);

/* ---- labelling ---- */
int orc_label(const orc_grid *g, int32_t n_target, const double *target_boxes,
              int32_t n_avoid, const double *avoid_boxes, int8_t *cls);

/* ---- LP by the sorting method ---- */
double orc_lp_sorted(int64_t n, const double *lo, const double *hi,
                     const double *val, int32_t maximise, double *p_out);

/* ---- interval iteration ---- */
/* optimistic = 0: pessimistic policy (the paper's IMDP_lower = true);
   optimistic = 1: optimistic policy (IMDP_lower = false).
   horizon = 0: infinite horizon (stop test on eps, cap max_sweeps);
   horizon = T > 0: finite horizon, exactly T sweeps per pass (Remark 5.1).
   self_stop = 1 (horizon 0): a pass stops once both iterates stop moving
   by more than eps in a sweep (Remark 5.2).
   n_dist >= 1: disturbances per (s, u); rows (s * n_inputs + u) * n_dist + w,
   the worst row valuing the input (eq. (5.1)). */
int orc_iterate(int64_t n_states, int32_t n_inputs, const int64_t *row_ptr,
                const int32_t *target, const double *lo, const double *hi,
                const int8_t *cls, int32_t spec_kind, double eps,
                int64_t max_sweeps, double *out_lo, double *out_hi,
                int32_t *policy, orc_iter_info *info, double *q0_last,
                int64_t hist_cap, double *hist_v0, double *hist_v1,
                int32_t optimistic, int64_t horizon, int32_t self_stop, int32_t n_dist);

#ifdef __cplusplus
}
#endif
#endif
