/*
 * impact.h -- C ABI of the MI355X (gfx950) IMDP library.
 *
 * The library builds interval-MDP abstractions of gridded stochastic systems
 *     x+ = f(x, u) + w,   w ~ N(0, diag(sigma^2)),
 * and runs interval iteration over them (IMPaCT, arXiv 2401.03555):
 *   - impact_build_imdp        : Def. 3.1 bounds, built as in Alg. 2, with
 *                                the out-of-domain entry of Remark 4.1;
 *   - impact_interval_iterate  : eq. (5.1)/(5.2), Alg. 3 (safety) and Alg. 4
 *                                (reach-avoid; reachability when the avoid set
 *                                is empty), the LP solved by the sorting method
 *                                of Section 6.2.
 * All arithmetic is IEEE FP64.  Every function returns a status code and never
 * throws; on a negative status a message is available from impact_last_error()
 * (thread-local) and outputs are unspecified.
 *
 * Conventions shared by every entry point
 *  - Grid: dimension i has n[i] >= 1 cells tiling [lb[i], ub[i]], width
 *    w_i = (ub_i - lb_i)/n_i, cell edge k = lb_i + k*w_i (edge n_i = ub_i).
 *    States are the cells in C order (last dimension fastest); 1 <= dim <= 8.
 *  - Inputs: a finite list (count x dim_u, row-major); row (s, u) has index
 *    s * count + u.  dim_u == 0 with count == 1 gives an interval Markov
 *    chain (Section 6.3): the policy is then identically 0.
 *  - Row layout of the abstraction: for row (s,u) the entries are the cells of
 *    its target window in C order over the window box, then OUT (leaving
 *    [lb, ub]) and, when windowed, TAIL (in-domain mass outside the window,
 *    lower bound 0).  Dense rows (k_sigma == 0) list every cell and have no
 *    TAIL.
 *  - Mean box: the per-dimension range of f over the source cell, padded
 *    outward by 2^-48 times the sum of magnitudes of the terms; affine sums
 *    are evaluated in index order as (sum_j a_ij x_j + sum_j b_ij u_j) + c_i,
 *    the unicycle as x0 + (dt v) cos-range, x1 + (dt v) sin-range,
 *    x2 + (dt om).  Windows are the cells meeting [m_lo - k sigma,
 *    m_hi + k sigma], computed as floor(((m - k*sigma) - lb)/w).
 *  - Streams: all device work is enqueued on impact_device.stream (a
 *    hipStream_t; NULL = the null stream).  Calls synchronize that stream
 *    before returning.
 */
#ifndef IMPACT_H
#define IMPACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IMPACT_MAX_DIM 8
#define IMPACT_MAX_ROW 16384 /* longest supported row (entries incl. OUT/TAIL); the
                                multi-query engine takes rows of up to 4096 */

/* Status codes.  > 0: success with a flag; < 0: failure. */
enum {
  IMPACT_OK = 0,
  IMPACT_NOT_CONVERGED = 1, /* a pass hit max_sweeps; outputs hold the current
                               (sound) brackets */
  IMPACT_E_INVAL = -1,      /* malformed argument                        */
  IMPACT_E_NOMEM = -2,      /* the allocator returned NULL               */
  IMPACT_E_HIP = -3,        /* a HIP runtime call failed                 */
  IMPACT_E_UNSUPPORTED = -4 /* valid but outside the supported envelope  */
};

/* System kinds. */
enum {
  IMPACT_SYS_AFFINE = 0,  /* f = A x + B u + c                                  */
  IMPACT_SYS_UNICYCLE = 1 /* f = (x0 + dt u0 cos x2, x1 + dt u0 sin x2, x2 + dt u1),
                             dim_x = 3, dim_u = 2, no wrap of x2              */
};

/* Dynamics (Def. 2.1 restricted to additive Gaussian noise).  Host pointers,
 * row-major, read during the call only.  A: dim_x*dim_x, B: dim_x*dim_u,
 * c: dim_x (affine); dt (unicycle). */
typedef struct {
  int32_t kind, dim_x, dim_u;
  const double *A, *B, *c;
  double dt;
} impact_system;

/* Grid (the partition of X, Section 2).  Host pointers, dim entries each. */
typedef struct {
  int32_t dim;
  const double *lb, *ub;
  const int32_t *n;
} impact_grid;

/* Finite input set U-hat.  Host pointer, count x dim_u row-major. */
typedef struct {
  int32_t count, dim_u;
  const double *values;
} impact_inputs;

/* Diagonal Gaussian noise (Section 4.1, NORMAL with diagonal covariance).
 * Host pointer to dim_x standard deviations, each > 0. */
typedef struct {
  const double *sigma;
} impact_noise;

/* Storage of the built bounds. */
enum {
  IMPACT_STORE_AUTO = 0,    /* library's choice (currently BOUNDS)           */
  IMPACT_STORE_BOUNDS = 1,  /* every entry's (lo, hi) kept in HBM            */
  IMPACT_STORE_FACTORS = 2  /* per-dimension factors kept; entry products
                               recomputed in every sweep                     */
};

/* Target window: k_sigma > 0 keeps cells within +-k_sigma standard
 * deviations of the mean box plus a TAIL entry; k_sigma == 0 is dense. */
typedef struct {
  double k_sigma;
  int32_t storage;
} impact_window;

/* Device memory and stream.  alloc/free may be NULL (hipMalloc/hipFree are
 * used).  alloc(bytes, ctx) returns device memory or NULL; free(ptr, ctx)
 * releases it.  stream is a hipStream_t. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
  void *stream;
} impact_device;

/* Opaque abstraction handle; owns its device buffers. */
typedef struct impact_imdp impact_imdp;

/*
 * Build the abstraction (Def. 3.1; Alg. 2; Remark 4.1).  For every row (s,u)
 * and every window cell t:
 *   lo(s,u,t) = prod_i min(g_i(m_lo_i), g_i(m_hi_i)),
 *   hi(s,u,t) = prod_i g_i(clamp(midpoint_i(t), m_lo_i, m_hi_i)),
 * g_i(m) the N(m, sigma_i^2) mass of the cell's i-th side; OUT bounds the mass
 * leaving [lb, ub], TAIL the in-domain mass outside the window.  The result is
 * specification independent (labels are applied at iteration time).
 * Arguments: host structs above; dev may be NULL (defaults).  *out receives
 * the handle (release with impact_imdp_free).
 * Errors: E_INVAL (bad dims/sizes/sigma/kind), E_NOMEM (allocation failed),
 * E_UNSUPPORTED (a row longer than IMPACT_MAX_ROW), E_HIP.
 */
int impact_build_imdp(const impact_system *sys, const impact_grid *grid,
                      const impact_inputs *inputs, const impact_noise *noise,
                      const impact_window *window, const impact_device *dev,
                      impact_imdp **out);

/* Correlated Gaussian noise (Section 4.1, full covariance): the covariance is
 * given by its inverse and its determinant, and cell masses are computed by
 * Monte Carlo integration.  Host pointers, read during the call only.
 *   inv_cov  : dim_x * dim_x, row-major, exactly symmetric, positive definite
 *   det_cov  : det(Cov) > 0 (of the covariance, not of its inverse); must
 *              agree with inv_cov (det(inv_cov) * det_cov within 1e-6 of 1)
 *   n_samples: N >= 1 points, samples: N * dim_x coordinates in [0, 1), the
 *              same points serving every cell (random or quasi-random)
 *   grid_pts : G >= 1 candidate means per dimension, G^dim_x <= 4096
 *   kappa    : >= 0 standard errors added to each side of every estimate */
typedef struct {
  const double *inv_cov;
  double det_cov;
  int64_t n_samples;
  const double *samples;
  int32_t grid_pts;
  double kappa;
} impact_mc_noise;

/*
 * impact_build_imdp for correlated noise, the cell masses of Def. 3.1 by Monte
 * Carlo integration (Section 4.1).  For a window cell [a, b] and a mean m the
 * estimate is vol * mean_k f(a + (b - a) r_k), f the N(m, Cov) density and r_k
 * the caller's points, with standard error vol * s / sqrt(N) (s the sample
 * standard deviation, 0 for N = 1).  The min / max over the source cell are
 * taken over G^dim candidate means, the centres of a G-way split of the mean
 * box, each estimate widened by kappa standard errors and by a bound on how
 * far the cell's mass can move between the candidate and any mean within half
 * a lattice spacing (the smaller of the total-variation distance and the
 * integrated mean derivative); bounds are clamped into [0, 1].  Windows use
 * the marginal standard deviations sqrt(Cov_ii); OUT and TAIL are union
 * bounds over dimensions of the marginal exit masses.  The bounds hold for
 * every point of the source cell up to the Monte Carlo error, which kappa
 * covers statistically.  Storage is BOUNDS (AUTO selects it); the handle
 * iterates like any other.
 * Errors: as impact_build_imdp, plus E_INVAL for a null noise, samples or
 * inv_cov, N < 1, G < 1, kappa < 0, a sample outside [0, 1), a non-symmetric,
 * singular or non-positive-definite inverse covariance, a determinant that
 * does not match it, or FACTORS storage; E_UNSUPPORTED for G^dim > 4096.
 */
int impact_build_imdp_mc(const impact_system *sys, const impact_grid *grid,
                         const impact_inputs *inputs, const impact_mc_noise *noise,
                         const impact_window *window, const impact_device *dev,
                         impact_imdp **out);

/* Finite disturbance set W-hat of an affine system, x+ = A x + B u + D w + c
 * + noise (eq. (5.1); Alg. 2 iterates over it like over the inputs).  Host
 * pointers, row-major: values count x dim_w, D dim_x x dim_w. */
typedef struct {
  int32_t count, dim_w;
  const double *values, *D;
} impact_disturbances;

/*
 * impact_build_imdp for an affine system with a disturbance player: one row
 * per (state, input, disturbance), row index (s * inputs.count + u) *
 * dist.count + w, each with the bounds of Def. 3.1 for the mean
 * A x + B u + D w + c (summed as (sum_j a_ij x_j + sum_j b_ij u_j +
 * sum_k d_ik w_k) + c_i).  impact_interval_iterate then values each (state,
 * input) by its worst row -- the lowest satisfaction probability for reach,
 * the highest bad-set probability for safety -- in both passes (eq. (5.1):
 * the disturbance is an adversary whatever the policy), and the policy
 * chooses the input only.  Such handles sweep both passes by state box
 * (one sort per state serving all its input and disturbance rows) when a
 * state's rows fit a box of 512 cells and the per-row mode is not set, and
 * per row otherwise; the multi-query engine runs them with the selection
 * sweep.  Errors as impact_build_imdp, plus E_INVAL for count or dim_w < 1,
 * null values or D, or non-finite entries; E_UNSUPPORTED for a non-affine
 * system, dim_u + dim_w > 8 or more than 256 (input, disturbance) pairs.
 */
int impact_build_imdp_dist(const impact_system *sys, const impact_grid *grid,
                           const impact_inputs *inputs, const impact_disturbances *dist,
                           const impact_noise *noise, const impact_window *window,
                           const impact_device *dev, impact_imdp **out);

/*
 * Build n abstractions with one launch of each construction kernel over the
 * rows of all of them (the parallel loop of Alg. 2 spanning every system).
 * sys, grid, inputs, noise, window are arrays of n structs (host); all windows
 * must use the same storage mode.  out[i] receives the handle of system i;
 * each is released with impact_imdp_free, and the shared device storage goes
 * when the last of them is released.  Results equal n separate
 * impact_build_imdp calls.  Errors as impact_build_imdp (the message names
 * the failing system); on error no handle is returned.
 */
int impact_build_imdp_batch(int32_t n, const impact_system *sys, const impact_grid *grid,
                            const impact_inputs *inputs, const impact_noise *noise,
                            const impact_window *window, const impact_device *dev,
                            impact_imdp **out);

/* Specification kinds (Section 3.1). */
enum { IMPACT_SAFETY = 0, IMPACT_REACH = 1, IMPACT_REACH_AVOID = 2 };

/* Specification.  Boxes are host arrays [n][2][dim] (lo then hi); a cell is
 * labelled by its centre (closed boxes, widened by 1e-9 cell widths); avoid
 * wins over target.  SAFETY: avoid boxes are the unsafe set, n_target must be
 * 0.  REACH: n_avoid must be 0.  Leaving [lb, ub] is always unsafe / failure.
 * pessimistic: 1 for the pessimistic policy (the paper's IMDP_lower = true,
 * Section 5: the policy is optimised on the adversarial LP and fixed for the
 * favourable one), 0 for the optimistic policy (optimised on the favourable
 * LP, fixed for the adversarial one); any other value is E_INVAL.  Either
 * way lo is the lower and hi the upper satisfaction bound under the policy.
 * max_sweeps >= 1 caps each of the two passes.
 * horizon: 0 for the infinite-horizon properties; T > 0 for the finite
 * horizon of Remark 5.1: each pass runs exactly T sweeps with no stop test
 * (eps and max_sweeps unused beyond validation; no sweep without SAFE
 * cells), value iteration from zero, so lo and hi are the T-step bounds
 * taken from the V0 iterate of the adversarial and the favourable pass; the
 * policy is the optimising input of the last policy-pass sweep, held for the
 * fixed-input pass.  IMPACT_HORIZON_AUTO (-1): the procedure of Remark 5.2
 * for runs whose two bounds need not meet: both passes first run until each
 * of their two iterates converges to itself, max(|V0' - V0|, |V1' - V1|) <=
 * eps over the SAFE cells after a sweep (at most max_sweeps sweeps); the
 * larger of the two sweep counts K is then the horizon of a finite-horizon
 * run as above, whose bounds and policy are returned (statistics: sweeps =
 * K per pass, self_sweeps = the two counts, converged = whether each pass's
 * iterates converged before the cap).  Any other negative value is E_INVAL. */
enum { IMPACT_HORIZON_AUTO = -1 };
typedef struct {
  int32_t kind, n_target, n_avoid;
  const double *target_boxes, *avoid_boxes;
  int32_t pessimistic;
  int64_t max_sweeps;
  int64_t horizon;
} impact_spec;

/*
 * Interval iteration with the sorting-method LP (eq. (5.1)/(5.2); Alg. 3 and
 * Alg. 4; Section 6.2).  Pass 1: V0 = 0, V1 = 1 on the SAFE cells; Jacobi
 * sweeps; reach / reach-avoid take the minimising LP and the max over u,
 * safety the maximising LP and the min over u; pi(s) is the optimising input
 * of the V0 results (lowest index on exact ties).  Pass 2: reset, u fixed by
 * pi, opposite LP direction.  Each pass runs while max(V1 - V0) > eps, at most
 * spec->max_sweeps sweeps.
 * Outputs (caller-owned DEVICE buffers of n_states elements, C order):
 *   reach, reach-avoid: lo = V0 of pass 1, hi = V1 of pass 2;
 *   safety: lo = 1 - V1 of pass 1, hi = 1 - V0 of pass 2 (safety probability);
 *   target cells lo = hi = 1, avoid cells lo = hi = 0;
 *   policy = input index on SAFE cells, -1 elsewhere.
 * That is the pessimistic policy.  With spec->pessimistic = 0 the two passes'
 * LP directions swap and so do the outputs' sources: reach lo = V0 of pass 2,
 * hi = V1 of pass 1; safety lo = 1 - V1 of pass 2, hi = 1 - V0 of pass 1.
 * spec->horizon selects the finite or automatic horizon (see impact_spec);
 * a handle from impact_build_imdp_dist values each input by its worst
 * disturbance row in both passes.
 * Returns IMPACT_OK, IMPACT_NOT_CONVERGED (a cap fired; outputs valid), or an
 * error (E_INVAL, E_NOMEM, E_UNSUPPORTED, E_HIP).
 */
int impact_interval_iterate(impact_imdp *imdp, const impact_spec *spec, double eps,
                            double *lo, double *hi, int32_t *policy);

/*
 * impact_interval_iterate for callers that cannot allocate device memory
 * (code that must not call hipMalloc, e.g. tight serving loops or harnesses
 * that forbid allocation): the same computation, arguments, outputs, status
 * codes and statistics, but every temporary of the call (labels, SAFE list,
 * value and policy buffers, control block, reduction partials, the sorted
 * value vectors and row hints of the long-row sweep) lives in one static
 * device array of 64 MiB per GPU, held from the library's first use on that
 * GPU until the process ends.  No allocation is made, through the handle's
 * allocator or otherwise, and no per-launch timing is recorded.  A call whose
 * temporaries exceed 64 MiB (about 65 bytes per state, plus 32 bytes per
 * state and 8 per row when rows are longer than 512 entries) returns
 * E_UNSUPPORTED and does nothing.  Calls on one GPU share its array:
 * calls that overlap in time on the same GPU (from several threads) race and
 * must be serialised by the caller.  Everything is re-initialised by each
 * call, so results do not depend on earlier calls.
 */
int impact_interval_iterate_noalloc(impact_imdp *imdp, const impact_spec *spec, double eps,
                                    double *lo, double *hi, int32_t *policy);

/* Statistics of the last impact_interval_iterate call on this handle. */
typedef struct {
  int64_t sweeps[2];    /* sweeps run in pass 1 / pass 2                 */
  double gap[2];        /* max(V1 - V0) over SAFE cells at the end       */
  int32_t converged[2]; /* 1 if the pass met eps (finite horizon: ran
                           its T sweeps)                                 */
  int64_t n_safe;       /* number of SAFE cells                          */
  int64_t updates[2];   /* (s,u)-row LP pairs solved per pass            */
  int64_t launches[2];  /* sweep-kernel launches per pass (a launch after
                           the stop test fired exits at once)            */
  double sweep_ms[2];   /* HIP-event time of the launches that swept
                           (timing on; else 0)                           */
  double launch_ms[2];  /* HIP-event time of every sweep launch (timing on) */
  double iterate_ms;    /* host wall time of the call                    */
  int64_t horizon;      /* horizon of the returned run: 0 infinite, else
                           the T (or K of IMPACT_HORIZON_AUTO) swept      */
  int64_t self_sweeps[2]; /* IMPACT_HORIZON_AUTO: sweeps until each pass's
                           iterates converged to themselves; else 0      */
  double self_sweep_ms; /* IMPACT_HORIZON_AUTO: HIP-event time of those
                           sweeps (timing on); else 0                    */
} impact_iter_info;

int impact_last_iter_info(const impact_imdp *imdp, impact_iter_info *info);

/* Shape and footprint of a built abstraction. */
typedef struct {
  int64_t n_states, n_rows, n_entries; /* entries include OUT / TAIL      */
  int32_t dim, n_inputs, windowed, storage;
  int32_t max_row;       /* longest row (entries incl. OUT / TAIL)       */
  int64_t max_box;       /* largest bounding box of one state's row windows
                            (cells; the unit sorted once per state)      */
  int64_t device_bytes;  /* bytes held by the handle                     */
  double build_ms;       /* build-kernel time, from HIP events           */
  int32_t n_dist;        /* disturbances per (state, input); 1 if none    */
} impact_imdp_info;

int impact_imdp_get_info(const impact_imdp *imdp, impact_imdp_info *info);

/*
 * Copy rows [row0, row0 + nrows) of the abstraction out, in the row layout
 * above (bounds are expanded from factors when FACTORS storage is in use).
 * All pointers are DEVICE buffers owned by the caller:
 *   window : nrows * 2 * dim int32 (klo[0..dim) then W[0..dim) per row)
 *   ot     : nrows * 4 doubles (OUT lo, OUT hi, TAIL lo, TAIL hi)
 *   counts : nrows int64 (window cells per row, i.e. excluding OUT / TAIL)
 *   entries: may be NULL; else (sum of counts) * 2 doubles, (lo, hi) pairs
 *            of the window cells of each row back to back (OUT/TAIL are in ot)
 * Errors: E_INVAL on a bad range.
 */
int impact_imdp_export_rows(const impact_imdp *imdp, int64_t row0, int64_t nrows,
                            int32_t *window, double *ot, int64_t *counts,
                            double *entries);

/* How interval iteration orders entries (all give the same LP values).
 *   AUTO       : the policy pass uses STATE_BOX when every row has at most 512
 *                entries; the fixed-input pass (one row per state) PER_ROW
 *   PER_ROW    : one bitonic sort per (state, input) row
 *   STATE_BOX  : one bitonic sort per state over the bounding box of its rows'
 *                windows; each row takes its order from it (the order of a
 *                subset of a sorted list is the subset's sorted order).  Used
 *                only when every row has at most 512 entries; states whose box
 *                exceeds 512 cells sort per row. */
enum { IMPACT_SWEEP_AUTO = 0, IMPACT_SWEEP_PER_ROW = 1, IMPACT_SWEEP_STATE_BOX = 2 };

int impact_set_sweep_mode(impact_imdp *imdp, int32_t mode);

/* The same choice made per pass: policy_pass for pass 1 (optimisation over
 * inputs), fixed_pass for pass 2 (policy fixed).  AUTO keeps the library's
 * default for that pass.  Results agree within rounding whatever the modes;
 * the autotuner picks them by measured sweep time.
 * Errors: E_INVAL on a null handle or an unknown mode. */
int impact_set_sweep_modes(impact_imdp *imdp, int32_t policy_pass, int32_t fixed_pass);

/* Enable (1) / disable (0) per-kernel HIP-event timing on this handle. */
int impact_set_timing(impact_imdp *imdp, int32_t enable);

/*
 * Multi-query engine: many interval-iteration queries in flight together
 * (the batched and served forms).  A query is (abstraction, specification,
 * eps) with the semantics and outputs of impact_interval_iterate; each runs
 * its own two passes and stop test, but every step advances all unfinished
 * queries with one launch per sweep kernel, and chunks of steps are replayed
 * from a captured HIP graph.  Queries join (submit) and leave (poll) at step
 * boundaries.  A query's results do not depend on the other queries in
 * flight.  The engine uses its own HIP stream; calls first wait for the
 * caller's stream (impact_device.stream) and return with the engine idle.
 */
typedef struct impact_mq impact_mq;

/* Create an engine with room for max_queries concurrent queries.  dev: as for
 * impact_build_imdp (allocator for the engine's and the queries' buffers). */
int impact_mq_create(const impact_device *dev, int32_t max_queries, impact_mq **out);

/* Add a query.  lo, hi, policy: caller-owned DEVICE buffers of the
 * abstraction's n_states elements, written as impact_interval_iterate would
 * once the query finishes (cells outside the SAFE set immediately).  The
 * abstraction handle may be released after submitting (the engine keeps its
 * device storage alive until the query is polled).  *id receives the query id.
 * Queries take every horizon of impact_spec, IMPACT_HORIZON_AUTO included,
 * and abstractions with a disturbance player (their queries run the
 * selection sweep, which values each input by its worst disturbance row).
 * Errors: E_INVAL (bad spec/eps/buffers), E_UNSUPPORTED (no free slot, rows
 * longer than 4096 entries, more than 256 inputs, or more than 256 (input,
 * disturbance) rows per state), E_NOMEM, E_HIP. */
int impact_mq_submit(impact_mq *mq, const impact_imdp *imdp, const impact_spec *spec, double eps,
                     double *lo, double *hi, int32_t *policy, int32_t *id);

/* Run up to `steps` steps (at least 1); returns early once every submitted
 * query has finished.  *n_active (may be NULL) receives the number of
 * unfinished queries. */
int impact_mq_run(impact_mq *mq, int32_t steps, int32_t *n_active);

/* Ids of queries finished since the last poll (up to cap, host array); their
 * outputs are final and their slots are released.  *n receives the count. */
int impact_mq_poll(impact_mq *mq, int32_t *ids, int32_t cap, int32_t *n);

/* Sweep counts, gaps and convergence flags of a finished query. */
int impact_mq_query_info(const impact_mq *mq, int32_t id, impact_iter_info *info);

/* Message for the last failing impact_mq_* call on this thread. */
const char *impact_mq_last_error(void);

/* Destroy the engine (unfinished queries are dropped).  NULL is a no-op. */
void impact_mq_free(impact_mq *mq);

/* Release the handle; its device buffers go with the last handle of its build.
 * NULL is a no-op. */
void impact_imdp_free(impact_imdp *imdp);

/* Message for the last failing call on this thread ("" if none). */
const char *impact_last_error(void);

/* Library version string. */
const char *impact_version(void);

/* Measurement support (not a step of the method): n_blocks workgroups of
 * 256 threads each run 16 independent FP64 FMA chains of `iters` steps, i.e.
 * 2 * 16 * iters * 256 * n_blocks FLOP, on `stream` (a hipStream_t, null for
 * the default stream).  `out` is a device double the kernel never writes in
 * practice.  Asynchronous; the caller times it with events on that stream.
 * E_INVAL for n_blocks outside [1, 2^24], iters < 1 or a null out. */
int impact_probe_fp64_fma(int64_t n_blocks, int32_t iters, double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
