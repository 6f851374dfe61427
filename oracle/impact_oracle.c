/*
 * impact_oracle.c -- reference CPU implementation (TEST INFRASTRUCTURE ONLY).
 *
 * Plain FP64, single-threaded, no blocking or fusion: each function is the
 * definition or algorithm step it cites, written out.  It is loaded only by
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark;
 * the GPU library never links or calls it, and it never reads a GPU result.
 *
 * Citations refer to arXiv 2401.03555 (IMPaCT): Def. 3.1 (IMDP bounds),
 * Section 3.1 (labels and absorbing target/avoid sets), Alg. 1/2 (construction),
 * Remark 4.1 (out-of-domain mass), Section 4.4 (low-cost abstraction),
 * eq. (5.1)/(5.2) (interval-iteration LP and update), Alg. 3/4 (pessimistic
 * safety and reach-avoid synthesis), Section 6.2 (sorting method).
 *
 * Readings where the paper is silent (closed-form bounds for the Gaussian
 * kernel, the +-k sigma window with its TAIL entry, the sweep cap, the output
 * pairing for safety) are stated at the function that implements them.
 */
#include "impact_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RSQRT2 0.70710678118654752440 /* 1/sqrt(2) rounded to double */
#define ORC_PAD_REL 3.552713678800501e-15 /* 2^-48: outward pad of the mean box */
#define ORC_TWO_PI 6.283185307179586
#define ORC_PI 3.141592653589793
#define ORC_HALF_PI 1.5707963267948966

/* ------------------------------------------------------------------------- */
/* Grid (Section 2 partitions; Alg. 2 "select finite partition").           */
/* Cells tile [lb, ub] with n cells of width w = (ub - lb)/n.  Edge k is      */
/* lb + k*w (product first, then the add), except edge n which is ub.         */
/* ------------------------------------------------------------------------- */
double orc_cell_edge(const orc_grid *g, int i, int64_t k) {
  double w = (g->ub[i] - g->lb[i]) / (double)g->n[i];
  if (k == g->n[i]) return g->ub[i];
  return g->lb[i] + (double)k * w;
}

static void unravel_state(const orc_grid *g, int64_t s, int64_t *k) {
  for (int i = g->dim - 1; i >= 0; --i) {
    k[i] = s % g->n[i];
    s /= g->n[i];
  }
}

/* Does a + 2*pi*j lie in [lo, hi] for some integer j? */
static int lattice_hit(double lo, double hi, double a) {
  double j = ceil((lo - a) / ORC_TWO_PI);
  return a + j * ORC_TWO_PI <= hi;
}

/* Range of cos over [lo, hi]: endpoint values, widened to +1 / -1 when a
 * maximiser 2j*pi / minimiser (2j+1)*pi lies inside the interval. */
void orc_interval_cos(double lo, double hi, double *cmin, double *cmax) {
  double c1 = cos(lo), c2 = cos(hi);
  *cmin = c1 < c2 ? c1 : c2;
  *cmax = c1 < c2 ? c2 : c1;
  if (lattice_hit(lo, hi, 0.0)) *cmax = 1.0;
  if (lattice_hit(lo, hi, ORC_PI)) *cmin = -1.0;
}

/* Range of sin over [lo, hi]; extrema at pi/2 + 2j*pi and -pi/2 + 2j*pi. */
void orc_interval_sin(double lo, double hi, double *smin, double *smax) {
  double s1 = sin(lo), s2 = sin(hi);
  *smin = s1 < s2 ? s1 : s2;
  *smax = s1 < s2 ? s2 : s1;
  if (lattice_hit(lo, hi, ORC_HALF_PI)) *smax = 1.0;
  if (lattice_hit(lo, hi, -ORC_HALF_PI)) *smin = -1.0;
}

/*
 * Interval of the noise-free successor f(x,u) over the source cell, per
 * dimension (Def. 3.1: the min/max over x in the partition; Alg. 2, the
 * parallel loop body).  Affine f: exact per-dimension range by the sign of
 * each coefficient.  Unicycle f: x and theta vary independently, with interval
 * cos/sin.  The result is padded outward by 2^-48 times the sum of the
 * magnitudes of the terms, which covers every rounding in the evaluation.
 * Evaluation order (fixed, so that window edges are reproducible):
 *   affine:   s_lo = sum_j a_ij * x_j^{lo or hi by sign of a_ij}  (j ascending)
 *             bu   = sum_j b_ij * u_j                              (j ascending)
 *             m_lo = (s_lo + bu) + c_i - pad,  m_hi likewise
 *   unicycle: t = dt*v; m0 = x0 + t*cos-range, m1 = x1 + t*sin-range,
 *             m2 = x2 + (dt*om).
 */
int orc_mean_box(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
                 int64_t state, int32_t input, double *mlo, double *mhi) {
  int d = g->dim;
  int64_t k[ORC_MAX_DIM];
  double xl[ORC_MAX_DIM], xh[ORC_MAX_DIM];
  unravel_state(g, state, k);
  for (int i = 0; i < d; ++i) {
    xl[i] = orc_cell_edge(g, i, k[i]);
    xh[i] = orc_cell_edge(g, i, k[i] + 1);
  }
  const double *u = in->dim_u > 0 ? in->values + (int64_t)input * in->dim_u : 0;
  if (sys->kind == ORC_SYS_AFFINE) {
    for (int i = 0; i < d; ++i) {
      double slo = 0.0, shi = 0.0, mag = 0.0;
      for (int j = 0; j < d; ++j) {
        double a = sys->A[i * d + j];
        if (a >= 0.0) {
          slo += a * xl[j];
          shi += a * xh[j];
        } else {
          slo += a * xh[j];
          shi += a * xl[j];
        }
        mag += fabs(a) * fmax(fabs(xl[j]), fabs(xh[j]));
      }
      double bu = 0.0;
      for (int j = 0; j < sys->dim_u; ++j) {
        double t = sys->B[i * sys->dim_u + j] * u[j];
        bu += t;
        mag += fabs(t);
      }
      mag += fabs(sys->c[i]);
      double pad = mag * ORC_PAD_REL;
      mlo[i] = (slo + bu) + sys->c[i] - pad;
      mhi[i] = (shi + bu) + sys->c[i] + pad;
    }
    return 0;
  }
  if (sys->kind == ORC_SYS_UNICYCLE) {
    if (d != 3 || in->dim_u != 2) return -1;
    double v = u[0], om = u[1];
    double cmin, cmax, smin, smax;
    orc_interval_cos(xl[2], xh[2], &cmin, &cmax);
    orc_interval_sin(xl[2], xh[2], &smin, &smax);
    double t = sys->dt * v;
    double pad0 = (fmax(fabs(xl[0]), fabs(xh[0])) + fabs(t)) * ORC_PAD_REL;
    double pad1 = (fmax(fabs(xl[1]), fabs(xh[1])) + fabs(t)) * ORC_PAD_REL;
    if (t >= 0.0) {
      mlo[0] = xl[0] + t * cmin - pad0;
      mhi[0] = xh[0] + t * cmax + pad0;
      mlo[1] = xl[1] + t * smin - pad1;
      mhi[1] = xh[1] + t * smax + pad1;
    } else {
      mlo[0] = xl[0] + t * cmax - pad0;
      mhi[0] = xh[0] + t * cmin + pad0;
      mlo[1] = xl[1] + t * smax - pad1;
      mhi[1] = xh[1] + t * smin + pad1;
    }
    double tw = sys->dt * om;
    double pad2 = (fmax(fabs(xl[2]), fabs(xh[2])) + fabs(tw)) * ORC_PAD_REL;
    mlo[2] = xl[2] + tw - pad2;
    mhi[2] = xh[2] + tw + pad2;
    return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------------- */
/* Gaussian masses (Def. 3.1 with T the Gaussian kernel of x+ = f + w).       */
/* ------------------------------------------------------------------------- */

/*
 * P(m + w in [a, b]) for w ~ N(0, sigma^2), i.e. Phi(zb) - Phi(za), evaluated
 * on whichever side keeps both terms in a tail so that nothing cancels:
 *   za >= 0: (erfc(za/sqrt2) - erfc(zb/sqrt2)) / 2
 *   zb <= 0: (erfc(-zb/sqrt2) - erfc(-za/sqrt2)) / 2
 *   else   : 1 - erfc(-za/sqrt2)/2 - erfc(zb/sqrt2)/2
 */
double orc_gauss_cell_mass(double a, double b, double m, double sigma) {
  double za = (a - m) / sigma;
  double zb = (b - m) / sigma;
  double g;
  if (za >= 0.0)
    g = 0.5 * (erfc(za * ORC_RSQRT2) - erfc(zb * ORC_RSQRT2));
  else if (zb <= 0.0)
    g = 0.5 * (erfc(-zb * ORC_RSQRT2) - erfc(-za * ORC_RSQRT2));
  else
    g = (1.0 - 0.5 * erfc(-za * ORC_RSQRT2)) - 0.5 * erfc(zb * ORC_RSQRT2);
  if (g < 0.0) g = 0.0;
  if (g > 1.0) g = 1.0;
  return g;
}

/*
 * min / max over m in [mlo, mhi] of the cell mass g(m) (Def. 3.1 min/max over
 * the source partition, specialised to one dimension).  g is unimodal in m
 * with its peak at the cell midpoint, so the minimum is at an end of the
 * interval and the maximum at the midpoint clamped into the interval.
 */
void orc_factor_bounds(double a, double b, double mlo, double mhi, double sigma,
                       double *flo, double *fhi) {
  double g1 = orc_gauss_cell_mass(a, b, mlo, sigma);
  double g2 = orc_gauss_cell_mass(a, b, mhi, sigma);
  double lo = g1 < g2 ? g1 : g2;
  double mid = 0.5 * (a + b);
  double mc = mid < mlo ? mlo : (mid > mhi ? mhi : mid);
  double hi = orc_gauss_cell_mass(a, b, mc, sigma);
  if (hi < lo) hi = lo;
  *flo = lo;
  *fhi = hi;
}

/* P(m + w outside [lb, ub]) for one dimension. */
double orc_exit_prob(double lb, double ub, double m, double sigma) {
  double q = 0.5 * erfc(((m - lb) / sigma) * ORC_RSQRT2) +
             0.5 * erfc(((ub - m) / sigma) * ORC_RSQRT2);
  return q > 1.0 ? 1.0 : q;
}

/* P(m + w outside [A, B]) where a missing side (has_a/has_b == 0) is open. */
static double window_exit_prob(double A, int has_a, double B, int has_b, double m,
                               double sigma) {
  double q = 0.0;
  if (has_a) q += 0.5 * erfc(((m - A) / sigma) * ORC_RSQRT2);
  if (has_b) q += 0.5 * erfc(((B - m) / sigma) * ORC_RSQRT2);
  return q > 1.0 ? 1.0 : q;
}

/* ------------------------------------------------------------------------- */
/* One row (s, u) of the abstraction (Alg. 2 loop body).                      */
/* ------------------------------------------------------------------------- */
typedef struct {
  double mlo[ORC_MAX_DIM], mhi[ORC_MAX_DIM];
  int64_t klo[ORC_MAX_DIM], W[ORC_MAX_DIM];
  double out_lo, out_hi, tail_lo, tail_hi;
  int64_t n_cells;
} row_geom;

/*
 * Target window per dimension: the cells that meet [mlo - k sigma, mhi + k
 * sigma], clipped to the grid (reading: the +-k sigma restriction; the mass
 * outside it is accounted by the TAIL entry, so the choice never affects
 * soundness).  k_sigma == 0 selects every cell (dense rows, no TAIL).
 */
static void row_window(const orc_grid *g, const double *sigma, double k_sigma,
                       row_geom *r) {
  r->n_cells = 1;
  for (int i = 0; i < g->dim; ++i) {
    int64_t n = g->n[i];
    if (k_sigma <= 0.0) {
      r->klo[i] = 0;
      r->W[i] = n;
    } else {
      double w = (g->ub[i] - g->lb[i]) / (double)n;
      double ks = k_sigma * sigma[i];
      double tl = ((r->mlo[i] - ks) - g->lb[i]) / w;
      double th = ((r->mhi[i] + ks) - g->lb[i]) / w;
      if (th < 0.0 || tl >= (double)n) {
        r->klo[i] = 0;
        r->W[i] = 0;
      } else {
        int64_t klo = tl <= 0.0 ? 0 : (int64_t)floor(tl);
        int64_t khi = th >= (double)n ? n - 1 : (int64_t)floor(th);
        if (khi > n - 1) khi = n - 1;
        r->klo[i] = klo;
        r->W[i] = khi - klo + 1;
      }
    }
    r->n_cells *= r->W[i];
  }
}

/*
 * OUT entry (Remark 4.1): mass leaving [lb, ub].  With independent noise the
 * in-domain mass is prod_i (1 - q_i(m_i)), q_i the per-dimension exit
 * probability, which is largest at the end of [mlo_i, mhi_i] and smallest at
 * the domain centre clamped into it.  OUT_lo = 1 - max in-domain mass,
 * OUT_hi = 1 - min in-domain mass, evaluated as -expm1(sum log1p(-q)).
 *
 * TAIL entry (reading for the +-k sigma window): an upper bound on the
 * in-domain mass that lands outside the window, the probability of leaving the
 * window box (open on sides where it reaches the domain edge) in some
 * dimension, maximised over the mean box, and never above 1 - OUT_lo.
 * Its lower bound is 0.
 */
static void row_out_tail(const orc_grid *g, const double *sigma, double k_sigma,
                         row_geom *r) {
  double smin = 0.0, smax = 0.0, stail = 0.0;
  for (int i = 0; i < g->dim; ++i) {
    double lb = g->lb[i], ub = g->ub[i];
    double qa = orc_exit_prob(lb, ub, r->mlo[i], sigma[i]);
    double qb = orc_exit_prob(lb, ub, r->mhi[i], sigma[i]);
    double qmax = qa > qb ? qa : qb;
    double ctr = 0.5 * (lb + ub);
    double mc = ctr < r->mlo[i] ? r->mlo[i] : (ctr > r->mhi[i] ? r->mhi[i] : ctr);
    double qmin = orc_exit_prob(lb, ub, mc, sigma[i]);
    if (qmin > qmax) qmin = qmax;
    smin += log1p(-qmin);
    smax += log1p(-qmax);
    if (k_sigma > 0.0) {
      double p;
      if (r->W[i] == 0) {
        p = 1.0;
      } else {
        int64_t khi = r->klo[i] + r->W[i] - 1;
        int has_a = r->klo[i] > 0, has_b = khi < g->n[i] - 1;
        double A = orc_cell_edge(g, i, r->klo[i]);
        double B = orc_cell_edge(g, i, khi + 1);
        double pa = window_exit_prob(A, has_a, B, has_b, r->mlo[i], sigma[i]);
        double pb = window_exit_prob(A, has_a, B, has_b, r->mhi[i], sigma[i]);
        p = pa > pb ? pa : pb;
      }
      stail += log1p(-p);
    }
  }
  r->out_lo = -expm1(smin);
  r->out_hi = -expm1(smax);
  r->tail_lo = 0.0;
  r->tail_hi = 0.0;
  if (k_sigma > 0.0) {
    double t = -expm1(stail);
    double cap = 1.0 - r->out_lo;
    if (t > cap) t = cap;
    if (t < 0.0) t = 0.0;
    r->tail_hi = t;
  }
}

static int row_geometry(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
                        const double *sigma, double k_sigma, int64_t row,
                        row_geom *r) {
  int64_t s = row / in->count;
  int32_t u = (int32_t)(row % in->count);
  if (orc_mean_box(sys, g, in, s, u, r->mlo, r->mhi) != 0) return -1;
  row_window(g, sigma, k_sigma, r);
  row_out_tail(g, sigma, k_sigma, r);
  return 0;
}

/*
 * Entry bounds of the window cells (Def. 3.1; Alg. 2 steps computing T_min and
 * T_max).  Transition mass to a box cell is the product of per-dimension masses,
 * each depending on its own mean coordinate only; the coordinates vary
 * independently over the mean box and the factors are non-negative, so the
 * min (max) of the product is the product of per-dimension mins (maxes).
 * Cells are listed in C order over the window (last dimension fastest),
 * followed by OUT and, in windowed mode, TAIL.
 */
static void row_entries(const orc_grid *g, const double *sigma, const row_geom *r,
                        int windowed, int32_t *target, double *lo, double *hi) {
  int d = g->dim;
  double *flo[ORC_MAX_DIM], *fhi[ORC_MAX_DIM];
  for (int i = 0; i < d; ++i) {
    flo[i] = (double *)malloc(sizeof(double) * (size_t)(r->W[i] > 0 ? r->W[i] : 1));
    fhi[i] = (double *)malloc(sizeof(double) * (size_t)(r->W[i] > 0 ? r->W[i] : 1));
    for (int64_t j = 0; j < r->W[i]; ++j) {
      int64_t k = r->klo[i] + j;
      orc_factor_bounds(orc_cell_edge(g, i, k), orc_cell_edge(g, i, k + 1), r->mlo[i],
                        r->mhi[i], sigma[i], &flo[i][j], &fhi[i][j]);
    }
  }
  int64_t stride[ORC_MAX_DIM];
  stride[d - 1] = 1;
  for (int i = d - 2; i >= 0; --i) stride[i] = stride[i + 1] * g->n[i + 1];
  for (int64_t slot = 0; slot < r->n_cells; ++slot) {
    int64_t rem = slot, t = 0;
    int64_t j[ORC_MAX_DIM];
    for (int i = d - 1; i >= 0; --i) {
      j[i] = rem % r->W[i];
      rem /= r->W[i];
    }
    double plo = 1.0, phi = 1.0;
    for (int i = 0; i < d; ++i) {
      plo *= flo[i][j[i]];
      phi *= fhi[i][j[i]];
      t += (r->klo[i] + j[i]) * stride[i];
    }
    target[slot] = (int32_t)t;
    lo[slot] = plo;
    hi[slot] = phi;
  }
  int64_t e = r->n_cells;
  target[e] = ORC_T_OUT;
  lo[e] = r->out_lo;
  hi[e] = r->out_hi;
  if (windowed) {
    target[e + 1] = ORC_T_TAIL;
    lo[e + 1] = r->tail_lo;
    hi[e + 1] = r->tail_hi;
  }
  for (int i = 0; i < d; ++i) {
    free(flo[i]);
    free(fhi[i]);
  }
}

/*
 * Build the abstraction for the listed rows (rows == NULL: every row
 * s * n_inputs + u in order).  Alg. 1 / Alg. 2 with the closed-form bounds
 * above in place of a numerical optimiser; target/avoid aggregation is done
 * at iteration time from labels (Section 3.1), so the rows do not depend on
 * the specification.
 */
int orc_build(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
              const double *sigma, double k_sigma, const int64_t *rows,
              int64_t n_rows, orc_imdp *out) {
  memset(out, 0, sizeof(*out));
  int d = g->dim;
  if (d < 1 || d > ORC_MAX_DIM || in->count < 1) return -1;
  int64_t n_states = 1;
  for (int i = 0; i < d; ++i) n_states *= g->n[i];
  int64_t total_rows = n_states * in->count;
  if (!rows) n_rows = total_rows;
  int windowed = k_sigma > 0.0;
  out->n_states = n_states;
  out->n_inputs = in->count;
  out->n_rows = n_rows;
  out->dim = d;
  out->windowed = windowed;
  out->win = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows * 2 * d));
  out->ot = (double *)malloc(sizeof(double) * (size_t)(n_rows * 4));
  out->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_rows + 1));
  if (!out->win || !out->ot || !out->row_ptr) return -2;
  row_geom r;
  out->row_ptr[0] = 0;
  for (int64_t q = 0; q < n_rows; ++q) {
    int64_t row = rows ? rows[q] : q;
    if (row < 0 || row >= total_rows) return -1;
    if (row_geometry(sys, g, in, sigma, k_sigma, row, &r) != 0) return -1;
    for (int i = 0; i < d; ++i) {
      out->win[q * 2 * d + i] = (int32_t)r.klo[i];
      out->win[q * 2 * d + d + i] = (int32_t)r.W[i];
    }
    out->ot[q * 4 + 0] = r.out_lo;
    out->ot[q * 4 + 1] = r.out_hi;
    out->ot[q * 4 + 2] = r.tail_lo;
    out->ot[q * 4 + 3] = r.tail_hi;
    out->row_ptr[q + 1] = out->row_ptr[q] + r.n_cells + 1 + windowed;
  }
  int64_t ne = out->row_ptr[n_rows];
  out->n_entries = ne;
  out->target = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
  out->lo = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  out->hi = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  if (!out->target || !out->lo || !out->hi) return -2;
  for (int64_t q = 0; q < n_rows; ++q) {
    int64_t row = rows ? rows[q] : q;
    row_geometry(sys, g, in, sigma, k_sigma, row, &r);
    int64_t b = out->row_ptr[q];
    row_entries(g, sigma, &r, windowed, out->target + b, out->lo + b, out->hi + b);
  }
  return 0;
}

void orc_imdp_free(orc_imdp *m) {
  free(m->win);
  free(m->ot);
  free(m->row_ptr);
  free(m->target);
  free(m->lo);
  free(m->hi);
  memset(m, 0, sizeof(*m));
}

/* ------------------------------------------------------------------------- */
/* Labels (Section 3.1; the representative point is the cell centre, Alg. 2). */
/* A cell is AVOID if its centre lies in a closed avoid box, else TARGET if in */
/* a target box, else SAFE; the boxes are widened by 1e-9 cell widths.         */
/* Box layout: [n][2][dim] -> lo = box[b*2*dim + i], hi = box[b*2*dim+dim+i]. */
/* ------------------------------------------------------------------------- */
static int centre_in_box(const orc_grid *g, const int64_t *k, const double *box) {
  int d = g->dim;
  for (int i = 0; i < d; ++i) {
    double w = (g->ub[i] - g->lb[i]) / (double)g->n[i];
    double c = g->lb[i] + ((double)k[i] + 0.5) * w;
    double tol = 1e-9 * w;
    if (c < box[i] - tol || c > box[d + i] + tol) return 0;
  }
  return 1;
}

int orc_label(const orc_grid *g, int32_t n_target, const double *target_boxes,
              int32_t n_avoid, const double *avoid_boxes, int8_t *cls) {
  int d = g->dim;
  int64_t n_states = 1;
  for (int i = 0; i < d; ++i) n_states *= g->n[i];
  int64_t k[ORC_MAX_DIM];
  for (int64_t s = 0; s < n_states; ++s) {
    unravel_state(g, s, k);
    int8_t c = ORC_SAFE;
    for (int32_t b = 0; b < n_target; ++b)
      if (centre_in_box(g, k, target_boxes + (int64_t)b * 2 * d)) c = ORC_TARGET;
    for (int32_t b = 0; b < n_avoid; ++b)
      if (centre_in_box(g, k, avoid_boxes + (int64_t)b * 2 * d)) c = ORC_AVOID;
    cls[s] = c;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* LP of eq. (5.1) over one row by the sorting method (Section 6.2): start at */
/* the lower bounds, then hand the remaining mass 1 - sum(lo) to the entries  */
/* in ascending value order (minimising LP) or descending order (maximising   */
/* LP), each up to its upper bound.  Ties are visited in index order.         */
/* ------------------------------------------------------------------------- */
typedef struct {
  double v;
  int64_t i;
} keyed;

static int cmp_asc(const void *a, const void *b) {
  const keyed *x = (const keyed *)a, *y = (const keyed *)b;
  if (x->v < y->v) return -1;
  if (x->v > y->v) return 1;
  return x->i < y->i ? -1 : (x->i > y->i);
}

static int cmp_desc(const void *a, const void *b) {
  const keyed *x = (const keyed *)a, *y = (const keyed *)b;
  if (x->v > y->v) return -1;
  if (x->v < y->v) return 1;
  return x->i < y->i ? -1 : (x->i > y->i);
}

double orc_lp_sorted(int64_t n, const double *lo, const double *hi,
                     const double *val, int32_t maximise, double *p_out) {
  double slo = 0.0;
  for (int64_t j = 0; j < n; ++j) slo += lo[j];
  double r = 1.0 - slo;
  if (r < 0.0) r = 0.0;
  keyed *ord = (keyed *)malloc(sizeof(keyed) * (size_t)(n > 0 ? n : 1));
  double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t j = 0; j < n; ++j) {
    ord[j].v = val[j];
    ord[j].i = j;
    p[j] = lo[j];
  }
  qsort(ord, (size_t)n, sizeof(keyed), maximise ? cmp_desc : cmp_asc);
  for (int64_t t = 0; t < n; ++t) {
    int64_t j = ord[t].i;
    double room = hi[j] - lo[j];
    if (room < 0.0) room = 0.0;
    double delta = room < r ? room : r;
    p[j] += delta;
    r -= delta;
  }
  double q = 0.0;
  for (int64_t j = 0; j < n; ++j) q += p[j] * val[j];
  if (p_out)
    for (int64_t j = 0; j < n; ++j) p_out[j] = p[j];
  free(ord);
  free(p);
  return q;
}

/* ------------------------------------------------------------------------- */
/* Interval iteration (eq. (5.1)/(5.2); Alg. 3 safety, Alg. 4 reach-avoid).   */
/* ------------------------------------------------------------------------- */

/*
 * Value of one entry in the LP objective (delta_1 R + delta_2 A + delta_3 T
 * of eq. (5.1), with the absorbing target / avoid sets of Section 3.1 kept as
 * labelled cells rather than summed rows):
 *   reach, reach-avoid: TARGET 1, AVOID 0, OUT 0, SAFE cell V(t)
 *   safety (reach the unsafe set, Section 5.1): AVOID 1, OUT 1, SAFE cell V(t)
 *   TAIL: 0 in a minimising LP, 1 in a maximising LP (the worst / best value
 *   any cell outside the window can hold).
 */
static double entry_value(int32_t t, const int8_t *cls, const double *V, int spec,
                          int maximise) {
  if (t == ORC_T_OUT) return spec == ORC_SAFETY ? 1.0 : 0.0;
  if (t == ORC_T_TAIL) return maximise ? 1.0 : 0.0;
  if (cls[t] == ORC_SAFE) return V[t];
  if (cls[t] == ORC_TARGET) return 1.0;
  return spec == ORC_SAFETY ? 1.0 : 0.0; /* AVOID */
}

static double row_lp(const int64_t *row_ptr, const int32_t *target, const double *lo,
                     const double *hi, const int8_t *cls, const double *V, int spec,
                     int maximise, int64_t row, double *val_buf) {
  int64_t b = row_ptr[row], e = row_ptr[row + 1];
  for (int64_t j = b; j < e; ++j)
    val_buf[j - b] = entry_value(target[j], cls, V, spec, maximise);
  return orc_lp_sorted(e - b, lo + b, hi + b, val_buf, maximise, 0);
}

/* Value of input u at state s against the disturbance player (eq. (5.1): the
   inner optimisation over w-hat): the worst of the n_dist rows (s, u, w) --
   the lowest satisfaction probability for reach, the highest probability of
   the bad set for safety.  Rows of (s, u) are (s * n_inputs + u) * n_dist + w. */
static double input_value(const int64_t *row_ptr, const int32_t *target, const double *lo,
                          const double *hi, const int8_t *cls, const double *V, int spec,
                          int maximise, int64_t s, int32_t u, int32_t n_inputs,
                          int32_t n_dist, double *val_buf) {
  int reach = spec != ORC_SAFETY;
  double worst = 0.0;
  for (int32_t w = 0; w < n_dist; ++w) {
    int64_t r = (s * n_inputs + u) * (int64_t)n_dist + w;
    double q = row_lp(row_ptr, target, lo, hi, cls, V, spec, maximise, r, val_buf);
    if (w == 0 || (reach ? q < worst : q > worst)) worst = q;
  }
  return worst;
}

static double max_gap(int64_t n, const int8_t *cls, const double *V0, const double *V1) {
  double gmax = 0.0;
  for (int64_t s = 0; s < n; ++s)
    if (cls[s] == ORC_SAFE && V1[s] - V0[s] > gmax) gmax = V1[s] - V0[s];
  return gmax;
}

/*
 * Pessimistic synthesis.  Pass 1 (policy): V0 = 0, V1 = 1 on S; Jacobi sweeps
 * V' = opt_u LP(V); reach-avoid / reach use the minimising LP and max over u
 * (Alg. 4), safety the maximising LP and min over u (Alg. 3); pi(s) is the
 * optimising u of the V0 results of each sweep (lowest u on exact ties).
 * Pass 2: reset V0 = 0, V1 = 1, fix u = pi(s), opposite LP direction.  Each
 * pass runs while max_S (V1 - V0) > eps, checked before every sweep, and at
 * most max_sweeps sweeps (reading: a cap, since the paper's loop need not
 * terminate when bounds cannot meet, Remark 5.2).
 * Outputs (reading: the sound outer pair):
 *   reach, reach-avoid: lo = V0 of pass 1, hi = V1 of pass 2;
 *   safety: lo = 1 - V1 of pass 1, hi = 1 - V0 of pass 2;
 *   TARGET cells lo = hi = 1; AVOID cells lo = hi = 0; policy -1 off S.
 * Finite horizon (Remark 5.1, horizon = T > 0): the while loops become for
 * loops, so each pass runs exactly T sweeps with no stop test (none without
 * SAFE states), and interval iteration reduces to value iteration: both
 * bounds come from the V0 iterate, which after k sweeps is the k-step value
 * from V0 = 0 (reach: lo = V0 of the adversarial pass, hi = V0 of the
 * favourable one; safety: 1 - V0 of each).  The policy is the optimising
 * input of the last pass-1 sweep (the first decision of the T-step game),
 * held fixed for pass 2, as above.
 * self_stop (Remark 5.2, with horizon = 0): each pass instead stops once both
 * of its iterates converge to themselves, max_S max(|V0' - V0|, |V1' - V1|)
 * <= eps after a sweep (at least one sweep when S is not empty; at most
 * max_sweeps); info->gap then holds that last move.
 * n_dist >= 1 disturbances (eq. (5.1)): each (s, u) has n_dist rows and is
 * valued by its worst one (the disturbance is always an adversary), in both
 * passes; the policy chooses u only.
 * Returns 0 if both passes met eps (or ran their T sweeps), 1 if a cap
 * fired, < 0 on bad input.
 */
int orc_iterate(int64_t n_states, int32_t n_inputs, const int64_t *row_ptr,
                const int32_t *target, const double *lo, const double *hi,
                const int8_t *cls, int32_t spec_kind, double eps,
                int64_t max_sweeps, double *out_lo, double *out_hi,
                int32_t *policy, orc_iter_info *info, double *q0_last,
                int64_t hist_cap, double *hist_v0, double *hist_v1,
                int32_t optimistic, int64_t horizon, int32_t self_stop, int32_t n_dist) {
  if (n_inputs < 1 || n_dist < 1 || max_sweeps < 1 || !(eps > 0.0) || horizon < 0) return -1;
  if (self_stop && horizon > 0) return -1;
  int64_t n_safe = 0, max_len = 1;
  for (int64_t s = 0; s < n_states; ++s) {
    if (spec_kind == ORC_SAFETY && cls[s] == ORC_TARGET) return -1;
    if (cls[s] != ORC_SAFE) continue;
    ++n_safe;
    for (int64_t k = 0; k < (int64_t)n_inputs * n_dist; ++k) {
      int64_t r = s * n_inputs * (int64_t)n_dist + k;
      if (row_ptr[r + 1] - row_ptr[r] > max_len) max_len = row_ptr[r + 1] - row_ptr[r];
    }
  }
  double *V0 = (double *)calloc((size_t)n_states, sizeof(double));
  double *V1 = (double *)calloc((size_t)n_states, sizeof(double));
  double *N0 = (double *)calloc((size_t)n_states, sizeof(double));
  double *N1 = (double *)calloc((size_t)n_states, sizeof(double));
  double *vb = (double *)malloc(sizeof(double) * (size_t)max_len);
  int32_t *pi = (int32_t *)calloc((size_t)n_states, sizeof(int32_t));
  int capped = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int reach = spec_kind != ORC_SAFETY;
    /* pessimistic policy (Sec. 5, IMDP_lower = true): pass 1 takes the
       adversarial LP -- reach: min LP, max over u; safety (probability of
       the bad set): max LP, min over u -- and pass 2 the other direction
       with u fixed by pi.  optimistic policy: the passes' LP directions are
       swapped, the policy comes from the favourable LP. */
    int adverse = pass == 0 ? !optimistic : optimistic;
    int maximise = adverse ? !reach : reach;
    for (int64_t s = 0; s < n_states; ++s) {
      V0[s] = 0.0;
      V1[s] = 1.0;
    }
    int64_t sweeps = 0;
    double gap, last_delta = 0.0;
    int converged;
    for (;;) {
      gap = n_safe > 0 ? max_gap(n_states, cls, V0, V1) : 0.0;
      if (self_stop)
        gap = last_delta;
      if (horizon > 0) {
        if (n_safe == 0 || sweeps >= horizon) {
          converged = 1;
          break;
        }
      } else if (self_stop) {
        if (n_safe == 0 || (sweeps > 0 && last_delta <= eps)) {
          converged = 1;
          break;
        }
        if (sweeps >= max_sweeps) {
          converged = 0;
          break;
        }
      } else if (gap <= eps) {
        converged = 1;
        break;
      } else if (sweeps >= max_sweeps) {
        converged = 0;
        break;
      }
      for (int64_t s = 0; s < n_states; ++s) {
        if (cls[s] != ORC_SAFE) continue;
        if (pass == 0) {
          double best0 = 0.0, best1 = 0.0;
          int32_t arg = 0;
          for (int32_t u = 0; u < n_inputs; ++u) {
            double q0 = input_value(row_ptr, target, lo, hi, cls, V0, spec_kind, maximise, s, u,
                                    n_inputs, n_dist, vb);
            double q1 = input_value(row_ptr, target, lo, hi, cls, V1, spec_kind, maximise, s, u,
                                    n_inputs, n_dist, vb);
            if (q0_last) q0_last[s * n_inputs + u] = q0;
            if (u == 0) {
              best0 = q0;
              best1 = q1;
              arg = 0;
              continue;
            }
            if (reach ? (q0 > best0) : (q0 < best0)) {
              best0 = q0;
              arg = u;
            }
            if (reach ? (q1 > best1) : (q1 < best1)) best1 = q1;
          }
          N0[s] = best0;
          N1[s] = best1;
          pi[s] = arg;
        } else {
          N0[s] = input_value(row_ptr, target, lo, hi, cls, V0, spec_kind, maximise, s, pi[s],
                              n_inputs, n_dist, vb);
          N1[s] = input_value(row_ptr, target, lo, hi, cls, V1, spec_kind, maximise, s, pi[s],
                              n_inputs, n_dist, vb);
        }
      }
      double delta = 0.0; /* largest move of either iterate in this sweep */
      for (int64_t s = 0; s < n_states; ++s) {
        if (cls[s] != ORC_SAFE) continue;
        delta = fmax(delta, fmax(fabs(N0[s] - V0[s]), fabs(N1[s] - V1[s])));
        V0[s] = N0[s];
        V1[s] = N1[s];
      }
      last_delta = delta;
      if (pass == 0 && sweeps < hist_cap) {
        if (hist_v0) memcpy(hist_v0 + sweeps * n_states, V0, sizeof(double) * (size_t)n_states);
        if (hist_v1) memcpy(hist_v1 + sweeps * n_states, V1, sizeof(double) * (size_t)n_states);
      }
      ++sweeps;
    }
    if (!converged) capped = 1;
    if (info) {
      info->sweeps[pass] = sweeps;
      info->gap[pass] = gap;
      info->converged[pass] = converged;
      info->n_safe = n_safe;
    }
    /* the adversarial pass bounds the satisfaction probability from below
       (reach: its V0; safety: 1 - V1 of the bad set), the favourable pass
       from above (reach: V1; safety: 1 - V0) */
    for (int64_t s = 0; s < n_states; ++s) {
      double v;
      if (cls[s] == ORC_SAFE && horizon > 0)
        v = reach ? V0[s] : 1.0 - V0[s]; /* value iteration: both from V0 = 0 */
      else if (cls[s] == ORC_SAFE)
        v = adverse ? (reach ? V0[s] : 1.0 - V1[s]) : (reach ? V1[s] : 1.0 - V0[s]);
      else if (cls[s] == ORC_TARGET)
        v = 1.0;
      else
        v = 0.0;
      if (adverse)
        out_lo[s] = v;
      else
        out_hi[s] = v;
      if (pass == 0) policy[s] = cls[s] == ORC_SAFE ? pi[s] : -1;
    }
  }
  free(V0);
  free(V1);
  free(N0);
  free(N1);
  free(vb);
  free(pi);
  return capped;
}

/* ------------------------------------------------------------------------- */
/* Correlated Gaussian noise by Monte Carlo integration (Section 4.1: a full  */
/* covariance given by its inverse and its determinant, cell masses by Monte  */
/* Carlo integration with a user-chosen number of samples).                   */
/*                                                                            */
/* Readings (the section names the integrator, not the bound construction):   */
/*  - the integral over a target cell is the plain Monte Carlo estimate: the   */
/*    density N(y; m, Cov) at the caller's points of [0,1)^d mapped onto the   */
/*    cell, averaged and multiplied by the cell volume; the points are an      */
/*    input, shared by every cell;                                            */
/*  - the min / max over the source cell (Def. 3.1), which the paper hands to  */
/*    a numerical optimiser, is taken over a lattice of G^d candidate means,   */
/*    the centres of a G-per-dimension split of the mean box, each estimate    */
/*    widened by a bound on how far the cell's mass can move between the      */
/*    candidate and any mean of its half-spacing box (orc_mc_shift_bound), so  */
/*    the bounds hold for the whole mean box up to the Monte Carlo error;     */
/*  - the Monte Carlo error is covered by kappa standard errors of each        */
/*    estimate (sample standard deviation / sqrt(N)) on each side;            */
/*  - windows use the marginal standard deviations sqrt(Cov_ii); OUT and TAIL  */
/*    use union bounds over dimensions of the marginal exit masses, which     */
/*    hold for any correlation.                                               */
/* ------------------------------------------------------------------------- */

/*
 * Marginal standard deviations sqrt(Cov_ii) from the inverse covariance:
 * Gauss-Jordan inversion with partial pivoting.  Returns 0, or -1 for a
 * singular matrix or a non-positive diagonal of the inverse.
 */
int orc_marginal_sigma(int d, const double *inv_cov, double *sigma) {
  double a[ORC_MAX_DIM][2 * ORC_MAX_DIM];
  if (d < 1 || d > ORC_MAX_DIM) return -1;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < 2 * d; ++j)
      a[i][j] = j < d ? inv_cov[i * d + j] : (j - d == i ? 1.0 : 0.0);
  for (int col = 0; col < d; ++col) {
    int piv = col;
    for (int r = col + 1; r < d; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (!(fabs(a[piv][col]) > 0.0)) return -1;
    if (piv != col)
      for (int j = 0; j < 2 * d; ++j) {
        double t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    double p = a[col][col];
    for (int j = 0; j < 2 * d; ++j) a[col][j] /= p;
    for (int r = 0; r < d; ++r) {
      if (r == col) continue;
      double f = a[r][col];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * d; ++j) a[r][j] -= f * a[col][j];
    }
  }
  for (int i = 0; i < d; ++i) {
    double v = a[i][d + i];
    if (!(v > 0.0) || !isfinite(v)) return -1;
    sigma[i] = sqrt(v);
  }
  return 0;
}

/* e^T P e, summed as sum_i e_i * (sum_j P_ij e_j), both sums in index order. */
static double quad_form(int d, const double *P, const double *e) {
  double q = 0.0;
  for (int i = 0; i < d; ++i) {
    double t = 0.0;
    for (int j = 0; j < d; ++j) t += P[i * d + j] * e[j];
    q += e[i] * t;
  }
  return q;
}

/*
 * Covering radius of the candidate lattice: with G candidates per dimension at
 * the centres of a G-way split of [mlo, mhi], every mean of the box lies
 * within h_i / 2 of its nearest candidate in each dimension (h_i = (mhi_i -
 * mlo_i) / G).  Returns rho, the largest Mahalanobis length sqrt(e^T P e) over
 * that half-spacing box, attained at one of its corners (a convex form is
 * largest at a vertex).
 */
double orc_mc_cover_radius(int d, const double *inv_cov, const double *mlo, const double *mhi,
                           int G) {
  double half[ORC_MAX_DIM], e[ORC_MAX_DIM];
  for (int i = 0; i < d; ++i) half[i] = 0.5 * ((mhi[i] - mlo[i]) / (double)G);
  double best = 0.0;
  for (int corner = 0; corner < (1 << d); ++corner) {
    for (int i = 0; i < d; ++i) e[i] = (corner >> i) & 1 ? half[i] : -half[i];
    double q = quad_form(d, inv_cov, e);
    if (q > best) best = q;
  }
  return sqrt(best);
}

/*
 * How far the N(m, Cov) mass of a cell of volume vol can move when the mean
 * moves from a candidate by a shift of Mahalanobis length at most rho, with
 * every y - m (y in the cell, m within the candidate's half-spacing box) in
 * the box [zlo, zhi].  Two bounds, the smaller taken:
 *  - total variation: no set's mass moves by more than erf(rho / (2 sqrt 2))
 *    = 2 Phi(rho / 2) - 1 between N(m, Cov) and N(m', Cov);
 *  - the mean-derivative of the cell mass along the shift, integrated over the
 *    cell: |d^T P z| f(z) <= rho r f(z) with r = sqrt(z^T P z) (Cauchy-Schwarz
 *    in the P inner product) and f(z) = norm exp(-r^2 / 2), so the change is
 *    at most vol norm rho g(r_lb), g(r) = r exp(-r^2 / 2) at r >= 1 and
 *    exp(-1/2) below (g's maximum), r_lb = max_i dist(0, [zlo_i, zhi_i]) /
 *    sigma_i a lower bound on r over the box (|z_i| <= sigma_i r).
 */
double orc_mc_shift_bound(int d, const double *sigma, double norm, double rho, double vol,
                          const double *zlo, const double *zhi) {
  double tv = erf((rho * 0.5) * ORC_RSQRT2);
  double r = 0.0;
  for (int i = 0; i < d; ++i) {
    double dist = zlo[i] > 0.0 ? zlo[i] : (zhi[i] < 0.0 ? -zhi[i] : 0.0);
    double t = dist / sigma[i];
    if (t > r) r = t;
  }
  double g = r > 1.0 ? r * exp(-0.5 * (r * r)) : exp(-0.5);
  double lip = ((vol * norm) * rho) * g;
  return lip < tv ? lip : tv;
}

/* 1 / sqrt((2 pi)^d det(Cov)), the Gaussian density's constant. */
static double mc_norm(int d, double det_cov) {
  double t = 1.0;
  for (int i = 0; i < d; ++i) t *= 2.0 * ORC_PI;
  return 1.0 / sqrt(t * det_cov);
}

/*
 * Plain Monte Carlo estimate of the N(m, Cov) mass of the box [a, b]:
 * p = vol * mean_k f(y_k), y_k = a + (b - a) * r_k, f the density, and its
 * standard error vol * s / sqrt(N), s^2 the unbiased sample variance of
 * f(y_k) (0 when N = 1).  Samples are summed in index order.
 */
void orc_mc_cell_estimate(int d, const double *inv_cov, double norm, const double *a,
                          const double *b, const double *m, int64_t n, const double *samples,
                          double *p, double *se) {
  double wd[ORC_MAX_DIM], e[ORC_MAX_DIM];
  double vol = 1.0;
  for (int i = 0; i < d; ++i) {
    wd[i] = b[i] - a[i];
    vol *= wd[i];
  }
  double S = 0.0, S2 = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    for (int i = 0; i < d; ++i) {
      double y = a[i] + wd[i] * samples[k * d + i];
      e[i] = y - m[i];
    }
    double z = norm * exp(-0.5 * quad_form(d, inv_cov, e));
    S += z;
    S2 += z * z;
  }
  double mean = S / (double)n;
  double var = 0.0;
  if (n > 1) {
    var = (S2 - ((double)n * mean) * mean) / (double)(n - 1);
    if (var < 0.0) var = 0.0;
  }
  *p = vol * mean;
  *se = vol * sqrt(var / (double)n);
}

/*
 * OUT and TAIL of one row under correlated noise.  The exit event is the
 * union of the per-dimension exits, each depending on its own mean coordinate
 * and marginal standard deviation only, so
 *   OUT_lo = max_i min over the mean interval of q_i (at the domain centre
 *            clamped into it), OUT_hi = min(1, sum_i max of q_i (at an end));
 * landing in the domain but outside the window needs an exit through an
 * interior side of the window in some dimension, so
 *   TAIL_hi = min(1 - OUT_lo, sum_i max over the mean interval of that exit
 *             mass), TAIL_lo = 0.
 */
static void row_out_tail_union(const orc_grid *g, const double *sigma, double k_sigma,
                               row_geom *r) {
  double out_lo = 0.0, out_hi = 0.0, tail = 0.0;
  for (int i = 0; i < g->dim; ++i) {
    double lb = g->lb[i], ub = g->ub[i];
    double qa = orc_exit_prob(lb, ub, r->mlo[i], sigma[i]);
    double qb = orc_exit_prob(lb, ub, r->mhi[i], sigma[i]);
    double qmax = qa > qb ? qa : qb;
    double ctr = 0.5 * (lb + ub);
    double mc = ctr < r->mlo[i] ? r->mlo[i] : (ctr > r->mhi[i] ? r->mhi[i] : ctr);
    double qmin = orc_exit_prob(lb, ub, mc, sigma[i]);
    if (qmin > qmax) qmin = qmax;
    if (qmin > out_lo) out_lo = qmin;
    out_hi += qmax;
    if (k_sigma > 0.0) {
      double p;
      if (r->W[i] == 0) {
        p = 1.0;
      } else {
        int64_t khi = r->klo[i] + r->W[i] - 1;
        int has_a = r->klo[i] > 0, has_b = khi < g->n[i] - 1;
        double A = orc_cell_edge(g, i, r->klo[i]);
        double B = orc_cell_edge(g, i, khi + 1);
        double pa = window_exit_prob(A, has_a, B, has_b, r->mlo[i], sigma[i]);
        double pb = window_exit_prob(A, has_a, B, has_b, r->mhi[i], sigma[i]);
        p = pa > pb ? pa : pb;
      }
      tail += p;
    }
  }
  if (out_hi > 1.0) out_hi = 1.0;
  r->out_lo = out_lo;
  r->out_hi = out_hi;
  r->tail_lo = 0.0;
  r->tail_hi = 0.0;
  if (k_sigma > 0.0) {
    double cap = 1.0 - out_lo;
    if (tail > cap) tail = cap;
    if (tail < 0.0) tail = 0.0;
    r->tail_hi = tail;
  }
}

/*
 * Entry bounds of one row's window cells under correlated noise: for each
 * cell (C order over the window) the estimate at every candidate mean
 * (C order over the G^d lattice), lo = min(p - kappa se - shift) and
 * hi = max(p + kappa se + shift), shift the candidate's orc_mc_shift_bound,
 * both clamped into [0, 1]; then OUT and,
 * when windowed, TAIL.
 */
static void row_entries_mc(const orc_grid *g, const orc_mc_noise *mc, const double *sigma,
                           const row_geom *r, int windowed, int32_t *target, double *lo,
                           double *hi) {
  int d = g->dim, G = mc->grid_pts;
  double norm = mc_norm(d, mc->det_cov);
  double rho = orc_mc_cover_radius(d, mc->inv_cov, r->mlo, r->mhi, G);
  double h[ORC_MAX_DIM];
  for (int i = 0; i < d; ++i) h[i] = (r->mhi[i] - r->mlo[i]) / (double)G;
  int64_t n_cand = 1;
  for (int i = 0; i < d; ++i) n_cand *= G;
  int64_t stride[ORC_MAX_DIM];
  stride[d - 1] = 1;
  for (int i = d - 2; i >= 0; --i) stride[i] = stride[i + 1] * g->n[i + 1];
  double a[ORC_MAX_DIM], b[ORC_MAX_DIM], m[ORC_MAX_DIM], zlo[ORC_MAX_DIM], zhi[ORC_MAX_DIM];
  for (int64_t slot = 0; slot < r->n_cells; ++slot) {
    int64_t rem = slot, t = 0;
    int64_t j[ORC_MAX_DIM];
    for (int i = d - 1; i >= 0; --i) {
      j[i] = rem % r->W[i];
      rem /= r->W[i];
    }
    for (int i = 0; i < d; ++i) {
      int64_t k = r->klo[i] + j[i];
      a[i] = orc_cell_edge(g, i, k);
      b[i] = orc_cell_edge(g, i, k + 1);
      t += k * stride[i];
    }
    double vol = 1.0;
    for (int i = 0; i < d; ++i) vol *= b[i] - a[i];
    double L = 0.0, U = 0.0;
    for (int64_t c = 0; c < n_cand; ++c) {
      int64_t cr = c;
      for (int i = d - 1; i >= 0; --i) {
        int64_t ci = cr % G;
        cr /= G;
        m[i] = r->mlo[i] + ((double)ci + 0.5) * h[i];
        zlo[i] = a[i] - (m[i] + 0.5 * h[i]);
        zhi[i] = b[i] - (m[i] - 0.5 * h[i]);
      }
      double p, se;
      orc_mc_cell_estimate(d, mc->inv_cov, norm, a, b, m, mc->n_samples, mc->samples, &p, &se);
      double mv = orc_mc_shift_bound(d, sigma, norm, rho, vol, zlo, zhi);
      double l = (p - mc->kappa * se) - mv, u = (p + mc->kappa * se) + mv;
      if (c == 0 || l < L) L = l;
      if (c == 0 || u > U) U = u;
    }
    target[slot] = (int32_t)t;
    lo[slot] = L < 0.0 ? 0.0 : (L > 1.0 ? 1.0 : L);
    hi[slot] = U < 0.0 ? 0.0 : (U > 1.0 ? 1.0 : U);
  }
  int64_t e = r->n_cells;
  target[e] = ORC_T_OUT;
  lo[e] = r->out_lo;
  hi[e] = r->out_hi;
  if (windowed) {
    target[e + 1] = ORC_T_TAIL;
    lo[e + 1] = r->tail_lo;
    hi[e + 1] = r->tail_hi;
  }
}

/*
 * Validation shared by the Monte Carlo build: sizes, samples in [0, 1), a
 * positive determinant that matches the inverse (det(P) * det_cov within
 * 1e-6 of 1, det(P) from the same elimination as the marginals).
 */
static int mc_validate(int d, const orc_mc_noise *mc, double *sigma) {
  if (!mc || !mc->inv_cov || !mc->samples || mc->n_samples < 1 || mc->grid_pts < 1) return -1;
  if (!(mc->det_cov > 0.0) || !isfinite(mc->det_cov) || !(mc->kappa >= 0.0)) return -1;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double x = mc->inv_cov[i * d + j];
      if (!isfinite(x) || x != mc->inv_cov[j * d + i]) return -1;
    }
  for (int64_t k = 0; k < mc->n_samples * d; ++k)
    if (!(mc->samples[k] >= 0.0 && mc->samples[k] < 1.0)) return -1;
  if (orc_marginal_sigma(d, mc->inv_cov, sigma) != 0) return -1;
  /* det(P) by elimination with partial pivoting */
  double a[ORC_MAX_DIM][ORC_MAX_DIM], det = 1.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) a[i][j] = mc->inv_cov[i * d + j];
  for (int col = 0; col < d; ++col) {
    int piv = col;
    for (int r = col + 1; r < d; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < d; ++j) {
        double t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
      det = -det;
    }
    det *= a[col][col];
    for (int r = col + 1; r < d; ++r) {
      double f = a[r][col] / a[col][col];
      for (int j = col; j < d; ++j) a[r][j] -= f * a[col][j];
    }
  }
  if (!(det > 0.0) || fabs(det * mc->det_cov - 1.0) > 1e-6) return -1;
  return 0;
}

/*
 * Build under correlated noise (Section 4.1 full covariance; Alg. 2 loop with
 * Monte Carlo cell masses).  Same row layout as orc_build.  Returns 0, or -1
 * for invalid arguments (see mc_validate), -2 on allocation failure.
 */
int orc_build_mc(const orc_system *sys, const orc_grid *g, const orc_inputs *in,
                 const orc_mc_noise *mc, double k_sigma, const int64_t *rows,
                 int64_t n_rows, orc_imdp *out) {
  memset(out, 0, sizeof(*out));
  int d = g->dim;
  if (d < 1 || d > ORC_MAX_DIM || in->count < 1) return -1;
  double sigma[ORC_MAX_DIM];
  if (mc_validate(d, mc, sigma) != 0) return -1;
  int64_t n_states = 1;
  for (int i = 0; i < d; ++i) n_states *= g->n[i];
  int64_t total_rows = n_states * in->count;
  if (!rows) n_rows = total_rows;
  int windowed = k_sigma > 0.0;
  out->n_states = n_states;
  out->n_inputs = in->count;
  out->n_rows = n_rows;
  out->dim = d;
  out->windowed = windowed;
  out->win = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows * 2 * d));
  out->ot = (double *)malloc(sizeof(double) * (size_t)(n_rows * 4));
  out->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_rows + 1));
  if (!out->win || !out->ot || !out->row_ptr) return -2;
  row_geom r;
  out->row_ptr[0] = 0;
  for (int64_t q = 0; q < n_rows; ++q) {
    int64_t row = rows ? rows[q] : q;
    if (row < 0 || row >= total_rows) return -1;
    int64_t s = row / in->count;
    int32_t u = (int32_t)(row % in->count);
    if (orc_mean_box(sys, g, in, s, u, r.mlo, r.mhi) != 0) return -1;
    row_window(g, sigma, k_sigma, &r);
    row_out_tail_union(g, sigma, k_sigma, &r);
    for (int i = 0; i < d; ++i) {
      out->win[q * 2 * d + i] = (int32_t)r.klo[i];
      out->win[q * 2 * d + d + i] = (int32_t)r.W[i];
    }
    out->ot[q * 4 + 0] = r.out_lo;
    out->ot[q * 4 + 1] = r.out_hi;
    out->ot[q * 4 + 2] = r.tail_lo;
    out->ot[q * 4 + 3] = r.tail_hi;
    out->row_ptr[q + 1] = out->row_ptr[q] + r.n_cells + 1 + windowed;
  }
  int64_t ne = out->row_ptr[n_rows];
  out->n_entries = ne;
  out->target = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
  out->lo = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  out->hi = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  if (!out->target || !out->lo || !out->hi) return -2;
  for (int64_t q = 0; q < n_rows; ++q) {
    int64_t row = rows ? rows[q] : q;
    int64_t s = row / in->count;
    int32_t u = (int32_t)(row % in->count);
    orc_mean_box(sys, g, in, s, u, r.mlo, r.mhi);
    row_window(g, sigma, k_sigma, &r);
    row_out_tail_union(g, sigma, k_sigma, &r);
    int64_t b = out->row_ptr[q];
    row_entries_mc(g, mc, sigma, &r, windowed, out->target + b, out->lo + b, out->hi + b);
  }
  return 0;
}
