// impact_device.hpp -- device-side definitions shared by the build and sweep
// kernels of the gfx950 IMDP library (IMPaCT, arXiv 2401.03555).
//
// Everything here is FP64 and evaluated in a fixed order with no FMA
// contraction (the library is compiled with -ffp-contract=off), so window
// edges are reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace impact {

constexpr int kMaxDim = 8;
constexpr int kMaxRow = 16384;     // longest row (entries incl. OUT / TAIL)
constexpr int kMaxRowBlock = 4096; // longest row of the multi-query engine
constexpr int kMaxFactors = 1024;  // longest per-row factor list (sum of window widths)

constexpr double kRsqrt2 = 0.70710678118654752440;
constexpr double kPadRel = 0x1p-48;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kPi = 3.141592653589793;
constexpr double kHalfPi = 1.5707963267948966;

// Loops over the dimensions of a system, unrolled to the compile-time maximum
// so that per-dimension arrays are indexed statically and stay in registers.
#define IMPACT_FOR_DIMS(i, d) \
  _Pragma("unroll") for (int i = 0; i < kMaxDim; ++i) if (i < (d))
#define IMPACT_FOR_DIMS_REV(i, d) \
  _Pragma("unroll") for (int i = kMaxDim - 1; i >= 0; --i) if (i < (d))

enum SysKind : int32_t { kAffine = 0, kUnicycle = 1 };
enum CellClass : int8_t { kSafe = 0, kTarget = 1, kAvoid = 2 };

// Dynamics + grid + noise of one system, resident in device memory and read
// with uniform (scalar) loads.
struct SysParams {
  int32_t kind, d, du, nu;
  int32_t windowed, pad0;
  double dt, k_sigma;
  double A[kMaxDim * kMaxDim];
  double B[kMaxDim * kMaxDim];
  double c[kMaxDim];
  double lb[kMaxDim], ub[kMaxDim], w[kMaxDim], sigma[kMaxDim];
  int32_t n[kMaxDim];
  int64_t stride[kMaxDim];  // C-order state strides
  int64_t n_states, n_rows;
  // Placement of this system inside a (possibly multi-system) build.
  const double* U;          // its inputs, nu x du (device)
  int64_t row_base;         // first global row
  int64_t state_base;       // first global state
  int64_t win_base;         // offset of its window table (int32 elements)
  int64_t fac_base;         // offset of its factor table (double2 elements)
  int32_t fs, pad1;         // factor stride (max over its rows of sum_i W_i)
  // Correlated noise with Monte Carlo cell masses (mc = 1); sigma[] then holds
  // the marginal standard deviations sqrt(Cov_ii).
  int32_t mc, mc_grid;      // flag; candidate means per dimension (G)
  int64_t mc_n;             // sample points
  double mc_norm;           // 1 / sqrt((2 pi)^d det Cov)
  double mc_kappa;          // standard errors added on each side
  const double* mc_samples; // mc_n x d points of [0, 1) (device)
  double mc_P[kMaxDim * kMaxDim];  // inverse covariance, row-major (d x d)
};

// Instances of one build: row r belongs to the last i with row_base[i] <= r.
struct BuildTable {
  const SysParams* sys;       // n entries
  const int64_t* row_base;    // n + 1
  const int64_t* state_base;  // n + 1
  int32_t n;
};

__device__ __forceinline__ int find_base(const int64_t* __restrict__ base, int n, int64_t r) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per-iteration-pass control block in device memory (sweep stop test on the
// device; the host only polls it between launch batches).
struct Ctrl {
  unsigned long long gap_bits;  // running max of (V1 - V0) for the sweep in flight
  int32_t done, converged;
  int64_t sweeps, cap;
  double gap, eps;
  int32_t err, pad;
};

__device__ __forceinline__ double cell_edge(const SysParams& p, int i, int64_t k) {
  return k == p.n[i] ? p.ub[i] : p.lb[i] + (double)k * p.w[i];
}

// a + 2*pi*j in [lo, hi] for some integer j?
__device__ __forceinline__ bool lattice_hit(double lo, double hi, double a) {
  double j = ceil((lo - a) / kTwoPi);
  return a + j * kTwoPi <= hi;
}

// Range of the noise-free successor over the source cell (Def. 3.1 min/max
// over the partition), padded outward by 2^-48 * (sum of term magnitudes).
__device__ inline void mean_box(const SysParams& p, const double* __restrict__ U,
                                int64_t s, int32_t u, double* mlo, double* mhi) {
  const int d = p.d;
  double xl[kMaxDim], xh[kMaxDim];
  int64_t rem = s;
  IMPACT_FOR_DIMS_REV(i, d) {
    int64_t k = rem % p.n[i];
    rem /= p.n[i];
    xl[i] = cell_edge(p, i, k);
    xh[i] = cell_edge(p, i, k + 1);
  }
  const double* uv = U + (int64_t)u * p.du;
  if (p.kind == kAffine) {
    IMPACT_FOR_DIMS(i, d) {
      double slo = 0.0, shi = 0.0, mag = 0.0;
      IMPACT_FOR_DIMS(j, d) {
        double a = p.A[i * d + j];
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
      for (int j = 0; j < p.du; ++j) {
        double t = p.B[i * p.du + j] * uv[j];
        bu += t;
        mag += fabs(t);
      }
      mag += fabs(p.c[i]);
      double pad = mag * kPadRel;
      mlo[i] = (slo + bu) + p.c[i] - pad;
      mhi[i] = (shi + bu) + p.c[i] + pad;
    }
  } else {  // unicycle: interval cos / sin over the heading cell
    double v = uv[0], om = uv[1];
    double c1 = cos(xl[2]), c2 = cos(xh[2]);
    double cmin = c1 < c2 ? c1 : c2, cmax = c1 < c2 ? c2 : c1;
    if (lattice_hit(xl[2], xh[2], 0.0)) cmax = 1.0;
    if (lattice_hit(xl[2], xh[2], kPi)) cmin = -1.0;
    double s1 = sin(xl[2]), s2 = sin(xh[2]);
    double smin = s1 < s2 ? s1 : s2, smax = s1 < s2 ? s2 : s1;
    if (lattice_hit(xl[2], xh[2], kHalfPi)) smax = 1.0;
    if (lattice_hit(xl[2], xh[2], -kHalfPi)) smin = -1.0;
    double t = p.dt * v;
    double pad0 = (fmax(fabs(xl[0]), fabs(xh[0])) + fabs(t)) * kPadRel;
    double pad1 = (fmax(fabs(xl[1]), fabs(xh[1])) + fabs(t)) * kPadRel;
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
    double tw = p.dt * om;
    double pad2 = (fmax(fabs(xl[2]), fabs(xh[2])) + fabs(tw)) * kPadRel;
    mlo[2] = xl[2] + tw - pad2;
    mhi[2] = xh[2] + tw + pad2;
  }
}

// N(m, sigma^2) mass of [a, b], tail-aware so that neither term cancels.
__device__ inline double gauss_mass(double a, double b, double m, double sigma) {
  double za = (a - m) / sigma;
  double zb = (b - m) / sigma;
  double g;
  if (za >= 0.0)
    g = 0.5 * (erfc(za * kRsqrt2) - erfc(zb * kRsqrt2));
  else if (zb <= 0.0)
    g = 0.5 * (erfc(-zb * kRsqrt2) - erfc(-za * kRsqrt2));
  else
    g = (1.0 - 0.5 * erfc(-za * kRsqrt2)) - 0.5 * erfc(zb * kRsqrt2);
  return g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
}

// min / max of the cell mass over the mean interval: min at an end, max at the
// cell midpoint clamped into the interval (g is unimodal in m).
__device__ inline void factor_bounds(double a, double b, double mlo, double mhi,
                                     double sigma, double* flo, double* fhi) {
  double g1 = gauss_mass(a, b, mlo, sigma);
  double g2 = gauss_mass(a, b, mhi, sigma);
  double lo = g1 < g2 ? g1 : g2;
  double mid = 0.5 * (a + b);
  double mc = mid < mlo ? mlo : (mid > mhi ? mhi : mid);
  double hi = gauss_mass(a, b, mc, sigma);
  *flo = lo;
  *fhi = hi < lo ? lo : hi;
}

__device__ __forceinline__ double exit_prob(double lb, double ub, double m, double sigma) {
  double q = 0.5 * erfc(((m - lb) / sigma) * kRsqrt2) + 0.5 * erfc(((ub - m) / sigma) * kRsqrt2);
  return q > 1.0 ? 1.0 : q;
}

__device__ __forceinline__ double window_exit_prob(double A, bool has_a, double B, bool has_b,
                                                   double m, double sigma) {
  double q = 0.0;
  if (has_a) q += 0.5 * erfc(((m - A) / sigma) * kRsqrt2);
  if (has_b) q += 0.5 * erfc(((B - m) / sigma) * kRsqrt2);
  return q > 1.0 ? 1.0 : q;
}

// Per-dimension target window: cells meeting [mlo - k sigma, mhi + k sigma].
__device__ inline void window_dim(const SysParams& p, int i, double mlo, double mhi,
                                  int32_t* klo, int32_t* W) {
  const int64_t n = p.n[i];
  if (!p.windowed) {
    *klo = 0;
    *W = (int32_t)n;
    return;
  }
  double ks = p.k_sigma * p.sigma[i];
  double tl = ((mlo - ks) - p.lb[i]) / p.w[i];
  double th = ((mhi + ks) - p.lb[i]) / p.w[i];
  if (th < 0.0 || tl >= (double)n) {
    *klo = 0;
    *W = 0;
    return;
  }
  int64_t lo = tl <= 0.0 ? 0 : (int64_t)floor(tl);
  int64_t hi = th >= (double)n ? n - 1 : (int64_t)floor(th);
  if (hi > n - 1) hi = n - 1;
  *klo = (int32_t)lo;
  *W = (int32_t)(hi - lo + 1);
}

// OUT (Remark 4.1) and TAIL bounds of one row.
__device__ inline void out_tail(const SysParams& p, const double* mlo, const double* mhi,
                                const int32_t* klo, const int32_t* W, double4* ot) {
  double smin = 0.0, smax = 0.0, stail = 0.0;
  IMPACT_FOR_DIMS(i, p.d) {
    double lb = p.lb[i], ub = p.ub[i], sg = p.sigma[i];
    double qa = exit_prob(lb, ub, mlo[i], sg);
    double qb = exit_prob(lb, ub, mhi[i], sg);
    double qmax = qa > qb ? qa : qb;
    double ctr = 0.5 * (lb + ub);
    double mc = ctr < mlo[i] ? mlo[i] : (ctr > mhi[i] ? mhi[i] : ctr);
    double qmin = exit_prob(lb, ub, mc, sg);
    if (qmin > qmax) qmin = qmax;
    smin += log1p(-qmin);
    smax += log1p(-qmax);
    if (p.windowed) {
      double pw;
      if (W[i] == 0) {
        pw = 1.0;
      } else {
        int64_t khi = (int64_t)klo[i] + W[i] - 1;
        bool has_a = klo[i] > 0, has_b = khi < p.n[i] - 1;
        double A = cell_edge(p, i, klo[i]);
        double B = cell_edge(p, i, khi + 1);
        double pa = window_exit_prob(A, has_a, B, has_b, mlo[i], sg);
        double pb = window_exit_prob(A, has_a, B, has_b, mhi[i], sg);
        pw = pa > pb ? pa : pb;
      }
      stail += log1p(-pw);
    }
  }
  double out_lo = -expm1(smin), out_hi = -expm1(smax), tail_hi = 0.0;
  if (p.windowed) {
    double t = -expm1(stail);
    double cap = 1.0 - out_lo;
    if (t > cap) t = cap;
    if (t < 0.0) t = 0.0;
    tail_hi = t;
  }
  *ot = make_double4(out_lo, out_hi, 0.0, tail_hi);
}

// OUT and TAIL bounds of one row under correlated noise: union bounds over
// the dimensions of the marginal exit masses (valid for any correlation).
// OUT_lo = max_i min q_i, OUT_hi = min(1, sum_i max q_i); TAIL_hi =
// min(1 - OUT_lo, sum_i max exit mass through the window's interior sides).
__device__ inline void out_tail_union(const SysParams& p, const double* mlo, const double* mhi,
                                      const int32_t* klo, const int32_t* W, double4* ot) {
  double out_lo = 0.0, out_hi = 0.0, tail = 0.0;
  IMPACT_FOR_DIMS(i, p.d) {
    double lb = p.lb[i], ub = p.ub[i], sg = p.sigma[i];
    double qa = exit_prob(lb, ub, mlo[i], sg);
    double qb = exit_prob(lb, ub, mhi[i], sg);
    double qmax = qa > qb ? qa : qb;
    double ctr = 0.5 * (lb + ub);
    double mc = ctr < mlo[i] ? mlo[i] : (ctr > mhi[i] ? mhi[i] : ctr);
    double qmin = exit_prob(lb, ub, mc, sg);
    if (qmin > qmax) qmin = qmax;
    if (qmin > out_lo) out_lo = qmin;
    out_hi += qmax;
    if (p.windowed) {
      double pw;
      if (W[i] == 0) {
        pw = 1.0;
      } else {
        int64_t khi = (int64_t)klo[i] + W[i] - 1;
        bool has_a = klo[i] > 0, has_b = khi < p.n[i] - 1;
        double A = cell_edge(p, i, klo[i]);
        double B = cell_edge(p, i, khi + 1);
        double pa = window_exit_prob(A, has_a, B, has_b, mlo[i], sg);
        double pb = window_exit_prob(A, has_a, B, has_b, mhi[i], sg);
        pw = pa > pb ? pa : pb;
      }
      tail += pw;
    }
  }
  if (out_hi > 1.0) out_hi = 1.0;
  double tail_hi = 0.0;
  if (p.windowed) {
    double cap = 1.0 - out_lo;
    if (tail > cap) tail = cap;
    if (tail < 0.0) tail = 0.0;
    tail_hi = tail;
  }
  *ot = make_double4(out_lo, out_hi, 0.0, tail_hi);
}

}  // namespace impact
