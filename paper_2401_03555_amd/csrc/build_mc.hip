// build_mc.hip -- entry bounds under correlated Gaussian noise (IMPaCT,
// Section 4.1: a full covariance given by its inverse and determinant, cell
// masses by Monte Carlo integration).
//
//  k_mc_entries : one thread per window cell of every row.  For each of the
//                 G^d candidate means (centres of a G-way split of the row's
//                 mean box) the plain Monte Carlo estimate of the cell's mass,
//                 vol * mean_k f(a + (b - a) r_k), over the caller's points r_k
//                 (read with uniform loads: every lane of a wavefront walks the
//                 same sample at the same time), and its standard error; each
//                 estimate is widened by kappa standard errors and by a bound
//                 on how far the mass can move between the candidate and any
//                 mean of its half-spacing box; lo / hi are the min / max over
//                 the candidates, clamped into [0, 1].
//
// The work is FP64 ALU work (one exp per cell, candidate and sample), with no
// reuse across threads beyond the shared sample points, so the kernel is
// bound by the FP64 vector units, not by memory.
#include "impact_internal.hpp"

namespace impact {

constexpr int kMcThreads = 256;

// Row stride of the thread's copy of P: the dimension when it is a template
// argument, else the maximum, so that every index is a compile-time constant
// and the copy stays in registers.
template <int D>
constexpr int mc_stride() {
  return D > 0 ? D : kMaxDim;
}

// e^T P e as sum_i e_i * (sum_j P_ij e_j), both sums in index order.
template <int D>
__device__ __forceinline__ double mc_quad(const double* P, int d, const double* e) {
  constexpr int S = mc_stride<D>();
  double q = 0.0;
  IMPACT_FOR_DIMS(i, d) {
    double t = 0.0;
    IMPACT_FOR_DIMS(j, d) t += P[i * S + j] * e[j];
    q += e[i] * t;
  }
  return q;
}

// Largest sqrt(e^T P e) over the corners e of the half-spacing box +-half.
template <int D>
__device__ __forceinline__ double mc_cover_radius(const double* P, int d, const double* half) {
  double best = 0.0, e[kMaxDim];
  for (int corner = 0; corner < (1 << d); ++corner) {
    IMPACT_FOR_DIMS(i, d) e[i] = (corner >> i) & 1 ? half[i] : -half[i];
    const double q = mc_quad<D>(P, d, e);
    if (q > best) best = q;
  }
  return sqrt(best);
}

// Bound on the change of the cell's mass between the candidate and any mean
// of its half-spacing box: the smaller of the total-variation distance at
// Mahalanobis distance rho, erf(rho / (2 sqrt 2)), and the integrated mean
// derivative vol * norm * rho * g(r_lb), g(r) = r exp(-r^2/2) for r > 1 and
// exp(-1/2) otherwise, r_lb = max_i dist(0, [zlo_i, zhi_i]) / sigma_i.
__device__ __forceinline__ double mc_shift_bound(const SysParams& p, int d, double rho, double vol,
                                                 const double* zlo, const double* zhi) {
  const double tv = erf((rho * 0.5) * kRsqrt2);
  double r = 0.0;
  IMPACT_FOR_DIMS(i, d) {
    const double dist = zlo[i] > 0.0 ? zlo[i] : (zhi[i] < 0.0 ? -zhi[i] : 0.0);
    const double t = dist / p.sigma[i];
    if (t > r) r = t;
  }
  const double g = r > 1.0 ? r * exp(-0.5 * (r * r)) : exp(-0.5);
  const double lip = ((vol * p.mc_norm) * rho) * g;
  return lip < tv ? lip : tv;
}

template <int D>
__global__ __launch_bounds__(kMcThreads) void k_mc_entries(const SysParams* __restrict__ sys,
                                                           int64_t n_rows,
                                                           const int32_t* __restrict__ win,
                                                           const int64_t* __restrict__ row_off,
                                                           double2* __restrict__ ent) {
  const SysParams& p = *sys;
  const int64_t n_ent = row_off[n_rows];
  const int64_t g = (int64_t)blockIdx.x * kMcThreads + threadIdx.x;
  if (g >= n_ent) return;
  const int d = D > 0 ? D : p.d;
  // the row holding entry g: the last r with row_off[r] <= g
  int64_t lo = 0, hi = n_rows - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (row_off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t r = lo;
  const int64_t s = r / p.nu;
  const int32_t u = (int32_t)(r - s * p.nu);
  double mlo[kMaxDim], mhi[kMaxDim];
  mean_box(p, p.U, s, u, mlo, mhi);
  const int32_t* wr = win + r * 2 * d;
  // the cell: C-order digits of the slot over the window (last dimension fastest)
  int64_t rem = g - row_off[r];
  double a[kMaxDim], wd[kMaxDim], b[kMaxDim];
  IMPACT_FOR_DIMS_REV(i, d) {
    const int32_t Wi = wr[d + i];
    const int64_t ji = rem % Wi;
    rem /= Wi;
    const int64_t k = wr[i] + ji;
    a[i] = cell_edge(p, i, k);
    b[i] = cell_edge(p, i, k + 1);
  }
  double vol = 1.0;
  IMPACT_FOR_DIMS(i, d) {
    wd[i] = b[i] - a[i];
    vol *= wd[i];
  }
  constexpr int PS = mc_stride<D>();
  double P[PS * PS];
  IMPACT_FOR_DIMS(i, d) {
    IMPACT_FOR_DIMS(j, d) P[i * PS + j] = p.mc_P[i * d + j];
  }
  const int G = p.mc_grid;
  double h[kMaxDim], half[kMaxDim];
  IMPACT_FOR_DIMS(i, d) {
    h[i] = (mhi[i] - mlo[i]) / (double)G;
    half[i] = 0.5 * h[i];
  }
  const double rho = mc_cover_radius<D>(P, d, half);
  int64_t n_cand = 1;
  IMPACT_FOR_DIMS(i, d) n_cand *= G;
  const int64_t N = p.mc_n;
  const double* __restrict__ X = p.mc_samples;
  const double norm = p.mc_norm, kappa = p.mc_kappa;
  double L = 0.0, U = 0.0;
  for (int64_t c = 0; c < n_cand; ++c) {
    double m[kMaxDim], zlo[kMaxDim], zhi[kMaxDim];
    int64_t cr = c;
    IMPACT_FOR_DIMS_REV(i, d) {
      const int64_t ci = cr % G;
      cr /= G;
      m[i] = mlo[i] + ((double)ci + 0.5) * h[i];
      zlo[i] = a[i] - (m[i] + 0.5 * h[i]);
      zhi[i] = b[i] - (m[i] - 0.5 * h[i]);
    }
    double S = 0.0, S2 = 0.0;
    for (int64_t k = 0; k < N; ++k) {
      double e[kMaxDim];
      IMPACT_FOR_DIMS(i, d) {
        const double y = a[i] + wd[i] * X[k * d + i];
        e[i] = y - m[i];
      }
      const double z = norm * exp(-0.5 * mc_quad<D>(P, d, e));
      S += z;
      S2 += z * z;
    }
    const double mean = S / (double)N;
    double var = 0.0;
    if (N > 1) {
      var = (S2 - ((double)N * mean) * mean) / (double)(N - 1);
      if (var < 0.0) var = 0.0;
    }
    const double est = vol * mean;
    const double se = vol * sqrt(var / (double)N);
    const double mv = mc_shift_bound(p, d, rho, vol, zlo, zhi);
    const double l = (est - kappa * se) - mv, up = (est + kappa * se) + mv;
    if (c == 0 || l < L) L = l;
    if (c == 0 || up > U) U = up;
  }
  ent[g] = make_double2(L < 0.0 ? 0.0 : (L > 1.0 ? 1.0 : L), U < 0.0 ? 0.0 : (U > 1.0 ? 1.0 : U));
}

hipError_t launch_mc_entries(const SysParams* sys, int32_t d, int64_t n_rows, int64_t n_ent,
                             const int32_t* win, const int64_t* row_off, double2* ent,
                             hipStream_t st) {
  if (n_rows == 0 || n_ent == 0) return hipSuccess;
  const int64_t blocks = (n_ent + kMcThreads - 1) / kMcThreads;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  switch (d) {
    case 1: hipLaunchKernelGGL(k_mc_entries<1>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
    case 2: hipLaunchKernelGGL(k_mc_entries<2>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
    case 3: hipLaunchKernelGGL(k_mc_entries<3>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
    case 4: hipLaunchKernelGGL(k_mc_entries<4>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
    case 5: hipLaunchKernelGGL(k_mc_entries<5>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
    default: hipLaunchKernelGGL(k_mc_entries<0>, grid, dim3(kMcThreads), 0, st, sys, n_rows, win, row_off, ent); break;
  }
  return hipGetLastError();
}

}  // namespace impact
