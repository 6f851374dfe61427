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
#include "build_mc.hpp"

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

// ---------------------------------------------------------------------------
// Factored form.  With y = a + w r_k (w the grid's cell widths) and a
// candidate mean m, the offset is e = delta + s_k, delta = a - m, s_k = w r_k,
// and the density's exponent splits:
//   exp(-e^T P e / 2) = exp(-delta^T P delta / 2) * exp(-delta^T g_k)
//                       * exp(-s_k^T P s_k / 2),       g_k = P s_k,
// where exp(-delta^T g_k) = prod_i exp(-delta_i g_k,i) and delta_i depends on
// the cell's and the candidate's i-th coordinates only.  So per chunk of
// points a row needs the tables T_i[k][t_i G + c_i] = exp(-delta_i g_k,i)
// (W_i G per dimension and point; the point factor A_k = exp(-s_k^T P s_k/2)
// is folded into dimension 0; along the window each table row is a geometric
// progression, two exps per point, dimension and candidate digit), and each
// (cell, candidate, point) costs the products of d table entries instead of
// an exp and a quadratic form.  A
// thread takes a cell and all G^d candidates (their products share prefixes
// over the dimensions).  A row whose cross exponents could overflow (sum over
// dimensions of max |delta_i| max |g_i| above 600) is evaluated directly.
// ---------------------------------------------------------------------------
constexpr int kMcRowThreads = 128;
constexpr int kMcChunk = 32;       // points per table chunk
constexpr int kMcTableMax = 5120;  // doubles of tables per chunk (40 KiB)

// Per point: g_k = P (w r_k) and A_k = exp(-(w r_k)^T P (w r_k) / 2); and per
// dimension max_k |g_k,i|.  One workgroup.
__global__ __launch_bounds__(256) void k_mc_prep(const SysParams* __restrict__ sys,
                                                 double* __restrict__ gA,
                                                 double* __restrict__ gmax) {
  const SysParams& p = *sys;
  const int d = p.d;
  __shared__ double red[256][kMaxDim];
  double mx[kMaxDim];
  IMPACT_FOR_DIMS(i, d) mx[i] = 0.0;
  for (int64_t k = threadIdx.x; k < p.mc_n; k += 256) {
    double sv[kMaxDim];
    IMPACT_FOR_DIMS(i, d) sv[i] = p.w[i] * p.mc_samples[k * d + i];
    double q = 0.0;
    IMPACT_FOR_DIMS(i, d) {
      double t = 0.0;
      IMPACT_FOR_DIMS(j, d) t += p.mc_P[i * d + j] * sv[j];
      gA[k * (d + 1) + i] = t;
      mx[i] = fmax(mx[i], fabs(t));
      q += sv[i] * t;
    }
    gA[k * (d + 1) + d] = exp(-0.5 * q);
  }
  IMPACT_FOR_DIMS(i, d) red[threadIdx.x][i] = mx[i];
  __syncthreads();
  if (threadIdx.x < (unsigned)d) {
    double m = 0.0;
    for (int t = 0; t < 256; ++t) m = fmax(m, red[t][threadIdx.x]);
    gmax[threadIdx.x] = m;
  }
}

// One workgroup per row.  Cells go to the threads in groups of CPT cells per
// thread, so that a group's accumulators (two per cell and candidate) stay in
// registers; the tables are rebuilt per group and chunk of points.
template <int D, int G>
__global__ __launch_bounds__(kMcRowThreads) void k_mc_rows(const SysParams* __restrict__ sys,
                                                           const int32_t* __restrict__ win,
                                                           const int64_t* __restrict__ row_off,
                                                           const double* __restrict__ gA,
                                                           const double* __restrict__ gmax,
                                                           double2* __restrict__ ent) {
  constexpr int C = (D == 1 ? G : D == 2 ? G * G : D == 3 ? G * G * G : D == 4 ? G * G * G * G
                                                                            : G * G * G * G * G);
  constexpr int CPT = C >= 8 ? 1 : 8 / C;  // cells per thread and group
  __shared__ double tab[kMcTableMax];
  const SysParams& p = *sys;
  const int64_t r = blockIdx.x;
  const int64_t base = row_off[r];
  const int64_t n_cells = row_off[r + 1] - base;
  if (n_cells == 0) return;
  const int64_t s = r / p.nu;
  const int32_t u = (int32_t)(r - s * p.nu);
  double mlo[kMaxDim], mhi[kMaxDim];
  mean_box(p, p.U, s, u, mlo, mhi);
  const int32_t* wr = win + r * 2 * D;
  int32_t klo[D], W[D], toff[D];
  double h[D];
  int tot = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    klo[i] = wr[i];
    W[i] = wr[D + i];
    toff[i] = tot;
    tot += W[i] * G;
    h[i] = (mhi[i] - mlo[i]) / (double)G;
  }
  // the cross exponents' bound: max |delta_i| is at the window's far ends
  double bound = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double a0 = cell_edge(p, i, klo[i]), a1 = cell_edge(p, i, klo[i] + W[i] - 1);
    const double m0 = mlo[i] + 0.5 * h[i], m1 = mlo[i] + ((double)(G - 1) + 0.5) * h[i];
    bound += fmax(fabs(a0 - m1), fabs(a1 - m0)) * gmax[i];
  }
  const double norm = p.mc_norm, kappa = p.mc_kappa;
  const int64_t N = p.mc_n;
  const bool factored = bound <= 600.0 && tot * kMcChunk <= kMcTableMax;
  double P[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) P[k] = p.mc_P[k];
  double rho;
  {
    double best = 0.0;
    for (int corner = 0; corner < (1 << D); ++corner) {
      double e[D];
#pragma unroll
      for (int i = 0; i < D; ++i) e[i] = (corner >> i) & 1 ? 0.5 * h[i] : -(0.5 * h[i]);
      double q = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) t += P[i * D + j] * e[j];
        q += e[i] * t;
      }
      if (q > best) best = q;
    }
    rho = sqrt(best);
  }
  constexpr int T = kMcRowThreads;
  const int64_t per_group = (int64_t)T * CPT;
  for (int64_t g0 = 0; g0 < n_cells; g0 += per_group) {
    int32_t tj[CPT][D];
    bool live[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
      const int64_t slot = g0 + (int64_t)e * T + threadIdx.x;
      live[e] = slot < n_cells;
      int64_t rem = live[e] ? slot : 0;
#pragma unroll
      for (int i = D - 1; i >= 0; --i) {
        tj[e][i] = (int32_t)(rem % W[i]);
        rem /= W[i];
      }
    }
    double S[CPT][C], S2[CPT][C];
#pragma unroll
    for (int e = 0; e < CPT; ++e)
#pragma unroll
      for (int c = 0; c < C; ++c) S[e][c] = S2[e][c] = 0.0;
    if (factored) {
      for (int64_t k0 = 0; k0 < N; k0 += kMcChunk) {
        const int K = (int)(N - k0 < kMcChunk ? N - k0 : kMcChunk);
        __syncthreads();  // the previous chunk's readers are done
        // one thread per (point, dimension, candidate digit): along the
        // window, delta_i grows by the cell width w_i, so the row of table
        // entries is a geometric progression from the window's first cell
        for (int e = threadIdx.x; e < K * D * G; e += T) {
          const int k = e / (D * G), rem = e - k * (D * G);
          const int i = rem / G, ci = rem - i * G;
          const double* gk = gA + (k0 + k) * (D + 1);
          const double delta0 = cell_edge(p, i, klo[i]) - (mlo[i] + ((double)ci + 0.5) * h[i]);
          double val = exp(-(delta0 * gk[i]));
          if (i == 0) val *= gk[D];
          const double ratio = exp(-(p.w[i] * gk[i]));
          double* row = tab + k * tot + toff[i] + ci;
          for (int t = 0; t < W[i]; ++t) {
            row[t * G] = val;
            val *= ratio;
          }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
          if (!live[e]) continue;
          for (int k = 0; k < K; ++k) {
            const double* tk = tab + k * tot;
            double pr[C];
#pragma unroll
            for (int c0 = 0; c0 < G; ++c0) pr[c0] = tk[toff[0] + tj[e][0] * G + c0];
            int len = G;
#pragma unroll
            for (int i = 1; i < D; ++i) {
              // extend the products by dimension i (candidate digits, last fastest)
#pragma unroll
              for (int c = C - 1; c >= 0; --c) {
                if (c < len * G) {
                  const int up = c / G, ci = c - up * G;
                  pr[c] = pr[up] * tk[toff[i] + tj[e][i] * G + ci];
                }
              }
              len *= G;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
              S[e][c] += pr[c];
              S2[e][c] = __builtin_fma(pr[c], pr[c], S2[e][c]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
      if (!live[e]) continue;
      double a[D], b[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        a[i] = cell_edge(p, i, klo[i] + tj[e][i]);
        b[i] = cell_edge(p, i, klo[i] + tj[e][i] + 1);
      }
      if (!factored) {
        // direct evaluation (rows whose factored exponents could overflow)
        for (int64_t k = 0; k < N; ++k) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            double ev[D];
            int cr = c;
#pragma unroll
            for (int i = D - 1; i >= 0; --i) {
              const int ci = cr % G;
              cr /= G;
              const double y = a[i] + (b[i] - a[i]) * p.mc_samples[k * D + i];
              ev[i] = y - (mlo[i] + ((double)ci + 0.5) * h[i]);
            }
            double q = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
              double t = 0.0;
#pragma unroll
              for (int j = 0; j < D; ++j) t += P[i * D + j] * ev[j];
              q += ev[i] * t;
            }
            const double z = exp(-0.5 * q);
            S[e][c] += z;
            S2[e][c] += z * z;
          }
        }
      }
      double vol = 1.0;
#pragma unroll
      for (int i = 0; i < D; ++i) vol *= b[i] - a[i];
      double L = 0.0, U = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double m[D], zlo[D], zhi[D], dl[D];
        int cr = c;
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
          const int ci = cr % G;
          cr /= G;
          m[i] = mlo[i] + ((double)ci + 0.5) * h[i];
          zlo[i] = a[i] - (m[i] + 0.5 * h[i]);
          zhi[i] = b[i] - (m[i] - 0.5 * h[i]);
          dl[i] = a[i] - m[i];
        }
        // the candidate's factor exp(-delta^T P delta / 2) and the density's constant
        double f = norm;
        if (factored) {
          double q = 0.0;
#pragma unroll
          for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) t += P[i * D + j] * dl[j];
            q += dl[i] * t;
          }
          f = norm * exp(-0.5 * q);
        }
        const double Sc = f * S[e][c], S2c = (f * f) * S2[e][c];
        const double mean = Sc / (double)N;
        double var = 0.0;
        if (N > 1) {
          var = (S2c - ((double)N * mean) * mean) / (double)(N - 1);
          if (var < 0.0) var = 0.0;
        }
        const double est = vol * mean;
        const double se = vol * sqrt(var / (double)N);
        const double mv = mc_shift_bound(p, D, rho, vol, zlo, zhi);
        const double l = (est - kappa * se) - mv, up = (est + kappa * se) + mv;
        if (c == 0 || l < L) L = l;
        if (c == 0 || up > U) U = up;
      }
      const int64_t slot = g0 + (int64_t)e * T + threadIdx.x;
      ent[base + slot] = make_double2(L < 0.0 ? 0.0 : (L > 1.0 ? 1.0 : L),
                                      U < 0.0 ? 0.0 : (U > 1.0 ? 1.0 : U));
    }
  }
}

// The factored kernel's shapes: at most 16 candidates per cell.
static bool mc_rows_shape(int32_t d, int32_t G) {
  switch (d) {
    case 1: return G <= 4;
    case 2: return G <= 4;
    case 3: return G <= 2;
    case 4: return G <= 2;
    case 5: return G <= 1;
    default: return false;
  }
}

hipError_t launch_mc_rows(const SysParams* sys, int32_t d, int64_t n_rows, int64_t n_ent,
                          const int32_t* win, const int64_t* row_off, double2* ent,
                          hipStream_t st, int32_t G, double* gA, double* gmax) {
  if (n_rows == 0 || n_ent == 0) return hipSuccess;
  if (!mc_rows_shape(d, G)) return launch_mc_entries(sys, d, n_rows, n_ent, win, row_off, ent, st);
  {
    if (n_rows > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mc_prep, dim3(1), dim3(256), 0, st, sys, gA, gmax);
    const dim3 grid((unsigned)n_rows), blk(kMcRowThreads);
#define MCR(DD, GG) \
  hipLaunchKernelGGL((k_mc_rows<DD, GG>), grid, blk, 0, st, sys, win, row_off, gA, gmax, ent)
    switch (d * 16 + G) {
      case 16 + 1: MCR(1, 1); break;
      case 16 + 2: MCR(1, 2); break;
      case 16 + 3: MCR(1, 3); break;
      case 16 + 4: MCR(1, 4); break;
      case 32 + 1: MCR(2, 1); break;
      case 32 + 2: MCR(2, 2); break;
      case 32 + 3: MCR(2, 3); break;
      case 32 + 4: MCR(2, 4); break;
      case 48 + 1: MCR(3, 1); break;
      case 48 + 2: MCR(3, 2); break;
      case 64 + 1: MCR(4, 1); break;
      case 64 + 2: MCR(4, 2); break;
      default: MCR(5, 1); break;
    }
#undef MCR
    return hipGetLastError();
  }
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
