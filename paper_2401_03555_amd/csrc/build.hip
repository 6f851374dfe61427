// build.hip -- abstraction construction kernels (Def. 3.1 bounds built as in
// Alg. 2: one work item per (source cell, input) row).
//
//  k_row_geom : one thread per row -- mean box, per-dimension windows, OUT and
//               TAIL bounds (Remark 4.1), window cell count.
//  k_expand   : tiles of rows -- per-dimension factor bounds from shared edge
//               erfc values (into LDS, or HBM for FACTORS storage), then the
//               entry products lo = prod_i flo_i, hi = prod_i fhi_i over the
//               window in C order, written as coalesced (lo, hi) pairs.
//  k_export   : copies rows out in the ABI row layout.
#include "impact_internal.hpp"

namespace impact {

constexpr int kGeomThreads = 256;
constexpr int kRowsPerBlock = 4;  // one wavefront per row

__device__ __forceinline__ int wave_max_i32(int x) {
  for (int off = 32; off > 0; off >>= 1) {
    int y = __shfl_xor(x, off);
    x = x > y ? x : y;
  }
  return x;
}

__global__ __launch_bounds__(kGeomThreads) void k_row_geom(BuildTable T, int64_t n_rows,
                                                           int32_t* __restrict__ win,
                                                           double4* __restrict__ ot,
                                                           int64_t* __restrict__ cnt,
                                                           int32_t* __restrict__ maxima) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int row_len = 0, fsum = 0, inst = 0;
  if (r < n_rows) {
    inst = T.n == 1 ? 0 : find_base(T.row_base, T.n, r);
    const SysParams& p = T.sys[inst];
    const int d = p.d;
    const int64_t rl = r - p.row_base;
    const int64_t s = rl / p.nu;
    const int32_t u = (int32_t)(rl - s * p.nu);
    double mlo[kMaxDim], mhi[kMaxDim];
    mean_box(p, p.U, s, u, mlo, mhi);
    int32_t klo[kMaxDim], W[kMaxDim];
    int64_t ncell = 1;
    IMPACT_FOR_DIMS(i, d) {
      window_dim(p, i, mlo[i], mhi[i], &klo[i], &W[i]);
      ncell *= W[i];
      fsum += W[i];
    }
    int32_t* wr = win + p.win_base + rl * 2 * d;
    IMPACT_FOR_DIMS(i, d) {
      wr[i] = klo[i];
      wr[d + i] = W[i];
    }
    double4 o;
    if (p.mc)
      out_tail_union(p, mlo, mhi, klo, W, &o);
    else
      out_tail(p, mlo, mhi, klo, W, &o);
    ot[r] = o;
    cnt[r] = ncell;
    const int64_t len = ncell + 1 + p.windowed;
    row_len = len > 0x3fffffff ? 0x3fffffff : (int)len;
  } else {
    inst = T.n - 1;
  }
  // per-instance maxima: one atomic per wavefront when it holds one instance
  const int first = __shfl(inst, 0);
  if (__all(inst == first)) {
    row_len = wave_max_i32(row_len);
    fsum = wave_max_i32(fsum);
    if ((threadIdx.x & 63) == 0) {
      atomicMax(&maxima[2 * inst], row_len);
      atomicMax(&maxima[2 * inst + 1], fsum);
    }
  } else if (r < n_rows) {
    atomicMax(&maxima[2 * inst], row_len);
    atomicMax(&maxima[2 * inst + 1], fsum);
  }
}

// Mixed-radix digits of v in the window radices W (last dimension fastest).
__device__ __forceinline__ void unravel(int64_t v, const int32_t* W, int d, int32_t* j) {
  IMPACT_FOR_DIMS_REV(i, d) {
    j[i] = (int32_t)(v % W[i]);
    v /= W[i];
  }
}

// k_expand: a workgroup takes a tile of B rows.
//   A. one thread per row: mean box (LDS) and the row's window (LDS);
//   B. one thread per (row, dimension, window edge): erfc(|z|/sqrt2) of the
//      edge at both ends of the mean interval, z = (edge - m)/sigma, stored
//      with the sign of z -- every interior edge is shared by two cells;
//   C. one thread per (row, dimension, window cell): the cell mass at each end
//      of the mean interval from its two edges (the same operations as the
//      tail-aware formula), min of the two, and the max at the clamped
//      midpoint (an end value, or a direct evaluation when the midpoint lies
//      inside the interval);
//   D. one wavefront per row: the window's products in C order, coalesced.
// B is chosen by the host so that the tile fits in LDS.
struct ExpandShape {
  int32_t B;        // rows per workgroup
  int32_t es;       // per-row stride of the edge table (>= sum_i (W_i + 1))
  int32_t fs;       // per-row stride of the LDS factor table (>= sum_i W_i)
  int32_t d;        // per-row stride / 2 of the mean-box and window tables
  int32_t with_products;
};

// Byte offsets of the LDS tables of one tile (16-byte aligned).
struct ExpandLayout {
  size_t mb, wn, ev, fv, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline ExpandLayout expand_layout(const ExpandShape& sh) {
  ExpandLayout L;
  L.mb = 0;
  L.wn = align16(L.mb + (size_t)sh.B * 2 * sh.d * sizeof(double));
  L.ev = align16(L.wn + (size_t)sh.B * (2 * sh.d + 1) * sizeof(int32_t));
  L.fv = align16(L.ev + (size_t)sh.B * sh.es * 2 * sizeof(double));
  L.total = align16(L.fv + (sh.with_products ? (size_t)sh.B * sh.fs * 2 * sizeof(double) : 0));
  return L;
}

// erfc(|z|/sqrt2) with the sign of z attached: +e for z > 0, -e for z < 0,
// and 2 (an impossible erfc value) for z == 0, so that the branch of the
// tail-aware formula is recovered exactly.
__device__ __forceinline__ double enc_erfc(double z) {
  if (z == 0.0) return 2.0;
  const double e = erfc(fabs(z) * kRsqrt2);
  return z > 0.0 ? e : -e;
}

__device__ __forceinline__ double dec_erfc(double x) { return x == 2.0 ? 1.0 : fabs(x); }

// Cell mass from the encoded edge values at its two edges (tail-aware form).
__device__ __forceinline__ double mass_from_edges(double ea, double eb) {
  const bool za_nonneg = !signbit(ea);
  const bool zb_nonpos = signbit(eb) || eb == 2.0;
  const double a = dec_erfc(ea), b = dec_erfc(eb);
  double g;
  if (za_nonneg)
    g = 0.5 * (a - b);
  else if (zb_nonpos)
    g = 0.5 * (b - a);
  else
    g = (1.0 - 0.5 * a) - 0.5 * b;
  return g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
}

__global__ __launch_bounds__(256) void k_expand(BuildTable T, int64_t n_rows,
                                                const int32_t* __restrict__ win,
                                                const int64_t* __restrict__ row_off,
                                                double2* __restrict__ ent, double2* __restrict__ fac,
                                                ExpandShape sh) {
  extern __shared__ double4 lds_raw[];
  char* lds = (char*)lds_raw;
  const int B = sh.B, es = sh.es, fs = sh.fs, D = sh.d;
  const int64_t r0 = (int64_t)blockIdx.x * B;
  const int nb = (int)(n_rows - r0 < B ? n_rows - r0 : B);
  const ExpandLayout lay = expand_layout(sh);
  double* mb = (double*)(lds + lay.mb);     // B * 2D: mlo then mhi
  int32_t* wn = (int32_t*)(lds + lay.wn);   // B * (2D + 1): klo, W, instance
  double* ev = (double*)(lds + lay.ev);     // B * es * 2 encoded edge values
  double2* fv = (double2*)(lds + lay.fv);   // B * fs factor bounds (BOUNDS only)

  // A. mean boxes and windows
  for (int r = threadIdx.x; r < nb; r += blockDim.x) {
    const int64_t row = r0 + r;
    const int inst = T.n == 1 ? 0 : find_base(T.row_base, T.n, row);
    const SysParams& p = T.sys[inst];
    const int d = p.d;
    const int64_t rl = row - p.row_base;
    const int64_t s = rl / p.nu;
    const int32_t u = (int32_t)(rl - s * p.nu);
    double mlo[kMaxDim], mhi[kMaxDim];
    mean_box(p, p.U, s, u, mlo, mhi);
    const int32_t* wr = win + p.win_base + rl * 2 * d;
    IMPACT_FOR_DIMS(i, d) {
      mb[r * 2 * D + i] = mlo[i];
      mb[r * 2 * D + D + i] = mhi[i];
      wn[r * (2 * D + 1) + i] = wr[i];
      wn[r * (2 * D + 1) + D + i] = wr[d + i];
    }
    wn[r * (2 * D + 1) + 2 * D] = inst;
  }
  __syncthreads();

  // B. edge values at both ends of the mean interval
  for (int t = threadIdx.x; t < nb * es; t += blockDim.x) {
    const int r = t / es, e = t - r * es;
    const int32_t* w = wn + r * (2 * D + 1);
    const SysParams& p = T.sys[w[2 * D]];
    const int d = p.d;
    int i = -1, j = e, acc = 0;
    IMPACT_FOR_DIMS(ii, d) {
      if (i < 0 && e < acc + w[D + ii] + 1) {
        i = ii;
        j = e - acc;
      }
      acc += w[D + ii] + 1;
    }
    if (i < 0 || w[D + i] == 0) continue;
    const double E = cell_edge(p, i, (int64_t)w[i] + j);
    const double sg = p.sigma[i];
    ev[(r * es + e) * 2 + 0] = enc_erfc((E - mb[r * 2 * D + i]) / sg);
    ev[(r * es + e) * 2 + 1] = enc_erfc((E - mb[r * 2 * D + D + i]) / sg);
  }
  __syncthreads();

  // C. per-dimension factor bounds
  for (int t = threadIdx.x; t < nb * fs; t += blockDim.x) {
    const int r = t / fs, c = t - r * fs;
    const int32_t* w = wn + r * (2 * D + 1);
    const SysParams& p = T.sys[w[2 * D]];
    const int d = p.d;
    int i = -1, j = c, acc = 0, eacc = 0, eo = 0;
    IMPACT_FOR_DIMS(ii, d) {
      if (i < 0 && c < acc + w[D + ii]) {
        i = ii;
        j = c - acc;
        eo = eacc;
      }
      acc += w[D + ii];
      eacc += w[D + ii] + 1;
    }
    if (i < 0) continue;
    const int64_t k = (int64_t)w[i] + j;
    const double* e0 = ev + (r * es + eo + j) * 2;
    const double g1 = mass_from_edges(e0[0], e0[2]);
    const double g2 = mass_from_edges(e0[1], e0[3]);
    const double lo = g1 < g2 ? g1 : g2;
    const double a = cell_edge(p, i, k), b = cell_edge(p, i, k + 1);
    const double mid = 0.5 * (a + b);
    const double mlo = mb[r * 2 * D + i], mhi = mb[r * 2 * D + D + i];
    double hi;
    if (mid < mlo)
      hi = g1;
    else if (mid > mhi)
      hi = g2;
    else
      hi = gauss_mass(a, b, mid, p.sigma[i]);
    if (hi < lo) hi = lo;
    if (fac)
      fac[p.fac_base + (r0 + r - p.row_base) * (int64_t)p.fs + c] = make_double2(lo, hi);
    else
      fv[r * fs + c] = make_double2(lo, hi);
  }
  if (fac) return;
  __syncthreads();

  // D. products, one wavefront per row
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  for (int r = wv; r < nb; r += nwv) {
    const int32_t* w = wn + r * (2 * D + 1);
    const int d = T.sys[w[2 * D]].d;
    int32_t W[kMaxDim], fo[kMaxDim], j[kMaxDim], inc[kMaxDim];
    int64_t ncell = 1;
    int tot = 0;
    IMPACT_FOR_DIMS(i, d) {
      W[i] = w[D + i];
      fo[i] = tot;
      tot += W[i];
      ncell *= W[i];
    }
    if (ncell == 0) continue;
    int64_t a0 = lane, a1 = 64;
    IMPACT_FOR_DIMS_REV(i, d) {
      j[i] = (int32_t)(a0 % W[i]);
      a0 /= W[i];
      inc[i] = (int32_t)(a1 % W[i]);
      a1 /= W[i];
    }
    const double2* f = fv + r * fs;
    const int64_t base = row_off[r0 + r];
    for (int64_t slot = lane; slot < ncell; slot += 64) {
      double lo = 1.0, hi = 1.0;
      IMPACT_FOR_DIMS(i, d) {
        const double2 x = f[fo[i] + j[i]];
        lo *= x.x;
        hi *= x.y;
      }
      ent[base + slot] = make_double2(lo, hi);
      int carry = 0;
      IMPACT_FOR_DIMS_REV(i, d) {
        j[i] += inc[i] + carry;
        carry = j[i] >= W[i];
        if (carry) j[i] -= W[i];
      }
    }
  }
}

__global__ __launch_bounds__(64 * kRowsPerBlock) void k_export(
    int64_t row0, int64_t nrows, const int32_t* __restrict__ win, const double4* __restrict__ ot,
    const int64_t* __restrict__ row_off, const double2* __restrict__ ent,
    const double2* __restrict__ fac, int32_t fs, int32_t d, int32_t* __restrict__ win_out,
    double* __restrict__ ot_out, int64_t* __restrict__ counts_out,
    double* __restrict__ entries_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * kRowsPerBlock + wv;
  if (q >= nrows) return;
  const int64_t r = row0 + q;
  if (lane < 2 * d) win_out[q * 2 * d + lane] = win[r * 2 * d + lane];
  const int64_t ncell = row_off[r + 1] - row_off[r];
  if (lane == 0) {
    const double4 o = ot[r];
    ot_out[q * 4 + 0] = o.x;
    ot_out[q * 4 + 1] = o.y;
    ot_out[q * 4 + 2] = o.z;
    ot_out[q * 4 + 3] = o.w;
    counts_out[q] = ncell;
  }
  if (!entries_out) return;
  const int64_t dst = row_off[r] - row_off[row0];
  int32_t W[kMaxDim], fo[kMaxDim];
  int tot = 0;
  IMPACT_FOR_DIMS(i, d) {
    W[i] = win[r * 2 * d + d + i];
    fo[i] = tot;
    tot += W[i];
  }
  for (int64_t slot = lane; slot < ncell; slot += 64) {
    double2 e;
    if (ent) {
      e = ent[row_off[r] + slot];
    } else {
      int32_t j[kMaxDim];
      unravel(slot, W, d, j);
      double lo = 1.0, hi = 1.0;
      IMPACT_FOR_DIMS(i, d) {
        const double2 fv = fac[r * fs + fo[i] + j[i]];
        lo *= fv.x;
        hi *= fv.y;
      }
      e = make_double2(lo, hi);
    }
    entries_out[2 * (dst + slot)] = e.x;
    entries_out[2 * (dst + slot) + 1] = e.y;
  }
}

hipError_t launch_row_geom(const BuildTable& T, int64_t n_rows, int32_t* win, double4* ot,
                           int64_t* cnt, int32_t* maxima, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  const int64_t blocks = (n_rows + kGeomThreads - 1) / kGeomThreads;
  hipLaunchKernelGGL(k_row_geom, dim3((unsigned)blocks), dim3(kGeomThreads), 0, st, T, n_rows, win,
                     ot, cnt, maxima);
  return hipGetLastError();
}

hipError_t launch_expand(const BuildTable& T, int64_t n_rows, const int32_t* win,
                         const int64_t* row_off, double2* ent, double2* fac, int32_t fs_max,
                         int32_t d_max, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  ExpandShape sh;
  sh.fs = fs_max;
  sh.es = fs_max + d_max;
  sh.d = d_max;
  sh.with_products = fac ? 0 : 1;
  const size_t budget = 48 * 1024;
  int B = 64;
  for (; B > 1; B /= 2) {
    sh.B = B;
    if (expand_layout(sh).total <= budget) break;
  }
  sh.B = B;
  const size_t lds = expand_layout(sh).total;
  const int64_t blocks = (n_rows + B - 1) / B;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)blocks), dim3(256), lds, st, T, n_rows, win, row_off,
                     ent, fac, sh);
  return hipGetLastError();
}

hipError_t launch_export(const SysParams*, int64_t row0, int64_t nrows, const int32_t* win,
                         const double4* ot, const int64_t* row_off, const double2* ent,
                         const double2* fac, int32_t fs, int32_t d, int32_t,
                         int32_t* win_out, double* ot_out, int64_t* counts_out,
                         double* entries_out, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const int64_t blocks = (nrows + kRowsPerBlock - 1) / kRowsPerBlock;
  hipLaunchKernelGGL(k_export, dim3((unsigned)blocks), dim3(64 * kRowsPerBlock), 0, st, row0,
                     nrows, win, ot, row_off, ent, fac, fs, d, win_out, ot_out, counts_out,
                     entries_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (row offsets, SAFE-cell compaction).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t x, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    int64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int64_t* __restrict__ in,
                                                             int64_t* __restrict__ out, int64_t n,
                                                             int64_t* __restrict__ tile_sum) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  const int64_t incl = wave_incl_scan_i64(s, lane);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int64_t excl = incl - s;
  for (int w = 0; w < wv; ++w) excl += wsum[w];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = excl;
    excl += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = excl;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ tile_sum, int64_t ntiles,
                                                   int64_t* __restrict__ total_out) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry_sh;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (int64_t c = 0; c < ntiles; c += 1024) {
    const int64_t i = c + threadIdx.x;
    const int64_t v = i < ntiles ? tile_sum[i] : 0;
    const int64_t incl = wave_incl_scan_i64(v, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int64_t pre = carry_sh;
    for (int w = 0; w < wv; ++w) pre += wsum[w];
    if (i < ntiles) tile_sum[i] = pre + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < 16; ++w) t += wsum[w];
      carry_sh += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *total_out = carry_sh;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n,
                           const int64_t* __restrict__ tile_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                              int64_t tmp_elems, hipStream_t st) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (tmp_elems < ntiles + 1) return hipErrorInvalidValue;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in, out,
                       n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, tmp, ntiles, out + n);
  if (ntiles > 1)
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n,
                       (const int64_t*)tmp);
  return hipGetLastError();
}

}  // namespace impact
