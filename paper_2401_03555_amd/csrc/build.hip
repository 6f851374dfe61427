// build.hip -- abstraction construction kernels (Def. 3.1 bounds built as in
// Alg. 2: one work item per (source cell, input) row).
//
//  k_row_geom : one thread per row -- mean box, per-dimension windows, OUT and
//               TAIL bounds (Remark 4.1), window cell count.
//  k_expand   : one wavefront per row -- per-dimension factor bounds into LDS
//               (or HBM for FACTORS storage), then the entry products
//               lo = prod_i flo_i, hi = prod_i fhi_i over the window in C order,
//               written as coalesced (lo, hi) pairs.
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

__global__ __launch_bounds__(kGeomThreads) void k_row_geom(const SysParams* __restrict__ sp,
                                                           const double* __restrict__ U,
                                                           int64_t n_rows, int32_t* __restrict__ win,
                                                           double4* __restrict__ ot,
                                                           int64_t* __restrict__ cnt,
                                                           int32_t* __restrict__ maxima) {
  const SysParams& p = *sp;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int row_len = 0, fsum = 0;
  if (r < n_rows) {
    const int d = p.d;
    const int64_t s = r / p.nu;
    const int32_t u = (int32_t)(r - s * p.nu);
    double mlo[kMaxDim], mhi[kMaxDim];
    mean_box(p, U, s, u, mlo, mhi);
    int32_t klo[kMaxDim], W[kMaxDim];
    int64_t ncell = 1;
    for (int i = 0; i < d; ++i) {
      window_dim(p, i, mlo[i], mhi[i], &klo[i], &W[i]);
      ncell *= W[i];
      fsum += W[i];
    }
    for (int i = 0; i < d; ++i) {
      win[r * 2 * d + i] = klo[i];
      win[r * 2 * d + d + i] = W[i];
    }
    double4 o;
    out_tail(p, mlo, mhi, klo, W, &o);
    ot[r] = o;
    cnt[r] = ncell;
    int64_t len = ncell + 1 + p.windowed;
    row_len = len > 0x3fffffff ? 0x3fffffff : (int)len;
  }
  row_len = wave_max_i32(row_len);
  fsum = wave_max_i32(fsum);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&maxima[0], row_len);
    atomicMax(&maxima[1], fsum);
  }
}

// Mixed-radix digits of v in the window radices W (last dimension fastest).
__device__ __forceinline__ void unravel(int64_t v, const int32_t* W, int d, int32_t* j) {
  for (int i = d - 1; i >= 0; --i) {
    j[i] = (int32_t)(v % W[i]);
    v /= W[i];
  }
}

__global__ __launch_bounds__(64 * kRowsPerBlock) void k_expand(
    const SysParams* __restrict__ sp, const double* __restrict__ U, int64_t n_rows,
    const int32_t* __restrict__ win, const int64_t* __restrict__ row_off,
    double2* __restrict__ ent, double2* __restrict__ fac, int32_t fs) {
  extern __shared__ double2 sh_fac[];
  const SysParams& p = *sp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + wv;
  const bool live = r < n_rows;
  const int d = p.d;
  double2* f = sh_fac + wv * fs;
  int32_t klo[kMaxDim], W[kMaxDim], fo[kMaxDim];
  int64_t ncell = 0;
  if (live) {
    const int64_t s = r / p.nu;
    const int32_t u = (int32_t)(r - s * p.nu);
    double mlo[kMaxDim], mhi[kMaxDim];
    mean_box(p, U, s, u, mlo, mhi);
    int tot = 0;
    ncell = 1;
    for (int i = 0; i < d; ++i) {
      klo[i] = win[r * 2 * d + i];
      W[i] = win[r * 2 * d + d + i];
      fo[i] = tot;
      tot += W[i];
      ncell *= W[i];
    }
    for (int idx = lane; idx < tot; idx += 64) {
      int i = 0;
      while (i + 1 < d && idx >= fo[i + 1]) ++i;
      const int64_t k = (int64_t)klo[i] + (idx - fo[i]);
      double flo, fhi;
      factor_bounds(cell_edge(p, i, k), cell_edge(p, i, k + 1), mlo[i], mhi[i], p.sigma[i], &flo,
                    &fhi);
      if (fac)
        fac[r * fs + idx] = make_double2(flo, fhi);
      else
        f[idx] = make_double2(flo, fhi);
    }
  }
  __syncthreads();
  if (!live || fac || ncell == 0) return;
  int32_t j[kMaxDim], inc[kMaxDim];
  unravel(lane, W, d, j);
  unravel(64, W, d, inc);
  const int64_t base = row_off[r];
  for (int64_t slot = lane; slot < ncell; slot += 64) {
    double lo = 1.0, hi = 1.0;
    for (int i = 0; i < d; ++i) {
      const double2 fv = f[fo[i] + j[i]];
      lo *= fv.x;
      hi *= fv.y;
    }
    ent[base + slot] = make_double2(lo, hi);
    int carry = 0;
    for (int i = d - 1; i >= 0; --i) {
      j[i] += inc[i] + carry;
      carry = j[i] >= W[i];
      if (carry) j[i] -= W[i];
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
  for (int i = 0; i < d; ++i) {
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
      for (int i = 0; i < d; ++i) {
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

hipError_t launch_row_geom(const SysParams* sys, const double* U, int64_t n_rows, int32_t* win,
                           double4* ot, int64_t* cnt, int32_t* maxima, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  const int64_t blocks = (n_rows + kGeomThreads - 1) / kGeomThreads;
  hipLaunchKernelGGL(k_row_geom, dim3((unsigned)blocks), dim3(kGeomThreads), 0, st, sys, U,
                     n_rows, win, ot, cnt, maxima);
  return hipGetLastError();
}

hipError_t launch_expand(const SysParams* sys, const double* U, int64_t n_rows,
                         const int32_t* win, const int64_t* row_off, double2* ent, double2* fac,
                         int32_t fs, int32_t d, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  const int64_t blocks = (n_rows + kRowsPerBlock - 1) / kRowsPerBlock;
  const size_t lds = fac ? 0 : (size_t)kRowsPerBlock * fs * sizeof(double2);
  hipLaunchKernelGGL(k_expand, dim3((unsigned)blocks), dim3(64 * kRowsPerBlock), lds, st, sys, U,
                     n_rows, win, row_off, ent, fac, fs);
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
