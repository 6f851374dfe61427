// sweep_sel.hip -- interval-iteration sweep for long rows (more than 512
// entries) by selection of the critical value instead of a sort per row.
//
// The sorting method of Section 6.2 hands the free mass r = 1 - sum(lo) to the
// entries of a row in value order (ascending for a minimising LP, descending
// for a maximising one), each up to its width hi - lo, until r runs out.  All
// entries before the one where r runs out receive their full width and all
// entries after it nothing, so the LP value (eq. (5.1)) needs only that
// critical value v*.  For a minimising LP, with F(x) the summed width of the
// entries of value <= x and F<(x) that of the entries of value < x:
//   v* = the smallest entry value with F(v*) > r,
//   q  = sum(lo v) + sum_{v < v*} (hi - lo) v + (r - F<(v*)) v*;
// entries tied at v* share the remainder and the value does not depend on how
// (a maximising LP is the same on negated values).  Every entry value is a
// value of the value vector, so v* is found by bisection over the value vector
// sorted once per sweep (k_vsort_*, of the signed values): about log2(cells) rounds of one compare
// and one masked add per entry.  The first round checks the critical cell of
// the same row in the previous sweep, which most sweeps keep; a hit ends the
// search at once.  The result does not depend on the search path.
//
// OUT and TAIL have the values 0 or 1, the two ends of every order, and are
// handed their share before or after the window cells in closed form.
//
// One workgroup (NW wavefronts) per SAFE state; the state's rows (all inputs
// in the policy pass, the policy's input in the fixed-input pass) are solved
// one after another, each by the whole workgroup with E window cells per
// thread held in registers (width and both values), cell slot e * 64NW + tid.
#include "sweep_common.hpp"

namespace impact {

constexpr int kSortChunk = 2048;  // keys per workgroup of the chunk sort

// Chunk sort of both components of the value vector, times sg (+1, or -1
// for a maximising LP): out[vec * n + i] holds sg * component vec of vin,
// ascending within each chunk of kSortChunk.
__global__ __launch_bounds__(256) void k_vsort_chunk(const Ctrl* __restrict__ c,
                                                     const double2* __restrict__ vin, int64_t n,
                                                     double sg, double* __restrict__ out) {
  if (c && c->done) return;
  __shared__ double s[kSortChunk];
  const int vec = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int i = threadIdx.x; i < kSortChunk; i += 256) {
    const int64_t g = base + i;
    double v = __builtin_inf();
    if (g < n) {
      const double2 x = vin[g];
      v = sg * (vec ? x.y : x.x) + 0.0;
    }
    s[i] = v;
  }
  __syncthreads();
  for (int k = 2; k <= kSortChunk; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kSortChunk / 2; i += 256) {
        const int lo = 2 * i - (i & (j - 1)), hi = lo + j;
        const bool asc = (lo & k) == 0;
        const double x = s[lo], y = s[hi];
        if ((x > y) == asc) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kSortChunk; i += 256) {
    const int64_t g = base + i;
    if (g < n) out[vec * n + g] = s[i];
  }
}

// One merge pass: sorted runs of length L (pairs [2pL, 2pL + L), [2pL + L,
// 2pL + 2L)) into runs of 2L.  Each key finds its place by a binary search in
// the other run; ties keep the first run's keys first.
__global__ __launch_bounds__(256) void k_vsort_merge(const Ctrl* __restrict__ c,
                                                     const double* __restrict__ in, int64_t n,
                                                     int64_t L, double* __restrict__ out) {
  if (c && c->done) return;
  const int vec = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* src = in + vec * n;
  const int64_t start = (i / (2 * L)) * (2 * L);
  const int64_t mid = start + L < n ? start + L : n;
  const int64_t end = start + 2 * L < n ? start + 2 * L : n;
  const double key = src[i];
  int64_t pos;
  if (i < mid) {
    int64_t lo = mid, hi = end;  // keys of the second run below key
    while (lo < hi) {
      const int64_t m = (lo + hi) >> 1;
      if (src[m] < key)
        lo = m + 1;
      else
        hi = m;
    }
    pos = i + (lo - mid);
  } else {
    int64_t lo = start, hi = mid;  // keys of the first run not above key
    while (lo < hi) {
      const int64_t m = (lo + hi) >> 1;
      if (src[m] <= key)
        lo = m + 1;
      else
        hi = m;
    }
    pos = (i - mid) + lo;
  }
  out[vec * n + pos] = key;
}

int value_sort_passes(int64_t n) {
  int p = 0;
  for (int64_t L = kSortChunk; L < n; L <<= 1) ++p;
  return p;
}

hipError_t launch_value_sort(const Ctrl* c, const double2* vin, int64_t n, double sg,
                             double* buf0, double* buf1, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned chunks = (unsigned)((n + kSortChunk - 1) / kSortChunk);
  hipLaunchKernelGGL(k_vsort_chunk, dim3(chunks, 2), dim3(256), 0, st, c, vin, n, sg, buf0);
  double* src = buf0;
  double* dst = buf1;
  for (int64_t L = kSortChunk; L < n; L <<= 1) {
    hipLaunchKernelGGL(k_vsort_merge, dim3((unsigned)((n + 255) / 256), 2), dim3(256), 0, st, c,
                       src, n, L, dst);
    double* t = src;
    src = dst;
    dst = t;
  }
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

constexpr int kTail = 128;  // candidates left for the one-wavefront sort of the search

template <int NW>
struct SelLds {
  double red[2][NW][12];       // block sums, double-buffered
  double2 fac[kMaxFactors];    // the row's factors (FACTORS storage)
  double qb0[kMaxItems], qb1[kMaxItems];
  double2 htau[kMaxItems];     // per row of the state: the hint cells' signed values
  int32_t hok[kMaxItems];      // ... whether the row has hints
  int64_t hbase[kMaxItems];    // ... the offset of its cells
  int32_t hnw[kMaxItems];      // ... and their count
  int32_t hit[2];              // a cell holding the critical value, per vector
  double cx[2][kTail], cw[2][kTail];  // gathered candidates (signed value, width)
  int32_t tcnt[2][NW];         // candidates per wavefront
  double tres[2];              // critical value found by the candidate sort
};

// One reduce-scatter level across lane bit M (32 or 16): lanes where bit M
// is clear keep the first half of the K partial sums and receive their
// partner's copy of it, lanes where it is set the second half.  The gfx950
// lane swaps do the exchange in the VALU: v_permlane32_swap trades the upper
// 32 lanes of its first operand with the lower 32 of its second, and
// v_permlane16_swap the odd 16-lane rows of the first with the even rows of
// the second, so swapping (x[k], x[k + K/2]) leaves every lane its own and
// its partner's copy of the value it keeps.
template <int M>
__device__ __forceinline__ double swap_add(double first, double second) {
  const uint64_t a = dbits(first), b = dbits(second);
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  uint32_t d0, d1, s0, s1;
  if constexpr (M == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
    d0 = l[0]; s0 = l[1]; d1 = h[0]; s1 = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
    d0 = l[0]; s0 = l[1]; d1 = h[0]; s1 = h[1];
  }
  return bitsd(((uint64_t)d1 << 32) | d0) + bitsd(((uint64_t)s1 << 32) | s0);
}

template <int M, int K>
__device__ __forceinline__ void scatter_half(const double (&x)[K], double (&y)[K / 2],
                                             int lane) {
  (void)lane;
#pragma unroll
  for (int k = 0; k < K / 2; ++k) y[k] = swap_add<M>(x[k], x[k + K / 2]);
}

// Sums over the workgroup of K per-thread values, the same on every thread.
// Within a wavefront the K values (padded with zeros to a multiple of 4) are
// reduce-scattered across lane bits 32 and 16, which leaves each 16-lane row
// a quarter of them to sum inside the row; a single value (an integer count)
// takes a plain butterfly.  Every value is added in the same order whatever
// K and its place among them, so a sum formed in the load pass equals the
// same sum formed by the closing pass bit for bit.  Then the wavefronts'
// partials are added in a fixed order.
template <int NW, int K>
__device__ __forceinline__ void block_sums(double (&x)[K], SelLds<NW>& L, int tid, int& par) {
  static_assert(K <= 12, "block_sums holds at most 12 values per wavefront");
  const int lane = tid & 63, wv = tid >> 6;
  if (NW == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = uniform_f64(wave_sum(x[k]));
    return;
  }
  if constexpr (K == 1) {
    x[0] = wave_sum(x[0]);
    if (lane == 0) L.red[par][wv][0] = x[0];
  } else {
    constexpr int P = (K + 3) / 4 * 4;
    double xp[P], h[P / 2], q[P / 4];
#pragma unroll
    for (int k = 0; k < P; ++k) xp[k] = k < K ? x[k] : 0.0;
    scatter_half<32, P>(xp, h, lane);
    scatter_half<16, P / 2>(h, q, lane);
    // the row sums read neighbouring lanes: every lane takes part
#pragma unroll
    for (int k = 0; k < P / 4; ++k) q[k] = group_sum_dpp<16>(q[k]);
    if ((lane & 15) == 0) {
      const int b = ((lane & 32) ? P / 2 : 0) + ((lane & 16) ? P / 4 : 0);
#pragma unroll
      for (int k = 0; k < P / 4; ++k)
        if (b + k < K) L.red[par][wv][b + k] = q[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += L.red[par][w][k];
    x[k] = uniform_f64(s);
  }
  par ^= 1;
}

// The cells of one row as one thread walks them: slot tid, then every 64 NW
// slots.  Holds the slot's window multi-index j, its cell index t, and the
// digits of the stride (last dimension fastest) with the cell-index
// correction of each carry; fo: offsets of the dimensions' factor lists.
struct RowWalk {
  int32_t W[kMaxDim], fo[kMaxDim], j[kMaxDim], dT[kMaxDim], corr[kMaxDim];
  int32_t t, dt;
};

template <int D>
__device__ __forceinline__ void walk_init(const SysParams& p, const int32_t* wr, int d, int tid,
                                          int stride, RowWalk& rw, int& tot) {
  int rem = tid, remT = stride;
  tot = 0;
  rw.t = 0;
  rw.dt = 0;
  IMPACT_FOR_DIMS_REV(i, d) {
    rw.W[i] = wr[d + i];
    const int Wi = rw.W[i] > 0 ? rw.W[i] : 1;
    divmod_small(rem, Wi, rem, rw.j[i]);
    divmod_small(remT, Wi, remT, rw.dT[i]);
  }
  IMPACT_FOR_DIMS(i, d) {
    const int32_t st = (int32_t)p.stride[i];
    rw.t += (wr[i] + rw.j[i]) * st;
    rw.dt += rw.dT[i] * st;
    rw.corr[i] = (i > 0 ? (int32_t)p.stride[i - 1] : 0) - rw.W[i] * st;
    rw.fo[i] = tot;
    tot += rw.W[i];
  }
}

// Next slot of the thread: add the stride's digits with carries.
template <int D>
__device__ __forceinline__ void walk_step(RowWalk& rw, int d) {
  int cy = 0;
  rw.t += rw.dt;
  IMPACT_FOR_DIMS_REV(i, d) {
    const int ji = rw.j[i] + rw.dT[i] + cy;
    cy = ji >= rw.W[i];
    rw.j[i] = cy ? ji - rw.W[i] : ji;
    rw.t += cy ? rw.corr[i] : 0;
  }
}

// Critical values of the vectors not settled by the hint check (found[v]
// false), from the signed values x0, x1 and widths w of the first EC slots of
// every thread (later slots and slots past the row's cells hold width 0 and
// value +inf): tc[v] = the smallest value with F(tc) > r1, fl[v] = F<(tc),
// ql[v] = the summed width * value of the entries below tc.  Bisects over the
// sorted value vector, then stores cells holding the critical values as the
// row's hints for the next sweep.
template <int NW, int EC, int E, int D>
__device__ __forceinline__ void sel_search(const SweepArgs& a, int64_t row, int tid, SelLds<NW>& L,
                                           int& par, const RowWalk& rw0, int nw,
                                           const double (&w)[E], const double (&x0)[E],
                                           const double (&x1)[E], double r1, bool found0,
                                           bool found1, double (&tc)[2], double (&fl)[2],
                                           double (&ql)[2]) {
  constexpr int T = 64 * NW;
  const int64_t N = a.n_cells;
  const double* sv0 = a.vsort;
  const double* sv1 = a.vsort + N;
  // k-th smallest signed value (the sort was of the signed values)
  auto pivot = [&](const double* sv, int64_t k) -> double { return sv[k]; };
  // one pass at pivots (ta, tb): F<, F<= and the width * value below, per vector
  double s[6];
  auto check = [&](double ta, double tb) {
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = 0.0;
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      const bool a_lt = x0[e] < ta, a_le = x0[e] <= ta;
      const bool b_lt = x1[e] < tb, b_le = x1[e] <= tb;
      s[0] += a_lt ? w[e] : 0.0;
      s[1] += a_le ? w[e] : 0.0;
      s[2] += a_lt ? w[e] * x0[e] : 0.0;
      s[3] += b_lt ? w[e] : 0.0;
      s[4] += b_le ? w[e] : 0.0;
      s[5] += b_lt ? w[e] * x1[e] : 0.0;
    }
    block_sums<NW, 6>(s, L, tid, par);
  };

  // Bisection over the sorted values for the vectors still searching: the
  // bracket [lo, hi] of sorted positions holds the smallest k with
  // F(<= sv[k]) > r1 (the largest sorted value counts every entry).  The
  // row's entries in the bracket -- values in (sv[lo - 1], sv[hi]] -- are its
  // candidates, counted every round.  A vector stops when the bracket is one
  // position, when every sorted value in it is the same, or when at most kTail
  // candidates are left: those are gathered into LDS, and one wavefront sorts
  // them and walks their widths from F(<= sv[lo - 1]).
  const int lane = tid & 63, wv = tid >> 6;
  const double* svv[2] = {sv0, sv1};
  const bool found[2] = {found0, found1};
  bool on[2], tail[2] = {false, false};
  int64_t lo[2], hi[2];
  double f_lo[2], n_lo[2], n_hi[2], pv_lo[2], pv_hi[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    on[v] = !found[v];
    lo[v] = 0;
    hi[v] = N - 1;
    f_lo[v] = 0.0;
    n_lo[v] = 0.0;
    pv_lo[v] = -__builtin_inf();
    pv_hi[v] = on[v] ? pivot(svv[v], N - 1) : 0.0;
  }
  {
    // every cell of the row is a candidate at first (slots past the row's
    // cells hold +inf)
    double c[1];
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < EC; ++e) cnt += __popcll(__ballot(x0[e] < __builtin_inf()));
    c[0] = lane == 0 ? (double)cnt : 0.0;
    block_sums<NW, 1>(c, L, tid, par);
    n_hi[0] = n_hi[1] = c[0];
  }
#pragma unroll
  for (int v = 0; v < 2; ++v)
    if (on[v] && n_hi[v] <= kTail) {
      on[v] = false;
      tail[v] = true;
    }
  while (on[0] || on[1]) {
    int64_t m[2];
    double p[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      m[v] = (lo[v] + hi[v]) >> 1;
      p[v] = on[v] ? pivot(svv[v], m[v]) : 0.0;
    }
    double b[4] = {0.0, 0.0, 0.0, 0.0};
    int c0 = 0, c1 = 0;
    if (on[0]) {
#pragma unroll
      for (int e = 0; e < EC; ++e) {
        const bool le = x0[e] <= p[0];
        b[0] += le ? w[e] : 0.0;
        c0 += __popcll(__ballot(le));
      }
    }
    if (on[1]) {
#pragma unroll
      for (int e = 0; e < EC; ++e) {
        const bool le = x1[e] <= p[1];
        b[1] += le ? w[e] : 0.0;
        c1 += __popcll(__ballot(le));
      }
    }
    b[2] = lane == 0 ? (double)c0 : 0.0;
    b[3] = lane == 0 ? (double)c1 : 0.0;
    block_sums<NW, 4>(b, L, tid, par);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (!on[v]) continue;
      if (b[v] > r1) {
        hi[v] = m[v];
        n_hi[v] = b[2 + v];
        pv_hi[v] = p[v];
      } else {
        lo[v] = m[v] + 1;
        f_lo[v] = b[v];
        n_lo[v] = b[2 + v];
        pv_lo[v] = p[v];
      }
      if (lo[v] == hi[v]) {
        on[v] = false;
        tc[v] = pivot(svv[v], lo[v]);
      } else if (pivot(svv[v], lo[v]) == pv_hi[v]) {
        on[v] = false;
        tc[v] = pv_hi[v];  // every sorted value left in the bracket is this one
      } else if (n_hi[v] - n_lo[v] <= kTail) {
        on[v] = false;
        tail[v] = true;
      }
    }
  }
  if (tail[0] || tail[1]) {
    // candidates per wavefront, then each one's place in the LDS list
    auto count = [&](const double(&xv)[E], int v) {
      int cnt = 0;
#pragma unroll
      for (int e = 0; e < EC; ++e)
        cnt += __popcll(__ballot(xv[e] > pv_lo[v] && xv[e] <= pv_hi[v]));
      if (lane == 0) L.tcnt[v][wv] = cnt;
    };
    auto gather = [&](const double(&xv)[E], int v) {
      int base = 0;
      for (int k = 0; k < wv; ++k) base += L.tcnt[v][k];
#pragma unroll
      for (int e = 0; e < EC; ++e) {
        const bool c = xv[e] > pv_lo[v] && xv[e] <= pv_hi[v];
        const uint64_t mk = (uint64_t)__ballot(c);
        const int below = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
        if (c) {
          L.cx[v][base + below] = xv[e];
          L.cw[v][base + below] = w[e];
        }
        base += __popcll(mk);
      }
    };
    if (tail[0]) count(x0, 0);
    if (tail[1]) count(x1, 1);
    __syncthreads();
    if (tail[0]) gather(x0, 0);
    if (tail[1]) gather(x1, 1);
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!tail[v]) continue;
        const int cnt = (int)(n_hi[v] - n_lo[v]);
        uint64_t key[2];
        double ww[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int pos = lane * 2 + k;
          if (pos < cnt) {
            const uint64_t bits = dbits(L.cx[v][pos]);
            key[k] = (bits >> 63) ? ~bits : (bits | (1ull << 63));  // order-preserving
            ww[k] = L.cw[v][pos];
          } else {
            key[k] = ~0ull;
            ww[k] = 0.0;
          }
        }
        bitonic_sort<2, 1, double>(key, ww, lane, nullptr);
        // the first sorted candidate at which F(<= sv[lo - 1]) plus the
        // widths so far exceeds r1
        const double excl = wave_excl_scan(ww[0] + ww[1], lane);
        const double i0 = f_lo[v] + excl + ww[0], i1 = i0 + ww[1];
        const bool h0 = i0 > r1 && 2 * lane < cnt, h1 = i1 > r1 && 2 * lane + 1 < cnt;
        const uint64_t mk = (uint64_t)__ballot(h0 || h1);
        int pos = cnt - 1;  // rounding: the largest candidate
        if (mk) {
          const int ln = __builtin_ctzll(mk);
          pos = 2 * ln + (__shfl((int)h0, ln) ? 0 : 1);
        }
        const uint64_t k0 = (uint64_t)__shfl((long long)key[0], pos >> 1);
        const uint64_t k1 = (uint64_t)__shfl((long long)key[1], pos >> 1);
        const uint64_t kx = (pos & 1) ? k1 : k0;
        const uint64_t bits = (kx >> 63) ? (kx & ~(1ull << 63)) : ~kx;
        if (lane == 0) L.tres[v] = bitsd(bits);
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 2; ++v)
      if (tail[v]) tc[v] = uniform_f64(L.tres[v]);
  }
  check(tc[0], tc[1]);
  if (!found0) {
    fl[0] = s[0];
    ql[0] = s[2];
  }
  if (!found1) {
    fl[1] = s[3];
    ql[1] = s[5];
  }

  // a cell holding each critical value (with positive width), for the next sweep
  if (tid == 0) {
    L.hit[0] = -1;
    L.hit[1] = -1;
  }
  __syncthreads();
  {
    const int d = D > 0 ? D : a.d;
    RowWalk rw = rw0;
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      if (e * T + tid < nw && w[e] > 0.0) {
        if (!found0 && x0[e] == tc[0]) L.hit[0] = rw.t;
        if (!found1 && x1[e] == tc[1]) L.hit[1] = rw.t;
      }
      walk_step<D>(rw, d);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int32_t* hint = a.hint + row * 2;
    if (!found0) hint[0] = L.hit[0];
    if (!found1) hint[1] = L.hit[1];
  }
}

// Both LP values of one row from its first EC slots per thread (see sel_row).
// The load pass also checks the hint values (tau0, tau1): F<, F<= and the
// width * value below each, so that a row whose critical cells did not move
// costs one pass.
template <int NW, int EC, int E, int D, int ST>
__device__ __forceinline__ void sel_row_body(const SweepArgs& a, int64_t row, int tid,
                                             SelLds<NW>& L, int& par, const RowWalk& rw0,
                                             int nw, int64_t base, bool have_hint, double tau0,
                                             double tau1, double& q0, double& q1) {
  constexpr int T = 64 * NW;
  const int d = D > 0 ? D : a.d;
  const bool mx = a.maximise != 0;
  const double sg = mx ? -1.0 : 1.0;
  const bool factors = ST == 0 ? a.storage == IMPACT_STORE_FACTORS : ST == 2;

  // the cells: width and both signed values per slot; loads use a valid
  // address for slots past the row's cells so that none waits on a branch
  double w[E], x0[E], x1[E];
  // sum lo, sum w, lo v0, lo v1, w v0, w v1, then the hint checks of V0 and V1
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  {
    RowWalk rw = rw0;
#pragma unroll
    for (int e = 0; e < EC; ++e) {
      const int slot = e * T + tid;
      const bool ok = slot < nw;
      double lo, hi;
      if (factors) {
        lo = 1.0;
        hi = 1.0;
        IMPACT_FOR_DIMS(i, d) {
          const double2 f = L.fac[rw.fo[i] + (ok ? rw.j[i] : 0)];
          lo *= f.x;
          hi *= f.y;
        }
      } else {
        const double2 b = a.ent[base + (ok ? slot : 0)];
        lo = b.x;
        hi = b.y;
      }
      const double2 V = a.vin[ok ? rw.t : 0];
      lo = ok ? lo : 0.0;
      const double wd = ok ? hi - lo : 0.0;
      w[e] = wd;
      x0[e] = ok ? sg * V.x : __builtin_inf();
      x1[e] = ok ? sg * V.y : __builtin_inf();
      acc[0] += lo;
      acc[1] += wd;
      acc[2] += lo * V.x;
      acc[3] += lo * V.y;
      acc[4] += wd * V.x;
      acc[5] += wd * V.y;
      const bool a_lt = x0[e] < tau0, a_le = x0[e] <= tau0;
      const bool b_lt = x1[e] < tau1, b_le = x1[e] <= tau1;
      acc[6] += a_lt ? wd : 0.0;
      acc[7] += a_le ? wd : 0.0;
      acc[8] += a_lt ? wd * x0[e] : 0.0;
      acc[9] += b_lt ? wd : 0.0;
      acc[10] += b_le ? wd : 0.0;
      acc[11] += b_lt ? wd * x1[e] : 0.0;
      walk_step<D>(rw, d);
    }
  }
  block_sums<NW, 12>(acc, L, tid, par);

  // OUT and TAIL: value out_val and the end value of the order
  const double4 o = a.ot[row];
  const double v_first = mx ? 1.0 : 0.0;  // the value visited first
  const double tail_w = a.windowed ? o.w - o.z : 0.0;
  const double tail_lo = a.windowed ? o.z : 0.0;
  double r = 1.0 - ((acc[0] + o.x) + tail_lo);
  if (r < 0.0) r = 0.0;
  // handed out before the cells: TAIL (value v_first) and OUT if it has
  // that value; OUT otherwise after them
  const bool out_first = a.out_val == v_first;
  double r1 = r, qf = 0.0;
  {
    double dl = tail_w < r1 ? tail_w : r1;
    r1 -= dl;
    qf += dl * v_first;
    if (out_first) {
      const double ow = o.y - o.x;
      dl = ow < r1 ? ow : r1;
      r1 -= dl;
      qf += dl * a.out_val;
    }
  }
  const double base0 = acc[2] + o.x * a.out_val + tail_lo * v_first + qf;
  const double base1 = acc[3] + o.x * a.out_val + tail_lo * v_first + qf;
  const double sw = acc[1];
  if (!(sw > r1)) {
    // every cell gets its full width; what is left goes to OUT if it comes last
    double qlast = 0.0;
    if (!out_first) {
      const double r2 = r1 - sw, ow = o.y - o.x;
      qlast = (ow < r2 ? ow : r2) * a.out_val;
    }
    q0 = base0 + acc[4] + qlast;
    q1 = base1 + acc[5] + qlast;
    return;
  }
  // the hint values are the critical values when F< <= r1 < F<= at them
  const bool found0 = have_hint && acc[6] <= r1 && acc[7] > r1;
  const bool found1 = have_hint && acc[9] <= r1 && acc[10] > r1;
  double tc[2] = {tau0, tau1}, fl[2] = {acc[6], acc[9]}, ql[2] = {acc[8], acc[11]};
  if (!(found0 && found1))
    sel_search<NW, EC, E, D>(a, row, tid, L, par, rw0, nw, w, x0, x1, r1, found0, found1, tc, fl,
                             ql);
  q0 = base0 + sg * (ql[0] + (r1 - fl[0]) * tc[0]);
  q1 = base1 + sg * (ql[1] + (r1 - fl[1]) * tc[1]);
}

// Both LP values (V0 and V1) of one row.  Values are held signed (negated for
// a maximising LP) so that both directions search for the smallest critical
// value in ascending order.  The thread's slots are processed by a body
// unrolled over the smallest of 4, 8, 12 and E slots that covers the row.
// ST: the storage of the bounds, 1 stored, 2 factors, 0 read from the
// arguments (the engine's kernels, whose queries may differ).
template <int NW, int E, int D, int ST>
__device__ __forceinline__ void sel_row(const SweepArgs& a, int64_t row, int tid, SelLds<NW>& L,
                                        int& par, bool have_hint, double tau0, double tau1,
                                        int64_t base, int nw, double& q0, double& q1) {
  constexpr int T = 64 * NW;
  const SysParams& p = *a.sys;
  const int d = D > 0 ? D : a.d;
  const int32_t* wr = a.win + row * 2 * d;
  RowWalk rw;
  int tot;
  walk_init<D>(p, wr, d, tid, T, rw, tot);
  if (ST == 0 ? a.storage == IMPACT_STORE_FACTORS : ST == 2) {
    __syncthreads();  // the previous row's readers are done with L.fac
    const double2* fr = a.fac + row * (int64_t)a.fs;
    for (int k = tid; k < tot; k += T) L.fac[k] = fr[k];
    __syncthreads();
  }
  const int Erow = (nw + T - 1) / T;
  if (Erow == 0)
    sel_row_body<NW, 1, E, D, ST>(a, row, tid, L, par, rw, nw, base, have_hint, tau0, tau1, q0, q1);
  else if (E <= 4 || Erow <= 4)
    sel_row_body<NW, (E < 4 ? E : 4), E, D, ST>(a, row, tid, L, par, rw, nw, base, have_hint, tau0,
                                            tau1, q0, q1);
  else if (E <= 8 || Erow <= 8)
    sel_row_body<NW, (E < 8 ? E : 8), E, D, ST>(a, row, tid, L, par, rw, nw, base, have_hint, tau0,
                                            tau1, q0, q1);
  else if (E <= 12 || Erow <= 12)
    sel_row_body<NW, (E < 12 ? E : 12), E, D, ST>(a, row, tid, L, par, rw, nw, base, have_hint,
                                              tau0, tau1, q0, q1);
  else
    sel_row_body<NW, E, E, D, ST>(a, row, tid, L, par, rw, nw, base, have_hint, tau0, tau1, q0, q1);
}

// One SAFE state s: its rows (all inputs in the policy pass, PASS 0; the
// policy's input in the fixed-input pass, PASS 1) solved one after another by
// the workgroup; writes vout[s] (and pi[s] in the policy pass) and returns
// the state's V1 - V0 on every thread.  With a disturbance player (nw > 1)
// every (state, input) has nw rows and is valued by its worst one (eq. (5.1)).
template <int NW, int E, int PASS, int D, int ST>
__device__ __forceinline__ double sel_state(const SweepArgs& a, int64_t s, SelLds<NW>& L) {
  const int tid = threadIdx.x;
  const int U = PASS == 0 ? a.nu : 1;
  const int NWD = a.nw > 1 ? a.nw : 1;
  const double sg = a.maximise ? -1.0 : 1.0;
  // the previous sweep's critical cells of a row and their values (only the
  // row itself rewrites its hints)
  auto hint_of = [&](int m, bool& ok, double& t0, double& t1) {
    const int ui = m / NWD, wi = m - ui * NWD;
    const int u = PASS == 0 ? ui : a.pi[s];
    const int32_t* hint = a.hint + ((s * a.nu + u) * NWD + wi) * 2;
    const int32_t h0 = hint[0], h1 = hint[1];
    ok = h0 >= 0 && h1 >= 0;
    t0 = ok ? sg * a.vin[h0].x : 0.0;
    t1 = ok ? sg * a.vin[h1].y : 0.0;
  };
  if (PASS == 0) {
    // every row's, read up front: a row's load pass then starts without
    // waiting on the two dependent loads
    for (int m = tid; m < U * NWD; m += 64 * NW) {
      bool ok;
      double t0, t1;
      hint_of(m, ok, t0, t1);
      L.hok[m] = ok;
      L.htau[m] = make_double2(t0, t1);
      const int64_t row = (s * a.nu + m / NWD) * NWD + (m - (m / NWD) * NWD);
      const int64_t b0 = a.row_off[row];
      L.hbase[m] = b0;
      L.hnw[m] = (int)(a.row_off[row + 1] - b0);
    }
    __syncthreads();
  }
  int par = 0;
  for (int m = 0; m < U * NWD; ++m) {
    const int ui = m / NWD, wi = m - ui * NWD;
    const int u = PASS == 0 ? ui : a.pi[s];
    double q0, q1;
    const int64_t row = (s * a.nu + u) * NWD + wi;
    bool ok;
    double t0, t1;
    int64_t base;
    int nw;
    if (PASS == 0) {
      ok = L.hok[m] != 0;
      t0 = L.htau[m].x;
      t1 = L.htau[m].y;
      base = L.hbase[m];
      nw = L.hnw[m];
    } else {
      hint_of(m, ok, t0, t1);
      base = a.row_off[row];
      nw = (int)(a.row_off[row + 1] - base);
    }
    sel_row<NW, E, D, ST>(a, row, tid, L, par, ok, t0, t1, base, nw, q0, q1);
    if (tid == 0) {
      L.qb0[m] = q0;
      L.qb1[m] = q1;
    }
  }
  __syncthreads();
  // an input is worth its worst row over the disturbances: the minimum for
  // reach, the maximum of the bad mass for safety
  auto worst = [&](const double* q, int ui) {
    double v = q[ui * NWD];
    for (int w = 1; w < NWD; ++w) {
      const double x = q[ui * NWD + w];
      v = a.reach ? fmin(v, x) : fmax(v, x);
    }
    return v;
  };
  double b0 = worst(L.qb0, 0), b1 = worst(L.qb1, 0);
  int arg = 0;
  for (int ui = 1; ui < U; ++ui) {
    const double q0 = worst(L.qb0, ui), q1 = worst(L.qb1, ui);
    if (a.reach ? (q0 > b0) : (q0 < b0)) {
      b0 = q0;
      arg = ui;
    }
    if (a.reach ? (q1 > b1) : (q1 < b1)) b1 = q1;
  }
  __syncthreads();  // every thread has read qb before the next state writes it
  if (tid == 0) {
    a.vout[s] = make_double2(b0, b1);
    if (PASS == 0) a.pi[s] = arg;
  }
  const double g = b1 - b0;
  return g > 0.0 ? g : 0.0;
}

// The fixed-input pass without a disturbance player has one row per state:
// a workgroup takes kSelFixedStates states (states[0 .. cnt)), reads their
// rows' hints and offsets up front, and solves the rows one after another;
// each state's V1 - V0 goes to its own partial gap[m].
constexpr int kSelFixedStates = 8;

template <int NW, int E, int D, int ST>
__device__ __forceinline__ void sel_fixed_states(const SweepArgs& a, const int32_t* states,
                                                 double* gap, int cnt, SelLds<NW>& L) {
  const int tid = threadIdx.x;
  const double sg = a.maximise ? -1.0 : 1.0;
  for (int m = tid; m < cnt; m += 64 * NW) {
    const int64_t s = states[m];
    const int64_t row = s * a.nu + a.pi[s];
    const int32_t* hint = a.hint + row * 2;
    const int32_t h0 = hint[0], h1 = hint[1];
    const bool ok = h0 >= 0 && h1 >= 0;
    L.hok[m] = ok;
    L.htau[m] = make_double2(ok ? sg * a.vin[h0].x : 0.0, ok ? sg * a.vin[h1].y : 0.0);
    const int64_t b0 = a.row_off[row];
    L.hbase[m] = b0;
    L.hnw[m] = (int)(a.row_off[row + 1] - b0);
  }
  __syncthreads();
  int par = 0;
  for (int m = 0; m < cnt; ++m) {
    const int64_t s = states[m];
    const int64_t row = s * a.nu + a.pi[s];
    double q0, q1;
    sel_row<NW, E, D, ST>(a, row, tid, L, par, L.hok[m] != 0, L.htau[m].x, L.htau[m].y,
                          L.hbase[m], L.hnw[m], q0, q1);
    if (tid == 0) {
      a.vout[s] = make_double2(q0, q1);
      const double g = q1 - q0;
      gap[m] = g > 0.0 ? g : 0.0;
    }
  }
}

// Two waves per SIMD at least: without the bound the compiler reaches for the
// accumulation registers and leaves one wave per SIMD, which doubles the sweep.
template <int NW, int E, int PASS, int D, int ST>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_sweep_sel(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ SelLds<NW> L;
  if (PASS == 1 && a.nw <= 1) {
    const int64_t s0 = (int64_t)blockIdx.x * kSelFixedStates;
    const int64_t left = a.n_safe - s0;
    sel_fixed_states<NW, E, D, ST>(a, a.safe + s0, a.gap_part + s0,
                                   left < kSelFixedStates ? (int)left : kSelFixedStates, L);
    return;
  }
  const int64_t si = blockIdx.x;
  const double g = sel_state<NW, E, PASS, D, ST>(a, a.safe[si], L);
  if (threadIdx.x == 0) a.gap_part[si] = g;
}

template <int PASS, int D, int ST>
static hipError_t launch_sel_pds(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  const int64_t per = (PASS == 1 && a.nw <= 1) ? kSelFixedStates : 1;
  const dim3 g((unsigned)((a.n_safe + per - 1) / per));
  const int cells = max_row;  // upper bound on window cells per row
  if (cells <= 256 * 8)
    hipLaunchKernelGGL((k_sweep_sel<4, 8, PASS, D, ST>), g, dim3(256), 0, st, a);
  else if (cells <= 256 * 16)
    hipLaunchKernelGGL((k_sweep_sel<4, 16, PASS, D, ST>), g, dim3(256), 0, st, a);
  else if (cells <= 512 * 16)
    hipLaunchKernelGGL((k_sweep_sel<8, 16, PASS, D, ST>), g, dim3(512), 0, st, a);
  else if (cells <= 1024 * 16)
    hipLaunchKernelGGL((k_sweep_sel<16, 16, PASS, D, ST>), g, dim3(1024), 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// The storage of the bounds as a template argument: the load pass then holds
// no per-slot branch between the stored and the factored form.
template <int PASS, int D>
static hipError_t launch_sel_pd(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  return a.storage == IMPACT_STORE_FACTORS ? launch_sel_pds<PASS, D, 2>(a, max_row, st)
                                           : launch_sel_pds<PASS, D, 1>(a, max_row, st);
}

template <int PASS>
static hipError_t launch_sel_p(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  switch (a.d) {
    case 5: return launch_sel_pd<PASS, 5>(a, max_row, st);
    default: return launch_sel_pd<PASS, 0>(a, max_row, st);
  }
}

hipError_t launch_sweep_sel(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  if (a.n_safe == 0) return hipSuccess;
  if ((int64_t)a.nu * (a.nw > 1 ? a.nw : 1) > kMaxItems || !a.vsort || !a.hint)
    return hipErrorInvalidValue;
  return a.pass == 0 ? launch_sel_p<0>(a, max_row, st) : launch_sel_p<1>(a, max_row, st);
}

// ---- multi-query engine: queries whose rows exceed 512 entries ------------

// The value vector of every listed query in a sweeping phase, both components
// signed by the LP direction of its current pass, chunk-sorted into its
// buffer vs[0] (queries in a closing or finished phase skip).
__global__ __launch_bounds__(256) void k_mq_vsort_chunk(const QueryDesc* __restrict__ desc,
                                                        const QueryCtrl* __restrict__ ctrl,
                                                        const int32_t* __restrict__ qlist) {
  __shared__ double s[kSortChunk];
  const int q = qlist[blockIdx.y >> 1], vec = blockIdx.y & 1;
  const int phase = ctrl[q].phase;
  if (phase != 0 && phase != 2) return;
  const QueryDesc& D = desc[q];
  const int64_t n = D.a.n_cells;
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  if (base >= n) return;
  const double2* vin = (ctrl[q].step & 1) ? D.vb1 : D.vb0;
  const double sg = D.max_lp[phase >> 1] ? -1.0 : 1.0;
  for (int i = threadIdx.x; i < kSortChunk; i += 256) {
    const int64_t g = base + i;
    double v = __builtin_inf();
    if (g < n) {
      const double2 x = vin[g];
      v = sg * (vec ? x.y : x.x) + 0.0;
    }
    s[i] = v;
  }
  __syncthreads();
  for (int k = 2; k <= kSortChunk; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kSortChunk / 2; i += 256) {
        const int lo = 2 * i - (i & (j - 1)), hi = lo + j;
        const bool asc = (lo & k) == 0;
        const double x = s[lo], y = s[hi];
        if ((x > y) == asc) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  double* out = D.vs[0] + vec * n;
  for (int i = threadIdx.x; i < kSortChunk; i += 256) {
    const int64_t g = base + i;
    if (g < n) out[g] = s[i];
  }
}

// One merge pass (runs of L into 2L) of every listed sweeping query, from
// vs[from] to vs[1 - from]; a query whose value vector is no longer than L
// is copied.
__global__ __launch_bounds__(256) void k_mq_vsort_merge(const QueryDesc* __restrict__ desc,
                                                        const QueryCtrl* __restrict__ ctrl,
                                                        const int32_t* __restrict__ qlist,
                                                        int64_t L, int from) {
  const int q = qlist[blockIdx.y >> 1], vec = blockIdx.y & 1;
  const int phase = ctrl[q].phase;
  if (phase != 0 && phase != 2) return;
  const QueryDesc& D = desc[q];
  const int64_t n = D.a.n_cells;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* src = D.vs[from] + vec * n;
  double* dst = D.vs[1 - from] + vec * n;
  const int64_t start = (i / (2 * L)) * (2 * L);
  const int64_t mid = start + L < n ? start + L : n;
  const int64_t end = start + 2 * L < n ? start + 2 * L : n;
  const double key = src[i];
  int64_t pos;
  if (i < mid) {
    int64_t lo = mid, hi = end;
    while (lo < hi) {
      const int64_t m = (lo + hi) >> 1;
      if (src[m] < key)
        lo = m + 1;
      else
        hi = m;
    }
    pos = i + (lo - mid);
  } else {
    int64_t lo = start, hi = mid;
    while (lo < hi) {
      const int64_t m = (lo + hi) >> 1;
      if (src[m] <= key)
        lo = m + 1;
      else
        hi = m;
    }
    pos = (i - mid) + lo;
  }
  dst[pos] = key;
}

hipError_t launch_mq_value_sort(const QueryDesc* desc, const QueryCtrl* ctrl,
                                const int32_t* qlist, int32_t nq, int64_t max_cells,
                                hipStream_t st) {
  if (nq == 0 || max_cells == 0) return hipSuccess;
  const unsigned chunks = (unsigned)((max_cells + kSortChunk - 1) / kSortChunk);
  hipLaunchKernelGGL(k_mq_vsort_chunk, dim3(chunks, 2 * nq), dim3(256), 0, st, desc, ctrl, qlist);
  int from = 0;
  for (int64_t L = kSortChunk; L < max_cells; L <<= 1) {
    hipLaunchKernelGGL(k_mq_vsort_merge, dim3((unsigned)((max_cells + 255) / 256), 2 * nq),
                       dim3(256), 0, st, desc, ctrl, qlist, L, from);
    from ^= 1;
  }
  return hipGetLastError();
}

// One workgroup per (query, SAFE state) item of the long-row queries, each
// query at its own phase and step: a sweep of the state (phases 0 and 2) or
// the close of a pass (phases 1 and 3).  In the fixed-input pass of a query
// without a disturbance player the workgroup of every kSelFixedStates-th item
// of the query's segment (items begin + item, counted in the whole work list)
// solves that item and the next ones of the same query, as the single-query
// sweep does, and the others return.  ST: the storage of every query in the
// launch (0: mixed, tested per query).
template <int NW, int E, int D, int ST>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_mq_sweep_sel(
    const QueryDesc* __restrict__ desc, const QueryCtrl* __restrict__ ctrl,
    const int32_t* __restrict__ wq, const int32_t* __restrict__ ws, int64_t n_items,
    int64_t begin, double* __restrict__ gap_item) {
  __shared__ SelLds<NW> L;
  const int64_t item = blockIdx.x;
  if (item >= n_items) return;
  const int q = wq[item];
  const int phase = ctrl[q].phase;
  const int64_t step = ctrl[q].step;
  const QueryDesc& Dq = desc[q];
  double g = 0.0;
  if (phase == 0 || phase == 2) {
    SweepArgs a = Dq.a;
    a.vin = (step & 1) ? Dq.vb1 : Dq.vb0;
    a.vout = (step & 1) ? Dq.vb0 : Dq.vb1;
    a.reach = !Dq.safety;
    a.pass = phase >> 1;
    a.maximise = Dq.max_lp[phase >> 1];
    if (phase == 2 && a.nw <= 1) {
      const int64_t at = begin + item;
      if ((at - Dq.work_begin) % kSelFixedStates != 0) return;
      const int64_t left = Dq.work_end - at;
      sel_fixed_states<NW, E, D, ST>(a, ws + item, gap_item + item,
                                     left < kSelFixedStates ? (int)left : kSelFixedStates, L);
      return;
    }
    if (phase == 0)
      g = sel_state<NW, E, 0, D, ST>(a, ws[item], L);
    else
      g = sel_state<NW, E, 1, D, ST>(a, ws[item], L);
  } else if ((phase == 1 || phase == 3) && threadIdx.x == 0) {
    mq_close_state(Dq, ctrl[q], phase, ws[item]);
  }
  if (threadIdx.x == 0) gap_item[item] = g;
}

template <int D, int ST>
static hipError_t launch_mq_sel_ds(const QueryDesc* desc, const QueryCtrl* ctrl,
                                   const int32_t* wq, const int32_t* ws, int64_t n_items,
                                   int64_t begin, double* gap_item, int32_t max_row,
                                   hipStream_t st) {
  const dim3 g((unsigned)n_items);
  if (max_row <= 256 * 8)
    hipLaunchKernelGGL((k_mq_sweep_sel<4, 8, D, ST>), g, dim3(256), 0, st, desc, ctrl, wq, ws,
                       n_items, begin, gap_item);
  else if (max_row <= 256 * 16)
    hipLaunchKernelGGL((k_mq_sweep_sel<4, 16, D, ST>), g, dim3(256), 0, st, desc, ctrl, wq, ws,
                       n_items, begin, gap_item);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int D>
static hipError_t launch_mq_sel_d(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                                  const int32_t* ws, int64_t n_items, int64_t begin,
                                  double* gap_item, int32_t max_row, int32_t storage,
                                  hipStream_t st) {
  switch (storage) {
    case IMPACT_STORE_BOUNDS:
      return launch_mq_sel_ds<D, 1>(desc, ctrl, wq, ws, n_items, begin, gap_item, max_row, st);
    case IMPACT_STORE_FACTORS:
      return launch_mq_sel_ds<D, 2>(desc, ctrl, wq, ws, n_items, begin, gap_item, max_row, st);
    default:
      return launch_mq_sel_ds<D, 0>(desc, ctrl, wq, ws, n_items, begin, gap_item, max_row, st);
  }
}

hipError_t launch_mq_sweep_sel(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                               const int32_t* ws, int64_t n_items, int64_t begin,
                               double* gap_item, int32_t max_row, int32_t d, int32_t storage,
                               hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  return d == 5 ? launch_mq_sel_d<5>(desc, ctrl, wq, ws, n_items, begin, gap_item, max_row,
                                     storage, st)
                : launch_mq_sel_d<0>(desc, ctrl, wq, ws, n_items, begin, gap_item, max_row,
                                     storage, st);
}

}  // namespace impact
