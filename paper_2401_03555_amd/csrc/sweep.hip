// sweep.hip -- interval-iteration kernels (eq. (5.1)/(5.2); Alg. 3 and
// Alg. 4; the LP of each (state, input) row solved by the sorting method of
// Section 6.2).
//
// k_sweep: one workgroup (4 wavefronts) per group of SAFE states.  For every
// (state, input) row it
//   1. gathers the row's (lo, hi) bounds and the current (V0, V1) value of
//      each entry's target (window cells, OUT, TAIL),
//   2. starts from p = lo, r = 1 - sum(lo),
//   3. bitonic-sorts the entries by value (ascending for a minimising LP,
//      descending for a maximising one), keys in registers, exchanges across
//      lanes by shuffles and across wavefronts through LDS,
//   4. hands r out greedily as an exclusive prefix sum of (hi - lo) in sorted
//      order: delta = clamp(r - prefix, 0, hi - lo),
//   5. returns q = sum(lo * v) + sum(delta * v),
// once with V0 and once with V1.  Rows of up to 512 entries are solved by one
// wavefront each (several rows in flight per workgroup); longer rows (up to
// 4096) by the whole workgroup.  The per-state max (reach) / min (safety) over
// inputs, the policy (lowest input on exact ties) and the state's V1 - V0 are
// then formed in LDS; the sweep's max gap goes to the control block by a
// 64-bit atomic max (order independent, so results are deterministic).
#include "impact_internal.hpp"

namespace impact {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxItems = 256;  // (state, input) rows per workgroup

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
  return x;
}

// Exclusive prefix sum across the wavefront (lane 0 gets 0).
__device__ __forceinline__ double wave_excl_scan(double x, int lane) {
  double incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    double y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  double e = __shfl_up(incl, 1);
  return lane == 0 ? 0.0 : e;
}

// Reduction / scan over a group of NW wavefronts (NW == 1: one wavefront).
template <int NW>
struct Group {
  double* red;  // 2 * NW doubles of LDS (double-buffered)
  int tid, lane, wv;
  int par;
  __device__ Group(double* r, int t) : red(r), tid(t), lane(t & 63), wv(t >> 6), par(0) {}

  __device__ double sum(double x) {
    x = wave_sum(x);
    if (NW == 1) return x;
    if (lane == 0) red[par * NW + wv] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[par * NW + w];
    par ^= 1;
    return s;
  }

  __device__ double excl_scan(double x) {
    double e = wave_excl_scan(x, lane);
    if (NW == 1) return e;
    if (lane == 63) red[par * NW + wv] = e + x;
    __syncthreads();
    double pre = 0.0;
    for (int w = 0; w < wv; ++w) pre += red[par * NW + w];
    par ^= 1;
    return pre + e;
  }
};

// Compare-exchange of two elements held by one thread.
template <int E>
__device__ __forceinline__ void ce_local(uint64_t (&key)[E], double (&val)[E], int e, int e2,
                                         bool asc) {
  const bool sw = asc ? (key[e] > key[e2]) : (key[e] < key[e2]);
  if (sw) {
    uint64_t tk = key[e];
    key[e] = key[e2];
    key[e2] = tk;
    double tv = val[e];
    val[e] = val[e2];
    val[e2] = tv;
  }
}

// All stages of merge step k whose stride j < E (both partners in one thread).
template <int E>
__device__ __forceinline__ void intra_stages(uint64_t (&key)[E], double (&val)[E], int tid,
                                             int k) {
#pragma unroll
  for (int j = E / 2; j > 0; j >>= 1) {
    if (j < k) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int e2 = e ^ j;
        if (e2 > e) ce_local<E>(key, val, e, e2, ((tid * E + e) & k) == 0);
      }
    }
  }
}

// Bitonic sort of P = 64 * NW * E keys, thread t holding positions
// [t*E, t*E + E) ("blocked" layout), ascending by key; val travels along.
template <int E, int NW>
__device__ void bitonic_sort(uint64_t (&key)[E], double (&val)[E], int tid, uint64_t* xk) {
  constexpr int P = 64 * NW * E;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j >= E; j >>= 1) {
      const int tm = j / E;  // partner thread = tid ^ tm
      const bool lower = (tid & tm) == 0;
      if (tm < 64) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool asc = ((tid * E + e) & k) == 0;
          const uint64_t pk = (uint64_t)__shfl_xor((long long)key[e], tm);
          const double pv = __shfl_xor(val[e], tm);
          const bool take = (asc == lower) ? !(key[e] < pk) : !(key[e] > pk);
          if (take) {
            key[e] = pk;
            val[e] = pv;
          }
        }
      } else {
        uint64_t pk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) xk[tid * E + e] = key[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) pk[e] = xk[(tid ^ tm) * E + e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) xk[tid * E + e] = dbits(val[e]);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool asc = ((tid * E + e) & k) == 0;
          const bool take = (asc == lower) ? !(key[e] < pk[e]) : !(key[e] > pk[e]);
          const double pv = bitsd(xk[(tid ^ tm) * E + e]);
          if (take) {
            key[e] = pk[e];
            val[e] = pv;
          }
        }
        __syncthreads();
      }
    }
    intra_stages<E>(key, val, tid, k);
  }
}

// One row's entries as seen by one thread: positions [first, first + E).
template <int E>
struct RowSlice {
  double lo[E], dd[E], v0[E], v1[E];
  bool pad[E];
};

template <int E>
__device__ void load_row(const SweepArgs& a, const SysParams& p, int64_t row, int first,
                         RowSlice<E>& rs) {
  const int d = a.d;
  const int64_t base = a.row_off[row];
  const int nw = (int)(a.row_off[row + 1] - base);
  const int32_t* wr = a.win + row * 2 * d;
  int32_t klo[kMaxDim], W[kMaxDim], j[kMaxDim], fo[kMaxDim];
  int64_t t = 0;
  int tot = 0;
  {
    int64_t rem = first < nw ? first : 0;
    for (int i = d - 1; i >= 0; --i) {
      W[i] = wr[d + i];
      klo[i] = wr[i];
      j[i] = nw > 0 ? (int32_t)(rem % W[i]) : 0;
      rem = nw > 0 ? rem / W[i] : 0;
    }
    for (int i = 0; i < d; ++i) {
      t += ((int64_t)klo[i] + j[i]) * p.stride[i];
      fo[i] = tot;
      tot += W[i];
    }
  }
  const double4 o = a.ot[row];
  const double tail_v = a.maximise ? 1.0 : 0.0;
  const double2* fr = a.fac ? a.fac + row * (int64_t)a.fs : nullptr;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int slot = first + e;
    double lo = 0.0, hi = 0.0, v0 = 0.0, v1 = 0.0;
    bool pad = false;
    if (slot < nw) {
      if (a.storage == IMPACT_STORE_FACTORS) {
        lo = 1.0;
        hi = 1.0;
        for (int i = 0; i < d; ++i) {
          const double2 fv = fr[fo[i] + j[i]];
          lo *= fv.x;
          hi *= fv.y;
        }
      } else {
        const double2 b = a.ent[base + slot];
        lo = b.x;
        hi = b.y;
      }
      const double2 V = a.vin[t];
      v0 = V.x;
      v1 = V.y;
      // advance the window multi-index by one (last dimension fastest)
      for (int i = d - 1; i >= 0; --i) {
        ++j[i];
        t += p.stride[i];
        if (j[i] < W[i]) break;
        j[i] = 0;
        t -= (int64_t)W[i] * p.stride[i];
      }
    } else if (slot == nw) {
      lo = o.x;
      hi = o.y;
      v0 = v1 = a.out_val;
    } else if (slot == nw + 1 && a.windowed) {
      lo = o.z;
      hi = o.w;
      v0 = v1 = tail_v;
    } else {
      pad = true;
    }
    rs.lo[e] = lo;
    rs.dd[e] = pad ? 0.0 : hi - lo;
    rs.v0[e] = v0;
    rs.v1[e] = v1;
    rs.pad[e] = pad;
  }
}

// Sorting-method LP value for one value vector (v), given r = 1 - sum(lo).
template <int E, int NW>
__device__ double lp_value(const RowSlice<E>& rs, const double (&v)[E], double r, bool maximise,
                           Group<NW>& g, uint64_t* xk) {
  double slv = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) slv += rs.lo[e] * v[e];
  slv = g.sum(slv);
  uint64_t key[E];
  double dk[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t b = dbits(v[e] + 0.0);
    key[e] = rs.pad[e] ? ~0ull : (maximise ? ~b : b);
    dk[e] = rs.dd[e];
  }
  bitonic_sort<E, NW>(key, dk, g.tid, xk);
  double ls = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) ls += dk[e];
  double acc = g.excl_scan(ls);
  double sdv = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double room = r - acc;
    const double delta = room <= 0.0 ? 0.0 : (dk[e] < room ? dk[e] : room);
    const double val = bitsd(maximise ? ~key[e] : key[e]);
    if (delta > 0.0) sdv += delta * val;
    acc += dk[e];
  }
  sdv = g.sum(sdv);
  return slv + sdv;
}

template <int E, int NW>
__device__ void solve_row(const SweepArgs& a, const SysParams& p, int64_t row, int tid,
                          double* red, uint64_t* xk, double& q0, double& q1) {
  // a single-wavefront group works in lane coordinates; a workgroup group
  // first waits for every wavefront to leave the previous row's reductions
  const int gtid = NW == 1 ? (tid & 63) : tid;
  if (NW > 1) __syncthreads();
  Group<NW> g(red, gtid);
  RowSlice<E> rs;
  load_row<E>(a, p, row, gtid * E, rs);
  double slo = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) slo += rs.lo[e];
  slo = g.sum(slo);
  double r = 1.0 - slo;
  if (r < 0.0) r = 0.0;
  const bool mx = a.maximise != 0;
  q0 = lp_value<E, NW>(rs, rs.v0, r, mx, g, xk);
  q1 = lp_value<E, NW>(rs, rs.v1, r, mx, g, xk);
}

template <int PASS>
__device__ __forceinline__ int64_t item_row(const SweepArgs& a, int64_t s0, int m, int U) {
  const int gi = m / U, ui = m - gi * U;
  const int64_t s = a.safe[s0 + gi];
  const int u = PASS == 0 ? ui : a.pi[s];
  return s * a.nu + u;
}

// WAVE_E: largest per-lane element count of single-wavefront rows (row
// length <= 64 * WAVE_E); BLOCK_E: largest per-thread count of workgroup rows
// (row length <= 256 * BLOCK_E), 0 when every row fits one wavefront.
// PASS 0: all inputs (policy pass); PASS 1: the input fixed by the policy.
// The two passes are separate kernel symbols so that profiles tell them apart.
template <int WAVE_E, int BLOCK_E, int PASS>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ uint64_t xk[BLOCK_E > 0 ? 64 * kWaves * BLOCK_E : 1];
  __shared__ double red[2 * kWaves];
  __shared__ double qb0[kMaxItems], qb1[kMaxItems];
  __shared__ double gapw[kWaves];
  const SysParams& p = *a.sys;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int G = a.states_per_block, U = a.inputs_per_state;
  const int64_t s0 = (int64_t)blockIdx.x * G;
  const int nst = (int)(a.n_safe - s0 < G ? a.n_safe - s0 : G);
  const int items = nst * U;
  const int extra = 1 + a.windowed;

  if constexpr (BLOCK_E > 0) {
    // rows longer than one wavefront's capacity: the whole workgroup
    for (int m = 0; m < items; ++m) {
      const int64_t row = item_row<PASS>(a, s0, m, U);
      const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + extra;
      if (n <= 64 * WAVE_E) continue;
      double q0, q1;
      if (BLOCK_E <= 4 || n <= 1024)
        solve_row<4, kWaves>(a, p, row, tid, red, xk, q0, q1);
      else if (BLOCK_E <= 8 || n <= 2048)
        solve_row<(BLOCK_E < 8 ? BLOCK_E : 8), kWaves>(a, p, row, tid, red, xk, q0, q1);
      else
        solve_row<BLOCK_E, kWaves>(a, p, row, tid, red, xk, q0, q1);
      if (tid == 0) {
        qb0[m] = q0;
        qb1[m] = q1;
      }
    }
  }
  // short rows: one wavefront each
  for (int m = wv; m < items; m += kWaves) {
    const int64_t row = item_row<PASS>(a, s0, m, U);
    const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + extra;
    if (n > 64 * WAVE_E) continue;
    double q0, q1;
    if (WAVE_E == 1 || n <= 64)
      solve_row<1, 1>(a, p, row, tid, red, xk, q0, q1);
    else if (WAVE_E == 2 || n <= 128)
      solve_row<(WAVE_E < 2 ? WAVE_E : 2), 1>(a, p, row, tid, red, xk, q0, q1);
    else if (WAVE_E == 4 || n <= 256)
      solve_row<(WAVE_E < 4 ? WAVE_E : 4), 1>(a, p, row, tid, red, xk, q0, q1);
    else
      solve_row<WAVE_E, 1>(a, p, row, tid, red, xk, q0, q1);
    if (lane == 0) {
      qb0[m] = q0;
      qb1[m] = q1;
    }
  }
  __syncthreads();

  double gap = 0.0;
  if (tid < nst) {
    const int64_t s = a.safe[s0 + tid];
    double b0 = qb0[tid * U], b1 = qb1[tid * U];
    int arg = 0;
    for (int ui = 1; ui < U; ++ui) {
      const double q0 = qb0[tid * U + ui], q1 = qb1[tid * U + ui];
      if (a.reach ? (q0 > b0) : (q0 < b0)) {
        b0 = q0;
        arg = ui;
      }
      if (a.reach ? (q1 > b1) : (q1 < b1)) b1 = q1;
    }
    a.vout[s] = make_double2(b0, b1);
    if (PASS == 0) a.pi[s] = arg;
    gap = b1 - b0;
    if (!(gap > 0.0)) gap = 0.0;
  }
  gap = wave_max(gap);
  if (lane == 0) gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = gapw[0];
    for (int w = 1; w < kWaves; ++w) gm = fmax(gm, gapw[w]);
    atomicMax(&a.ctrl->gap_bits, (unsigned long long)dbits(gm));
  }
}

// Close one sweep: record its gap, count it, stop on eps or the cap.
__global__ void k_finish(Ctrl* c) {
  if (threadIdx.x != 0 || c->done) return;
  const double gap = bitsd(c->gap_bits);
  c->gap_bits = 0ull;
  c->sweeps += 1;
  c->gap = gap;
  if (gap <= c->eps) {
    c->done = 1;
    c->converged = 1;
  } else if (c->sweeps >= c->cap) {
    c->done = 1;
  }
}

__global__ void k_ctrl_init(Ctrl* c, double eps, int64_t cap) {
  if (threadIdx.x != 0) return;
  c->gap_bits = 0ull;
  c->done = 0;
  c->converged = 0;
  c->sweeps = 0;
  c->cap = cap;
  c->gap = 1.0;
  c->eps = eps;
  c->err = 0;
}

// Labels (Section 3.1): centre of each cell against closed boxes, avoid wins.
__global__ void k_label(const SysParams* __restrict__ sp, const double* __restrict__ tb, int32_t nt,
                        const double* __restrict__ ab, int32_t na, int8_t* __restrict__ cls,
                        int64_t* __restrict__ flag) {
  const SysParams& p = *sp;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= p.n_states) return;
  const int d = p.d;
  double c[kMaxDim], tol[kMaxDim];
  int64_t rem = s;
  for (int i = d - 1; i >= 0; --i) {
    const int64_t k = rem % p.n[i];
    rem /= p.n[i];
    c[i] = p.lb[i] + ((double)k + 0.5) * p.w[i];
    tol[i] = 1e-9 * p.w[i];
  }
  int8_t cl = kSafe;
  for (int b = 0; b < nt; ++b) {
    const double* box = tb + (int64_t)b * 2 * d;
    bool in = true;
    for (int i = 0; i < d; ++i) in = in && !(c[i] < box[i] - tol[i] || c[i] > box[d + i] + tol[i]);
    if (in) cl = kTarget;
  }
  for (int b = 0; b < na; ++b) {
    const double* box = ab + (int64_t)b * 2 * d;
    bool in = true;
    for (int i = 0; i < d; ++i) in = in && !(c[i] < box[i] - tol[i] || c[i] > box[d + i] + tol[i]);
    if (in) cl = kAvoid;
  }
  cls[s] = cl;
  flag[s] = cl == kSafe ? 1 : 0;
}

__global__ void k_compact(const int8_t* __restrict__ cls, const int64_t* __restrict__ pos,
                          int64_t n, int32_t* __restrict__ safe) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && cls[s] == kSafe) safe[pos[s]] = (int32_t)s;
}

// V0 = 0, V1 = 1 on SAFE cells; constant class values elsewhere (both buffers).
__global__ void k_init_values(const int8_t* __restrict__ cls, int64_t n, int32_t safety,
                              double2* __restrict__ v0, double2* __restrict__ v1,
                              int32_t* __restrict__ pi) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double2 v;
  if (cls[s] == kSafe)
    v = make_double2(0.0, 1.0);
  else if (cls[s] == kTarget)
    v = make_double2(1.0, 1.0);
  else
    v = safety ? make_double2(1.0, 1.0) : make_double2(0.0, 0.0);
  v0[s] = v;
  v1[s] = v;
  if (pi) pi[s] = 0;
}

// Outputs: pass 0 writes lo and the policy, pass 1 writes hi.
__global__ void k_finalize(const int8_t* __restrict__ cls, int64_t n, const double2* __restrict__ v,
                           const int32_t* __restrict__ pi, int32_t pass, int32_t safety,
                           double* __restrict__ out, int32_t* __restrict__ policy) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double o;
  if (cls[s] == kSafe) {
    const double2 x = v[s];
    if (pass == 0)
      o = safety ? 1.0 - x.y : x.x;
    else
      o = safety ? 1.0 - x.x : x.y;
  } else {
    o = cls[s] == kTarget ? 1.0 : 0.0;
  }
  out[s] = o;
  if (pass == 0) policy[s] = cls[s] == kSafe ? pi[s] : -1;
}

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_label(const SysParams* sys, int64_t n, const double* tb, int32_t nt,
                        const double* ab, int32_t na, int8_t* cls, int64_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_label, dim3(blocks_for(n, 256)), dim3(256), 0, st, sys, tb, nt, ab, na, cls,
                     flag);
  return hipGetLastError();
}

hipError_t launch_compact(const int8_t* cls, const int64_t* pos, int64_t n, int32_t* safe,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3(blocks_for(n, 256)), dim3(256), 0, st, cls, pos, n, safe);
  return hipGetLastError();
}

hipError_t launch_init_values(const int8_t* cls, int64_t n, int32_t safety, double2* v0,
                              double2* v1, int32_t* pi, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_values, dim3(blocks_for(n, 256)), dim3(256), 0, st, cls, n, safety, v0,
                     v1, pi);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* c, double eps, int64_t cap, hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, c, eps, cap);
  return hipGetLastError();
}

template <int PASS>
static hipError_t launch_sweep_pass(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  const int64_t blocks = (a.n_safe + a.states_per_block - 1) / a.states_per_block;
  const dim3 g((unsigned)blocks), b(kBlock);
  if (max_row <= 64)
    hipLaunchKernelGGL((k_sweep<1, 0, PASS>), g, b, 0, st, a);
  else if (max_row <= 128)
    hipLaunchKernelGGL((k_sweep<2, 0, PASS>), g, b, 0, st, a);
  else if (max_row <= 256)
    hipLaunchKernelGGL((k_sweep<4, 0, PASS>), g, b, 0, st, a);
  else if (max_row <= 512)
    hipLaunchKernelGGL((k_sweep<8, 0, PASS>), g, b, 0, st, a);
  else if (max_row <= 1024)
    hipLaunchKernelGGL((k_sweep<8, 4, PASS>), g, b, 0, st, a);
  else if (max_row <= 2048)
    hipLaunchKernelGGL((k_sweep<8, 8, PASS>), g, b, 0, st, a);
  else if (max_row <= kMaxRow)
    hipLaunchKernelGGL((k_sweep<8, 16, PASS>), g, b, 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  if (a.n_safe == 0) return hipSuccess;
  return a.pass == 0 ? launch_sweep_pass<0>(a, max_row, st) : launch_sweep_pass<1>(a, max_row, st);
}

hipError_t launch_finish(Ctrl* c, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_finalize(const int8_t* cls, int64_t n, const double2* v, const int32_t* pi,
                           int32_t pass, int32_t safety, double* out, int32_t* policy,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 256)), dim3(256), 0, st, cls, n, v, pi, pass,
                     safety, out, policy);
  return hipGetLastError();
}

}  // namespace impact
