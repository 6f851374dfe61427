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
#include "sweep_common.hpp"

namespace impact {

// Shared memory of the workgroup sweep.
template <int BLOCK_E>
struct BlockLds {
  uint64_t xk[BLOCK_E > 0 ? 64 * kWaves * BLOCK_E : 1];
  double red[2 * kWaves];
  double qb0[kMaxItems], qb1[kMaxItems];
  double gapw[kWaves];
};

// Sweep update of nst SAFE states (states[0..nst)) on one workgroup, all
// their (state, input) rows; returns, on thread t < nst, state t's V1 - V0.
// WAVE_E: largest per-lane element count of single-wavefront rows (row
// length <= 64 * WAVE_E); BLOCK_E: largest per-thread count of workgroup rows
// (row length <= 256 * BLOCK_E), 0 when every row fits one wavefront.
// D > 0: the grid dimension is the compile-time D; D == 0: read at run time.
template <int WAVE_E, int BLOCK_E, int PASS, int D>
__device__ double block_sweep_states(const SweepArgs& a, const int32_t* __restrict__ states,
                                     int nst, BlockLds<BLOCK_E>& L) {
  const SysParams& p = *a.sys;
  const int tid = threadIdx.x, lane = tid & 63, wv = uniform_i32(tid >> 6);
  // rows per state: (inputs swept) x (disturbances), disturbance fastest
  const int NW = a.nw > 1 ? a.nw : 1;
  const int U = (PASS == 0 ? a.nu : 1) * NW;
  const int items = nst * U;
  const int extra = 1 + a.windowed;
  constexpr bool UN = WAVE_E < 8 && BLOCK_E == 0;
  auto row_of = [&](int m) -> int64_t {
    const int gi = m / U, ui = m - gi * U;
    const int64_t s = states[gi];
    const int ku = ui / NW, w = ui - ku * NW;
    const int u = PASS == 0 ? ku : a.pi[s];
    return (s * a.nu + u) * NW + w;
  };

  if constexpr (BLOCK_E > 0) {
    // rows longer than one wavefront's capacity: the whole workgroup
    for (int m = 0; m < items; ++m) {
      const int64_t row = row_of(m);
      const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + extra;
      if (n <= 64 * WAVE_E) continue;
      double q0, q1;
      if (BLOCK_E <= 4 || n <= 1024)
        solve_row<4, kWaves, D, false>(a, p, row, tid, L.red, L.xk, q0, q1);
      else if (BLOCK_E <= 8 || n <= 2048)
        solve_row<(BLOCK_E < 8 ? BLOCK_E : 8), kWaves, D, false>(a, p, row, tid, L.red, L.xk, q0, q1);
      else
        solve_row<BLOCK_E, kWaves, D, false>(a, p, row, tid, L.red, L.xk, q0, q1);
      if (tid == 0) {
        L.qb0[m] = q0;
        L.qb1[m] = q1;
      }
    }
  }
  // short rows: one wavefront each
  for (int m = wv; m < items; m += kWaves) {
    const int64_t row = row_of(m);
    const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + extra;
    if (n > 64 * WAVE_E) continue;
    double q0, q1;
    if (WAVE_E == 1 || n <= 64)
      solve_row<1, 1, D, UN>(a, p, row, tid, L.red, L.xk, q0, q1);
    else if (WAVE_E == 2 || n <= 128)
      solve_row<(WAVE_E < 2 ? WAVE_E : 2), 1, D, UN>(a, p, row, tid, L.red, L.xk, q0, q1);
    else if (WAVE_E == 4 || n <= 256)
      solve_row<(WAVE_E < 4 ? WAVE_E : 4), 1, D, UN>(a, p, row, tid, L.red, L.xk, q0, q1);
    else
      solve_row<WAVE_E, 1, D, UN>(a, p, row, tid, L.red, L.xk, q0, q1);
    if (lane == 0) {
      L.qb0[m] = q0;
      L.qb1[m] = q1;
    }
  }
  __syncthreads();

  double gap = 0.0;
  if (tid < nst) {
    const int64_t s = states[tid];
    // an input is worth its worst row over the disturbances (eq. (5.1)):
    // the minimum for reach, the maximum of the bad mass for safety
    auto worst = [&](const double* q, int ku) {
      double v = q[tid * U + ku * NW];
      for (int w = 1; w < NW; ++w) {
        const double x = q[tid * U + ku * NW + w];
        v = a.reach ? fmin(v, x) : fmax(v, x);
      }
      return v;
    };
    double b0 = worst(L.qb0, 0), b1 = worst(L.qb1, 0);
    int arg = 0;
    for (int ku = 1; ku < U / NW; ++ku) {
      const double q0 = worst(L.qb0, ku), q1 = worst(L.qb1, ku);
      if (a.reach ? (q0 > b0) : (q0 < b0)) {
        b0 = q0;
        arg = ku;
      }
      if (a.reach ? (q1 > b1) : (q1 < b1)) b1 = q1;
    }
    a.vout[s] = make_double2(b0, b1);
    if (PASS == 0) a.pi[s] = arg;
    gap = b1 - b0;
    if (!(gap > 0.0)) gap = 0.0;
  }
  return gap;
}

// PASS 0: all inputs (policy pass); PASS 1: the input fixed by the policy.
// The two passes are separate kernel symbols so that profiles tell them apart.
template <int WAVE_E, int BLOCK_E, int PASS, int D>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ BlockLds<BLOCK_E> L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int G = a.states_per_block;
  const int64_t s0 = (int64_t)blockIdx.x * G;
  const int nst = (int)(a.n_safe - s0 < G ? a.n_safe - s0 : G);
  double gap = block_sweep_states<WAVE_E, BLOCK_E, PASS, D>(a, a.safe + s0, nst, L);
  gap = wave_max(gap);
  if (lane == 0) L.gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = L.gapw[0];
    for (int w = 1; w < kWaves; ++w) gm = fmax(gm, L.gapw[w]);
    a.gap_part[blockIdx.x] = gm;
  }
}

// Fixed-input pass with short rows: each GW-lane group of the workgroup
// solves one SAFE state's row (the policy's input), GW = 16 or 32 lanes with
// E keys each, so a wavefront carries 64 / GW rows at once.
template <int E, int GW, int D>
__global__ __launch_bounds__(kBlock) void k_sweep_rows_g(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ double gapw[kWaves];
  constexpr int G = kBlock / GW;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int grp = tid / GW, gl = tid % GW;
  const int64_t si = (int64_t)blockIdx.x * G + grp;
  double gap = 0.0;
  if (si < a.n_safe) {
    const int64_t s = a.safe[si];
    const int64_t row = s * a.nu + a.pi[s];
    double q0, q1;
    solve_row_g<E, GW, D>(a, *a.sys, row, gl, q0, q1);
    if (gl == 0) {
      a.vout[s] = make_double2(q0, q1);
      gap = q1 - q0 > 0.0 ? q1 - q0 : 0.0;
    }
  }
  gap = wave_max(gap);
  if (lane == 0) gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = gapw[0];
    for (int w = 1; w < kWaves; ++w) gm = fmax(gm, gapw[w]);
    a.gap_part[blockIdx.x] = gm;
  }
}

// States per workgroup of k_sweep_rows_g for rows of at most max_row entries,
// or 0 when the rows are too long for it.
int rows_g_states_per_block(int32_t max_row) {
  return max_row <= 128 ? kBlock / 16 : max_row <= 256 ? kBlock / 32 : 0;
}

// Multi-query fixed-input pass for queries whose rows fit a wavefront: one
// wavefront per (query, SAFE state) item in the fixed-input phase (others are
// left to k_mq_sweep_sb), the row of the policy's input solved like the
// single-query per-row sweep does (element count by the row's own length, up
// to WAVE_E).
template <int WAVE_E, int DIM>
__global__ __launch_bounds__(kBlock) void k_mq_sweep_row(
    const QueryDesc* __restrict__ desc, const QueryCtrl* __restrict__ ctrl,
    const int32_t* __restrict__ wq, const int32_t* __restrict__ ws, int64_t n_items,
    double* __restrict__ gap_item) {
  const int lane = threadIdx.x & 63, wv = uniform_i32(threadIdx.x >> 6);
  const int64_t item = (int64_t)blockIdx.x * kWaves + wv;
  if (item >= n_items) return;
  const int q = uniform_i32(wq[item]);
  if (uniform_i32(ctrl[q].phase) != 2) return;
  const int64_t s = uniform_i32(ws[item]);
  const int64_t step = uniform_i64(ctrl[q].step);
  const QueryDesc& D = desc[q];
  SweepArgs a = D.a;
  a.vin = (step & 1) ? D.vb1 : D.vb0;
  a.vout = (step & 1) ? D.vb0 : D.vb1;
  a.reach = !D.safety;
  a.pass = 1;
  a.maximise = D.max_lp[1];
  const SysParams& p = *a.sys;
  const int64_t row = s * a.nu + a.pi[s];
  const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + 1 + a.windowed;
  double q0, q1;
  if (WAVE_E == 1 || n <= 64)
    solve_row<1, 1, DIM, (WAVE_E < 8)>(a, p, row, lane, nullptr, nullptr, q0, q1);
  else if (WAVE_E == 2 || n <= 128)
    solve_row<(WAVE_E < 2 ? WAVE_E : 2), 1, DIM, (WAVE_E < 8)>(a, p, row, lane, nullptr, nullptr, q0, q1);
  else if (WAVE_E == 4 || n <= 256)
    solve_row<(WAVE_E < 4 ? WAVE_E : 4), 1, DIM, (WAVE_E < 8)>(a, p, row, lane, nullptr, nullptr, q0, q1);
  else
    solve_row<WAVE_E, 1, DIM, (WAVE_E < 8)>(a, p, row, lane, nullptr, nullptr, q0, q1);
  if (lane == 0) {
    a.vout[s] = make_double2(q0, q1);
    const double g = q1 - q0;
    gap_item[item] = g > 0.0 ? g : 0.0;
  }
}

// The engine's fixed-input pass for rows of at most 256 entries: one
// (query, SAFE state) item per GW-lane group, as k_sweep_rows_g.
template <int E, int GW, int DIM>
__global__ __launch_bounds__(kBlock) void k_mq_sweep_rows_g(
    const QueryDesc* __restrict__ desc, const QueryCtrl* __restrict__ ctrl,
    const int32_t* __restrict__ wq, const int32_t* __restrict__ ws, int64_t n_items,
    double* __restrict__ gap_item) {
  constexpr int G = kBlock / GW;
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int64_t item = (int64_t)blockIdx.x * G + grp;
  if (item >= n_items) return;
  const int q = wq[item];
  if (ctrl[q].phase != 2) return;
  const int64_t s = ws[item];
  const int64_t step = ctrl[q].step;
  const QueryDesc& D = desc[q];
  SweepArgs a = D.a;
  a.vin = (step & 1) ? D.vb1 : D.vb0;
  a.vout = (step & 1) ? D.vb0 : D.vb1;
  a.reach = !D.safety;
  a.pass = 1;
  a.maximise = D.max_lp[1];
  const int64_t row = s * a.nu + a.pi[s];
  double q0, q1;
  solve_row_g<E, GW, DIM>(a, *a.sys, row, gl, q0, q1);
  if (gl == 0) {
    a.vout[s] = make_double2(q0, q1);
    const double g = q1 - q0;
    gap_item[item] = g > 0.0 ? g : 0.0;
  }
}

hipError_t launch_mq_sweep_row(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                               const int32_t* ws, int64_t n_items, double* gap_item,
                               int32_t max_row, int32_t d, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  if (max_row > 512) return hipErrorInvalidValue;
  if (max_row <= 256) {
    const int gw = max_row <= 128 ? 16 : 32;
    const dim3 gg((unsigned)((n_items + kBlock / gw - 1) / (kBlock / gw))), bb(kBlock);
#define MG(GW1, D)                                                                            \
  hipLaunchKernelGGL((k_mq_sweep_rows_g<8, GW1, D>), gg, bb, 0, st, desc, ctrl, wq, ws, \
                     n_items, gap_item)
#define MGD(GW1)                \
  switch (d) {                  \
    case 2: MG(GW1, 2); break;  \
    case 3: MG(GW1, 3); break;  \
    case 5: MG(GW1, 5); break;  \
    default: MG(GW1, 0); break; \
  }
    if (gw == 16) {
      MGD(16)
    } else {
      MGD(32)
    }
#undef MGD
#undef MG
    return hipGetLastError();
  }
  const dim3 g((unsigned)((n_items + kWaves - 1) / kWaves)), b(kBlock);
#define MR(E1, D)                                                                           \
  hipLaunchKernelGGL((k_mq_sweep_row<E1, D>), g, b, 0, st, desc, ctrl, wq, ws, n_items, \
                     gap_item)
#define MRD(E1)                \
  switch (d) {                 \
    case 2: MR(E1, 2); break;  \
    case 3: MR(E1, 3); break;  \
    case 5: MR(E1, 5); break;  \
    default: MR(E1, 0); break; \
  }
  if (max_row <= 64) {
    MRD(1)
  } else if (max_row <= 128) {
    MRD(2)
  } else if (max_row <= 256) {
    MRD(4)
  } else {
    MRD(8)
  }
#undef MRD
#undef MR
  return hipGetLastError();
}

// Close one sweep: reduce the workgroups' gap partials, count the sweep, stop
// on eps or the cap.
__global__ __launch_bounds__(1024) void k_finish(Ctrl* c, const double* __restrict__ part,
                                                 int64_t n_part) {
  __shared__ double wmax[16];
  if (c->done) return;
  double g = 0.0;
  for (int64_t i = threadIdx.x; i < n_part; i += blockDim.x) g = fmax(g, part[i]);
  g = wave_max(g);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) g = fmax(g, wmax[w]);
  g = fmax(g, wmax[0]);
  c->sweeps += 1;
  c->gap = g;
  if (g <= c->eps) {
    c->done = 1;
    c->converged = 1;
  } else if (c->sweeps >= c->cap) {
    c->done = 1;
  }
}

// Self-convergence measure of one sweep (Remark 5.2): per workgroup, the
// largest change of either iterate, max(|V0' - V0|, |V1' - V1|), over its
// share of the SAFE states (grid-stride).
__global__ __launch_bounds__(256) void k_self_delta(const Ctrl* __restrict__ c,
                                                    const int32_t* __restrict__ safe,
                                                    int64_t n_safe,
                                                    const double2* __restrict__ vin,
                                                    const double2* __restrict__ vout,
                                                    double* __restrict__ part) {
  __shared__ double wmax[4];
  if (c->done) return;
  double g = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_safe;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = safe[i];
    const double2 o = vin[s], n = vout[s];
    g = fmax(g, fmax(fabs(n.x - o.x), fabs(n.y - o.y)));
  }
  g = wave_max(g);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}

hipError_t launch_self_delta(const Ctrl* c, const int32_t* safe, int64_t n_safe,
                             const double2* vin, const double2* vout, double* part, int64_t n_part,
                             hipStream_t st) {
  if (n_safe == 0 || n_part < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_self_delta, dim3((unsigned)n_part), dim3(256), 0, st, c, safe, n_safe, vin,
                     vout, part);
  return hipGetLastError();
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
                           const int32_t* __restrict__ pi, int32_t upper, int32_t safety,
                           int32_t finite, double* __restrict__ out,
                           int32_t* __restrict__ policy) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  out[s] = cls[s] == kSafe ? bound_of(v[s], upper != 0, safety != 0, finite != 0)
                           : (cls[s] == kTarget ? 1.0 : 0.0);
  if (policy) policy[s] = cls[s] == kSafe ? pi[s] : -1;
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

template <int PASS, int D>
static hipError_t launch_sweep_pass_d(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  const int64_t blocks = (a.n_safe + a.states_per_block - 1) / a.states_per_block;
  const dim3 g((unsigned)blocks), b(kBlock);
  if (PASS == 1 && a.states_per_block == rows_g_states_per_block(max_row)) {
    // one row per state: several rows per wavefront
    if (max_row <= 128)
      hipLaunchKernelGGL((k_sweep_rows_g<8, 16, D>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_sweep_rows_g<8, 32, D>), g, b, 0, st, a);
    return hipGetLastError();
  }
  if (max_row <= 64)
    hipLaunchKernelGGL((k_sweep<1, 0, PASS, D>), g, b, 0, st, a);
  else if (max_row <= 128)
    hipLaunchKernelGGL((k_sweep<2, 0, PASS, D>), g, b, 0, st, a);
  else if (max_row <= 256)
    hipLaunchKernelGGL((k_sweep<4, 0, PASS, D>), g, b, 0, st, a);
  else if (max_row <= 512)
    hipLaunchKernelGGL((k_sweep<8, 0, PASS, D>), g, b, 0, st, a);
  else
    return hipErrorInvalidValue;  // longer rows: the selection sweep
  return hipGetLastError();
}

// Kernels specialised on the grid dimension for the case-study dimensions.
template <int PASS>
static hipError_t launch_sweep_pass(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  switch (a.d) {
    case 2: return launch_sweep_pass_d<PASS, 2>(a, max_row, st);
    case 3: return launch_sweep_pass_d<PASS, 3>(a, max_row, st);
    case 5: return launch_sweep_pass_d<PASS, 5>(a, max_row, st);
    default: return launch_sweep_pass_d<PASS, 0>(a, max_row, st);
  }
}

hipError_t launch_sweep(const SweepArgs& a, int32_t max_row, hipStream_t st) {
  if (a.n_safe == 0) return hipSuccess;
  return a.pass == 0 ? launch_sweep_pass<0>(a, max_row, st) : launch_sweep_pass<1>(a, max_row, st);
}

hipError_t launch_finish(Ctrl* c, const double* part, int64_t n_part, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, st, c, part, n_part);
  return hipGetLastError();
}

int64_t sweep_blocks(const SweepArgs& a, bool box_path) {
  if (box_path) return (a.n_safe + kSbWavesPerBlock - 1) / kSbWavesPerBlock;
  return (a.n_safe + a.states_per_block - 1) / a.states_per_block;
}

hipError_t launch_finalize(const int8_t* cls, int64_t n, const double2* v, const int32_t* pi,
                           int32_t upper, int32_t safety, int32_t finite, double* out,
                           int32_t* policy, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(blocks_for(n, 256)), dim3(256), 0, st, cls, n, v, pi, upper,
                     safety, finite, out, policy);
  return hipGetLastError();
}

}  // namespace impact
