// sweep_sb.hip -- interval-iteration sweep with one sort per state.
//
// The rows (s, u) of one state have target windows that overlap almost
// entirely (the input moves the mean by a fraction of the window).  The LP of
// a row (eq. (5.1), sorting method of Section 6.2) only needs the row's
// entries in value order, and the order of a subset of a sorted list is the
// subset's own sorted order.  So one wavefront per SAFE state
//   1. forms the bounding box B of its rows' windows,
//   2. gathers (V0, V1) over the cells of B and bitonic-sorts B twice
//      (keys: IEEE bits of the value, complemented for a maximising LP;
//      payload: the cell's position in B),
//   3. for each input: clears an LDS staging array over B, scatters the row's
//      (lo, hi) to the positions of its window cells, and runs the prefix-sum
//      greedy along each sorted order -- cells of B outside the row's window
//      carry zero mass and drop out,
//   4. keeps the max (reach) / min (safety) over inputs and the policy.
// OUT and TAIL have values exactly 0 or 1, the extremes of every order, so
// they sit before or after all cells and are handled in closed form.
// States whose box exceeds a wavefront's capacity fall back to one sort per
// row.  The result equals the per-row sort's LP values up to summation order.
#include "sweep_common.hpp"

namespace impact {

constexpr int kSbWaves = kSbWavesPerBlock;

__device__ __forceinline__ int wave_min_i32(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int y = xor_lane_i32(x, off);
    x = y < x ? y : x;
  }
  return x;
}

__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int y = xor_lane_i32(x, off);
    x = y > x ? y : x;
  }
  return x;
}

// LDS writes of one wavefront made visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct StateBox {
  int32_t blo[kMaxDim], ext[kMaxDim];
  int32_t bstride[kMaxDim];
  int64_t P;  // cells in the box (0: every row has an empty window)
};

template <int PASS>
__device__ __forceinline__ int row_input(const SweepArgs& a, int64_t s, int ui) {
  return PASS == 0 ? ui : a.pi[s];
}

// Bounding box of the windows of the state's rows (rows whose window is empty
// in some dimension hold no cells and are ignored).  D > 0: the grid dimension
// is the compile-time D (every dimension loop unrolls to straight-line code);
// D == 0: read at run time.
template <int PASS, int D>
__device__ void state_box(const SweepArgs& a, int64_t s, int U, int lane, StateBox& b) {
  const int d = D > 0 ? D : a.d;
  int lo[kMaxDim], hi[kMaxDim];
  IMPACT_FOR_DIMS(i, d) {
    lo[i] = 0x7fffffff;
    hi[i] = -0x7fffffff;
  }
  for (int ui = lane; ui < U; ui += 64) {
    const int64_t row = s * a.nu + row_input<PASS>(a, s, ui);
    const int32_t* wr = a.win + row * 2 * d;
    bool empty = false;
    IMPACT_FOR_DIMS(i, d) empty = empty || wr[d + i] == 0;
    if (!empty)
      IMPACT_FOR_DIMS(i, d) {
        lo[i] = wr[i] < lo[i] ? wr[i] : lo[i];
        hi[i] = wr[i] + wr[d + i] > hi[i] ? wr[i] + wr[d + i] : hi[i];
      }
  }
  int64_t P = 1;
  IMPACT_FOR_DIMS(i, d) {
    const int l = uniform_i32(wave_min_i32(lo[i])), h = uniform_i32(wave_max_i32(hi[i]));
    b.blo[i] = l;
    b.ext[i] = h > l ? h - l : 0;
    P *= b.ext[i];
  }
  int32_t st = 1;
  IMPACT_FOR_DIMS_REV(i, d) {
    b.bstride[i] = st;
    st = (int32_t)((int64_t)st * b.ext[i] > 0x3fffffff ? 0x3fffffff : st * b.ext[i]);
  }
  b.P = P;
}

// OUT / TAIL: value exactly 0 or 1, so first or last in every sorted order.
struct Specials {
  double lo[2], dd[2], v[2];
  int n;
};

__device__ __forceinline__ bool special_front(double v, bool mx) { return mx ? v == 1.0 : v == 0.0; }

// Reductions over the GW-lane group a lane belongs to (GW = 16, 32 or 64).
template <int GW>
__device__ __forceinline__ double group_sum(double x) {
  return group_sum_dpp<GW>(x);
}

// Bitonic sort of two key sets at once (same network, independent data),
// 64 lanes x E keys each, blocked layout, ascending.
template <int E>
__device__ void bitonic_sort2(uint64_t (&ka)[E], int32_t (&pa)[E], uint64_t (&kb)[E],
                              int32_t (&pb)[E], int lane) {
  constexpr int P = 64 * E;
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j >= E; j >>= 1) {
      const int tm = j / E;
      const bool lower = (lane & tm) == 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool asc = ((lane * E + e) & k) == 0;
        const uint64_t qa = xor_lane_u64(ka[e], tm);
        const uint64_t qb = xor_lane_u64(kb[e], tm);
        const int32_t ra = xor_lane_i32(pa[e], tm);
        const int32_t rb = xor_lane_i32(pb[e], tm);
        const bool keep_min = asc == lower;
        if (keep_min ? !(ka[e] < qa) : !(ka[e] > qa)) {
          ka[e] = qa;
          pa[e] = ra;
        }
        if (keep_min ? !(kb[e] < qb) : !(kb[e] > qb)) {
          kb[e] = qb;
          pb[e] = rb;
        }
      }
    }
    intra_stages<E, int32_t>(ka, pa, lane, k);
    intra_stages<E, int32_t>(kb, pb, lane, k);
  }
}

// Rows of a state are processed by NG lane groups of GW = 64/NG lanes at a
// time, each lane holding 8 sorted positions: NG = 4 for boxes of up to 128
// cells, 2 for 256, 1 for 512.
template <int P>
struct SbShape {
  static constexpr int NG = P <= 128 ? 4 : (P <= 256 ? 2 : 1);
  static constexpr int GW = 64 / NG;
  static constexpr int R = P / GW;
};

// Per-wavefront LDS of the state-box path (P = box capacity).
template <int P>
struct SbLds {
  int32_t ord[2][P];                 // box position of the j-th entry of each order
  double val[2][P];                  // its value
  double2 stg[SbShape<P>::NG][P];    // (lo, hi) over the box, one array per lane group
};

// Sorting-method LP of one row along one sorted order, on a GW-lane group:
// lane gl holds sorted positions [gl*R, gl*R + R).
template <int R, int GW>
__device__ double sb_lp_group(const int32_t* __restrict__ ord, const double* __restrict__ val,
                          const double2* __restrict__ stg, int64_t P, double r, bool mx,
                          const Specials& sp, int gl) {
  double dd[R], vv[R];
  double lane_d = 0.0, lane_q = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int j = gl * R + k;
    const int o = ord[j];
    if (o < P) {
      const double2 b = stg[o];
      dd[k] = b.y - b.x;
      vv[k] = val[j];
      lane_q += b.x * vv[k];
    } else {
      dd[k] = 0.0;
      vv[k] = 0.0;
    }
    lane_d += dd[k];
  }
  double front = 0.0, q_sp = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= sp.n || !special_front(sp.v[k], mx)) continue;
    const double room = r - front;
    const double delta = room <= 0.0 ? 0.0 : (sp.dd[k] < room ? sp.dd[k] : room);
    q_sp += (sp.lo[k] + delta) * sp.v[k];
    front += sp.dd[k];
  }
  double total;
  const double excl = group_excl_scan_dpp<GW>(lane_d, gl, total);
  double acc = front + excl;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double room = r - acc;
    const double delta = room <= 0.0 ? 0.0 : (dd[k] < room ? dd[k] : room);
    if (delta > 0.0) lane_q += delta * vv[k];
    acc += dd[k];
  }
  double back = front + total;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= sp.n || special_front(sp.v[k], mx)) continue;
    const double room = r - back;
    const double delta = room <= 0.0 ? 0.0 : (sp.dd[k] < room ? sp.dd[k] : room);
    q_sp += (sp.lo[k] + delta) * sp.v[k];
    back += sp.dd[k];
  }
  return group_sum<GW>(lane_q) + q_sp;
}

// One SAFE state on one wavefront, box of at most 64*E cells.  The box is
// sorted with 64 lanes; then the NG lane groups take rows u = g, g+NG, ...
template <int E, int PASS, int D>
__device__ void sb_state(const SweepArgs& a, const SysParams& p, int64_t s, int U,
                         const StateBox& b, int lane, SbLds<64 * E>& L, double& best0,
                         double& best1, int& arg) {
  constexpr int P = 64 * E;
  constexpr int NG = SbShape<P>::NG, GW = SbShape<P>::GW, R = SbShape<P>::R;
  const int d = D > 0 ? D : a.d;
  const bool mx = a.maximise != 0;
  const int64_t PB = b.P;
  {
    uint64_t k0[E], k1[E];
    int32_t p0[E], p1[E];
    // values over the box, blocked layout: lane holds positions lane*E + e
    int32_t c[kMaxDim];
    int64_t rem = (int64_t)lane * E < PB ? (int64_t)lane * E : 0;
    int64_t t = 0;
    IMPACT_FOR_DIMS_REV(i, d) {
      c[i] = PB > 0 ? (int32_t)(rem % b.ext[i]) : 0;
      rem = PB > 0 ? rem / b.ext[i] : 0;
    }
    IMPACT_FOR_DIMS(i, d) t += ((int64_t)b.blo[i] + c[i]) * p.stride[i];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int bi = lane * E + e;
      p0[e] = bi;
      p1[e] = bi;
      if (bi < PB) {
        const double2 V = a.vin[t];
        const uint64_t b0 = dbits(V.x + 0.0), b1 = dbits(V.y + 0.0);
        k0[e] = mx ? ~b0 : b0;
        k1[e] = mx ? ~b1 : b1;
        IMPACT_FOR_DIMS_REV(i, d) {
          ++c[i];
          t += p.stride[i];
          if (c[i] < b.ext[i]) break;
          c[i] = 0;
          t -= (int64_t)b.ext[i] * p.stride[i];
        }
      } else {
        k0[e] = ~0ull;
        k1[e] = ~0ull;
      }
    }
    bitonic_sort2<E>(k0, p0, k1, p1, lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = lane * E + e;
      L.ord[0][j] = p0[e];
      L.ord[1][j] = p1[e];
      L.val[0][j] = p0[e] < PB ? bitsd(mx ? ~k0[e] : k0[e]) : 0.0;
      L.val[1][j] = p1[e] < PB ? bitsd(mx ? ~k1[e] : k1[e]) : 0.0;
    }
  }
  wave_lds_sync();

  const int g = lane / GW, gl = lane % GW;
  double2* stg = L.stg[g];
  const double tail_v = mx ? 1.0 : 0.0;
  const double worst = a.reach ? -1.0 : 2.0;
  double g0 = worst, g1 = worst;
  int garg = 0x7fffffff;
  for (int ui0 = 0; ui0 < U; ui0 += NG) {
    const int ui = ui0 + g;
    const bool act = ui < U;
#pragma unroll
    for (int k = 0; k < R; ++k) stg[gl * R + k] = make_double2(0.0, 0.0);
    wave_lds_sync();
    int u = 0;
    int64_t row = 0;
    double lane_lo = 0.0;
    if (act) {
      u = row_input<PASS>(a, s, ui);
      row = s * a.nu + u;
      const int64_t base = a.row_off[row];
      const int nw = (int)(a.row_off[row + 1] - base);
      if (nw > 0) {
        const int32_t* wr = a.win + row * 2 * d;
        int32_t W[kMaxDim], off[kMaxDim], j[kMaxDim], inc[kMaxDim], fo[kMaxDim];
        int tot = 0;
        IMPACT_FOR_DIMS(i, d) {
          W[i] = wr[d + i];
          off[i] = wr[i] - b.blo[i];
          fo[i] = tot;
          tot += W[i];
        }
        int64_t r0 = gl, r1 = GW;
        IMPACT_FOR_DIMS_REV(i, d) {
          j[i] = (int32_t)(r0 % W[i]);
          r0 /= W[i];
          inc[i] = (int32_t)(r1 % W[i]);
          r1 /= W[i];
        }
        const double2* fr = a.fac ? a.fac + row * (int64_t)a.fs : nullptr;
        for (int slot = gl; slot < nw; slot += GW) {
          int bi = 0;
          IMPACT_FOR_DIMS(i, d) bi += (off[i] + j[i]) * b.bstride[i];
          double2 e;
          if (a.storage == IMPACT_STORE_FACTORS) {
            double lo = 1.0, hi = 1.0;
            IMPACT_FOR_DIMS(i, d) {
              const double2 fv = fr[fo[i] + j[i]];
              lo *= fv.x;
              hi *= fv.y;
            }
            e = make_double2(lo, hi);
          } else {
            e = a.ent[base + slot];
          }
          stg[bi] = e;
          lane_lo += e.x;
          int carry = 0;
          IMPACT_FOR_DIMS_REV(i, d) {
            j[i] += inc[i] + carry;
            carry = j[i] >= W[i];
            if (carry) j[i] -= W[i];
          }
        }
      }
    }
    wave_lds_sync();
    if (act) {
      const double4 o = a.ot[row];
      Specials sp;
      sp.n = 1 + a.windowed;
      sp.lo[0] = o.x;
      sp.dd[0] = o.y - o.x;
      sp.v[0] = a.out_val;
      sp.lo[1] = o.z;
      sp.dd[1] = o.w - o.z;
      sp.v[1] = tail_v;
      double slo = group_sum<GW>(lane_lo) + o.x;
      if (a.windowed) slo += o.z;
      double r = 1.0 - slo;
      if (r < 0.0) r = 0.0;
      const double q0 = sb_lp_group<R, GW>(L.ord[0], L.val[0], stg, PB, r, mx, sp, gl);
      const double q1 = sb_lp_group<R, GW>(L.ord[1], L.val[1], stg, PB, r, mx, sp, gl);
      // rows of a group come in increasing u: a strict improvement keeps the lowest u
      if (a.reach ? (q0 > g0) : (q0 < g0)) {
        g0 = q0;
        garg = u;
      }
      if (a.reach ? (q1 > g1) : (q1 < g1)) g1 = q1;
    }
    wave_lds_sync();
  }
  // combine the lane groups: best value, lowest input on exact ties
#pragma unroll
  for (int off = GW; off < 64; off <<= 1) {
    const double o0 = __shfl_xor(g0, off), o1 = __shfl_xor(g1, off);
    const int oa = __shfl_xor(garg, off);
    const bool better = a.reach ? (o0 > g0 || (o0 == g0 && oa < garg))
                                : (o0 < g0 || (o0 == g0 && oa < garg));
    if (better) {
      g0 = o0;
      garg = oa;
    }
    g1 = a.reach ? fmax(g1, o1) : fmin(g1, o1);
  }
  best0 = g0;
  best1 = g1;
  arg = garg;
}

// ESB: per-lane element count of the largest state box handled by the box
// path (box <= 64 * ESB cells); EROW > 0: per-lane count of the per-row
// fallback for states whose box is larger (rows <= 64 * EROW entries).
// Sweep update of one SAFE state s on one wavefront: writes vout[s] (and
// pi[s] in the policy pass); returns the state's V1 - V0 (>= 0).
template <int ESB, int EROW, int PASS, int D>
__device__ double sb_sweep_state(const SweepArgs& a, int64_t s, int lane, SbLds<64 * ESB>& L) {
  const SysParams& p = *a.sys;
  const int U = PASS == 0 ? a.nu : 1;
  StateBox b;
  state_box<PASS, D>(a, s, U, lane, b);
  double best0 = 0.0, best1 = 0.0;
  int arg = 0;
  if (b.P <= 64 * ESB) {
    if (ESB == 1 || b.P <= 64)
      sb_state<1, PASS, D>(a, p, s, U, b, lane, *(SbLds<64>*)&L, best0, best1, arg);
    else if (ESB == 2 || b.P <= 128)
      sb_state<(ESB < 2 ? ESB : 2), PASS, D>(a, p, s, U, b, lane,
                                          *(SbLds<64 * (ESB < 2 ? ESB : 2)>*)&L, best0, best1,
                                          arg);
    else if (ESB == 4 || b.P <= 256)
      sb_state<(ESB < 4 ? ESB : 4), PASS, D>(a, p, s, U, b, lane,
                                          *(SbLds<64 * (ESB < 4 ? ESB : 4)>*)&L, best0, best1,
                                          arg);
    else
      sb_state<ESB, PASS, D>(a, p, s, U, b, lane, L, best0, best1, arg);
  } else if constexpr (EROW > 0) {
    const int extra = 1 + a.windowed;
    for (int ui = 0; ui < U; ++ui) {
      const int u = row_input<PASS>(a, s, ui);
      const int64_t row = s * a.nu + u;
      const int n = (int)(a.row_off[row + 1] - a.row_off[row]) + extra;
      double q0, q1;
      if (EROW == 1 || n <= 64)
        solve_row<1, 1, 0>(a, p, row, lane, nullptr, nullptr, q0, q1);
      else if (EROW == 2 || n <= 128)
        solve_row<(EROW < 2 ? EROW : 2), 1, 0>(a, p, row, lane, nullptr, nullptr, q0, q1);
      else if (EROW == 4 || n <= 256)
        solve_row<(EROW < 4 ? EROW : 4), 1, 0>(a, p, row, lane, nullptr, nullptr, q0, q1);
      else
        solve_row<EROW, 1, 0>(a, p, row, lane, nullptr, nullptr, q0, q1);
      if (ui == 0) {
        best0 = q0;
        best1 = q1;
        arg = u;
      } else {
        if (a.reach ? (q0 > best0) : (q0 < best0)) {
          best0 = q0;
          arg = u;
        }
        if (a.reach ? (q1 > best1) : (q1 < best1)) best1 = q1;
      }
    }
  }
  if (lane == 0) {
    a.vout[s] = make_double2(best0, best1);
    if (PASS == 0) a.pi[s] = arg;
  }
  const double gap = best1 - best0;
  return gap > 0.0 ? gap : 0.0;
}

template <int ESB, int EROW, int PASS, int D>
__global__ __launch_bounds__(64 * kSbWaves) void k_sweep_sb(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ SbLds<64 * ESB> lds[kSbWaves];
  __shared__ double gapw[kSbWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = uniform_i32(tid >> 6);
  const int64_t si = (int64_t)blockIdx.x * kSbWaves + wv;
  double gap = 0.0;
  if (si < a.n_safe) {
    const int64_t s = uniform_i64(a.safe[si]);
    gap = sb_sweep_state<ESB, EROW, PASS, D>(a, s, lane, lds[wv]);
  }
  if (lane == 0) gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = gapw[0];
    for (int w = 1; w < kSbWaves; ++w) gm = fmax(gm, gapw[w]);
    a.gap_part[blockIdx.x] = gm;
  }
}

// Close a pass for one state of a query (phase 1: lo, policy and the reset of
// the values for pass 2; phase 3: hi).
__device__ __forceinline__ void mq_close_state(const QueryDesc& D, int64_t step, int phase,
                                               int64_t s) {
  const double2* vin = (step & 1) ? D.vb1 : D.vb0;
  double2* vout = (step & 1) ? D.vb0 : D.vb1;
  const double2 V = vin[s];
  if (phase == 1) {
    D.lo[s] = D.safety ? 1.0 - V.y : V.x;
    D.pol[s] = D.a.pi[s];
    vout[s] = make_double2(0.0, 1.0);
  } else {
    D.hi[s] = D.safety ? 1.0 - V.x : V.y;
  }
}

// The state-box update of one item, specialised on its grid dimension when
// the kernel has no per-row fallback (EROW == 0).
template <int ESB, int EROW, int PASS>
__device__ double mq_sb_pass(const SweepArgs& a, int d, int64_t s, int lane,
                             SbLds<64 * ESB>& L) {
  if constexpr (EROW == 0) {
    switch (d) {
      case 2: return sb_sweep_state<ESB, 0, PASS, 2>(a, s, lane, L);
      case 3: return sb_sweep_state<ESB, 0, PASS, 3>(a, s, lane, L);
      case 5: return sb_sweep_state<ESB, 0, PASS, 5>(a, s, lane, L);
      default: return sb_sweep_state<ESB, 0, PASS, 0>(a, s, lane, L);
    }
  } else {
    return sb_sweep_state<ESB, EROW, PASS, 0>(a, s, lane, L);
  }
}

template <int ESB, int EROW>
__device__ double mq_sb_dispatch(const SweepArgs& a, int d, bool policy_pass, int64_t s,
                                 int lane, SbLds<64 * ESB>& L) {
  return policy_pass ? mq_sb_pass<ESB, EROW, 0>(a, d, s, lane, L)
                     : mq_sb_pass<ESB, EROW, 1>(a, d, s, lane, L);
}

// Multi-query state-box sweep: one wavefront per (query, SAFE state) item,
// each query at its own phase and step.
template <int ESB, int EROW>
__global__ __launch_bounds__(64 * kSbWaves) void k_mq_sweep_sb(
    const QueryDesc* __restrict__ desc, const QueryCtrl* __restrict__ ctrl,
    const int32_t* __restrict__ wq, const int32_t* __restrict__ ws, int64_t n_items,
    double* __restrict__ gap_item) {
  __shared__ SbLds<64 * ESB> lds[kSbWaves];
  const int lane = threadIdx.x & 63, wv = uniform_i32(threadIdx.x >> 6);
  const int64_t item = (int64_t)blockIdx.x * kSbWaves + wv;
  if (item >= n_items) return;
  const int q = uniform_i32(wq[item]);
  const int64_t s = uniform_i32(ws[item]);
  const int phase = uniform_i32(ctrl[q].phase);
  const int64_t step = uniform_i64(ctrl[q].step);
  const QueryDesc& D = desc[q];
  double g = 0.0;
  if (phase == 0 || phase == 2) {
    SweepArgs a = D.a;
    a.vin = (step & 1) ? D.vb1 : D.vb0;
    a.vout = (step & 1) ? D.vb0 : D.vb1;
    a.reach = !D.safety;
    a.pass = phase == 0 ? 0 : 1;
    a.maximise = phase == 0 ? D.safety : !D.safety;
    g = mq_sb_dispatch<ESB, EROW>(a, uniform_i32(a.d), phase == 0, s, lane, lds[wv]);
  } else if ((phase == 1 || phase == 3) && lane == 0) {
    mq_close_state(D, step, phase, s);
  }
  if (lane == 0) gap_item[item] = g;
}

static inline int lanes_elems(int64_t n) {
  return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 0;
}

template <int PASS>
static hipError_t launch_sb_pass(const SweepArgs& a, int64_t max_box, int32_t max_row,
                                 hipStream_t st) {
  const int64_t blocks = (a.n_safe + kSbWaves - 1) / kSbWaves;
  const dim3 g((unsigned)blocks), bl(64 * kSbWaves);
  const int er = lanes_elems(max_row);
  if (er == 0) return hipErrorInvalidValue;
  const int eb = lanes_elems(max_box);
#define SB(E1, E2, D) hipLaunchKernelGGL((k_sweep_sb<E1, E2, PASS, D>), g, bl, 0, st, a)
#define SBD(E1)                       \
  switch (a.d) {                      \
    case 2: SB(E1, 0, 2); break;      \
    case 3: SB(E1, 0, 3); break;      \
    case 5: SB(E1, 0, 5); break;      \
    default: SB(E1, 0, 0); break;     \
  }
  switch (eb) {
    case 1: SBD(1); break;
    case 2: SBD(2); break;
    case 4: SBD(4); break;
    case 8: SBD(8); break;
    default:  // some boxes exceed 512 cells: per-row sorts for those states
      switch (er) {
        case 1: SB(8, 1, 0); break;
        case 2: SB(8, 2, 0); break;
        case 4: SB(8, 4, 0); break;
        default: SB(8, 8, 0); break;
      }
  }
#undef SBD
#undef SB
  return hipGetLastError();
}

hipError_t launch_mq_sweep_sb(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                              const int32_t* ws, int64_t n_items, double* gap_item,
                              int64_t max_box, int32_t max_row, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const dim3 g((unsigned)((n_items + kSbWaves - 1) / kSbWaves)), bl(64 * kSbWaves);
  const int er = lanes_elems(max_row);
  if (er == 0) return hipErrorInvalidValue;
  const int eb = lanes_elems(max_box);
#define MQ(E1, E2) \
  hipLaunchKernelGGL((k_mq_sweep_sb<E1, E2>), g, bl, 0, st, desc, ctrl, wq, ws, n_items, gap_item)
  switch (eb) {
    case 1: MQ(1, 0); break;
    case 2: MQ(2, 0); break;
    case 4: MQ(4, 0); break;
    case 8: MQ(8, 0); break;
    default:
      switch (er) {
        case 1: MQ(8, 1); break;
        case 2: MQ(8, 2); break;
        case 4: MQ(8, 4); break;
        default: MQ(8, 8); break;
      }
  }
#undef MQ
  return hipGetLastError();
}

hipError_t launch_sweep_sb(const SweepArgs& a, int64_t max_box, int32_t max_row, hipStream_t st) {
  if (a.n_safe == 0) return hipSuccess;
  // pass 2 uses one row per state: its box is the row's own window
  return a.pass == 0 ? launch_sb_pass<0>(a, max_box, max_row, st)
                     : launch_sb_pass<1>(a, max_row, max_row, st);
}

// Largest state box of every instance (one thread per global state).
__global__ void k_state_box_max(BuildTable T, int64_t n_states, const int32_t* __restrict__ win,
                                unsigned long long* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long P = 0;
  int inst = T.n - 1;
  if (g < n_states) {
    inst = T.n == 1 ? 0 : find_base(T.state_base, T.n, g);
    const SysParams& p = T.sys[inst];
    const int64_t s = g - p.state_base;
    const int d = p.d;
    int lo[kMaxDim], hi[kMaxDim];
    IMPACT_FOR_DIMS(i, d) {
      lo[i] = 0x7fffffff;
      hi[i] = -0x7fffffff;
    }
    for (int u = 0; u < p.nu; ++u) {
      const int32_t* wr = win + p.win_base + (s * p.nu + u) * 2 * d;
      bool empty = false;
      IMPACT_FOR_DIMS(i, d) empty = empty || wr[d + i] == 0;
      if (empty) continue;
      IMPACT_FOR_DIMS(i, d) {
        lo[i] = wr[i] < lo[i] ? wr[i] : lo[i];
        hi[i] = wr[i] + wr[d + i] > hi[i] ? wr[i] + wr[d + i] : hi[i];
      }
    }
    P = 1;
    IMPACT_FOR_DIMS(i, d) P *= (unsigned long long)(hi[i] > lo[i] ? hi[i] - lo[i] : 0);
  }
  const int first = __shfl(inst, 0);
  if (__all(inst == first)) {
    for (int off = 32; off > 0; off >>= 1) {
      unsigned long long y = __shfl_xor(P, off);
      P = y > P ? y : P;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(&out[inst], P);
  } else if (g < n_states) {
    atomicMax(&out[inst], P);
  }
}

hipError_t launch_state_box_max(const BuildTable& T, int64_t n_states, const int32_t* win,
                                unsigned long long* out, hipStream_t st) {
  if (n_states == 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_box_max, dim3((unsigned)((n_states + 255) / 256)), dim3(256), 0, st,
                     T, n_states, win, out);
  return hipGetLastError();
}

}  // namespace impact
