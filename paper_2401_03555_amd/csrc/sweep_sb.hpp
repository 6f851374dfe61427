// sweep_sb.hpp -- interval-iteration sweep with one sort per state (or per
// group of its inputs).
//
// The rows (s, u) of one state have target windows that overlap almost
// entirely (the input moves the mean by a fraction of the window).  The LP of
// a row (eq. (5.1), sorting method of Section 6.2) only needs the row's
// entries in value order, and the order of a subset of a sorted list is the
// subset's own sorted order.  So one wavefront per SAFE state
//   1. takes its inputs in consecutive groups whose windows' bounding box B
//      fits the wavefront (every input at once when the whole box fits),
//   2. gathers (V0, V1) over the cells of B into LDS and bitonic-sorts B
//      twice (keys: IEEE bits of the value, complemented for a maximising LP;
//      payload: the cell's position in B), keeping each cell's position in
//      both orders,
//   3. for each input of the group: lanes hold the row's window cells with
//      their widths hi - lo and order positions; the greedy of the sorting
//      method fills widths in order until the budget 1 - sum(lo) runs out at
//      one critical cell, found by bisection over order positions on group
//      sums of the widths below a position,
//   4. keeps the max (reach) / min (safety) over inputs and the policy.
// OUT and TAIL have values exactly 0 or 1, the extremes of every order, so
// they sit before or after all cells and are handled in closed form.
// The result equals the per-row sort's LP values up to summation order.
#pragma once

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

// Inclusive prefix min / max across the wavefront (lane l: over lanes 0..l).
__device__ __forceinline__ int wave_prefix_min_i32(int x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ int wave_prefix_max_i32(int x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x = y > x ? y : x;
  }
  return x;
}

// The next group of consecutive inputs [g0, g1) of state s whose windows'
// bounding box holds at most cap cells: the longest run from g0 (at most 64
// inputs) for which it does, or the single input g0 when its own window is
// larger.  Rows whose window is empty in some dimension hold no cells and do
// not widen the box.  D > 0: the grid dimension is the compile-time D (every
// dimension loop unrolls to straight-line code); D == 0: read at run time.
template <int PASS, int D>
__device__ __forceinline__ int group_box(const SweepArgs& a, int64_t s, int g0, int U, int64_t cap, int lane,
                         StateBox& b) {
  const int d = D > 0 ? D : a.d;
  int lo[kMaxDim], hi[kMaxDim];
  IMPACT_FOR_DIMS(i, d) {
    lo[i] = 0x7fffffff;
    hi[i] = -0x7fffffff;
  }
  const int ui = g0 + lane;
  if (ui < U) {
    const int64_t row = s * a.nu + row_input<PASS>(a, s, ui);
    const int32_t* wr = a.win + row * 2 * d;
    bool empty = false;
    IMPACT_FOR_DIMS(i, d) empty = empty || wr[d + i] == 0;
    if (!empty)
      IMPACT_FOR_DIMS(i, d) {
        lo[i] = wr[i];
        hi[i] = wr[i] + wr[d + i];
      }
  }
  int64_t P = 1;
  IMPACT_FOR_DIMS(i, d) {
    lo[i] = wave_prefix_min_i32(lo[i], lane);
    hi[i] = wave_prefix_max_i32(hi[i], lane);
    P *= hi[i] > lo[i] ? (int64_t)(hi[i] - lo[i]) : 0;
  }
  // first lane whose prefix box is too large ends the group (at least one row)
  const bool over = ui < U && P > cap;
  const uint64_t m = (uint64_t)__ballot(over);
  const int n_in = U - g0 < 64 ? U - g0 : 64;
  int len = m ? __builtin_ctzll(m) : n_in;
  if (len == 0) len = 1;
  const int last = len - 1;
  int64_t PB = 1;
  IMPACT_FOR_DIMS(i, d) {
    const int l = uniform_i32(__shfl(lo[i], last)), h = uniform_i32(__shfl(hi[i], last));
    b.blo[i] = l;
    b.ext[i] = h > l ? h - l : 0;
    PB *= b.ext[i];
  }
  int32_t st = 1;
  IMPACT_FOR_DIMS_REV(i, d) {
    b.bstride[i] = st;
    st = (int32_t)((int64_t)st * b.ext[i] > 0x3fffffff ? 0x3fffffff : st * b.ext[i]);
  }
  b.P = PB;
  return g0 + len;
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

// Bitonic sort of one key set, 64 lanes x E keys, blocked layout, ascending.
template <int E>
__device__ void bitonic_sort1(uint64_t (&ka)[E], int32_t (&pa)[E], int lane) {
  constexpr int P = 64 * E;
  // fully unrolled (compile-time partner distances) up to 256 keys; the
  // 512-key network keeps its loops, which holds its register footprint
  constexpr int kUnroll = E >= 8 ? 1 : 16;
#pragma unroll kUnroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll kUnroll
    for (int j = k >> 1; j >= E; j >>= 1) {
      const int tm = j / E;
      const bool lower = (lane & tm) == 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool asc = ((lane * E + e) & k) == 0;
        const uint64_t qa = xor_lane_u64(ka[e], tm);
        const int32_t ra = xor_lane_i32(pa[e], tm);
        const bool keep_min = asc == lower;
        if (keep_min ? !(ka[e] < qa) : !(ka[e] > qa)) {
          ka[e] = qa;
          pa[e] = ra;
        }
      }
    }
    intra_stages<E, int32_t>(ka, pa, lane, k);
  }
}

// Bitonic sort of two key sets at once (same network, independent data),
// 64 lanes x E keys each, blocked layout, ascending.
template <int E>
__device__ void bitonic_sort2(uint64_t (&ka)[E], int32_t (&pa)[E], uint64_t (&kb)[E],
                              int32_t (&pb)[E], int lane) {
  constexpr int P = 64 * E;
  // fully unrolled (compile-time partner distances) up to 256 keys; the
  // 512-key network keeps its loops, which holds its register footprint
  constexpr int kUnroll = E >= 8 ? 1 : 16;
#pragma unroll kUnroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll kUnroll
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

// Per-wavefront LDS of the state-box path (P = box capacity): each box cell's
// (V0, V1) and its position in the two sorted orders; capacities of at most
// 128 cells also get one staging array of P (width, value) pairs per lane
// group for the scan form of the greedy (kernels of larger capacity use the
// bisection form for every group, so their smaller groups need no staging).
template <int P>
struct SbLdsCore {
  double2 vb[P];
  uint16_t rk[2][P];
  double2 stg[P <= 128 ? 4 : 1][P <= 128 ? P + P / 8 : 1];
};

// Staging slot of order position j: one pad slot after every 8 positions, so
// that lanes reading 8 consecutive positions each do not all start on the
// same LDS bank.
__device__ __forceinline__ int stg_slot(int j) { return j + (j >> 3); }
template <int P>
struct SbLds : SbLdsCore<P> {};

// Entries held per lane: a row of up to 8 * GW window cells on a GW-lane group.
constexpr int kSbEntriesPerLane = 8;

// A row entry held by a lane: its width dd = hi - lo and one packed word with
// its positions in the two sorted orders (bits 0-9, 10-19) and in the box
// (bits 20-29); kNoEntry marks an empty slot (positions 1023, beyond any box).
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;
__device__ __forceinline__ int entry_pos(uint32_t pk, int order) {
  return (int)((pk >> (10 * order)) & 1023u);
}
__device__ __forceinline__ int entry_box(uint32_t pk) { return (int)((pk >> 20) & 1023u); }

// Sorting-method LP of one row along one order, without walking the order:
// the greedy gives every entry its full width dd until the budget rb runs
// out at one critical entry, so the result only needs the critical position
// j* = max{ j : S(j) <= rb }, with S(j) the row's total dd over order
// positions below j.  S is monotone, so j* is found by bisection on group
// sums.  Entries at positions below j* add dd * v, the critical one adds the
// rest of the budget times its value.  Lane gl of the GW-lane group holds
// entries k = 0..EL-1; values come from the box's LDS copy.  Returns the group
// sum of the cells' greedy mass times value, and the cells' total width in
// `total`.
template <int EL, int GW, int P>
__device__ double sb_greedy(const double (&dd)[EL], const uint32_t (&pk)[EL], int order,
                            const SbLds<P>& L, int PB, double rb, double& total) {
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < EL; ++k) t += dd[k];
  total = group_sum_dpp<GW>(t);
  int lo = 0, hi = PB + 1;  // S(lo) <= rb (or lo == 0), S(hi) > rb (or hi == PB + 1)
  double s_lo = 0.0;
  if (total <= rb) {
    lo = PB;
    s_lo = total;
  } else {
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < EL; ++k) x += entry_pos(pk[k], order) < mid ? dd[k] : 0.0;
      x = group_sum_dpp<GW>(x);
      if (x <= rb) {
        lo = mid;
        s_lo = x;
      } else {
        hi = mid;
      }
    }
  }
  const double room = rb - s_lo;
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < EL; ++k) {
    const int ps = entry_pos(pk[k], order);
    if (ps <= lo && pk[k] != kNoEntry) {
      const double2 V = L.vb[entry_box(pk[k])];
      const double v = order == 0 ? V.x : V.y;
      if (ps < lo) {
        q += dd[k] * v;
      } else {
        const double delta = room <= 0.0 ? 0.0 : (dd[k] < room ? dd[k] : room);
        q += delta * v;
      }
    }
  }
  return group_sum_dpp<GW>(q);
}

// One row's LP value along one order (specials at the front or the back).
template <int EL, int GW, int P>
__device__ double sb_row_lp(const double (&dd)[EL], const uint32_t (&pk)[EL], int order,
                            const SbLds<P>& L, int PB, double r, double slv, bool mx,
                            const Specials& sp) {
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
  const double qc = sb_greedy<EL, GW, P>(dd, pk, order, L, PB, r - front, total);
  double back = front + total;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= sp.n || special_front(sp.v[k], mx)) continue;
    const double room = r - back;
    const double delta = room <= 0.0 ? 0.0 : (sp.dd[k] < room ? sp.dd[k] : room);
    q_sp += (sp.lo[k] + delta) * sp.v[k];
    back += sp.dd[k];
  }
  return slv + qc + q_sp;
}

// One row's LP value along one order in scan form (boxes of at most 128
// cells): the row's cells are placed at their order positions in the lane
// group's staging array (width, value; zero elsewhere), and the group walks
// the order once, R = 64E / GW positions per lane, with an exclusive prefix
// sum of the widths -- the sorting method's greedy as written.  Cheaper in
// VALU than the bisection when the box is small.
template <int EL, int GW, int E>
__device__ double sb_row_scan(const double (&dd)[EL], const uint32_t (&pk)[EL], int order,
                              const SbLds<64 * E>& L, double2* __restrict__ stg, int gl,
                              double r, double slv, bool mx, const Specials& sp) {
  constexpr int R = 64 * E / GW;
#pragma unroll
  for (int k = 0; k < R; ++k) stg[stg_slot(gl * R + k)] = make_double2(0.0, 0.0);
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < EL; ++k) {
    if (pk[k] != kNoEntry) {
      const double2 V = L.vb[entry_box(pk[k])];
      stg[stg_slot(entry_pos(pk[k], order))] = make_double2(dd[k], order == 0 ? V.x : V.y);
    }
  }
  wave_lds_sync();
  // two passes over the lane's positions (widths, then widths and values):
  // re-reading LDS is cheaper than holding 2R doubles in registers
  double lane_d = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) lane_d += stg[stg_slot(gl * R + k)].x;
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
  double acc = front + excl, lane_q = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double2 x = stg[stg_slot(gl * R + k)];
    const double room = r - acc;
    const double delta = room <= 0.0 ? 0.0 : (x.x < room ? x.x : room);
    lane_q += delta * x.y;
    acc += x.x;
  }
  wave_lds_sync();
  double back = front + total;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= sp.n || special_front(sp.v[k], mx)) continue;
    const double room = r - back;
    const double delta = room <= 0.0 ? 0.0 : (sp.dd[k] < room ? sp.dd[k] : room);
    q_sp += (sp.lo[k] + delta) * sp.v[k];
    back += sp.dd[k];
  }
  return slv + group_sum_dpp<GW>(lane_q) + q_sp;
}

// One group of inputs [g0, g1) of a SAFE state on one wavefront, box of at
// most 64*E cells.  The box is sorted with 64 lanes (once per order); then
// lane groups of GW lanes take rows u = g0 + g, g0 + g + 64/GW, ..., each lane
// holding up to 8 of the row's window cells with their widths, values and
// order positions.  The group's best is merged into (best0, best1, arg),
// which hold the earlier groups' (lower inputs') best.
template <int E, int GW, int PASS, int D, bool SCAN>
__device__ __forceinline__ void sb_state(const SweepArgs& a, const SysParams& p, int64_t s, int g0, int g1,
                         const StateBox& b, int lane, SbLds<64 * E>& L, double& best0,
                         double& best1, int& arg) {
  constexpr int NG = 64 / GW, EL = kSbEntriesPerLane;
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
        L.vb[bi] = V;
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
    if constexpr (E >= 8) {
      // one order at a time: half the registers of the paired network
      bitonic_sort1<E>(k0, p0, lane);
      bitonic_sort1<E>(k1, p1, lane);
    } else {
      bitonic_sort2<E>(k0, p0, k1, p1, lane);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = lane * E + e;
      if (p0[e] < PB) L.rk[0][p0[e]] = (uint16_t)j;
      if (p1[e] < PB) L.rk[1][p1[e]] = (uint16_t)j;
    }
  }
  wave_lds_sync();

  const int g = lane / GW, gl = lane % GW;
  const double tail_v = mx ? 1.0 : 0.0;
  const double worst = a.reach ? -1.0 : 2.0;
  double gb0 = worst, gb1 = worst;
  int garg = 0x7fffffff;
  for (int ui0 = g0; ui0 < g1; ui0 += NG) {
    const int ui = ui0 + g;
    const bool act = ui < g1;
    double dd[EL];
    uint32_t pk[EL];
    double lane_lo = 0.0, lq0 = 0.0, lq1 = 0.0;
#pragma unroll
    for (int k = 0; k < EL; ++k) {
      dd[k] = 0.0;
      pk[k] = kNoEntry;
    }
    int u = 0;
    int64_t row = 0;
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
        int64_t q0i = gl, q1i = GW;
        IMPACT_FOR_DIMS_REV(i, d) {
          j[i] = (int32_t)(q0i % W[i]);
          q0i /= W[i];
          inc[i] = (int32_t)(q1i % W[i]);
          q1i /= W[i];
        }
        const double2* fr = a.fac ? a.fac + row * (int64_t)a.fs : nullptr;
#pragma unroll
        for (int k = 0; k < EL; ++k) {
          const int slot = gl + k * GW;
          if (slot < nw) {
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
            const double2 V = L.vb[bi];
            dd[k] = e.y - e.x;
            pk[k] = (uint32_t)L.rk[0][bi] | ((uint32_t)L.rk[1][bi] << 10) | ((uint32_t)bi << 20);
            lane_lo += e.x;
            lq0 += e.x * V.x;
            lq1 += e.x * V.y;
            int carry = 0;
            IMPACT_FOR_DIMS_REV(i, d) {
              j[i] += inc[i] + carry;
              carry = j[i] >= W[i];
              if (carry) j[i] -= W[i];
            }
          }
        }
      }
    }
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
      const double s0 = group_sum<GW>(lq0), s1 = group_sum<GW>(lq1);
      double q0, q1;
      if constexpr (SCAN && E <= 2) {
        q0 = sb_row_scan<EL, GW, E>(dd, pk, 0, L, L.stg[g], gl, r, s0, mx, sp);
        q1 = sb_row_scan<EL, GW, E>(dd, pk, 1, L, L.stg[g], gl, r, s1, mx, sp);
      } else {
        q0 = sb_row_lp<EL, GW, 64 * E>(dd, pk, 0, L, (int)PB, r, s0, mx, sp);
        q1 = sb_row_lp<EL, GW, 64 * E>(dd, pk, 1, L, (int)PB, r, s1, mx, sp);
      }
      // rows of a group come in increasing u: a strict improvement keeps the lowest u
      if (a.reach ? (q0 > gb0) : (q0 < gb0)) {
        gb0 = q0;
        garg = u;
      }
      if (a.reach ? (q1 > gb1) : (q1 < gb1)) gb1 = q1;
    }
  }
  // combine the lane groups: best value, lowest input on exact ties
#pragma unroll
  for (int off = GW; off < 64; off <<= 1) {
    const double o0 = __shfl_xor(gb0, off), o1 = __shfl_xor(gb1, off);
    const int oa = __shfl_xor(garg, off);
    const bool better = a.reach ? (o0 > gb0 || (o0 == gb0 && oa < garg))
                                : (o0 < gb0 || (o0 == gb0 && oa < garg));
    if (better) {
      gb0 = o0;
      garg = oa;
    }
    gb1 = a.reach ? fmax(gb1, o1) : fmin(gb1, o1);
  }
  // earlier groups hold lower inputs: a strict improvement is needed to replace them
  if (a.reach ? (gb0 > best0) : (gb0 < best0)) {
    best0 = gb0;
    arg = garg;
  }
  best1 = a.reach ? fmax(best1, gb1) : fmin(best1, gb1);
}

// Sweep update of one SAFE state s on one wavefront: writes vout[s] (and
// pi[s] in the policy pass); returns the state's V1 - V0 (>= 0).  The inputs
// are taken in consecutive groups whose windows' box holds at most 64 * ESB
// cells (one sort per group); a single row always fits, because the state-box
// kernels run only on abstractions whose rows have at most 512 entries and
// ESB is 8 unless every state's whole box fits.
template <int ESB, int GW, int PASS, int D>
__device__ __forceinline__ double sb_sweep_state(const SweepArgs& a, int64_t s, int lane,
                                                SbLds<64 * ESB>& L) {
  const SysParams& p = *a.sys;
  const int U = PASS == 0 ? a.nu : 1;
  const double worst = a.reach ? -1.0 : 2.0;
  double best0 = worst, best1 = worst;
  int arg = 0x7fffffff;
  for (int g0 = 0; g0 < U;) {
    StateBox b;
    const int g1 = uniform_i32(group_box<PASS, D>(a, s, g0, U, 64 * ESB, lane, b));
    if (ESB == 1 || b.P <= 64)
      sb_state<1, GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane, *(SbLds<64>*)&L, best0, best1, arg);
    else if (ESB == 2 || b.P <= 128)
      sb_state<(ESB < 2 ? ESB : 2), GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane,
                                              *(SbLds<64 * (ESB < 2 ? ESB : 2)>*)&L, best0,
                                              best1, arg);
    else if (ESB == 4 || b.P <= 256)
      sb_state<(ESB < 4 ? ESB : 4), GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane,
                                              *(SbLds<64 * (ESB < 4 ? ESB : 4)>*)&L, best0,
                                              best1, arg);
    else
      sb_state<ESB, GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane, L, best0, best1, arg);
    g0 = g1;
    wave_lds_sync();
  }
  if (lane == 0) {
    a.vout[s] = make_double2(best0, best1);
    if (PASS == 0) a.pi[s] = arg;
  }
  const double gap = best1 - best0;
  return gap > 0.0 ? gap : 0.0;
}

template <int ESB, int GW, int PASS, int D>
__global__ __launch_bounds__(64 * kSbWaves) void k_sweep_sb(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ SbLds<64 * ESB> lds[kSbWaves];
  __shared__ double gapw[kSbWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = uniform_i32(tid >> 6);
  const int64_t si = (int64_t)blockIdx.x * kSbWaves + wv;
  double gap = 0.0;
  if (si < a.n_safe) {
    const int64_t s = uniform_i64(a.safe[si]);
    gap = sb_sweep_state<ESB, GW, PASS, D>(a, s, lane, lds[wv]);
  }
  if (lane == 0) gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = gapw[0];
    for (int w = 1; w < kSbWaves; ++w) gm = fmax(gm, gapw[w]);
    a.gap_part[blockIdx.x] = gm;
  }
}


// ---- the same sweep with a disturbance player (rows (s, u, w)) -------------
// Separate copies of the functions above, so that the kernels without a
// disturbance player keep their register allocation.  A lane group takes an
// item (an input, or the policy's input) and walks its disturbance rows,
// keeping the worst; an item's box covers all of its rows' windows.

// Row of item ui of state s (an input of the policy pass, the policy's input
// in the fixed-input pass) and disturbance w.
template <int PASS>
__device__ __forceinline__ int64_t dist_row(const SweepArgs& a, int64_t s, int ui, int w) {
  return (s * a.nu + row_input<PASS>(a, s, ui)) * a.nw + w;
}

template <int PASS, int D>
__device__ __forceinline__ int group_box_dist(const SweepArgs& a, int64_t s, int g0, int U, int64_t cap, int lane,
                         StateBox& b) {
  const int d = D > 0 ? D : a.d;
  int lo[kMaxDim], hi[kMaxDim];
  IMPACT_FOR_DIMS(i, d) {
    lo[i] = 0x7fffffff;
    hi[i] = -0x7fffffff;
  }
  const int ui = g0 + lane;
  if (ui < U) {
    // an item's box covers the windows of all its disturbance rows
    for (int w = 0; w < a.nw; ++w) {
      const int32_t* wr = a.win + dist_row<PASS>(a, s, ui, w) * 2 * d;
      bool empty = false;
      IMPACT_FOR_DIMS(i, d) empty = empty || wr[d + i] == 0;
      if (!empty)
        IMPACT_FOR_DIMS(i, d) {
          lo[i] = wr[i] < lo[i] ? wr[i] : lo[i];
          hi[i] = wr[i] + wr[d + i] > hi[i] ? wr[i] + wr[d + i] : hi[i];
        }
    }
  }
  int64_t P = 1;
  IMPACT_FOR_DIMS(i, d) {
    lo[i] = wave_prefix_min_i32(lo[i], lane);
    hi[i] = wave_prefix_max_i32(hi[i], lane);
    P *= hi[i] > lo[i] ? (int64_t)(hi[i] - lo[i]) : 0;
  }
  // first lane whose prefix box is too large ends the group (at least one row)
  const bool over = ui < U && P > cap;
  const uint64_t m = (uint64_t)__ballot(over);
  const int n_in = U - g0 < 64 ? U - g0 : 64;
  int len = m ? __builtin_ctzll(m) : n_in;
  if (len == 0) len = 1;
  const int last = len - 1;
  int64_t PB = 1;
  IMPACT_FOR_DIMS(i, d) {
    const int l = uniform_i32(__shfl(lo[i], last)), h = uniform_i32(__shfl(hi[i], last));
    b.blo[i] = l;
    b.ext[i] = h > l ? h - l : 0;
    PB *= b.ext[i];
  }
  int32_t st = 1;
  IMPACT_FOR_DIMS_REV(i, d) {
    b.bstride[i] = st;
    st = (int32_t)((int64_t)st * b.ext[i] > 0x3fffffff ? 0x3fffffff : st * b.ext[i]);
  }
  b.P = PB;
  return g0 + len;
}


template <int E, int GW, int PASS, int D, bool SCAN>
__device__ __forceinline__ void sb_state_dist(const SweepArgs& a, const SysParams& p, int64_t s, int g0, int g1,
                         const StateBox& b, int lane, SbLds<64 * E>& L, double& best0,
                         double& best1, int& arg) {
  constexpr int NG = 64 / GW, EL = kSbEntriesPerLane;
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
        L.vb[bi] = V;
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
    if constexpr (E >= 8) {
      // one order at a time: half the registers of the paired network
      bitonic_sort1<E>(k0, p0, lane);
      bitonic_sort1<E>(k1, p1, lane);
    } else {
      bitonic_sort2<E>(k0, p0, k1, p1, lane);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = lane * E + e;
      if (p0[e] < PB) L.rk[0][p0[e]] = (uint16_t)j;
      if (p1[e] < PB) L.rk[1][p1[e]] = (uint16_t)j;
    }
  }
  wave_lds_sync();

  const int g = lane / GW, gl = lane % GW;
  const double tail_v = mx ? 1.0 : 0.0;
  const double worst = a.reach ? -1.0 : 2.0;
  double gb0 = worst, gb1 = worst;
  int garg = 0x7fffffff;
  for (int ui0 = g0; ui0 < g1; ui0 += NG) {
    const int ui = ui0 + g;
    const bool act = ui < g1;
    int u = 0;
    // with a disturbance player the item's value is its worst row over them
    double wq0 = 0.0, wq1 = 0.0;
    // one row of the item: its LP values, folded into the item's value
    auto row_pass = [&](const int w) __attribute__((always_inline)) {
    double dd[EL];
    uint32_t pk[EL];
    double lane_lo = 0.0, lq0 = 0.0, lq1 = 0.0;
#pragma unroll
    for (int k = 0; k < EL; ++k) {
      dd[k] = 0.0;
      pk[k] = kNoEntry;
    }
    int64_t row = 0;
    if (act) {
      u = row_input<PASS>(a, s, ui);
      row = dist_row<PASS>(a, s, ui, w);
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
        int64_t q0i = gl, q1i = GW;
        IMPACT_FOR_DIMS_REV(i, d) {
          j[i] = (int32_t)(q0i % W[i]);
          q0i /= W[i];
          inc[i] = (int32_t)(q1i % W[i]);
          q1i /= W[i];
        }
        const double2* fr = a.fac ? a.fac + row * (int64_t)a.fs : nullptr;
#pragma unroll
        for (int k = 0; k < EL; ++k) {
          const int slot = gl + k * GW;
          if (slot < nw) {
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
            const double2 V = L.vb[bi];
            dd[k] = e.y - e.x;
            pk[k] = (uint32_t)L.rk[0][bi] | ((uint32_t)L.rk[1][bi] << 10) | ((uint32_t)bi << 20);
            lane_lo += e.x;
            lq0 += e.x * V.x;
            lq1 += e.x * V.y;
            int carry = 0;
            IMPACT_FOR_DIMS_REV(i, d) {
              j[i] += inc[i] + carry;
              carry = j[i] >= W[i];
              if (carry) j[i] -= W[i];
            }
          }
        }
      }
    }
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
      const double s0 = group_sum<GW>(lq0), s1 = group_sum<GW>(lq1);
      double q0, q1;
      if constexpr (SCAN && E <= 2) {
        q0 = sb_row_scan<EL, GW, E>(dd, pk, 0, L, L.stg[g], gl, r, s0, mx, sp);
        q1 = sb_row_scan<EL, GW, E>(dd, pk, 1, L, L.stg[g], gl, r, s1, mx, sp);
      } else {
        q0 = sb_row_lp<EL, GW, 64 * E>(dd, pk, 0, L, (int)PB, r, s0, mx, sp);
        q1 = sb_row_lp<EL, GW, 64 * E>(dd, pk, 1, L, (int)PB, r, s1, mx, sp);
      }
      wq0 = w == 0 ? q0 : (a.reach ? fmin(wq0, q0) : fmax(wq0, q0));
      wq1 = w == 0 ? q1 : (a.reach ? fmin(wq1, q1) : fmax(wq1, q1));
    }
    };
    for (int w = 0; w < a.nw; ++w) row_pass(w);
    // items of a group come in increasing u: a strict improvement keeps the lowest u
    if (act) {
      if (a.reach ? (wq0 > gb0) : (wq0 < gb0)) {
        gb0 = wq0;
        garg = u;
      }
      if (a.reach ? (wq1 > gb1) : (wq1 < gb1)) gb1 = wq1;
    }
  }
  // combine the lane groups: best value, lowest input on exact ties
#pragma unroll
  for (int off = GW; off < 64; off <<= 1) {
    const double o0 = __shfl_xor(gb0, off), o1 = __shfl_xor(gb1, off);
    const int oa = __shfl_xor(garg, off);
    const bool better = a.reach ? (o0 > gb0 || (o0 == gb0 && oa < garg))
                                : (o0 < gb0 || (o0 == gb0 && oa < garg));
    if (better) {
      gb0 = o0;
      garg = oa;
    }
    gb1 = a.reach ? fmax(gb1, o1) : fmin(gb1, o1);
  }
  // earlier groups hold lower inputs: a strict improvement is needed to replace them
  if (a.reach ? (gb0 > best0) : (gb0 < best0)) {
    best0 = gb0;
    arg = garg;
  }
  best1 = a.reach ? fmax(best1, gb1) : fmin(best1, gb1);
}

template <int ESB, int GW, int PASS, int D>
__device__ __forceinline__ double sb_sweep_state_dist(const SweepArgs& a, int64_t s, int lane,
                                                SbLds<64 * ESB>& L) {
  const SysParams& p = *a.sys;
  const int U = PASS == 0 ? a.nu : 1;
  const double worst = a.reach ? -1.0 : 2.0;
  double best0 = worst, best1 = worst;
  int arg = 0x7fffffff;
  for (int g0 = 0; g0 < U;) {
    StateBox b;
    const int g1 = uniform_i32(group_box_dist<PASS, D>(a, s, g0, U, 64 * ESB, lane, b));
    if (ESB == 1 || b.P <= 64)
      sb_state_dist<1, GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane, *(SbLds<64>*)&L, best0,
                                                 best1, arg);
    else if (ESB == 2 || b.P <= 128)
      sb_state_dist<(ESB < 2 ? ESB : 2), GW, PASS, D, (ESB <= 2)>(
          a, p, s, g0, g1, b, lane, *(SbLds<64 * (ESB < 2 ? ESB : 2)>*)&L, best0, best1, arg);
    else if (ESB == 4 || b.P <= 256)
      sb_state_dist<(ESB < 4 ? ESB : 4), GW, PASS, D, (ESB <= 2)>(
          a, p, s, g0, g1, b, lane, *(SbLds<64 * (ESB < 4 ? ESB : 4)>*)&L, best0, best1, arg);
    else
      sb_state_dist<ESB, GW, PASS, D, (ESB <= 2)>(a, p, s, g0, g1, b, lane, L, best0, best1,
                                                   arg);
    g0 = g1;
    wave_lds_sync();
  }
  if (lane == 0) {
    a.vout[s] = make_double2(best0, best1);
    if (PASS == 0) a.pi[s] = arg;
  }
  const double gap = best1 - best0;
  return gap > 0.0 ? gap : 0.0;
}

template <int ESB, int GW, int PASS, int D>
__global__ __launch_bounds__(64 * kSbWaves) void k_sweep_sb_dist(SweepArgs a) {
  if (a.ctrl->done) return;
  __shared__ SbLds<64 * ESB> lds[kSbWaves];
  __shared__ double gapw[kSbWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = uniform_i32(tid >> 6);
  const int64_t si = (int64_t)blockIdx.x * kSbWaves + wv;
  double gap = 0.0;
  if (si < a.n_safe) {
    const int64_t s = uniform_i64(a.safe[si]);
    gap = sb_sweep_state_dist<ESB, GW, PASS, D>(a, s, lane, lds[wv]);
  }
  if (lane == 0) gapw[wv] = gap;
  __syncthreads();
  if (tid == 0) {
    double gm = gapw[0];
    for (int w = 1; w < kSbWaves; ++w) gm = fmax(gm, gapw[w]);
    a.gap_part[blockIdx.x] = gm;
  }
}

// Multi-query state-box sweep of the policy pass (and the closing steps):
// one wavefront per (query, SAFE state) item,
// each query at its own phase and step.
template <int ESB, int GW, int DIM>
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
  // the fixed-input pass of these queries runs in k_mq_sweep_row
  if (phase == 2) return;
  double g = 0.0;
  if (phase == 0) {
    SweepArgs a = D.a;
    a.vin = (step & 1) ? D.vb1 : D.vb0;
    a.vout = (step & 1) ? D.vb0 : D.vb1;
    a.reach = !D.safety;
    a.pass = 0;
    a.maximise = D.max_lp[0];
    g = sb_sweep_state<ESB, GW, 0, DIM>(a, s, lane, lds[wv]);
  } else if ((phase == 1 || phase == 3) && lane == 0) {
    mq_close_state(D, ctrl[q], phase, s);
  }
  if (lane == 0) gap_item[item] = g;
}

inline int lanes_elems(int64_t n) {
  return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 0;
}

// Kernel variant for a largest state box of max_box cells (boxes beyond 512
// cells are split into input groups by the 512-cell variants) and rows of at
// most max_row entries (at most 512; a row's cells go to 16, 32 or 64 lanes,
// 8 per lane).  Returns the element count and lane-group width through eb/gw.
inline bool sb_variant(int64_t max_box, int32_t max_row, int& eb, int& gw) {
  if (max_row > 512) return false;
  gw = max_row <= 128 ? 16 : max_row <= 256 ? 32 : 64;
  eb = lanes_elems(max_box < 512 ? max_box : 512);
  const int need = gw == 16 ? 1 : gw == 32 ? 2 : 4;  // the box holds a whole row
  if (eb < need) eb = need;
  return true;
}

#define IMPACT_SB_SWITCH(LAUNCH)                    \
  switch (gw * 16 + eb) {                           \
    case 16 * 16 + 1: LAUNCH(1, 16); break;         \
    case 16 * 16 + 2: LAUNCH(2, 16); break;         \
    case 16 * 16 + 4: LAUNCH(4, 16); break;         \
    case 16 * 16 + 8: LAUNCH(8, 16); break;         \
    case 32 * 16 + 2: LAUNCH(2, 32); break;         \
    case 32 * 16 + 4: LAUNCH(4, 32); break;         \
    case 32 * 16 + 8: LAUNCH(8, 32); break;         \
    case 64 * 16 + 4: LAUNCH(4, 64); break;         \
    default: LAUNCH(8, 64); break;                  \
  }

// Launchers of the kernels of one grid dimension D (0: any other); each
// sweep_sb_d*.hip instantiates one D, so the variants compile in parallel.
template <int D>
hipError_t launch_sb_d(const SweepArgs& a, int pass, int64_t max_box, int32_t max_row,
                       hipStream_t st) {
  int eb = 0, gw = 0;
  if (!sb_variant(max_box, max_row, eb, gw)) return hipErrorInvalidValue;
  const int64_t blocks = (a.n_safe + kSbWaves - 1) / kSbWaves;
  const dim3 g((unsigned)blocks), bl(64 * kSbWaves);
#define SB(E1, G1)                                                         \
  if (pass == 0)                                                           \
    hipLaunchKernelGGL((k_sweep_sb<E1, G1, 0, D>), g, bl, 0, st, a);       \
  else                                                                     \
    hipLaunchKernelGGL((k_sweep_sb<E1, G1, 1, D>), g, bl, 0, st, a);
  IMPACT_SB_SWITCH(SB)
#undef SB
  return hipGetLastError();
}

// With a disturbance player (a.nw > 1): the kernels that value each item by
// its worst disturbance row (instantiated for dimensions 2, 3 and any other).  Every item's box (the union
// of its rows' windows) must fit the capacity: the caller passes the largest
// state box, at most 512 cells.
template <int D>
hipError_t launch_sb_dist(const SweepArgs& a, int pass, int64_t max_box, int32_t max_row,
                          hipStream_t st) {
  int eb = 0, gw = 0;
  if (max_box > 512 || !sb_variant(max_box, max_row, eb, gw)) return hipErrorInvalidValue;
  const int64_t blocks = (a.n_safe + kSbWaves - 1) / kSbWaves;
  const dim3 g((unsigned)blocks), bl(64 * kSbWaves);
#define SBW(E1, G1)                                                              \
  if (pass == 0)                                                                 \
    hipLaunchKernelGGL((k_sweep_sb_dist<E1, G1, 0, D>), g, bl, 0, st, a);       \
  else                                                                           \
    hipLaunchKernelGGL((k_sweep_sb_dist<E1, G1, 1, D>), g, bl, 0, st, a);
  IMPACT_SB_SWITCH(SBW)
#undef SBW
  return hipGetLastError();
}

template <int D>
hipError_t launch_mq_sb_d(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                          const int32_t* ws, int64_t n_items, double* gap_item, int64_t max_box,
                          int32_t max_row, hipStream_t st) {
  int eb = 0, gw = 0;
  if (!sb_variant(max_box, max_row, eb, gw)) return hipErrorInvalidValue;
  const dim3 g((unsigned)((n_items + kSbWaves - 1) / kSbWaves)), bl(64 * kSbWaves);
#define MQ(E1, G1)                                                                   \
  hipLaunchKernelGGL((k_mq_sweep_sb<E1, G1, D>), g, bl, 0, st, desc, ctrl, wq, ws, \
                     n_items, gap_item);
  IMPACT_SB_SWITCH(MQ)
#undef MQ
  return hipGetLastError();
}

#undef IMPACT_SB_SWITCH

#define IMPACT_SB_DECLARE(D)                                                                   \
  extern template hipError_t launch_sb_d<D>(const SweepArgs&, int, int64_t, int32_t,          \
                                            hipStream_t);                                       \
  extern template hipError_t launch_mq_sb_d<D>(const QueryDesc*, const QueryCtrl*,            \
                                               const int32_t*, const int32_t*, int64_t, double*, \
                                               int64_t, int32_t, hipStream_t);
IMPACT_SB_DECLARE(2)
IMPACT_SB_DECLARE(3)
IMPACT_SB_DECLARE(5)
IMPACT_SB_DECLARE(0)
#undef IMPACT_SB_DECLARE
extern template hipError_t launch_sb_dist<0>(const SweepArgs&, int, int64_t, int32_t,
                                             hipStream_t);
extern template hipError_t launch_sb_dist<2>(const SweepArgs&, int, int64_t, int32_t,
                                             hipStream_t);
extern template hipError_t launch_sb_dist<3>(const SweepArgs&, int, int64_t, int32_t,
                                             hipStream_t);

}  // namespace impact
