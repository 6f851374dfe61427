// sweep_common.hpp -- device building blocks of the interval-iteration
// sweep (eq. (5.1) by the sorting method of Section 6.2): wavefront /
// workgroup reductions and scans, a register/shuffle/LDS bitonic sort of
// 64-bit keys with a payload, row loading and the per-row LP.
#pragma once

#include "impact_internal.hpp"

namespace impact {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxItems = 256;  // (state, input) rows per workgroup

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

// Values that are equal on every lane of a wavefront, moved to scalar registers.
__device__ __forceinline__ int32_t uniform_i32(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t to_bits(double x) { return dbits(x); }
__device__ __forceinline__ uint64_t to_bits(int32_t x) { return (uint64_t)(uint32_t)x; }
template <class V>
__device__ __forceinline__ V from_bits(uint64_t b);
template <>
__device__ __forceinline__ double from_bits<double>(uint64_t b) {
  return bitsd(b);
}
template <>
__device__ __forceinline__ int32_t from_bits<int32_t>(uint64_t b) {
  return (int32_t)(uint32_t)b;
}

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
template <int E, class V>
__device__ __forceinline__ void ce_local(uint64_t (&key)[E], V (&val)[E], int e, int e2,
                                         bool asc) {
  const bool sw = asc ? (key[e] > key[e2]) : (key[e] < key[e2]);
  if (sw) {
    uint64_t tk = key[e];
    key[e] = key[e2];
    key[e2] = tk;
    V tv = val[e];
    val[e] = val[e2];
    val[e2] = tv;
  }
}

// All stages of merge step k whose stride j < E (both partners in one thread).
template <int E, class V>
__device__ __forceinline__ void intra_stages(uint64_t (&key)[E], V (&val)[E], int tid, int k) {
#pragma unroll
  for (int j = E / 2; j > 0; j >>= 1) {
    if (j < k) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int e2 = e ^ j;
        if (e2 > e) ce_local<E, V>(key, val, e, e2, ((tid * E + e) & k) == 0);
      }
    }
  }
}

// Bitonic sort of P = 64 * NW * E keys, thread t holding positions
// [t*E, t*E + E) ("blocked" layout), ascending by key; val travels along.
template <int E, int NW, class V>
__device__ void bitonic_sort(uint64_t (&key)[E], V (&val)[E], int tid, uint64_t* xk) {
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
          const V pv = __shfl_xor(val[e], tm);
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
        for (int e = 0; e < E; ++e) xk[tid * E + e] = to_bits(val[e]);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool asc = ((tid * E + e) & k) == 0;
          const bool take = (asc == lower) ? !(key[e] < pk[e]) : !(key[e] > pk[e]);
          const V pv = from_bits<V>(xk[(tid ^ tm) * E + e]);
          if (take) {
            key[e] = pk[e];
            val[e] = pv;
          }
        }
        __syncthreads();
      }
    }
    intra_stages<E, V>(key, val, tid, k);
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
    IMPACT_FOR_DIMS_REV(i, d) {
      W[i] = wr[d + i];
      klo[i] = wr[i];
      j[i] = nw > 0 ? (int32_t)(rem % W[i]) : 0;
      rem = nw > 0 ? rem / W[i] : 0;
    }
    IMPACT_FOR_DIMS(i, d) {
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
        IMPACT_FOR_DIMS(i, d) {
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
      IMPACT_FOR_DIMS_REV(i, d) {
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
  bitonic_sort<E, NW, double>(key, dk, g.tid, xk);
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

}  // namespace impact
