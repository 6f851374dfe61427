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
// q = n / w and r = n % w for 0 <= n < 2^22 and 1 <= w < 2^22: a float
// estimate of the quotient (off by at most one) corrected exactly, a handful
// of instructions instead of an integer division's expansion (the window and
// box digit decompositions of the sweeps divide small numbers by runtime
// extents).
__device__ __forceinline__ void divmod_small(int n, int w, int& q, int& r) {
  int qq = (int)((float)n * __builtin_amdgcn_rcpf((float)w));
  int rr = n - qq * w;
  if (rr < 0) {
    qq -= 1;
    rr += w;
  }
  if (rr >= w) {
    qq += 1;
    rr -= w;
  }
  q = qq;
  r = rr;
}

__device__ __forceinline__ int32_t uniform_i32(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double uniform_f64(double x) {
  return __longlong_as_double(uniform_i64(__double_as_longlong(x)));
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

// ---- cross-lane moves without the LDS address path --------------------------
// DPP (data-parallel primitives) move a VALU operand between lanes of a
// 16-lane row (or across rows for the broadcasts) with no LDS traffic;
// ds_swizzle permutes within 32-lane halves by a fixed bit pattern.  Lanes
// whose DPP source does not exist keep 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int32_t dpp_i32(int32_t x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  const uint32_t lo = (uint32_t)dpp_i32<CTRL, ROW_MASK>((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)dpp_i32<CTRL, ROW_MASK>((int32_t)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
  return __longlong_as_double((long long)dpp_u64<CTRL, ROW_MASK>((uint64_t)__double_as_longlong(x)));
}
template <int PATTERN>
__device__ __forceinline__ uint64_t swz_u64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int32_t)(uint32_t)x, PATTERN);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int32_t)(uint32_t)(x >> 32), PATTERN);
  return ((uint64_t)hi << 32) | lo;
}
template <int PATTERN>
__device__ __forceinline__ double swz_f64(double x) {
  return __longlong_as_double((long long)swz_u64<PATTERN>((uint64_t)__double_as_longlong(x)));
}

enum : int {
  kDppXor1 = 0xB1,        // quad_perm [1,0,3,2]
  kDppXor2 = 0x4E,        // quad_perm [2,3,0,1]
  kDppRowShr1 = 0x111,    // row_shr:n = 0x110 + n
  kDppWaveShr1 = 0x138,   // wave_shr:1
  kDppRowHalfMirror = 0x141,
  kDppRowMirror = 0x140,
  kDppBcast15 = 0x142,
  kDppBcast31 = 0x143,
};
// ds_swizzle bit-mask mode: lane' = ((lane & and) | or) ^ xor over 5 bits.
constexpr int swz_xor(int m) { return 0x1F | (m << 10); }
constexpr int kSwzLast16 = 0x10 | (0x0F << 5);  // lane 15 of each 16-lane group
constexpr int kSwzLast32 = 0x1F << 5;           // lane 31 of each 32-lane half

// x of lane (lane ^ m), m a power of two below 64.
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t x, int m) {
  switch (m) {
    case 1: return dpp_u64<kDppXor1>(x);
    case 2: return dpp_u64<kDppXor2>(x);
    case 4: return swz_u64<swz_xor(4)>(x);
    case 8: return swz_u64<swz_xor(8)>(x);
    case 16: return swz_u64<swz_xor(16)>(x);
    default: return (uint64_t)__shfl_xor((long long)x, 32);
  }
}
__device__ __forceinline__ int32_t xor_lane_i32(int32_t x, int m) {
  switch (m) {
    case 1: return dpp_i32<kDppXor1>(x);
    case 2: return dpp_i32<kDppXor2>(x);
    case 4: return __builtin_amdgcn_ds_swizzle(x, swz_xor(4));
    case 8: return __builtin_amdgcn_ds_swizzle(x, swz_xor(8));
    case 16: return __builtin_amdgcn_ds_swizzle(x, swz_xor(16));
    default: return __shfl_xor(x, 32);
  }
}

// Sum over the GW-lane group (GW = 16, 32, 64) of each lane, every lane of the
// group getting the same value: butterfly over pairs, quads, 8- and 16-lane
// mirrors, then the halves and the wave.
template <int GW>
__device__ __forceinline__ double group_sum_dpp(double x) {
  x += dpp_f64<kDppXor1>(x);
  x += dpp_f64<kDppXor2>(x);
  x += dpp_f64<kDppRowHalfMirror>(x);
  x += dpp_f64<kDppRowMirror>(x);
  if (GW >= 32) x += swz_f64<swz_xor(16)>(x);
  if (GW == 64) x += __shfl_xor(x, 32);
  return x;
}

// Inclusive prefix sum within GW-lane groups (Hillis-Steele inside 16-lane
// rows, then the row totals carried across rows).
template <int GW>
__device__ __forceinline__ double group_incl_scan_dpp(double x) {
  x += dpp_f64<kDppRowShr1>(x);
  x += dpp_f64<kDppRowShr1 + 1>(x);
  x += dpp_f64<kDppRowShr1 + 3>(x);
  x += dpp_f64<kDppRowShr1 + 7>(x);
  if (GW >= 32) x += dpp_f64<kDppBcast15, 0xA>(x);
  if (GW == 64) x += dpp_f64<kDppBcast31, 0xC>(x);
  return x;
}

// Exclusive prefix sum within GW-lane groups (group lane gl) and the group total.
template <int GW>
__device__ __forceinline__ double group_excl_scan_dpp(double x, int gl, double& total) {
  const double incl = group_incl_scan_dpp<GW>(x);
  if (GW == 16) total = swz_f64<kSwzLast16>(incl);
  else if (GW == 32) total = swz_f64<kSwzLast32>(incl);
  else total = __shfl(incl, 63);
  const double e = dpp_f64<kDppWaveShr1>(incl);
  return gl == 0 ? 0.0 : e;
}

template <class V>
__device__ __forceinline__ V xor_lane(V x, int m);
template <>
__device__ __forceinline__ int32_t xor_lane<int32_t>(int32_t x, int m) {
  return xor_lane_i32(x, m);
}
template <>
__device__ __forceinline__ double xor_lane<double>(double x, int m) {
  return __longlong_as_double((long long)xor_lane_u64((uint64_t)__double_as_longlong(x), m));
}

// Every lane of the wavefront active.
__device__ __forceinline__ double wave_sum(double x) { return group_sum_dpp<64>(x); }

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
  return x;
}

// Exclusive prefix sum across the wavefront (lane 0 gets 0); every lane active.
__device__ __forceinline__ double wave_excl_scan(double x, int lane) {
  double total;
  return group_excl_scan_dpp<64>(x, lane, total);
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

// Lane exchange at a compile-time xor distance M (< 64).
template <int M>
__device__ __forceinline__ uint64_t xor_lane_c(uint64_t x) {
  if constexpr (M == 1) return dpp_u64<kDppXor1>(x);
  else if constexpr (M == 2) return dpp_u64<kDppXor2>(x);
  else if constexpr (M == 4 || M == 8 || M == 16) return swz_u64<swz_xor(M)>(x);
  else return (uint64_t)__shfl_xor((long long)x, M);
}

// One merge stage across lanes at xor distance M: each key meets the key of
// the same slot on lane tid ^ M; selects, not branches.
template <int E, class V, int M>
__device__ __forceinline__ void lane_stage(uint64_t (&key)[E], V (&val)[E], int tid, int k) {
  const bool lower = (tid & M) == 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool asc = ((tid * E + e) & k) == 0;
    const uint64_t pk = xor_lane_c<M>(key[e]);
    const V pv = from_bits<V>(xor_lane_c<M>(to_bits(val[e])));
    const bool take = (asc == lower) ? !(key[e] < pk) : !(key[e] > pk);
    key[e] = take ? pk : key[e];
    val[e] = take ? pv : val[e];
  }
}

// Bitonic sort of P = 64 * NW * E keys, thread t holding positions
// [t*E, t*E + E) ("blocked" layout), ascending by key; val travels along.
// Stages between lanes of one wavefront pick their exchange primitive once
// per stage (the distance is uniform); stages between wavefronts go through
// xk (at least P words) in element-major order, xk[e * 64 * NW + t], so that
// a wavefront's accesses fall on consecutive words.
template <int E, int NW, class V, bool UNROLL = true>
__device__ void bitonic_sort(uint64_t (&key)[E], V (&val)[E], int tid, uint64_t* xk) {
  constexpr int P = 64 * NW * E;
  constexpr int T = 64 * NW;
  // fully unrolled (compile-time partner distances) up to 4 keys per thread;
  // larger networks, and every network of a kernel that also holds the large
  // ones (UNROLL false), keep their loops, which holds the register footprint
  constexpr int kUnroll = (E >= 8 || !UNROLL) ? 1 : 16;
#pragma unroll kUnroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll kUnroll
    for (int j = k >> 1; j >= E; j >>= 1) {
      const int tm = j / E;  // partner thread = tid ^ tm
      if (tm < 64) {
        switch (tm) {
          case 1: lane_stage<E, V, 1>(key, val, tid, k); break;
          case 2: lane_stage<E, V, 2>(key, val, tid, k); break;
          case 4: lane_stage<E, V, 4>(key, val, tid, k); break;
          case 8: lane_stage<E, V, 8>(key, val, tid, k); break;
          case 16: lane_stage<E, V, 16>(key, val, tid, k); break;
          default: lane_stage<E, V, 32>(key, val, tid, k); break;
        }
      } else {
        const bool lower = (tid & tm) == 0;
        const int pt = tid ^ tm;
        uint64_t pk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) xk[e * T + tid] = key[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) pk[e] = xk[e * T + pt];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) xk[e * T + tid] = to_bits(val[e]);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool asc = ((tid * E + e) & k) == 0;
          const bool take = (asc == lower) ? !(key[e] < pk[e]) : !(key[e] > pk[e]);
          const V pv = from_bits<V>(xk[e * T + pt]);
          key[e] = take ? pk[e] : key[e];
          val[e] = take ? pv : val[e];
        }
        __syncthreads();
      }
    }
    intra_stages<E, V>(key, val, tid, k);
  }
}

// Bitonic sort of GW * E keys held by a GW-lane group (GW <= 64, groups
// aligned within the wavefront), lane gl holding positions [gl*E, gl*E + E);
// every partner is in the same group.
template <int E, int GW, class V>
__device__ void bitonic_sort_g(uint64_t (&key)[E], V (&val)[E], int gl) {
  constexpr int P = GW * E;
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j >= E; j >>= 1) {
      const int tm = j / E;
      const bool lower = (gl & tm) == 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool asc = ((gl * E + e) & k) == 0;
        const uint64_t pk = xor_lane_u64(key[e], tm);
        const V pv = xor_lane<V>(val[e], tm);
        const bool take = (asc == lower) ? !(key[e] < pk) : !(key[e] > pk);
        if (take) {
          key[e] = pk;
          val[e] = pv;
        }
      }
    }
    intra_stages<E, V>(key, val, gl, k);
  }
}

// One row's entries as seen by one thread: positions [first, first + E).
template <int E>
struct RowSlice {
  double lo[E], dd[E], v0[E], v1[E];
  bool pad[E];
};

// D > 0: the grid dimension is the compile-time D; D == 0: read at run time.
template <int E, int D>
__device__ void load_row(const SweepArgs& a, const SysParams& p, int64_t row, int first,
                         RowSlice<E>& rs) {
  const int d = D > 0 ? D : a.d;
  const int64_t base = a.row_off[row];
  const int nw = (int)(a.row_off[row + 1] - base);
  const int32_t* wr = a.win + row * 2 * d;
  int32_t klo[kMaxDim], W[kMaxDim], j[kMaxDim], fo[kMaxDim];
  int64_t t = 0;
  int tot = 0;
  {
    int rem = first < nw ? first : 0;
    IMPACT_FOR_DIMS_REV(i, d) {
      W[i] = wr[d + i];
      klo[i] = wr[i];
      if (nw > 0)
        divmod_small(rem, W[i], rem, j[i]);
      else
        j[i] = 0;
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
template <int E, int NW, bool UNROLL = true>
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
  bitonic_sort<E, NW, double, UNROLL>(key, dk, g.tid, xk);
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

template <int E, int NW, int D, bool UNROLL = true>
__device__ void solve_row(const SweepArgs& a, const SysParams& p, int64_t row, int tid,
                          double* red, uint64_t* xk, double& q0, double& q1) {
  // a single-wavefront group works in lane coordinates; a workgroup group
  // first waits for every wavefront to leave the previous row's reductions
  const int gtid = NW == 1 ? (tid & 63) : tid;
  if (NW > 1) __syncthreads();
  Group<NW> g(red, gtid);
  RowSlice<E> rs;
  load_row<E, D>(a, p, row, gtid * E, rs);
  double slo = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) slo += rs.lo[e];
  slo = g.sum(slo);
  double r = 1.0 - slo;
  if (r < 0.0) r = 0.0;
  const bool mx = a.maximise != 0;
  q0 = lp_value<E, NW, UNROLL>(rs, rs.v0, r, mx, g, xk);
  q1 = lp_value<E, NW, UNROLL>(rs, rs.v1, r, mx, g, xk);
}

template <int PASS>
__device__ __forceinline__ int64_t item_row(const SweepArgs& a, int64_t s0, int m, int U) {
  const int gi = m / U, ui = m - gi * U;
  const int64_t s = a.safe[s0 + gi];
  const int u = PASS == 0 ? ui : a.pi[s];
  return s * a.nu + u;
}

// The same LP on a GW-lane group (several rows per wavefront, one per group;
// group sums and scans by DPP within the group).
template <int E, int GW>
__device__ double lp_value_g(const RowSlice<E>& rs, const double (&v)[E], double r,
                             bool maximise, int gl) {
  double slv = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) slv += rs.lo[e] * v[e];
  slv = group_sum_dpp<GW>(slv);
  uint64_t key[E];
  double dk[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t b = dbits(v[e] + 0.0);
    key[e] = rs.pad[e] ? ~0ull : (maximise ? ~b : b);
    dk[e] = rs.dd[e];
  }
  bitonic_sort_g<E, GW, double>(key, dk, gl);
  double ls = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) ls += dk[e];
  double total;
  double acc = group_excl_scan_dpp<GW>(ls, gl, total);
  double sdv = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double room = r - acc;
    const double delta = room <= 0.0 ? 0.0 : (dk[e] < room ? dk[e] : room);
    const double val = bitsd(maximise ? ~key[e] : key[e]);
    if (delta > 0.0) sdv += delta * val;
    acc += dk[e];
  }
  return slv + group_sum_dpp<GW>(sdv);
}

// One row (at most GW * E entries) on a GW-lane group: both LP values.
template <int E, int GW, int D>
__device__ void solve_row_g(const SweepArgs& a, const SysParams& p, int64_t row, int gl,
                            double& q0, double& q1) {
  RowSlice<E> rs;
  load_row<E, D>(a, p, row, gl * E, rs);
  double slo = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) slo += rs.lo[e];
  slo = group_sum_dpp<GW>(slo);
  double r = 1.0 - slo;
  if (r < 0.0) r = 0.0;
  const bool mx = a.maximise != 0;
  q0 = lp_value_g<E, GW>(rs, rs.v0, r, mx, gl);
  q1 = lp_value_g<E, GW>(rs, rs.v1, r, mx, gl);
}

// Satisfaction bound of a SAFE state from its converged (V0, V1): the
// adversarial pass gives the lower bound (reach: V0; safety, whose values are
// probabilities of the bad set: 1 - V1), the favourable pass the upper bound.
// Finite horizon: value iteration, both bounds from the V0 iterate.
__device__ __forceinline__ double bound_of(double2 V, bool upper, bool safety, bool finite) {
  if (finite) return safety ? 1.0 - V.x : V.x;
  return upper ? (safety ? 1.0 - V.x : V.y) : (safety ? 1.0 - V.y : V.x);
}

// Engine: close a pass for one state of a query (phase 1: the policy pass's
// bound, the policy and the reset of the values for the fixed-input pass;
// phase 3: the other bound, and under Remark 5.2's horizon at the end of the
// self-convergence stage the reset of the values for the finite stage).
__device__ __forceinline__ void mq_close_state(const QueryDesc& D, const QueryCtrl& c, int phase,
                                               int64_t s) {
  const int64_t step = c.step;
  const bool self_stage = D.auto_h && c.stage == 0;
  const bool finite = D.finite || (D.auto_h && c.stage == 1);
  const double2* vin = (step & 1) ? D.vb1 : D.vb0;
  double2* vout = (step & 1) ? D.vb0 : D.vb1;
  const double2 V = vin[s];
  const bool upper = (phase == 1) == (D.upper_first != 0);
  (upper ? D.hi : D.lo)[s] = bound_of(V, upper, D.safety != 0, finite);
  if (phase == 1) D.pol[s] = D.a.pi[s];
  if (phase == 1 || self_stage) vout[s] = make_double2(0.0, 1.0);
}

}  // namespace impact
