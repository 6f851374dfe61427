// sweep_sb.hip -- host dispatch of the state-box sweep kernels (which live in
// sweep_sb.hpp and are instantiated per grid dimension in sweep_sb_d*.hip),
// and the per-instance largest state box.
#include "sweep_sb.hpp"

namespace impact {

hipError_t launch_sweep_sb(const SweepArgs& a, int64_t max_box, int32_t max_row, hipStream_t st) {
  if (a.n_safe == 0) return hipSuccess;
  // a disturbance player: items of several rows, boxes up to the state's
  if (a.nw > 1) {
    switch (a.d) {
      case 2: return launch_sb_dist<2>(a, a.pass, max_box, max_row, st);
      case 3: return launch_sb_dist<3>(a, a.pass, max_box, max_row, st);
      default: return launch_sb_dist<0>(a, a.pass, max_box, max_row, st);
    }
  }
  // pass 2 uses one row per state: its box is the row's own window
  const int64_t box = a.pass == 0 ? max_box : max_row;
  switch (a.d) {
    case 2: return launch_sb_d<2>(a, a.pass, box, max_row, st);
    case 3: return launch_sb_d<3>(a, a.pass, box, max_row, st);
    case 5: return launch_sb_d<5>(a, a.pass, box, max_row, st);
    default: return launch_sb_d<0>(a, a.pass, box, max_row, st);
  }
}

// Every item's query has grid dimension d when d is 2, 3 or 5 (kernels
// specialised on it); any other d runs the generic variant.
hipError_t launch_mq_sweep_sb(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                              const int32_t* ws, int64_t n_items, double* gap_item,
                              int64_t max_box, int32_t max_row, int32_t d, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  switch (d) {
    case 2: return launch_mq_sb_d<2>(desc, ctrl, wq, ws, n_items, gap_item, max_box, max_row, st);
    case 3: return launch_mq_sb_d<3>(desc, ctrl, wq, ws, n_items, gap_item, max_box, max_row, st);
    case 5: return launch_mq_sb_d<5>(desc, ctrl, wq, ws, n_items, gap_item, max_box, max_row, st);
    default:
      return launch_mq_sb_d<0>(desc, ctrl, wq, ws, n_items, gap_item, max_box, max_row, st);
  }
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
