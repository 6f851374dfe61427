// impact_internal.hpp -- host-side declarations shared by the library's
// translation units (kernel launchers and the handle layout).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "impact.h"
#include "impact_device.hpp"

namespace impact {

// Kernel arguments of one interval-iteration sweep.
struct SweepArgs {
  const int64_t* row_off;  // n_rows + 1, offsets of the window cells
  const int32_t* win;      // n_rows * 2d (klo then W)
  const double4* ot;       // n_rows (OUT lo, OUT hi, TAIL lo, TAIL hi)
  const double2* ent;      // STORE: (lo, hi) of window cells
  const double2* fac;      // FACTORS: per-row factor lists at stride fs
  const SysParams* sys;
  const double2* vin;      // (V0, V1) per cell, read
  double2* vout;           // (V0, V1) per cell, written on SAFE cells
  int32_t* pi;             // policy per cell
  const int32_t* safe;     // SAFE cell list
  Ctrl* ctrl;
  double* gap_part;        // one max(V1 - V0) partial per workgroup
  int64_t n_safe;
  int32_t fs;              // factor stride (FACTORS)
  int32_t pass;            // 0: policy pass (all inputs), 1: fixed input
  int32_t maximise;        // LP direction
  int32_t reach;           // 1: combine over u by max (reach), 0: by min (safety)
  int32_t states_per_block;
  int32_t inputs_per_state;
  int32_t nu, d, windowed, storage;
  double out_val;          // objective value of OUT
};

// Scan: out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                              int64_t tmp_elems, hipStream_t st);
int64_t scan_tmp_elems(int64_t n);

// Build launchers.
hipError_t launch_row_geom(const BuildTable& T, int64_t n_rows, int32_t* win, double4* ot,
                           int64_t* cnt, int32_t* maxima, hipStream_t st);
hipError_t launch_expand(const BuildTable& T, int64_t n_rows, const int32_t* win,
                         const int64_t* row_off, double2* ent, double2* fac, int32_t fs_max,
                         int32_t d_max, hipStream_t st);
hipError_t launch_export(const SysParams* sys, int64_t row0, int64_t nrows, const int32_t* win,
                         const double4* ot, const int64_t* row_off, const double2* ent,
                         const double2* fac, int32_t fs, int32_t d, int32_t windowed,
                         int32_t* win_out, double* ot_out, int64_t* counts_out,
                         double* entries_out, hipStream_t st);

// Iteration launchers.
hipError_t launch_label(const SysParams* sys, int64_t n, const double* tboxes, int32_t nt,
                        const double* aboxes, int32_t na, int8_t* cls, int64_t* flag,
                        hipStream_t st);
hipError_t launch_compact(const int8_t* cls, const int64_t* pos, int64_t n, int32_t* safe,
                          hipStream_t st);
hipError_t launch_init_values(const int8_t* cls, int64_t n, int32_t safety, double2* v0,
                              double2* v1, int32_t* pi, hipStream_t st);
hipError_t launch_ctrl_init(Ctrl* c, double eps, int64_t cap, hipStream_t st);
hipError_t launch_sweep(const SweepArgs& a, int32_t max_row, hipStream_t st);
hipError_t launch_sweep_sb(const SweepArgs& a, int64_t max_box, int32_t max_row, hipStream_t st);
hipError_t launch_state_box_max(const BuildTable& T, int64_t n_states, const int32_t* win,
                                unsigned long long* out, hipStream_t st);
hipError_t launch_finish(Ctrl* c, const double* part, int64_t n_part, hipStream_t st);
constexpr int kSbWavesPerBlock = 2;  // state-box sweep: wavefronts (= states) per workgroup
int64_t sweep_blocks(const SweepArgs& a, bool box_path);
hipError_t launch_finalize(const int8_t* cls, int64_t n, const double2* v, const int32_t* pi,
                           int32_t pass, int32_t safety, double* out, int32_t* policy,
                           hipStream_t st);

}  // namespace impact
