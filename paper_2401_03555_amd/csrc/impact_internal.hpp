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
  int32_t nw;              // disturbances per (state, input), 0 or 1: none;
                           // rows of (s, u) are (s * nu + u) * nw + w
  double out_val;          // objective value of OUT
  // selection sweep (rows longer than 512 entries)
  const double* vsort;     // both components of vin, negated for a maximising LP, sorted
                           // ascending: [V0 | V1], n_cells each
  int32_t* hint;           // per (row, vector): a cell that held the critical value, or -1
  int64_t n_cells;         // cells of the grid (length of vin)
};

// One interval-iteration query of the multi-query engine (device table).
// a holds the abstraction's pointers and the query's value buffers; vin,
// vout, pass and maximise are set per step from the query's control block.
struct QueryDesc {
  SweepArgs a;
  double2* vb0;
  double2* vb1;
  double* lo;
  double* hi;
  int32_t* pol;
  int32_t safety;
  int32_t box_class;        // 1: state-box kernel class, 0: workgroup kernel class
  int32_t max_lp[2];        // LP direction of each pass (1: maximising)
  int32_t upper_first;      // 1: the policy pass yields the upper output (optimistic policy)
  int32_t finite;           // 1: finite horizon (cap sweeps per pass, no stop test)
  int32_t auto_h;           // 1: the horizon of Remark 5.2 (self-convergence stage, then
                            // a finite-horizon stage of the larger self sweep count)
  double eps;
  int64_t cap;
  int64_t work_begin, work_end;  // its items in its class's work list
  double* vs[2];             // rows beyond 512 entries: sort buffers (2 * n_cells each);
                             // a.vsort is the one the step's last merge pass writes
};

// Phase machine of one query: 0 policy pass, 1 close pass 1 (write lo and the
// policy, reset values), 2 fixed-input pass, 3 close pass 2 (write hi), 4 done.
struct QueryCtrl {
  int32_t phase, stage;  // stage: 0, or 1 for the finite-horizon stage of Remark 5.2
  int32_t converged[2];
  int64_t step;       // value-buffer steps applied (ping-pong parity)
  int64_t sweeps[2];
  double gap[2];
  int64_t horizon;          // Remark 5.2: the finite stage's horizon K
  int64_t self_sweeps[2];   // Remark 5.2: sweeps until each pass's iterates stopped moving
  int32_t self_conv[2];     // ... and whether they stopped before the cap
};

}  // namespace impact

#include <memory>
struct impact_imdp;

namespace impact {

// What the multi-query engine needs of a built abstraction.
struct ImdpView {
  SweepArgs a;  // abstraction pointers and sizes (query fields unset)
  const SysParams* dp;
  int64_t n_states, max_box;
  int32_t max_row, d, nu;
  int32_t nw;  // disturbances per (state, input); the engine takes 1 only
  std::shared_ptr<void> keep;  // the abstraction's device storage
};
int imdp_view(const impact_imdp* h, ImdpView* v);

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
hipError_t launch_mc_entries(const SysParams* sys, int32_t d, int64_t n_rows, int64_t n_ent,
                             const int32_t* win, const int64_t* row_off, double2* ent,
                             hipStream_t st);
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
// Selection sweep for long rows: the value vector sorted per sweep
// (launch_value_sort writes both components of vin times sg, sorted
// ascending, to buf0 after an even and to buf1 after an odd number of merge
// passes; sg = -1 for a maximising LP), then one workgroup per SAFE state
// (rows of up to kMaxRow entries).
int value_sort_passes(int64_t n);
hipError_t launch_value_sort(const Ctrl* c, const double2* vin, int64_t n, double sg,
                             double* buf0, double* buf1, hipStream_t st);
hipError_t launch_sweep_sel(const SweepArgs& a, int32_t max_row, hipStream_t st);
// p[0, n) = v
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_finish(Ctrl* c, const double* part, int64_t n_part, hipStream_t st);
// part[0, n_part) = per-workgroup max(|V0' - V0|, |V1' - V1|) over the SAFE
// states of one sweep from vin to vout (n_part workgroups of 256 threads;
// nothing if the control block is done).
hipError_t launch_self_delta(const Ctrl* c, const int32_t* safe, int64_t n_safe,
                             const double2* vin, const double2* vout, double* part, int64_t n_part,
                             hipStream_t st);
constexpr int kSbWavesPerBlock = 2;  // state-box sweep: wavefronts (= states) per workgroup
int64_t sweep_blocks(const SweepArgs& a, bool box_path);

// Multi-query engine launchers.
hipError_t launch_mq_sweep_sb(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                              const int32_t* ws, int64_t n_items, double* gap_item,
                              int64_t max_box, int32_t max_row, int32_t d, hipStream_t st);
int rows_g_states_per_block(int32_t max_row);
hipError_t launch_mq_sweep_row(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                               const int32_t* ws, int64_t n_items, double* gap_item,
                               int32_t max_row, int32_t d, hipStream_t st);
// Queries with rows beyond 512 entries (selection sweep): the value vectors of
// the listed query slots sorted (qlist in device memory, nq slots, max_cells
// their largest n_cells; the result lands in vs[p & 1], p =
// value_sort_passes(max_cells)), then one workgroup per item (wq, ws: the
// class's items, which start at position begin of the whole work list;
// storage: the common storage mode of the class's queries, 0 if mixed).
hipError_t launch_mq_value_sort(const QueryDesc* desc, const QueryCtrl* ctrl,
                                const int32_t* qlist, int32_t nq, int64_t max_cells,
                                hipStream_t st);
hipError_t launch_mq_sweep_sel(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                               const int32_t* ws, int64_t n_items, int64_t begin,
                               double* gap_item, int32_t max_row, int32_t d, int32_t storage,
                               hipStream_t st);
// Items of queries in the self-convergence stage of Remark 5.2: gap_item =
// max(|V0' - V0|, |V1' - V1|) of the item's state over this step's sweep.
hipError_t launch_mq_self_delta(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                                const int32_t* ws, int64_t n_items, double* gap_item,
                                hipStream_t st);
// out = the lower (upper = 0) or upper (upper = 1) satisfaction bound of
// every cell (finite = 1: from the V0 iterate of a finite-horizon pass);
// policy (may be null) = pi on SAFE cells, -1 elsewhere.
hipError_t launch_finalize(const int8_t* cls, int64_t n, const double2* v, const int32_t* pi,
                           int32_t upper, int32_t safety, int32_t finite, double* out,
                           int32_t* policy, hipStream_t st);

}  // namespace impact
