// abi.hip -- the C ABI declared in include/impact.h: argument validation,
// device allocation through the caller's allocator, and the host side of the
// build and of interval iteration (sweep batches with a device-side stop test).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "build_mc.hpp"
#include "impact_internal.hpp"

using namespace impact;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) throw HipError{_e, #expr};  \
  } while (0)

struct NoMem {
  size_t bytes;
};

}  // namespace

// Device buffers of one build (one or many systems), shared by the handles
// (views) of the systems it holds and released with the last of them.
struct Storage {
  impact_device dev{};
  hipStream_t st = nullptr;
  int device = 0;         // the device current when the build ran
  bool hip_used = false;  // set before the first HIP call
  std::vector<void*> owned;
  int64_t bytes = 0;
  SysParams* d_sys = nullptr;
  double* d_U = nullptr;
  int32_t* win = nullptr;
  double4* ot = nullptr;
  int64_t* row_off = nullptr;
  double2* ent = nullptr;
  double2* fac = nullptr;

  void sync() {
    if (hip_used) (void)hipStreamSynchronize(st);
  }
  void* alloc(size_t nbytes) {
    if (nbytes == 0) nbytes = 8;
    void* p = nullptr;
    if (dev.alloc) {
      p = dev.alloc(nbytes, dev.ctx);
    } else if (hipMalloc(&p, nbytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) throw NoMem{nbytes};
    return p;
  }
  void release(void* p) {
    if (!p) return;
    if (dev.free)
      dev.free(p, dev.ctx);
    else
      (void)hipFree(p);
  }
  template <class T>
  T* own(int64_t elems) {
    T* p = (T*)alloc((size_t)(elems > 0 ? elems : 1) * sizeof(T));
    owned.push_back(p);
    bytes += elems * (int64_t)sizeof(T);
    return p;
  }
  ~Storage() {
    sync();
    for (void* p : owned) release(p);
  }
};

// One system's abstraction: a view into a Storage.
struct impact_imdp {
  std::shared_ptr<Storage> store;
  int32_t inst = 0;
  hipStream_t st = nullptr;
  SysParams hp{};
  const SysParams* dp = nullptr;
  const int64_t* row_off = nullptr;  // indexed by this system's row
  const int32_t* win = nullptr;
  const double4* ot = nullptr;
  const double2* ent = nullptr;      // indexed by row_off values
  const double2* fac = nullptr;
  int64_t n_states = 0, n_rows = 0, n_cells = 0;
  int32_t d = 0, nu = 0, windowed = 0, storage = IMPACT_STORE_BOUNDS, max_row = 0, fs = 0;
  int32_t nw = 1;       // disturbances per (state, input); rows per state nu * nw
  int64_t max_box = 0;  // largest bounding box of one state's row windows (cells)
  int32_t sweep_mode[2] = {IMPACT_SWEEP_AUTO, IMPACT_SWEEP_AUTO};  // per pass
  impact_iter_info last{};
  bool timing = false;
  double build_ms = 0.0;

  void sync() { store->sync(); }
  void* alloc(size_t nbytes) { return store->alloc(nbytes); }
  void release(void* p) { store->release(p); }
};

namespace {

// Scoped temporaries of one call, returned to the caller's allocator on exit.
template <class Owner>
struct ScratchT {
  Owner* h;
  std::vector<void*> ps;
  explicit ScratchT(Owner* hh) : h(hh) {}
  template <class T>
  T* get(int64_t elems) {
    T* p = (T*)h->alloc((size_t)(elems > 0 ? elems : 1) * sizeof(T));
    ps.push_back(p);
    return p;
  }
  size_t need = 0, cap = 0;
  bool overflow() const { return false; }  // allocation failures throw NoMem
  ~ScratchT() {
    h->sync();
    for (void* p : ps) h->release(p);
  }
};
using Scratch = ScratchT<impact_imdp>;

// Temporaries of one call inside a fixed device region (the no-allocation
// entry point): bump allocation at 256-byte alignment; a request beyond the
// region's end returns null and marks the arena as overflowed.
struct Arena {
  char* base;
  size_t cap;
  size_t need = 0;
  template <class T>
  T* get(int64_t elems) {
    const size_t bytes = (size_t)(elems > 0 ? elems : 1) * sizeof(T);
    const size_t off = (need + 255) & ~(size_t)255;
    need = off + bytes;
    return need <= cap ? (T*)(base + off) : nullptr;
  }
  bool overflow() const { return need > cap; }
};

// HIP events of one call, destroyed on every exit path.
struct EventPool {
  std::vector<hipEvent_t> evs;
  hipEvent_t make() {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    evs.push_back(e);
    return e;
  }
  ~EventPool() {
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
};

bool is_finite(double x) { return std::isfinite(x); }

int validate_build(const impact_system* sys, const impact_grid* grid, const impact_inputs* in,
                   const impact_noise* noise, const impact_window* win) {
  if (!sys || !grid || !in || !noise || !win) return fail(IMPACT_E_INVAL, "null argument");
  const int d = grid->dim;
  if (d < 1 || d > IMPACT_MAX_DIM) return fail(IMPACT_E_INVAL, "grid.dim must be in [1, 8]");
  if (sys->dim_x != d) return fail(IMPACT_E_INVAL, "system.dim_x != grid.dim");
  if (!grid->lb || !grid->ub || !grid->n) return fail(IMPACT_E_INVAL, "grid arrays are null");
  int64_t ns = 1;
  for (int i = 0; i < d; ++i) {
    if (grid->n[i] < 1) return fail(IMPACT_E_INVAL, "grid.n must be >= 1");
    if (!is_finite(grid->lb[i]) || !is_finite(grid->ub[i]) || !(grid->lb[i] < grid->ub[i]))
      return fail(IMPACT_E_INVAL, "grid bounds must be finite with lb < ub");
    ns *= grid->n[i];
    if (ns > 0x7fffffffLL) return fail(IMPACT_E_UNSUPPORTED, "more than 2^31-1 states");
  }
  if (in->count < 1) return fail(IMPACT_E_INVAL, "inputs.count must be >= 1");
  if (in->dim_u < 0 || in->dim_u > IMPACT_MAX_DIM || in->dim_u != sys->dim_u)
    return fail(IMPACT_E_INVAL, "inputs.dim_u must equal system.dim_u and be in [0, 8]");
  if (in->dim_u > 0 && !in->values) return fail(IMPACT_E_INVAL, "inputs.values is null");
  for (int64_t k = 0; k < (int64_t)in->count * in->dim_u; ++k)
    if (!is_finite(in->values[k])) return fail(IMPACT_E_INVAL, "non-finite input value");
  if (!noise->sigma) return fail(IMPACT_E_INVAL, "noise.sigma is null");
  for (int i = 0; i < d; ++i)
    if (!is_finite(noise->sigma[i]) || !(noise->sigma[i] > 0.0))
      return fail(IMPACT_E_INVAL, "noise.sigma must be finite and > 0");
  if (!is_finite(win->k_sigma) || win->k_sigma < 0.0)
    return fail(IMPACT_E_INVAL, "window.k_sigma must be finite and >= 0");
  if (win->storage < IMPACT_STORE_AUTO || win->storage > IMPACT_STORE_FACTORS)
    return fail(IMPACT_E_INVAL, "unknown window.storage");
  if (sys->kind == IMPACT_SYS_AFFINE) {
    if (!sys->A || !sys->c || (sys->dim_u > 0 && !sys->B))
      return fail(IMPACT_E_INVAL, "affine system needs A, c (and B when dim_u > 0)");
    for (int k = 0; k < d * d; ++k)
      if (!is_finite(sys->A[k])) return fail(IMPACT_E_INVAL, "non-finite A");
    for (int k = 0; k < d * sys->dim_u; ++k)
      if (!is_finite(sys->B[k])) return fail(IMPACT_E_INVAL, "non-finite B");
    for (int k = 0; k < d; ++k)
      if (!is_finite(sys->c[k])) return fail(IMPACT_E_INVAL, "non-finite c");
  } else if (sys->kind == IMPACT_SYS_UNICYCLE) {
    if (d != 3 || sys->dim_u != 2) return fail(IMPACT_E_INVAL, "unicycle needs dim_x 3, dim_u 2");
    if (!is_finite(sys->dt)) return fail(IMPACT_E_INVAL, "non-finite dt");
  } else {
    return fail(IMPACT_E_INVAL, "unknown system kind");
  }
  return IMPACT_OK;
}

void fill_params(SysParams& p, const impact_system* sys, const impact_grid* g,
                 const impact_inputs* in, const impact_noise* nz, const impact_window* w) {
  std::memset(&p, 0, sizeof(p));
  const int d = g->dim;
  p.kind = sys->kind;
  p.d = d;
  p.du = in->dim_u;
  p.nu = in->count;
  p.windowed = w->k_sigma > 0.0;
  p.dt = sys->dt;
  p.k_sigma = w->k_sigma;
  if (sys->kind == IMPACT_SYS_AFFINE) {
    for (int k = 0; k < d * d; ++k) p.A[k] = sys->A[k];
    for (int k = 0; k < d * in->dim_u; ++k) p.B[k] = sys->B[k];
    for (int k = 0; k < d; ++k) p.c[k] = sys->c[k];
  }
  int64_t ns = 1;
  for (int i = 0; i < d; ++i) {
    p.lb[i] = g->lb[i];
    p.ub[i] = g->ub[i];
    p.n[i] = g->n[i];
    p.w[i] = (g->ub[i] - g->lb[i]) / (double)g->n[i];
    p.sigma[i] = nz->sigma[i];
    ns *= g->n[i];
  }
  int64_t s = 1;
  for (int i = d - 1; i >= 0; --i) {
    p.stride[i] = s;
    s *= g->n[i];
  }
  p.n_states = ns;
  p.n_rows = ns * in->count;
}

float event_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const NoMem& e) {
    return fail(IMPACT_E_NOMEM, "device allocation of " + std::to_string(e.bytes) + " bytes failed");
  } catch (const HipError& e) {
    return fail(IMPACT_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::exception& e) {
    return fail(IMPACT_E_INVAL, e.what());
  } catch (...) {
    return fail(IMPACT_E_INVAL, "unknown error");
  }
}

}  // namespace

namespace impact {
int imdp_view(const impact_imdp* h, ImdpView* v) {
  if (!h || !v) return IMPACT_E_INVAL;
  std::memset(&v->a, 0, sizeof(v->a));
  v->a.row_off = h->row_off;
  v->a.win = h->win;
  v->a.ot = h->ot;
  v->a.ent = h->ent;
  v->a.fac = h->fac;
  v->a.sys = h->dp;
  v->a.fs = h->fs;
  v->a.nu = h->nu;
  v->a.nw = h->nw;
  v->a.d = h->d;
  v->a.windowed = h->windowed;
  v->a.storage = h->storage;
  v->dp = h->dp;
  v->n_states = h->n_states;
  v->max_box = h->max_box;
  v->max_row = h->max_row;
  v->d = h->d;
  v->nu = h->nu;
  v->nw = h->nw;
  v->keep = h->store;
  return IMPACT_OK;
}
}  // namespace impact

// Temporaries of impact_interval_iterate_noalloc: one array per GPU, which
// each GPU the library runs on holds until the process ends.  Host code never
// uses this name as an address: it takes the device address from
// hipGetSymbolAddress once per device (scratch_base).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_base;  // device -> address of its scratch array

// The device address of `device`'s scratch array, looked up on the first call
// for that device with the device current.
int scratch_base(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_base.find(device);
  if (it != g_scratch_base.end()) {
    *out = it->second;
    return IMPACT_OK;
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return fail(IMPACT_E_HIP, "hipGetDevice failed");
  if (cur != device && hipSetDevice(device) != hipSuccess)
    return fail(IMPACT_E_HIP, "hipSetDevice failed");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return fail(IMPACT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_base[device] = p;
  *out = p;
  return IMPACT_OK;
}

}  // namespace

namespace {

// Arguments of impact_interval_iterate and its no-allocation variant.
int validate_iterate(const impact_imdp* h, const impact_spec* spec, double eps, const double* lo,
                     const double* hi, const int32_t* policy) {
  if (!h || !spec) return fail(IMPACT_E_INVAL, "null argument");
  if (!lo || !hi || !policy) return fail(IMPACT_E_INVAL, "lo/hi/policy must be device buffers");
  if (spec->kind < IMPACT_SAFETY || spec->kind > IMPACT_REACH_AVOID)
    return fail(IMPACT_E_INVAL, "unknown spec kind");
  if (spec->n_target < 0 || spec->n_avoid < 0) return fail(IMPACT_E_INVAL, "negative box count");
  if ((spec->n_target > 0 && !spec->target_boxes) || (spec->n_avoid > 0 && !spec->avoid_boxes))
    return fail(IMPACT_E_INVAL, "box array is null");
  if (spec->kind == IMPACT_SAFETY && spec->n_target != 0)
    return fail(IMPACT_E_INVAL, "safety takes no target boxes");
  if (spec->kind == IMPACT_REACH && spec->n_avoid != 0)
    return fail(IMPACT_E_INVAL, "reachability takes no avoid boxes (use reach-avoid)");
  if (spec->pessimistic != 0 && spec->pessimistic != 1)
    return fail(IMPACT_E_INVAL, "pessimistic must be 0 or 1");
  if (spec->max_sweeps < 1) return fail(IMPACT_E_INVAL, "max_sweeps must be >= 1");
  if (spec->horizon < IMPACT_HORIZON_AUTO)
    return fail(IMPACT_E_INVAL, "horizon must be >= 0 or IMPACT_HORIZON_AUTO");
  if (!is_finite(eps) || !(eps > 0.0)) return fail(IMPACT_E_INVAL, "eps must be finite and > 0");
  const int d = h->d;
  for (int64_t k = 0; k < (int64_t)spec->n_target * 2 * d; ++k)
    if (std::isnan(spec->target_boxes[k])) return fail(IMPACT_E_INVAL, "NaN in target box");
  for (int64_t k = 0; k < (int64_t)spec->n_avoid * 2 * d; ++k)
    if (std::isnan(spec->avoid_boxes[k])) return fail(IMPACT_E_INVAL, "NaN in avoid box");
  for (int b = 0; b < spec->n_target; ++b)
    for (int i = 0; i < d; ++i)
      if (spec->target_boxes[b * 2 * d + i] > spec->target_boxes[b * 2 * d + d + i])
        return fail(IMPACT_E_INVAL, "target box with lo > hi");
  for (int b = 0; b < spec->n_avoid; ++b)
    for (int i = 0; i < d; ++i)
      if (spec->avoid_boxes[b * 2 * d + i] > spec->avoid_boxes[b * 2 * d + d + i])
        return fail(IMPACT_E_INVAL, "avoid box with lo > hi");

  return IMPACT_OK;
}

// Interval iteration with the call's temporaries from tmp (the caller's
// allocator, or the static scratch array of the no-allocation variant).
template <class Tmp>
int iterate_body(impact_imdp* h, const impact_spec* spec, double eps, double* lo, double* hi,
                 int32_t* policy, Tmp& tmp, bool timing) {
  const int d = h->d;
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t N = h->n_states;
  const bool safety = spec->kind == IMPACT_SAFETY;
  double* tb = tmp.template get<double>((int64_t)spec->n_target * 2 * d);
  double* ab = tmp.template get<double>((int64_t)spec->n_avoid * 2 * d);
  int8_t* cls = tmp.template get<int8_t>(N);
  int64_t* flag = tmp.template get<int64_t>(N);
  int64_t* pos = tmp.template get<int64_t>(N + 1);
  const int64_t te = scan_tmp_elems(N);
  int64_t* stmp = tmp.template get<int64_t>(te);
  int32_t* safe = tmp.template get<int32_t>(N);
  double2* vb[2] = {tmp.template get<double2>(N), tmp.template get<double2>(N)};
  int32_t* pi = tmp.template get<int32_t>(N);
  Ctrl* ctrl = tmp.template get<Ctrl>(1);
  double* gap_part = tmp.template get<double>(std::max<int64_t>(1, N));
  // rows longer than a wavefront's sort: selection sweep, which needs the
  // value vector sorted per sweep and keeps a per-row hint
  const bool sel = h->max_row > 512;
  double* vs_buf[2] = {nullptr, nullptr};
  int32_t* hint = nullptr;
  if (sel) {
    vs_buf[0] = tmp.template get<double>(2 * N);
    vs_buf[1] = tmp.template get<double>(2 * N);
    hint = tmp.template get<int32_t>(2 * h->n_rows);
  }
  if (tmp.overflow())
    return fail(IMPACT_E_UNSUPPORTED,
                "the call needs " + std::to_string(tmp.need) + " bytes of temporaries, more than the " +
                    std::to_string(tmp.cap) + " of the static scratch array");
  h->store->hip_used = true;

  if (spec->n_target > 0)
    HIP_TRY(hipMemcpyAsync(tb, spec->target_boxes, sizeof(double) * spec->n_target * 2 * d,
                           hipMemcpyHostToDevice, h->st));
  if (spec->n_avoid > 0)
    HIP_TRY(hipMemcpyAsync(ab, spec->avoid_boxes, sizeof(double) * spec->n_avoid * 2 * d,
                           hipMemcpyHostToDevice, h->st));
  HIP_TRY(launch_label(h->dp, N, tb, spec->n_target, ab, spec->n_avoid, cls, flag, h->st));
  HIP_TRY(exclusive_scan_i64(flag, pos, N, stmp, te, h->st));
  int64_t n_safe = 0;
  HIP_TRY(hipMemcpyAsync(&n_safe, pos + N, sizeof(int64_t), hipMemcpyDeviceToHost, h->st));
  HIP_TRY(hipStreamSynchronize(h->st));
  HIP_TRY(launch_compact(cls, pos, N, safe, h->st));

  impact_iter_info info{};
  info.n_safe = n_safe;
  EventPool events;
  Ctrl hc{};
  // Both passes under one stop rule: self_rule stops a pass once both its
  // iterates stop moving (Remark 5.2); otherwise the gap rule, or exactly
  // `horizon` sweeps when horizon > 0 (Remark 5.1).
  auto run_passes = [&](bool self_rule, int64_t horizon) -> int {
  for (int pass = 0; pass < 2; ++pass) {
    // policy pass: one sort per state over its rows' window box when every
    // row fits a wavefront; the fixed-input pass has one row per state and
    // sorts per row unless the state-box mode is forced
    const int32_t mode = h->sweep_mode[pass];
    // (with a disturbance player the state box must hold a whole state's
    // rows; the fixed-input pass then also sweeps by state box, so that an
    // item's disturbance rows share one sort)
    const bool use_box = h->max_row <= 512 &&
                         (h->nw > 1 ? h->max_box <= 512 && mode != IMPACT_SWEEP_PER_ROW
                                    : (mode == IMPACT_SWEEP_STATE_BOX ||
                                       (mode == IMPACT_SWEEP_AUTO && pass == 0)));
    SweepArgs a{};
    a.row_off = h->row_off;
    a.win = h->win;
    a.ot = h->ot;
    a.ent = h->ent;
    a.fac = h->fac;
    a.sys = h->dp;
    a.pi = pi;
    a.safe = safe;
    a.ctrl = ctrl;
    a.gap_part = gap_part;
    a.n_safe = n_safe;
    a.fs = h->fs;
    a.pass = pass;
    a.reach = !safety;
    // the adversarial LP (reach: minimising; safety: maximising the bad
    // mass) runs in the policy pass for the pessimistic policy and in the
    // fixed-input pass for the optimistic one
    const bool adverse = (pass == 0) == (spec->pessimistic != 0);
    a.maximise = adverse ? safety : !safety;
    a.nu = h->nu;
    a.nw = h->nw;
    a.d = d;
    a.windowed = h->windowed;
    a.storage = h->storage;
    a.out_val = safety ? 1.0 : 0.0;
    a.inputs_per_state = (pass == 0 ? h->nu : 1) * h->nw;  // rows swept per state
    a.n_cells = N;
    a.hint = hint;
    double* vsorted = sel ? vs_buf[value_sort_passes(N) & 1] : nullptr;
    a.vsort = vsorted;
    int G = 1;
    if (h->max_row <= 512) G = std::max(1, 4 / a.inputs_per_state);
    while (G > 1 && G * a.inputs_per_state > 256) --G;
    if (a.inputs_per_state > 256)
      return fail(IMPACT_E_UNSUPPORTED, "more than 256 rows per state");
    // the fixed-input pass sorting per row runs several rows per wavefront
    if (pass == 1 && !use_box && h->nw == 1 && rows_g_states_per_block(h->max_row) > 0)
      G = rows_g_states_per_block(h->max_row);
    if (sel) G = 1;  // one workgroup per state
    a.states_per_block = G;
    if (sel) HIP_TRY(launch_fill_i32(hint, 2 * h->n_rows, -1, h->st));

    HIP_TRY(launch_init_values(cls, N, safety, vb[0], vb[1], pass == 0 ? pi : nullptr, h->st));
    // finite horizon: the device stop test never fires (gap >= 0 > -1) and
    // the cap is the horizon
    const bool finite = horizon > 0;
    const double eps_dev = finite ? -1.0 : eps;
    const int64_t cap = finite ? horizon : spec->max_sweeps;
    // workgroups of the self-convergence measure (within gap_part's N slots)
    const int64_t n_delta = std::min<int64_t>(1024, (n_safe + 255) / 256);
    HIP_TRY(launch_ctrl_init(ctrl, eps_dev, cap, h->st));
    int64_t sweeps = 0, launched = 0;
    double gap = n_safe > 0 ? 1.0 : 0.0;
    int converged = (finite || self_rule) ? n_safe == 0 : gap <= eps;
    float sweep_ms = 0.f, launch_ms = 0.f;
    if (!converged) {
      // Sweeps go out in batches between host polls of the control block.
      // A batch lasts about 2 ms of GPU time (from the last batch's per-sweep
      // time) and never exceeds the number of sweeps still needed if the
      // gap keeps contracting at its last observed rate, so few launches run
      // after the stop test has fired.
      int64_t chunk = 1, prev_sweeps = 0;
      double prev_gap = 1.0;
      std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
      for (;;) {
        const int64_t n = std::min<int64_t>(chunk, cap - launched);
        if (n <= 0) break;
        const auto c0 = std::chrono::steady_clock::now();
        for (int64_t k = 0; k < n; ++k) {
          const int64_t idx = launched + k;
          a.vin = vb[idx & 1];
          a.vout = vb[(idx + 1) & 1];
          // the sort is outside the timed pair: the events bracket the sweep kernel
          if (sel)
            HIP_TRY(launch_value_sort(ctrl, a.vin, N, a.maximise ? -1.0 : 1.0, vs_buf[0],
                                      vs_buf[1], h->st));
          hipEvent_t e0 = nullptr, e1 = nullptr;
          if (timing) {
            e0 = events.make();
            e1 = events.make();
            HIP_TRY(hipEventRecord(e0, h->st));
          }
          if (use_box)
            HIP_TRY(launch_sweep_sb(a, h->max_box, h->max_row, h->st));
          else if (sel)
            HIP_TRY(launch_sweep_sel(a, h->max_row, h->st));
          else
            HIP_TRY(launch_sweep(a, h->max_row, h->st));
          if (timing) {
            HIP_TRY(hipEventRecord(e1, h->st));
            marks.emplace_back(e0, e1);
          }
          if (self_rule) {
            HIP_TRY(launch_self_delta(ctrl, safe, n_safe, a.vin, a.vout, gap_part, n_delta,
                                      h->st));
            HIP_TRY(launch_finish(ctrl, gap_part, n_delta, h->st));
          } else {
            HIP_TRY(launch_finish(ctrl, gap_part, sweep_blocks(a, use_box), h->st));
          }
        }
        launched += n;
        HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->st));
        HIP_TRY(hipStreamSynchronize(h->st));
        if (hc.done) break;
        const double per_sweep_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0)
                .count() / (double)n;
        int64_t next = (int64_t)std::max(1.0, std::min(256.0, 2.0 / std::max(per_sweep_ms, 1e-3)));
        if (!finite && hc.sweeps > prev_sweeps && hc.gap > 0.0 && hc.gap < prev_gap) {
          const double rate = std::pow(hc.gap / prev_gap, 1.0 / (double)(hc.sweeps - prev_sweeps));
          if (rate > 0.0 && rate < 1.0) {
            const double need = std::ceil(std::log(eps / hc.gap) / std::log(rate));
            if (need >= 1.0 && need < (double)next) next = (int64_t)need;
          }
        }
        prev_sweeps = hc.sweeps;
        prev_gap = hc.gap;
        chunk = next;
      }
      sweeps = hc.sweeps;
      gap = hc.gap;
      converged = finite ? hc.sweeps == cap : hc.converged;
      for (int64_t k = 0; k < (int64_t)marks.size(); ++k) {
        const float ms = event_ms(marks[k].first, marks[k].second);
        launch_ms += ms;
        if (k < sweeps) sweep_ms += ms;
      }
    }
    info.sweeps[pass] = sweeps;
    info.gap[pass] = gap;
    info.converged[pass] = converged;
    info.updates[pass] = sweeps * n_safe * a.inputs_per_state;
    info.sweep_ms[pass] = sweep_ms;
    info.launch_ms[pass] = launch_ms;
    info.launches[pass] = launched;
    HIP_TRY(launch_finalize(cls, N, vb[sweeps & 1], pi, adverse ? 0 : 1, safety, finite,
                            adverse ? lo : hi, pass == 0 ? policy : nullptr, h->st));
  }
  info.horizon = horizon;
  return IMPACT_OK;
  };
  int rc;
  if (spec->horizon == IMPACT_HORIZON_AUTO) {
    // Remark 5.2: the sweeps each pass needs for both of its iterates to
    // converge to themselves; the larger count is the horizon of a
    // value-iteration run, whose outputs are returned
    if ((rc = run_passes(true, 0)) < 0) return rc;
    const int64_t s0 = info.sweeps[0], s1 = info.sweeps[1];
    const int32_t c0 = info.converged[0], c1 = info.converged[1];
    const double self_ms = info.sweep_ms[0] + info.sweep_ms[1];
    info = impact_iter_info{};
    info.n_safe = n_safe;
    if ((rc = run_passes(false, std::max<int64_t>(1, std::max(s0, s1)))) < 0) return rc;
    info.self_sweeps[0] = s0;
    info.self_sweeps[1] = s1;
    info.converged[0] = c0;
    info.converged[1] = c1;
    info.self_sweep_ms = self_ms;
  } else if ((rc = run_passes(false, spec->horizon)) < 0) {
    return rc;
  }
  HIP_TRY(hipStreamSynchronize(h->st));
  info.iterate_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
          .count();
  h->last = info;
  return (info.converged[0] && info.converged[1]) ? IMPACT_OK : IMPACT_NOT_CONVERGED;
}

}  // namespace

extern "C" {

const char* impact_last_error(void) { return g_err.c_str(); }

const char* impact_version(void) { return "impact-gfx950 0.1"; }

// Build n systems with one launch of each construction kernel over all of
// their rows (Alg. 2's parallel loop spans every system).
// Correlated noise of a Monte Carlo build, checked and prepared on the host.
struct McSetup {
  double P[IMPACT_MAX_DIM * IMPACT_MAX_DIM];  // inverse covariance, d x d row-major
  double sigma[IMPACT_MAX_DIM];               // marginal standard deviations
  double norm, kappa;
  int32_t G;
  int64_t N;
  const double* samples;  // host, N x d
};

static int build_many(int32_t n, const impact_system* sys, const impact_grid* grid,
                      const impact_inputs* inputs, const impact_noise* noise,
                      const impact_window* window, const impact_device* dev, impact_imdp** out,
                      const McSetup* mc = nullptr) {
  for (int32_t i = 0; i < n; ++i) out[i] = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    const int rc = validate_build(&sys[i], &grid[i], &inputs[i], &noise[i], &window[i]);
    if (rc != IMPACT_OK) {
      if (n > 1) g_err = "system " + std::to_string(i) + ": " + g_err;
      return rc;
    }
    const bool fi = window[i].storage == IMPACT_STORE_FACTORS;
    const bool f0 = window[0].storage == IMPACT_STORE_FACTORS;
    if (fi != f0) return fail(IMPACT_E_INVAL, "all systems of a batch share one storage mode");
  }
  auto store = std::make_shared<Storage>();
  if (dev) store->dev = *dev;
  store->st = (hipStream_t)store->dev.stream;
  if (hipGetDevice(&store->device) != hipSuccess) {
    (void)hipGetLastError();
    store->device = 0;
  }
  const bool factors = window[0].storage == IMPACT_STORE_FACTORS;
  std::vector<SysParams> hp(n);
  std::vector<int64_t> row_base(n + 1, 0), state_base(n + 1, 0), u_off(n + 1, 0);
  int64_t win_total = 0;
  int32_t d_max = 1;
  for (int32_t i = 0; i < n; ++i) {
    fill_params(hp[i], &sys[i], &grid[i], &inputs[i], &noise[i], &window[i]);
    if (mc) {
      const int d = hp[i].d;
      hp[i].mc = 1;
      hp[i].mc_grid = mc->G;
      hp[i].mc_n = mc->N;
      hp[i].mc_norm = mc->norm;
      hp[i].mc_kappa = mc->kappa;
      for (int k = 0; k < d * d; ++k) hp[i].mc_P[k] = mc->P[k];
    }
    hp[i].row_base = row_base[i];
    hp[i].state_base = state_base[i];
    hp[i].win_base = win_total;
    row_base[i + 1] = row_base[i] + hp[i].n_rows;
    state_base[i + 1] = state_base[i] + hp[i].n_states;
    u_off[i + 1] = u_off[i] + (int64_t)hp[i].nu * hp[i].du;
    win_total += hp[i].n_rows * 2 * hp[i].d;
    d_max = std::max(d_max, hp[i].d);
  }
  const int64_t R = row_base[n], S = state_base[n];
  std::vector<int64_t> fsz(n, 1);
  std::vector<int32_t> max_row(n, 0);
  std::vector<unsigned long long> bm(n, 0);
  int64_t total = 0;
  float build_ms = 0.f;
  const int rc = guarded([&]() -> int {
    Storage* st = store.get();
    // every allocation of the first phase is requested before the first HIP call
    st->d_sys = st->own<SysParams>(n);
    st->d_U = st->own<double>(std::max<int64_t>(1, u_off[n]));
    st->win = st->own<int32_t>(win_total);
    st->ot = st->own<double4>(R);
    st->row_off = st->own<int64_t>(R + 1);
    double* d_samples = mc ? st->own<double>(mc->N * hp[0].d) : nullptr;
    if (mc) hp[0].mc_samples = d_samples;
    ScratchT<Storage> tmp(st);
    int64_t* cnt = tmp.template get<int64_t>(R);
    int32_t* maxima = tmp.template get<int32_t>(2 * (int64_t)n);
    unsigned long long* boxmax = tmp.template get<unsigned long long>(n);
    int64_t* d_row_base = tmp.template get<int64_t>(n + 1);
    int64_t* d_state_base = tmp.template get<int64_t>(n + 1);
    const int64_t te = scan_tmp_elems(R);
    int64_t* stmp = tmp.template get<int64_t>(te);
    double* d_gA = mc ? tmp.template get<double>(mc->N * (hp[0].d + 1)) : nullptr;
    double* d_gmax = mc ? tmp.template get<double>(kMaxDim) : nullptr;
    std::vector<double> U_all(std::max<int64_t>(1, u_off[n]));
    for (int32_t i = 0; i < n; ++i) {
      hp[i].U = st->d_U + u_off[i];
      if (u_off[i + 1] > u_off[i])
        std::memcpy(U_all.data() + u_off[i], inputs[i].values,
                    sizeof(double) * (size_t)(u_off[i + 1] - u_off[i]));
    }
    st->hip_used = true;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipMemcpyAsync(st->d_U, U_all.data(), sizeof(double) * U_all.size(),
                           hipMemcpyHostToDevice, st->st));
    HIP_TRY(hipMemcpyAsync(st->d_sys, hp.data(), sizeof(SysParams) * n, hipMemcpyHostToDevice,
                           st->st));
    if (mc)
      HIP_TRY(hipMemcpyAsync(d_samples, mc->samples, sizeof(double) * mc->N * hp[0].d,
                             hipMemcpyHostToDevice, st->st));
    HIP_TRY(hipMemcpyAsync(d_row_base, row_base.data(), sizeof(int64_t) * (n + 1),
                           hipMemcpyHostToDevice, st->st));
    HIP_TRY(hipMemcpyAsync(d_state_base, state_base.data(), sizeof(int64_t) * (n + 1),
                           hipMemcpyHostToDevice, st->st));
    HIP_TRY(hipMemsetAsync(maxima, 0, 2 * sizeof(int32_t) * n, st->st));
    HIP_TRY(hipMemsetAsync(boxmax, 0, sizeof(unsigned long long) * n, st->st));
    const BuildTable T{st->d_sys, d_row_base, d_state_base, n};
    HIP_TRY(hipEventRecord(e0, st->st));
    HIP_TRY(launch_row_geom(T, R, st->win, st->ot, cnt, maxima, st->st));
    HIP_TRY(exclusive_scan_i64(cnt, st->row_off, R, stmp, te, st->st));
    std::vector<int32_t> mx(2 * (size_t)n);
    HIP_TRY(hipMemcpyAsync(&total, st->row_off + R, sizeof(int64_t), hipMemcpyDeviceToHost,
                           st->st));
    HIP_TRY(hipMemcpyAsync(mx.data(), maxima, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToHost,
                           st->st));
    HIP_TRY(hipStreamSynchronize(st->st));
    int64_t fac_total = 0;
    int32_t fs_max = 1;
    for (int32_t i = 0; i < n; ++i) {
      max_row[i] = mx[2 * i];
      const int32_t fs = mx[2 * i + 1] > 0 ? mx[2 * i + 1] : 1;
      if (max_row[i] > IMPACT_MAX_ROW)
        return fail(IMPACT_E_UNSUPPORTED,
                    (n > 1 ? "system " + std::to_string(i) + ": " : std::string()) + "a row has " +
                        std::to_string(max_row[i]) + " entries (max " +
                        std::to_string(IMPACT_MAX_ROW) + ")");
      if (fs > kMaxFactors)
        return fail(IMPACT_E_UNSUPPORTED, "per-row factor list longer than " +
                                              std::to_string(kMaxFactors));
      fsz[i] = fs;
      hp[i].fs = fs;
      hp[i].fac_base = fac_total;
      if (factors) fac_total += hp[i].n_rows * (int64_t)fs;
      fs_max = std::max(fs_max, fs);
    }
    HIP_TRY(hipMemcpyAsync(st->d_sys, hp.data(), sizeof(SysParams) * n, hipMemcpyHostToDevice,
                           st->st));
    if (factors)
      st->fac = st->own<double2>(fac_total);
    else
      st->ent = st->own<double2>(total);
    if (mc)
      HIP_TRY(launch_mc_rows(st->d_sys, hp[0].d, R, total, st->win, st->row_off, st->ent,
                             st->st, mc->G, d_gA, d_gmax));
    else
      HIP_TRY(launch_expand(T, R, st->win, st->row_off, st->ent, st->fac, fs_max, d_max,
                            st->st));
    HIP_TRY(hipEventRecord(e1, st->st));
    HIP_TRY(launch_state_box_max(T, S, st->win, boxmax, st->st));
    HIP_TRY(hipMemcpyAsync(bm.data(), boxmax, sizeof(unsigned long long) * n,
                           hipMemcpyDeviceToHost, st->st));
    HIP_TRY(hipStreamSynchronize(st->st));
    build_ms = event_ms(e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return IMPACT_OK;
  });
  if (rc != IMPACT_OK) return rc;
  // per-system views (row offsets of the last system end at the total)
  std::vector<int64_t> cells(n, 0);
  {
    std::vector<int64_t> starts(n + 1);
    const int r = guarded([&]() -> int {
      for (int32_t i = 0; i <= n; ++i)
        HIP_TRY(hipMemcpyAsync(&starts[i], store->row_off + row_base[i], sizeof(int64_t),
                               hipMemcpyDeviceToHost, store->st));
      HIP_TRY(hipStreamSynchronize(store->st));
      return IMPACT_OK;
    });
    if (r != IMPACT_OK) return r;
    for (int32_t i = 0; i < n; ++i) cells[i] = starts[i + 1] - starts[i];
  }
  for (int32_t i = 0; i < n; ++i) {
    impact_imdp* h = new impact_imdp();
    h->store = store;
    h->inst = i;
    h->st = store->st;
    h->hp = hp[i];
    h->dp = store->d_sys + i;
    h->row_off = store->row_off + hp[i].row_base;
    h->win = store->win + hp[i].win_base;
    h->ot = store->ot + hp[i].row_base;
    h->ent = store->ent;
    h->fac = store->fac ? store->fac + hp[i].fac_base : nullptr;
    h->n_states = hp[i].n_states;
    h->n_rows = hp[i].n_rows;
    h->n_cells = cells[i];
    h->d = hp[i].d;
    h->nu = hp[i].nu;
    h->windowed = hp[i].windowed;
    h->storage = factors ? IMPACT_STORE_FACTORS : IMPACT_STORE_BOUNDS;
    h->max_row = max_row[i];
    h->fs = (int32_t)fsz[i];
    h->max_box = (int64_t)bm[i];
    h->build_ms = build_ms;
    out[i] = h;
  }
  return IMPACT_OK;
}

int impact_build_imdp(const impact_system* sys, const impact_grid* grid,
                      const impact_inputs* inputs, const impact_noise* noise,
                      const impact_window* window, const impact_device* dev,
                      impact_imdp** out) {
  g_err.clear();
  if (!out) return fail(IMPACT_E_INVAL, "out is null");
  *out = nullptr;
  if (!sys || !grid || !inputs || !noise || !window) return fail(IMPACT_E_INVAL, "null argument");
  return build_many(1, sys, grid, inputs, noise, window, dev, out);
}

// Marginal standard deviations sqrt(Cov_ii) of Cov = P^-1: Gauss-Jordan
// elimination of [P | I] with partial pivoting.  False for a singular P or a
// non-positive diagonal of the inverse.
static bool mc_marginals(int d, const double* P, double* sigma) {
  double a[IMPACT_MAX_DIM][2 * IMPACT_MAX_DIM];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < 2 * d; ++j) a[i][j] = j < d ? P[i * d + j] : (j - d == i ? 1.0 : 0.0);
  for (int col = 0; col < d; ++col) {
    int piv = col;
    for (int r = col + 1; r < d; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (!(std::fabs(a[piv][col]) > 0.0)) return false;
    if (piv != col)
      for (int j = 0; j < 2 * d; ++j) std::swap(a[col][j], a[piv][j]);
    const double pv = a[col][col];
    for (int j = 0; j < 2 * d; ++j) a[col][j] /= pv;
    for (int r = 0; r < d; ++r) {
      if (r == col) continue;
      const double f = a[r][col];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * d; ++j) a[r][j] -= f * a[col][j];
    }
  }
  for (int i = 0; i < d; ++i) {
    const double v = a[i][d + i];
    if (!(v > 0.0) || !std::isfinite(v)) return false;
    sigma[i] = std::sqrt(v);
  }
  return true;
}

// det(P) by forward elimination with partial pivoting.
static double mc_det(int d, const double* P) {
  double a[IMPACT_MAX_DIM][IMPACT_MAX_DIM], det = 1.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) a[i][j] = P[i * d + j];
  for (int col = 0; col < d; ++col) {
    int piv = col;
    for (int r = col + 1; r < d; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < d; ++j) std::swap(a[col][j], a[piv][j]);
      det = -det;
    }
    det *= a[col][col];
    if (a[col][col] == 0.0) return 0.0;
    for (int r = col + 1; r < d; ++r) {
      const double f = a[r][col] / a[col][col];
      for (int j = col; j < d; ++j) a[r][j] -= f * a[col][j];
    }
  }
  return det;
}

int impact_build_imdp_mc(const impact_system* sys, const impact_grid* grid,
                         const impact_inputs* inputs, const impact_mc_noise* noise,
                         const impact_window* window, const impact_device* dev,
                         impact_imdp** out) {
  g_err.clear();
  if (!out) return fail(IMPACT_E_INVAL, "out is null");
  *out = nullptr;
  if (!sys || !grid || !inputs || !noise || !window) return fail(IMPACT_E_INVAL, "null argument");
  const int d = grid->dim;
  if (d < 1 || d > IMPACT_MAX_DIM) return fail(IMPACT_E_INVAL, "grid.dim must be in [1, 8]");
  if (!noise->inv_cov || !noise->samples) return fail(IMPACT_E_INVAL, "inv_cov or samples is null");
  if (noise->n_samples < 1) return fail(IMPACT_E_INVAL, "n_samples must be >= 1");
  if (noise->grid_pts < 1) return fail(IMPACT_E_INVAL, "grid_pts must be >= 1");
  if (!std::isfinite(noise->kappa) || noise->kappa < 0.0)
    return fail(IMPACT_E_INVAL, "kappa must be finite and >= 0");
  if (!std::isfinite(noise->det_cov) || !(noise->det_cov > 0.0))
    return fail(IMPACT_E_INVAL, "det_cov must be finite and > 0");
  if (window->storage == IMPACT_STORE_FACTORS)
    return fail(IMPACT_E_INVAL, "correlated noise has no per-dimension factors (use BOUNDS)");
  int64_t n_cand = 1;
  for (int i = 0; i < d; ++i) {
    n_cand *= noise->grid_pts;
    if (n_cand > 4096) return fail(IMPACT_E_UNSUPPORTED, "grid_pts^dim must be at most 4096");
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double x = noise->inv_cov[i * d + j];
      if (!std::isfinite(x) || x != noise->inv_cov[j * d + i])
        return fail(IMPACT_E_INVAL, "inv_cov must be finite and symmetric");
    }
  for (int64_t k = 0; k < noise->n_samples * d; ++k)
    if (!(noise->samples[k] >= 0.0 && noise->samples[k] < 1.0))
      return fail(IMPACT_E_INVAL, "samples must lie in [0, 1)");
  McSetup mc{};
  if (!mc_marginals(d, noise->inv_cov, mc.sigma))
    return fail(IMPACT_E_INVAL, "inv_cov is singular or not positive definite");
  const double detP = mc_det(d, noise->inv_cov);
  if (!(detP > 0.0) || std::fabs(detP * noise->det_cov - 1.0) > 1e-6)
    return fail(IMPACT_E_INVAL, "det_cov does not match inv_cov");
  for (int k = 0; k < d * d; ++k) mc.P[k] = noise->inv_cov[k];
  double t = 1.0;
  for (int i = 0; i < d; ++i) t *= 2.0 * kPi;
  mc.norm = 1.0 / std::sqrt(t * noise->det_cov);
  mc.kappa = noise->kappa;
  mc.G = noise->grid_pts;
  mc.N = noise->n_samples;
  mc.samples = noise->samples;
  const impact_noise marg{mc.sigma};
  impact_window w2 = *window;
  w2.storage = IMPACT_STORE_BOUNDS;
  return build_many(1, sys, grid, inputs, &marg, &w2, dev, out, &mc);
}

int impact_build_imdp_dist(const impact_system* sys, const impact_grid* grid,
                           const impact_inputs* inputs, const impact_disturbances* dist,
                           const impact_noise* noise, const impact_window* window,
                           const impact_device* dev, impact_imdp** out) {
  g_err.clear();
  if (!out) return fail(IMPACT_E_INVAL, "out is null");
  *out = nullptr;
  if (!sys || !grid || !inputs || !dist || !noise || !window)
    return fail(IMPACT_E_INVAL, "null argument");
  if (sys->kind != IMPACT_SYS_AFFINE)
    return fail(IMPACT_E_UNSUPPORTED, "disturbances need an affine system");
  const int d = grid->dim;
  if (d < 1 || d > IMPACT_MAX_DIM || sys->dim_x != d)
    return fail(IMPACT_E_INVAL, "grid.dim must equal system.dim_x and be in [1, 8]");
  if (dist->count < 1 || dist->dim_w < 1)
    return fail(IMPACT_E_INVAL, "disturbances.count and dim_w must be >= 1");
  if (!dist->values || !dist->D) return fail(IMPACT_E_INVAL, "disturbances.values or D is null");
  const int du = sys->dim_u, dw = dist->dim_w;
  if (du < 0 || inputs->dim_u != du || inputs->count < 1 || (du > 0 && (!inputs->values || !sys->B)))
    return fail(IMPACT_E_INVAL, "inputs must match system.dim_u and hold at least one input");
  if (du + dw > IMPACT_MAX_DIM) return fail(IMPACT_E_UNSUPPORTED, "dim_u + dim_w must be at most 8");
  if ((int64_t)inputs->count * dist->count > 256)
    return fail(IMPACT_E_UNSUPPORTED, "more than 256 (input, disturbance) pairs");
  for (int64_t k = 0; k < (int64_t)dist->count * dw; ++k)
    if (!is_finite(dist->values[k])) return fail(IMPACT_E_INVAL, "non-finite disturbance value");
  for (int64_t k = 0; k < (int64_t)d * dw; ++k)
    if (!is_finite(dist->D[k])) return fail(IMPACT_E_INVAL, "non-finite D");
  // one input per (u, w) pair, u-major, with input matrix [B | D]: the build
  // computes the mean A x + B u + D w + c of every row
  const int dc = du + dw;
  std::vector<double> B2((size_t)d * dc), U2((size_t)inputs->count * dist->count * dc);
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j < du; ++j) B2[(size_t)i * dc + j] = sys->B[(size_t)i * du + j];
    for (int k = 0; k < dw; ++k) B2[(size_t)i * dc + du + k] = dist->D[(size_t)i * dw + k];
  }
  for (int32_t u = 0; u < inputs->count; ++u)
    for (int32_t w = 0; w < dist->count; ++w) {
      double* r = U2.data() + ((size_t)u * dist->count + w) * dc;
      for (int j = 0; j < du; ++j) r[j] = inputs->values[(size_t)u * du + j];
      for (int k = 0; k < dw; ++k) r[du + k] = dist->values[(size_t)w * dw + k];
    }
  impact_system s2 = *sys;
  s2.dim_u = dc;
  s2.B = B2.data();
  impact_inputs i2{inputs->count * dist->count, dc, U2.data()};
  const int rc = build_many(1, &s2, grid, &i2, noise, window, dev, out);
  if (rc < 0) return rc;
  (*out)->nu = inputs->count;
  (*out)->nw = dist->count;
  return rc;
}

int impact_build_imdp_batch(int32_t n, const impact_system* sys, const impact_grid* grid,
                            const impact_inputs* inputs, const impact_noise* noise,
                            const impact_window* window, const impact_device* dev,
                            impact_imdp** out) {
  g_err.clear();
  if (!out) return fail(IMPACT_E_INVAL, "out is null");
  if (n < 1) return fail(IMPACT_E_INVAL, "n must be >= 1");
  if (!sys || !grid || !inputs || !noise || !window) return fail(IMPACT_E_INVAL, "null argument");
  return build_many(n, sys, grid, inputs, noise, window, dev, out);
}

int impact_set_timing(impact_imdp* h, int32_t enable) {
  if (!h) return fail(IMPACT_E_INVAL, "null handle");
  h->timing = enable != 0;
  return IMPACT_OK;
}

int impact_set_sweep_modes(impact_imdp* h, int32_t policy_pass, int32_t fixed_pass) {
  if (!h) return fail(IMPACT_E_INVAL, "null handle");
  for (int32_t mode : {policy_pass, fixed_pass})
    if (mode < IMPACT_SWEEP_AUTO || mode > IMPACT_SWEEP_STATE_BOX)
      return fail(IMPACT_E_INVAL, "unknown sweep mode");
  h->sweep_mode[0] = policy_pass;
  h->sweep_mode[1] = fixed_pass;
  return IMPACT_OK;
}

int impact_set_sweep_mode(impact_imdp* h, int32_t mode) {
  return impact_set_sweep_modes(h, mode, mode);
}

int impact_imdp_get_info(const impact_imdp* h, impact_imdp_info* info) {
  if (!h || !info) return fail(IMPACT_E_INVAL, "null argument");
  std::memset(info, 0, sizeof(*info));
  info->n_states = h->n_states;
  info->n_rows = h->n_rows;
  info->n_entries = h->n_cells + h->n_rows * (1 + h->windowed);
  info->dim = h->d;
  info->n_inputs = h->nu;
  info->windowed = h->windowed;
  info->storage = h->storage;
  info->max_row = h->max_row;
  info->max_box = h->max_box;
  info->device_bytes = h->store->bytes;
  info->build_ms = h->build_ms;
  info->n_dist = h->nw;
  return IMPACT_OK;
}

int impact_last_iter_info(const impact_imdp* h, impact_iter_info* info) {
  if (!h || !info) return fail(IMPACT_E_INVAL, "null argument");
  *info = h->last;
  return IMPACT_OK;
}

int impact_imdp_export_rows(const impact_imdp* hc, int64_t row0, int64_t nrows, int32_t* window,
                            double* ot, int64_t* counts, double* entries) {
  g_err.clear();
  if (!hc) return fail(IMPACT_E_INVAL, "null handle");
  impact_imdp* h = const_cast<impact_imdp*>(hc);
  if (row0 < 0 || nrows < 0 || row0 + nrows > h->n_rows)
    return fail(IMPACT_E_INVAL, "row range out of bounds");
  if (nrows > 0 && (!window || !ot || !counts))
    return fail(IMPACT_E_INVAL, "window/ot/counts must be device buffers");
  return guarded([&]() -> int {
    HIP_TRY(launch_export(h->dp, row0, nrows, h->win, h->ot, h->row_off, h->ent, h->fac, h->fs,
                          h->d, h->windowed, window, ot, counts, entries, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    return IMPACT_OK;
  });
}

int impact_interval_iterate(impact_imdp* h, const impact_spec* spec, double eps, double* lo,
                            double* hi, int32_t* policy) {
  g_err.clear();
  const int rc = validate_iterate(h, spec, eps, lo, hi, policy);
  if (rc != IMPACT_OK) return rc;
  return guarded([&]() -> int {
    Scratch tmp(h);
    return iterate_body(h, spec, eps, lo, hi, policy, tmp, h->timing);
  });
}

int impact_interval_iterate_noalloc(impact_imdp* h, const impact_spec* spec, double eps,
                                    double* lo, double* hi, int32_t* policy) {
  g_err.clear();
  const int rc = validate_iterate(h, spec, eps, lo, hi, policy);
  if (rc != IMPACT_OK) return rc;
  void* base = nullptr;
  const int rb = scratch_base(h->store->device, &base);
  if (rb != IMPACT_OK) return rb;
  return guarded([&]() -> int {
    Arena tmp{(char*)base, kScratchBytes};
    // no per-launch timing: event creation is left to the allocating variant
    return iterate_body(h, spec, eps, lo, hi, policy, tmp, false);
  });
}

void impact_imdp_free(impact_imdp* h) {
  if (!h) return;
  delete h;
}

}  // extern "C"
