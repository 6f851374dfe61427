// mq.hip -- many interval-iteration queries in flight on one device.
//
// Each query is a (built abstraction, specification, eps) triple with its own
// labels, SAFE list, (V0, V1) buffers, policy and outputs.  The engine runs
// all of them together: one step = one launch of each sweep kernel over the
// (query, SAFE state) items of every unfinished query, followed by one launch
// of k_mq_finish, which applies each query's own stop test and moves it along
// its phase machine (policy pass, close, fixed-input pass, close, done).  So
// queries of very different sizes and convergence speeds share launches, and
// a query's result does not depend on which others run beside it (every
// state's update reads only its own query's data).  Chunks of steps are
// captured once into a HIP graph and replayed; the host polls a done counter
// between replays, and queries join or leave at those boundaries.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "impact_internal.hpp"

using namespace impact;

namespace impact {

// Per-query stop test and phase machine (one workgroup per query slot).
__global__ __launch_bounds__(256) void k_mq_finish(const QueryDesc* __restrict__ desc,
                                                   QueryCtrl* __restrict__ ctrl,
                                                   const double* __restrict__ gp,
                                                   int32_t* __restrict__ done_count) {
  __shared__ double wmax[4];
  const int q = blockIdx.x;
  const int phase = ctrl[q].phase;
  if (phase == 4) return;
  const QueryDesc& D = desc[q];
  double g = 0.0;
  if (phase == 0 || phase == 2) {
    for (int64_t i = D.work_begin + threadIdx.x; i < D.work_end; i += blockDim.x)
      g = fmax(g, gp[i]);
    for (int off = 32; off > 0; off >>= 1) g = fmax(g, __shfl_xor(g, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = g;
    __syncthreads();
    g = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  }
  if (threadIdx.x != 0) return;
  QueryCtrl& c = ctrl[q];
  // Remark 5.2: a self-convergence stage (the items' partials are the moves
  // of the iterates, stop once they are <= eps), then a finite stage whose
  // horizon is the larger of its two sweep counts
  const bool self_stage = D.auto_h && c.stage == 0;
  const bool finite = D.finite || (D.auto_h && c.stage == 1);
  const double eps = finite ? -1.0 : D.eps;
  const int64_t cap = (D.auto_h && c.stage == 1) ? c.horizon : D.cap;
  if (phase == 0 || phase == 2) {
    const int pass = phase >> 1;
    c.sweeps[pass] += 1;
    c.gap[pass] = g;
    c.step += 1;
    if (g <= eps) {
      c.converged[pass] = 1;
      c.phase = phase + 1;
    } else if (c.sweeps[pass] >= cap) {
      c.converged[pass] = finite;
      c.phase = phase + 1;
    }
  } else if (phase == 1) {
    c.step += 1;
    // the fixed-input pass starts from a gap of 1: it runs no sweep if eps >= 1
    // (the self rule and a finite horizon always sweep)
    const bool skip = !self_stage && 1.0 <= eps;
    c.phase = skip ? 3 : 2;
    c.gap[1] = 1.0;
    c.converged[1] = skip;
  } else if (self_stage) {
    // the close wrote the reset values: the finite stage starts
    c.step += 1;
    c.self_sweeps[0] = c.sweeps[0];
    c.self_sweeps[1] = c.sweeps[1];
    c.self_conv[0] = c.converged[0];
    c.self_conv[1] = c.converged[1];
    const int64_t K = c.sweeps[0] > c.sweeps[1] ? c.sweeps[0] : c.sweeps[1];
    c.horizon = K > 1 ? K : 1;
    c.stage = 1;
    c.sweeps[0] = c.sweeps[1] = 0;
    c.converged[0] = c.converged[1] = 0;
    c.gap[0] = c.gap[1] = 1.0;
    c.phase = 0;
  } else {
    c.phase = 4;
    atomicAdd(done_count, 1);
  }
}

// Remark 5.2's stop rule: for items of queries in the self-convergence stage,
// replace the sweep's partial by the state's largest move of either iterate.
__global__ void k_mq_self_delta(const QueryDesc* __restrict__ desc,
                                const QueryCtrl* __restrict__ ctrl, const int32_t* __restrict__ wq,
                                const int32_t* __restrict__ ws, int64_t n_items,
                                double* __restrict__ gap_item) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_items) return;
  const int q = wq[item];
  const QueryDesc& D = desc[q];
  const QueryCtrl& c = ctrl[q];
  if (!D.auto_h || c.stage != 0 || (c.phase != 0 && c.phase != 2)) return;
  const int64_t s = ws[item];
  const double2* vin = (c.step & 1) ? D.vb1 : D.vb0;
  const double2* vout = (c.step & 1) ? D.vb0 : D.vb1;
  const double2 o = vin[s], n = vout[s];
  gap_item[item] = fmax(fabs(n.x - o.x), fabs(n.y - o.y));
}

hipError_t launch_mq_self_delta(const QueryDesc* desc, const QueryCtrl* ctrl, const int32_t* wq,
                                const int32_t* ws, int64_t n_items, double* gap_item,
                                hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mq_self_delta, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, st,
                     desc, ctrl, wq, ws, n_items, gap_item);
  return hipGetLastError();
}

// Work-list fill: segment k copies its query's SAFE list to [dst, dst + n).
struct MqSegment {
  const int32_t* safe;
  int64_t dst, n;
  int32_t slot, cls;
};

__global__ void k_mq_fill(const MqSegment* __restrict__ seg, int32_t* __restrict__ wq,
                          int32_t* __restrict__ ws) {
  const MqSegment S = seg[blockIdx.x];
  for (int64_t i = threadIdx.x; i < S.n; i += blockDim.x) {
    wq[S.dst + i] = S.slot;
    ws[S.dst + i] = S.safe[i];
  }
}

}  // namespace impact

namespace {

thread_local std::string g_mq_err;
int mq_fail(int code, const std::string& m) {
  g_mq_err = m;
  return code;
}

struct MqNoMem {};

// Kernel classes of the engine: the queries of one class share a launch of
// the kernel variant sized for them, the same variant a single query of that
// abstraction runs.  Wavefront classes by grid dimension (2, 3, 5, other),
// the per-lane element count of the largest state box (1, 2, 4, 8; boxes
// beyond 512 cells are split into input groups) and the lane-group width of
// the longest row (16, 32, 64): the policy pass runs the state-box kernel,
// the fixed-input pass the per-row kernel.  Workgroup classes for rows beyond
// 512 entries, which run the selection sweep (by grid dimension, 5 or other,
// and the longest row, up to 2048 or 4096 entries).
constexpr int kMqBoxClasses = 4 * 4 * 3;
constexpr int kMqClasses = kMqBoxClasses + 4;
constexpr int kMqDims[4] = {2, 3, 5, 0};

int elems_for(int64_t n) { return n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 0; }
int elems_slot(int e) { return e == 1 ? 0 : e == 2 ? 1 : e == 4 ? 2 : 3; }

struct MqClass {
  int64_t begin = 0, n = 0, max_box = 1;
  int32_t max_row = 1;
  int32_t storage = -1;  // common storage mode of its queries, 0 if mixed
  bool box = true;
};

struct MqQuery {
  int32_t id = -1;
  bool active = false;    // occupies its slot
  bool finished = false;  // reported by a poll
  int64_t n_safe = 0, n_states = 0;
  int32_t box_class = 1, max_row = 0, nu = 1, d = 0;
  int64_t max_box = 0;
  std::shared_ptr<void> keep;  // keeps the abstraction's storage alive
  std::vector<void*> bufs;
  int32_t* safe = nullptr;
};

}  // namespace

struct impact_mq {
  impact_device dev{};
  hipStream_t user_st = nullptr;  // the caller's stream
  hipStream_t st = nullptr;       // the engine's own stream (graphs are captured on it)
  int32_t cap = 0;
  std::vector<MqQuery> slots;
  int32_t next_id = 0;
  std::map<int32_t, impact_iter_info> finished_info;
  std::vector<int32_t> unreported;
  QueryDesc* d_desc = nullptr;
  QueryCtrl* d_ctrl = nullptr;
  int32_t* d_done = nullptr;
  std::vector<QueryDesc> h_desc;
  // one work list of (query slot, state) items, grouped by kernel class
  int32_t *wq = nullptr, *ws = nullptr;
  double* gap = nullptr;
  int64_t cap_items = 0, n_items = 0;
  MqClass cls[kMqClasses];
  // query slots with rows beyond 512 entries (their value vectors are sorted
  // every step) and the largest of their grids
  int32_t* d_long = nullptr;
  int32_t n_long = 0;
  int32_t n_auto = 0;  // live queries under Remark 5.2's horizon
  int64_t long_cells = 0;
  int32_t n_slots_used = 0;
  bool dirty = true;
  // captured chunk of steps
  hipGraphExec_t exec = nullptr;
  int32_t graph_steps = 0;
  int64_t live_submitted = 0;  // queries with SAFE states ever submitted
  int64_t steps_run = 0;
  bool hip_used = false;

  void* alloc(size_t nbytes) {
    if (nbytes == 0) nbytes = 8;
    void* p = nullptr;
    if (dev.alloc) {
      p = dev.alloc(nbytes, dev.ctx);
    } else if (hipMalloc(&p, nbytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) throw MqNoMem{};
    return p;
  }
  void release(void* p) {
    if (!p) return;
    if (dev.free)
      dev.free(p, dev.ctx);
    else
      (void)hipFree(p);
  }
  void sync() {
    if (hip_used) (void)hipStreamSynchronize(st);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    graph_steps = 0;
  }
  // Work submitted by the caller on its stream is complete before ours starts.
  void join_user() {
    if (!hip_used) return;
    (void)hipStreamSynchronize(user_st);
  }
  ~impact_mq() {
    sync();
    drop_graph();
    for (auto& q : slots)
      for (void* p : q.bufs) release(p);
    for (void* p : {(void*)d_desc, (void*)d_ctrl, (void*)d_done, (void*)wq, (void*)ws,
                    (void*)gap, (void*)d_long})
      release(p);
    if (st) (void)hipStreamDestroy(st);
  }
};

namespace {

struct MqHipError {
  hipError_t e;
  const char* what;
};

#define MQ_TRY(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) throw MqHipError{_e, #expr}; \
  } while (0)

template <class F>
int mq_guarded(F&& f) {
  try {
    return f();
  } catch (const MqNoMem&) {
    return mq_fail(IMPACT_E_NOMEM, "device allocation failed");
  } catch (const MqHipError& e) {
    return mq_fail(IMPACT_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (...) {
    return mq_fail(IMPACT_E_INVAL, "unknown error");
  }
}

// Grow a device array (contents are rebuilt by the caller).
template <class T>
void ensure(impact_mq* m, T*& p, int64_t& cap, int64_t need) {
  if (need <= cap && p) return;
  const int64_t nc = std::max<int64_t>(need, std::max<int64_t>(1024, cap * 2));
  if (p) m->release(p);
  p = nullptr;
  p = (T*)m->alloc((size_t)nc * sizeof(T));
  cap = nc;
}

int class_of(const MqQuery& q) {
  if (q.box_class) {
    const int ds = q.d == 2 ? 0 : q.d == 3 ? 1 : q.d == 5 ? 2 : 3;
    const int gs = q.max_row <= 128 ? 0 : q.max_row <= 256 ? 1 : 2;
    int eb = elems_for(std::min<int64_t>(q.max_box, 512));
    eb = std::max(eb, gs == 0 ? 1 : gs == 1 ? 2 : 4);  // the box holds a whole row
    return (ds * 4 + elems_slot(eb)) * 3 + gs;
  }
  return kMqBoxClasses + (q.d == 5 ? 2 : 0) + (q.max_row <= 2048 ? 0 : 1);
}

// Rebuild the work list from the live (unfinished) queries, grouped by class.
void rebuild(impact_mq* m) {
  std::vector<MqSegment> seg;
  MqClass cl[kMqClasses];
  for (int c = 0; c < kMqClasses; ++c) cl[c].box = c < kMqBoxClasses;
  for (int32_t k = 0; k < m->n_slots_used; ++k) {
    MqQuery& q = m->slots[k];
    m->h_desc[k].work_begin = m->h_desc[k].work_end = 0;
    if (!q.active || q.finished || q.n_safe == 0) continue;
    MqSegment S;
    S.safe = q.safe;
    S.n = q.n_safe;
    S.slot = k;
    S.cls = class_of(q);
    S.dst = 0;
    MqClass& c = cl[S.cls];
    c.n += q.n_safe;
    c.max_box = std::max(c.max_box, q.max_box);
    c.max_row = std::max(c.max_row, q.max_row);
    const int32_t sto = m->h_desc[k].a.storage;
    c.storage = c.storage < 0 || c.storage == sto ? sto : 0;
    seg.push_back(S);
  }
  // long-row queries: one sort of every one of them per step, over the
  // largest grid, so that all land in the same buffer of their pair
  std::vector<int32_t> longs;
  int64_t long_cells = 0;
  for (const MqSegment& S : seg)
    if (S.cls >= kMqBoxClasses) {
      longs.push_back(S.slot);
      long_cells = std::max(long_cells, m->slots[S.slot].n_states);
    }
  for (int32_t k : longs) {
    QueryDesc& D = m->h_desc[k];
    D.a.vsort = D.vs[value_sort_passes(long_cells) & 1];
  }
  if (m->d_long) m->release(m->d_long);
  m->d_long = nullptr;
  m->n_long = (int32_t)longs.size();
  m->n_auto = 0;
  for (const MqSegment& S : seg) m->n_auto += m->h_desc[S.slot].auto_h != 0;
  m->long_cells = long_cells;
  if (!longs.empty()) {
    m->d_long = (int32_t*)m->alloc(sizeof(int32_t) * longs.size());
    MQ_TRY(hipMemcpyAsync(m->d_long, longs.data(), sizeof(int32_t) * longs.size(),
                          hipMemcpyHostToDevice, m->st));
  }
  int64_t total = 0;
  for (int c = 0; c < kMqClasses; ++c) {
    cl[c].begin = total;
    total += cl[c].n;
  }
  int64_t at[kMqClasses];
  for (int c = 0; c < kMqClasses; ++c) at[c] = cl[c].begin;
  for (MqSegment& S : seg) {
    S.dst = at[S.cls];
    at[S.cls] += S.n;
    m->h_desc[S.slot].work_begin = S.dst;
    m->h_desc[S.slot].work_end = S.dst + S.n;
  }
  int64_t c1 = m->cap_items, c2 = m->cap_items, c3 = m->cap_items;
  ensure(m, m->wq, c1, total);
  ensure(m, m->ws, c2, total);
  ensure(m, m->gap, c3, total);
  m->cap_items = std::min({c1, c2, c3});
  m->n_items = total;
  for (int c = 0; c < kMqClasses; ++c) m->cls[c] = cl[c];
  if (!seg.empty()) {
    MqSegment* d_seg = (MqSegment*)m->alloc(sizeof(MqSegment) * seg.size());
    MQ_TRY(hipMemcpyAsync(d_seg, seg.data(), sizeof(MqSegment) * seg.size(),
                          hipMemcpyHostToDevice, m->st));
    hipLaunchKernelGGL(k_mq_fill, dim3((unsigned)seg.size()), dim3(256), 0, m->st, d_seg, m->wq,
                       m->ws);
    MQ_TRY(hipGetLastError());
    MQ_TRY(hipStreamSynchronize(m->st));
    m->release(d_seg);
  }
  MQ_TRY(hipMemcpyAsync(m->d_desc, m->h_desc.data(), sizeof(QueryDesc) * m->n_slots_used,
                        hipMemcpyHostToDevice, m->st));
  m->drop_graph();
  m->dirty = false;
}

void enqueue_step(impact_mq* m) {
  if (m->n_slots_used == 0) return;
  if (m->n_long > 0)
    MQ_TRY(launch_mq_value_sort(m->d_desc, m->d_ctrl, m->d_long, m->n_long, m->long_cells,
                                m->st));
  for (int c = 0; c < kMqClasses; ++c) {
    const MqClass& k = m->cls[c];
    if (k.n == 0) continue;
    if (k.box) {
      const int d = kMqDims[c / 12];
      MQ_TRY(launch_mq_sweep_sb(m->d_desc, m->d_ctrl, m->wq + k.begin, m->ws + k.begin, k.n,
                                m->gap + k.begin, k.max_box, k.max_row, d, m->st));
      MQ_TRY(launch_mq_sweep_row(m->d_desc, m->d_ctrl, m->wq + k.begin, m->ws + k.begin, k.n,
                                 m->gap + k.begin, k.max_row, d, m->st));
    } else {
      MQ_TRY(launch_mq_sweep_sel(m->d_desc, m->d_ctrl, m->wq + k.begin, m->ws + k.begin, k.n,
                                 k.begin, m->gap + k.begin, k.max_row,
                                 (c - kMqBoxClasses) >= 2 ? 5 : 0, k.storage, m->st));
    }
  }
  if (m->n_auto > 0)
    MQ_TRY(launch_mq_self_delta(m->d_desc, m->d_ctrl, m->wq, m->ws, m->n_items, m->gap, m->st));
  hipLaunchKernelGGL(k_mq_finish, dim3((unsigned)m->n_slots_used), dim3(256), 0, m->st,
                     (const QueryDesc*)m->d_desc, m->d_ctrl, (const double*)m->gap, m->d_done);
  MQ_TRY(hipGetLastError());
}

// Capture `steps` steps into a graph (replayed until the set of queries changes).
void capture(impact_mq* m, int32_t steps) {
  m->drop_graph();
  hipGraph_t g = nullptr;
  MQ_TRY(hipStreamBeginCapture(m->st, hipStreamCaptureModeThreadLocal));
  for (int32_t k = 0; k < steps; ++k) enqueue_step(m);
  MQ_TRY(hipStreamEndCapture(m->st, &g));
  MQ_TRY(hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0));
  (void)hipGraphDestroy(g);
  m->graph_steps = steps;
}

}  // namespace

extern "C" {

const char* impact_mq_last_error(void) { return g_mq_err.c_str(); }

int impact_mq_create(const impact_device* dev, int32_t max_queries, impact_mq** out) {
  g_mq_err.clear();
  if (!out) return mq_fail(IMPACT_E_INVAL, "out is null");
  *out = nullptr;
  if (max_queries < 1 || max_queries > (1 << 20))
    return mq_fail(IMPACT_E_INVAL, "max_queries must be in [1, 2^20]");
  impact_mq* m = new impact_mq();
  if (dev) m->dev = *dev;
  m->user_st = (hipStream_t)m->dev.stream;
  m->cap = max_queries;
  const int rc = mq_guarded([&]() -> int {
    m->d_desc = (QueryDesc*)m->alloc(sizeof(QueryDesc) * (size_t)max_queries);
    m->d_ctrl = (QueryCtrl*)m->alloc(sizeof(QueryCtrl) * (size_t)max_queries);
    m->d_done = (int32_t*)m->alloc(sizeof(int32_t));
    m->slots.resize(max_queries);
    m->h_desc.resize(max_queries);
    m->hip_used = true;
    MQ_TRY(hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking));
    std::vector<QueryCtrl> c(max_queries);
    for (auto& x : c) {
      std::memset(&x, 0, sizeof(x));
      x.phase = 4;
    }
    MQ_TRY(hipMemcpyAsync(m->d_ctrl, c.data(), sizeof(QueryCtrl) * c.size(),
                          hipMemcpyHostToDevice, m->st));
    const int32_t zero = 0;
    MQ_TRY(hipMemcpyAsync(m->d_done, &zero, sizeof(zero), hipMemcpyHostToDevice, m->st));
    MQ_TRY(hipStreamSynchronize(m->st));
    return IMPACT_OK;
  });
  if (rc != IMPACT_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return IMPACT_OK;
}

int impact_mq_submit(impact_mq* m, const impact_imdp* h, const impact_spec* spec, double eps,
                     double* lo, double* hi, int32_t* policy, int32_t* id_out) {
  g_mq_err.clear();
  if (!m || !h || !spec || !id_out) return mq_fail(IMPACT_E_INVAL, "null argument");
  if (!lo || !hi || !policy) return mq_fail(IMPACT_E_INVAL, "lo/hi/policy must be device buffers");
  if (spec->kind < IMPACT_SAFETY || spec->kind > IMPACT_REACH_AVOID)
    return mq_fail(IMPACT_E_INVAL, "unknown spec kind");
  if (spec->n_target < 0 || spec->n_avoid < 0) return mq_fail(IMPACT_E_INVAL, "negative box count");
  if ((spec->n_target > 0 && !spec->target_boxes) || (spec->n_avoid > 0 && !spec->avoid_boxes))
    return mq_fail(IMPACT_E_INVAL, "box array is null");
  if (spec->kind == IMPACT_SAFETY && spec->n_target != 0)
    return mq_fail(IMPACT_E_INVAL, "safety takes no target boxes");
  if (spec->kind == IMPACT_REACH && spec->n_avoid != 0)
    return mq_fail(IMPACT_E_INVAL, "reachability takes no avoid boxes (use reach-avoid)");
  if (spec->pessimistic != 0 && spec->pessimistic != 1)
    return mq_fail(IMPACT_E_INVAL, "pessimistic must be 0 or 1");
  if (spec->max_sweeps < 1) return mq_fail(IMPACT_E_INVAL, "max_sweeps must be >= 1");
  if (spec->horizon < IMPACT_HORIZON_AUTO)
    return mq_fail(IMPACT_E_INVAL, "horizon must be >= 0 or IMPACT_HORIZON_AUTO");
  if (!std::isfinite(eps) || !(eps > 0.0)) return mq_fail(IMPACT_E_INVAL, "eps must be > 0");
  ImdpView v;
  if (imdp_view(h, &v) != IMPACT_OK) return mq_fail(IMPACT_E_INVAL, "bad abstraction handle");
  // the selection sweep holds a state's row values in LDS, 256 of them
  if ((int64_t)v.nu * (v.nw > 1 ? v.nw : 1) > 256)
    return mq_fail(IMPACT_E_UNSUPPORTED, "more than 256 (input, disturbance) rows per state");
  const int d = v.d;
  for (int b = 0; b < spec->n_target; ++b)
    for (int i = 0; i < d; ++i)
      if (!(spec->target_boxes[b * 2 * d + i] <= spec->target_boxes[b * 2 * d + d + i]))
        return mq_fail(IMPACT_E_INVAL, "target box with lo > hi");
  for (int b = 0; b < spec->n_avoid; ++b)
    for (int i = 0; i < d; ++i)
      if (!(spec->avoid_boxes[b * 2 * d + i] <= spec->avoid_boxes[b * 2 * d + d + i]))
        return mq_fail(IMPACT_E_INVAL, "avoid box with lo > hi");
  if (v.nu > 256) return mq_fail(IMPACT_E_UNSUPPORTED, "more than 256 inputs per state");
  if (v.max_row > kMaxRowBlock)
    return mq_fail(IMPACT_E_UNSUPPORTED, "rows longer than " + std::to_string(kMaxRowBlock) +
                                             " entries run through impact_interval_iterate");
  // a free slot
  int32_t k = -1;
  for (int32_t i = 0; i < m->cap; ++i)
    if (!m->slots[i].active) {
      k = i;
      break;
    }
  if (k < 0) return mq_fail(IMPACT_E_UNSUPPORTED, "no free query slot (poll finished queries)");
  return mq_guarded([&]() -> int {
    m->join_user();
    MqQuery q;
    const int64_t N = v.n_states;
    const bool safety = spec->kind == IMPACT_SAFETY;
    auto get = [&](size_t bytes) {
      void* p = m->alloc(bytes);
      q.bufs.push_back(p);
      return p;
    };
    std::vector<void*> temps;
    auto tget = [&](size_t bytes) {
      void* p = m->alloc(bytes);
      temps.push_back(p);
      return p;
    };
    struct TempFree {
      impact_mq* m;
      std::vector<void*>* t;
      ~TempFree() {
        m->sync();
        for (void* p : *t) m->release(p);
      }
    } tf{m, &temps};
    int8_t* cls = (int8_t*)get((size_t)std::max<int64_t>(1, N));
    int32_t* safe = (int32_t*)get(sizeof(int32_t) * (size_t)std::max<int64_t>(1, N));
    double2* vb0 = (double2*)get(sizeof(double2) * (size_t)std::max<int64_t>(1, N));
    double2* vb1 = (double2*)get(sizeof(double2) * (size_t)std::max<int64_t>(1, N));
    int32_t* pi = (int32_t*)get(sizeof(int32_t) * (size_t)std::max<int64_t>(1, N));
    double* tb = (double*)tget(sizeof(double) * (size_t)std::max(1, spec->n_target * 2 * d));
    double* ab = (double*)tget(sizeof(double) * (size_t)std::max(1, spec->n_avoid * 2 * d));
    int64_t* flag = (int64_t*)tget(sizeof(int64_t) * (size_t)std::max<int64_t>(1, N));
    int64_t* pos = (int64_t*)tget(sizeof(int64_t) * (size_t)(N + 1));
    const int64_t te = scan_tmp_elems(N);
    int64_t* stmp = (int64_t*)tget(sizeof(int64_t) * (size_t)te);
    if (spec->n_target > 0)
      MQ_TRY(hipMemcpyAsync(tb, spec->target_boxes, sizeof(double) * spec->n_target * 2 * d,
                            hipMemcpyHostToDevice, m->st));
    if (spec->n_avoid > 0)
      MQ_TRY(hipMemcpyAsync(ab, spec->avoid_boxes, sizeof(double) * spec->n_avoid * 2 * d,
                            hipMemcpyHostToDevice, m->st));
    MQ_TRY(launch_label(v.dp, N, tb, spec->n_target, ab, spec->n_avoid, cls, flag, m->st));
    MQ_TRY(exclusive_scan_i64(flag, pos, N, stmp, te, m->st));
    int64_t n_safe = 0;
    MQ_TRY(hipMemcpyAsync(&n_safe, pos + N, sizeof(int64_t), hipMemcpyDeviceToHost, m->st));
    MQ_TRY(hipStreamSynchronize(m->st));
    MQ_TRY(launch_compact(cls, pos, N, safe, m->st));
    MQ_TRY(launch_init_values(cls, N, safety, vb0, vb1, pi, m->st));
    // outputs of non-SAFE cells now (SAFE cells are written when the passes close)
    MQ_TRY(launch_finalize(cls, N, vb0, pi, 0, safety, 0, lo, policy, m->st));
    MQ_TRY(launch_finalize(cls, N, vb0, pi, 1, safety, 0, hi, nullptr, m->st));
    QueryDesc D;
    std::memset(&D, 0, sizeof(D));
    D.a = v.a;
    D.a.pi = pi;
    D.a.n_safe = n_safe;
    D.a.out_val = safety ? 1.0 : 0.0;
    D.a.reach = !safety;
    D.vb0 = vb0;
    D.vb1 = vb1;
    D.lo = lo;
    D.hi = hi;
    D.pol = policy;
    D.safety = safety;
    // the adversarial LP first for the pessimistic policy, second for the optimistic one
    D.upper_first = spec->pessimistic ? 0 : 1;
    D.max_lp[0] = spec->pessimistic ? safety : !safety;
    D.max_lp[1] = spec->pessimistic ? !safety : safety;
    // a disturbance player (eq. (5.1)) takes the selection sweep, which values
    // each (state, input) by its worst disturbance row in both passes
    D.box_class = v.max_row <= 512 && v.nw <= 1;
    if (!D.box_class) {
      // selection sweep: two sort buffers of both value components, row hints
      D.vs[0] = (double*)get(sizeof(double) * 2 * (size_t)std::max<int64_t>(1, N));
      D.vs[1] = (double*)get(sizeof(double) * 2 * (size_t)std::max<int64_t>(1, N));
      const int64_t rows = N * v.nu * (v.nw > 1 ? v.nw : 1);
      D.a.hint = (int32_t*)get(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(1, rows));
      D.a.n_cells = N;
      MQ_TRY(launch_fill_i32(D.a.hint, 2 * rows, -1, m->st));
    }
    // finite horizon: no stop test (gap >= 0 > -1), exactly `horizon` sweeps per pass
    D.finite = spec->horizon > 0;
    D.auto_h = spec->horizon == IMPACT_HORIZON_AUTO;
    D.eps = D.finite ? -1.0 : eps;
    D.cap = D.finite ? spec->horizon : spec->max_sweeps;
    QueryCtrl c;
    std::memset(&c, 0, sizeof(c));
    c.gap[0] = c.gap[1] = n_safe > 0 ? 1.0 : 0.0;
    if (n_safe == 0) {
      c.phase = 4;  // nothing to iterate: outputs are final
      c.converged[0] = c.converged[1] = 1;
    } else {
      // the self rule of Remark 5.2 and a finite horizon always sweep
      const bool skip = !D.auto_h && 1.0 <= D.eps;
      c.phase = skip ? 1 : 0;
      c.converged[0] = skip;
    }
    MQ_TRY(hipMemcpyAsync(m->d_ctrl + k, &c, sizeof(c), hipMemcpyHostToDevice, m->st));
    MQ_TRY(hipStreamSynchronize(m->st));
    q.id = m->next_id++;
    q.active = true;
    q.finished = false;
    q.n_safe = n_safe;
    q.n_states = N;
    q.box_class = D.box_class;
    q.max_row = v.max_row;
    q.max_box = v.max_box;
    q.nu = v.nu;
    q.d = v.d;
    q.keep = v.keep;
    q.safe = safe;
    m->slots[k] = q;
    m->h_desc[k] = D;
    m->n_slots_used = std::max(m->n_slots_used, k + 1);
    m->dirty = true;
    if (n_safe == 0) {
      // report at the next poll without running anything
      m->finished_info[q.id] = impact_iter_info{};
      m->finished_info[q.id].n_safe = 0;
      m->finished_info[q.id].converged[0] = m->finished_info[q.id].converged[1] = 1;
      m->finished_info[q.id].horizon = D.finite ? D.cap : (D.auto_h ? 1 : 0);
      m->slots[k].finished = true;
      m->unreported.push_back(q.id);
    } else {
      m->live_submitted += 1;
    }
    *id_out = q.id;
    return IMPACT_OK;
  });
}

int impact_mq_run(impact_mq* m, int32_t steps, int32_t* n_active) {
  g_mq_err.clear();
  if (!m || steps < 1) return mq_fail(IMPACT_E_INVAL, "bad argument");
  return mq_guarded([&]() -> int {
    m->join_user();
    if (m->dirty) rebuild(m);
    // d_done counts every query that reached the done phase since creation
    int32_t done = 0;
    MQ_TRY(hipMemcpyAsync(&done, m->d_done, sizeof(int32_t), hipMemcpyDeviceToHost, m->st));
    MQ_TRY(hipStreamSynchronize(m->st));
    int32_t left = steps;
    const int32_t chunk_max = 64;
    while (left > 0 && done < m->live_submitted && m->n_items > 0) {
      const int32_t c = std::min(left, chunk_max);
      if (!m->exec || m->graph_steps != c) capture(m, c);
      MQ_TRY(hipGraphLaunch(m->exec, m->st));
      MQ_TRY(hipMemcpyAsync(&done, m->d_done, sizeof(int32_t), hipMemcpyDeviceToHost, m->st));
      MQ_TRY(hipStreamSynchronize(m->st));
      m->steps_run += c;
      left -= c;
    }
    if (n_active) *n_active = (int32_t)std::max<int64_t>(0, m->live_submitted - done);
    return IMPACT_OK;
  });
}

int impact_mq_poll(impact_mq* m, int32_t* ids, int32_t cap, int32_t* n_out) {
  g_mq_err.clear();
  if (!m || !n_out || cap < 0 || (cap > 0 && !ids)) return mq_fail(IMPACT_E_INVAL, "bad argument");
  return mq_guarded([&]() -> int {
    std::vector<QueryCtrl> c(std::max(1, m->n_slots_used));
    if (m->n_slots_used > 0) {
      MQ_TRY(hipMemcpyAsync(c.data(), m->d_ctrl, sizeof(QueryCtrl) * m->n_slots_used,
                            hipMemcpyDeviceToHost, m->st));
      MQ_TRY(hipStreamSynchronize(m->st));
    }
    for (int32_t k = 0; k < m->n_slots_used; ++k) {
      MqQuery& q = m->slots[k];
      if (!q.active || q.finished || c[k].phase != 4) continue;
      impact_iter_info info{};
      for (int p = 0; p < 2; ++p) {
        info.sweeps[p] = c[k].sweeps[p];
        info.gap[p] = c[k].gap[p];
        info.converged[p] = c[k].converged[p];
        info.updates[p] = c[k].sweeps[p] * q.n_safe * (p == 0 ? q.nu : 1);
      }
      info.n_safe = q.n_safe;
      info.horizon = m->h_desc[k].finite ? m->h_desc[k].cap : 0;
      if (m->h_desc[k].auto_h) {
        // Remark 5.2: the returned run is the finite stage; converged tells
        // whether each pass's iterates stopped moving before the cap
        info.horizon = c[k].horizon;
        for (int p = 0; p < 2; ++p) {
          info.self_sweeps[p] = c[k].self_sweeps[p];
          info.converged[p] = c[k].self_conv[p];
        }
      }
      m->finished_info[q.id] = info;
      q.finished = true;
      m->unreported.push_back(q.id);
    }
    int32_t n = 0;
    std::vector<int32_t> keep;
    for (int32_t id : m->unreported) {
      if (n < cap)
        ids[n++] = id;
      else
        keep.push_back(id);
    }
    m->unreported = keep;
    // reported queries give their buffers and slots back
    for (int32_t k = 0; k < m->n_slots_used; ++k) {
      MqQuery& q = m->slots[k];
      if (!q.active || !q.finished) continue;
      if (std::find(m->unreported.begin(), m->unreported.end(), q.id) != m->unreported.end())
        continue;
      for (void* p : q.bufs) m->release(p);
      q.bufs.clear();
      q.keep.reset();
      q.active = false;
      m->dirty = true;
    }
    while (m->n_slots_used > 0 && !m->slots[m->n_slots_used - 1].active) --m->n_slots_used;
    *n_out = n;
    return IMPACT_OK;
  });
}

int impact_mq_query_info(const impact_mq* m, int32_t id, impact_iter_info* info) {
  if (!m || !info) return mq_fail(IMPACT_E_INVAL, "null argument");
  auto it = m->finished_info.find(id);
  if (it == m->finished_info.end()) return mq_fail(IMPACT_E_INVAL, "query not finished / unknown");
  *info = it->second;
  return IMPACT_OK;
}

void impact_mq_free(impact_mq* m) { delete m; }

}  // extern "C"
