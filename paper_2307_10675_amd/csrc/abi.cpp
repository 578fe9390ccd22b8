// extern "C" entry points of libifci (declared in include/ifci.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

namespace ifci {
static thread_local std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }
}  // namespace ifci

using namespace ifci;

namespace {

// Makes the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

ifci_status dev_err(hipError_t e, const char* where) {
  set_error(std::string(where) + ": " + hipGetErrorString(e));
  return IFCI_ERR_DEVICE;
}

#define HIP_TRY(expr, where)                 \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return dev_err(e_, where); \
  } while (0)

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

template <typename T>
void free_one(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Free what earlier batched device-wide solves kept alive (graphs, host
// copies of uploaded arrays) once their work has run; `all` waits for it.
void release_in_flight(ifci_plan_s* P, bool all) {
  std::vector<ifci_plan_s::InFlight> keep;
  for (ifci_plan_s::InFlight& f : P->in_flight) {
    bool done = true;
    if (f.done) {
      if (all)
        (void)hipEventSynchronize(f.done);
      else
        done = hipEventQuery(f.done) == hipSuccess;
    }
    if (!done) {
      keep.push_back(std::move(f));
      continue;
    }
    for (hipGraphExec_t g : f.graphs) (void)hipGraphExecDestroy(g);
    if (f.done) (void)hipEventDestroy(f.done);
  }
  P->in_flight = std::move(keep);
}

void free_device(ifci_plan_s* P) {
  free_one(P->d_inc);
  free_one(P->d_orbs);
  free_one(P->d_tables);
  free_one(P->d_order);
  free_one(P->d_sub_ptr);
  free_one(P->d_sub_idx);
  free_one(P->d_inc_size);
  free_one(P->d_rdm_off);
  free_one(P->d_loc);
  free_one(P->d_w_inc);
  free_one(P->d_keep);
  free_one(P->group_ctl);
  P->group_ctl_bytes = 0;
  release_in_flight(P, true);
  if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
  P->capture_stream = nullptr;
  for (hipEvent_t& e : P->poll_event) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (P->pinned) (void)hipHostFree(P->pinned);
  P->pinned = nullptr;
  for (hipStream_t s : P->slot_streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : P->slot_events) (void)hipEventDestroy(e);
  if (P->fork_event) (void)hipEventDestroy(P->fork_event);
  P->slot_streams.clear();
  P->slot_events.clear();
  P->fork_event = nullptr;
  P->on_device = false;
}

// Upload the plan's small tables to its device (first use of the device).
ifci_status ensure_device(ifci_plan_s* P) {
  if (P->on_device) return IFCI_OK;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&P->d_inc, P->inc);
  if (e == hipSuccess) e = upload(&P->d_orbs, P->orbs);
  if (e == hipSuccess) e = upload(&P->d_tables, P->tables);
  if (e == hipSuccess) e = upload(&P->d_order, P->order_all);
  if (e == hipSuccess) e = upload(&P->d_sub_ptr, P->h_sub_ptr);
  if (e == hipSuccess) e = upload(&P->d_sub_idx, P->h_sub_idx);
  if (e == hipSuccess) e = upload(&P->d_inc_size, P->h_inc_size);
  if (e == hipSuccess) e = upload(&P->d_rdm_off, P->rdm_off);
  if (e == hipSuccess) e = upload(&P->d_loc, P->h_loc);
  if (e == hipSuccess) e = upload(&P->d_w_inc, P->h_w_inc);
  if (e == hipSuccess && !P->keep.empty()) e = upload(&P->d_keep, P->keep);
  if (e != hipSuccess) {
    free_device(P);
    return dev_err(e, "uploading plan tables");
  }
  // the static scratch array's address on this device, for the
  // allocation-free entry point
  e = static_scratch(nullptr);
  if (e != hipSuccess) {
    free_device(P);
    return dev_err(e, "static scratch address");
  }
  P->on_device = true;
  return IFCI_OK;
}

ifci_status check_plan(ifci_plan_t p) {
  if (!p) {
    set_error("null plan");
    return IFCI_ERR_ARG;
  }
  return IFCI_OK;
}

ifci_status need_ws(ifci_plan_t p) {
  if (!p->ws) {
    set_error("no workspace set (ifci_set_workspace)");
    return IFCI_ERR_STATE;
  }
  return IFCI_OK;
}

ifci_status need_ints(ifci_plan_t p) {
  ifci_status s = need_ws(p);
  if (s != IFCI_OK) return s;
  if (!p->integrals_set) {
    set_error("integrals not set (ifci_set_integrals)");
    return IFCI_ERR_STATE;
  }
  return IFCI_OK;
}

// LDS the batched solver asks for when running increments `ids`: enough
// for every wave's FP64 E slice, capped at the hardware limit.
int batch_lds(const ifci_plan_s* P, const std::vector<int32_t>& ids) {
  int64_t need = 0;
  for (int32_t i : ids) {
    const IncDev& d = P->inc[i];
    need = std::max(need, batched_lds_want(d.k, d.n_str, d.n_link));
  }
  return (int)std::min<int64_t>(kMaxLds, (need + 255) & ~int64_t(255));
}

// Iterations captured per graph of the batched device-wide solver; without
// IFCI_FLAG_ASYNC_WIDE the host reads the live count after every graph (one
// graph behind the device).
constexpr int kWideChunk = 4;

// Copy of v kept in `keep`; returns the copy's bytes (stable: moving the
// outer vector does not move them).
template <typename T>
const char* push_bytes(std::vector<std::vector<char>>& keep, const std::vector<T>& v) {
  keep.emplace_back((const char*)v.data(), (const char*)v.data() + v.size() * sizeof(T));
  return keep.back().data();
}

// Layout of a control block for n items: item pointers, live counts and
// lists, output positions (each 256-byte aligned).
struct CtlBlock {
  WideItem** ptrs;
  int* ctl;
  int32_t* pos;
};
int64_t ctl_block_bytes(int n) {
  auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
  return up((int64_t)n * 8) + up((int64_t)wide_ctl_ints(n) * 4) + up((int64_t)n * 4);
}
CtlBlock ctl_block(char* base, int n) {
  auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
  CtlBlock c;
  c.ptrs = (WideItem**)base;
  c.ctl = (int*)(base + up((int64_t)n * 8));
  c.pos = (int32_t*)((char*)c.ctl + up((int64_t)wide_ctl_ints(n) * 4));
  return c;
}

// The increments of one plan that a batched device-wide solve takes, with
// where their outputs go.
struct WideMember {
  ifci_plan_s* P;
  std::vector<int32_t> ids;
  int64_t first;
  double* e_out;
  int32_t* status_out;
  int32_t* iters_out;
  double* resid_out;
  const uint8_t* evict;
};

// Batched device-wide solve of the members' increments: grouped by shape
// across plans, each plan contributing at most its wide_cap increments to a
// batch; every batch set up, iterated with device-side control (graph
// replays of kWideChunk iterations) and its outputs written.  `owner` keeps
// the streams, events, pinned counts and (for several plans) the control
// block; the options (precision, tolerances, iterations, flags) are owner's.
ifci_status run_wide(ifci_plan_s* owner, std::vector<WideMember>& members, hipStream_t st) {
  ifci_plan_s* O = owner;
  for (WideMember& m : members) {
    release_in_flight(m.P, false);
    if (!m.ids.empty() && m.P->wide_cap < 1) {
      set_error("ifci_davidson: the workspace has no slots for device-wide increments");
      return IFCI_ERR_STATE;
    }
  }
  HIP_TRY(wide_prepare(0), "ifci_davidson wide");
  if (!O->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&O->capture_stream, hipStreamNonBlocking), "stream");
  if (!O->pinned) HIP_TRY(hipHostMalloc((void**)&O->pinned, 2 * sizeof(int32_t), hipHostMallocDefault), "pinned");
  for (hipEvent_t& e : O->poll_event)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  const bool async = (O->opt.flags & IFCI_FLAG_ASYNC_WIDE) != 0;
  const bool group = members.size() > 1;
  ifci_plan_s::InFlight fl;
  // (shape) -> per member, its increments of that shape, in the given order
  std::vector<std::pair<int, int>> shapes;
  for (WideMember& m : members)
    for (int32_t i : m.ids) {
      const std::pair<int, int> key(m.P->inc[i].k, m.P->inc[i].na);
      if (std::find(shapes.begin(), shapes.end(), key) == shapes.end()) shapes.push_back(key);
    }
  for (const std::pair<int, int>& key : shapes) {
    std::vector<std::vector<int32_t>> todo(members.size());
    size_t left = 0;
    for (size_t mi = 0; mi < members.size(); ++mi)
      for (int32_t i : members[mi].ids)
        if (members[mi].P->inc[i].k == key.first && members[mi].P->inc[i].na == key.second) todo[mi].push_back(i);
    for (auto& t : todo) left += t.size();
    std::vector<size_t> next(members.size(), 0);
    while (left > 0) {
      // one batch: up to wide_cap increments of each member
      std::vector<WideItem*> ptrs;
      std::vector<int32_t> pos;
      std::vector<std::pair<size_t, std::pair<int, int>>> spans;  // member, (offset, count)
      IncDev shape{};
      for (size_t mi = 0; mi < members.size(); ++mi) {
        WideMember& m = members[mi];
        ifci_plan_s* P = m.P;
        const int take = (int)std::min<size_t>((size_t)P->wide_cap, todo[mi].size() - next[mi]);
        if (take <= 0) continue;
        WideItem* d_items = (WideItem*)(P->ws + P->off_wide_ctl);
        std::vector<WideItem> items(take);
        for (int j = 0; j < take; ++j) {
          const int32_t i = todo[mi][next[mi] + j];
          const IncDev& d = P->inc[i];
          const WideSlot sl = wide_slot(d);
          double* slot = (double*)(P->ws + P->off_wide) + (int64_t)j * P->wide_slot_doubles;
          WideItem& w = items[j];
          std::memset(&w, 0, sizeof(w));
          w.d = d;
          w.B = P->ws_ints() + d.int_off;
          w.tabs = P->d_tables;
          w.Vb = P->ws_dav() + d.vec_off;
          w.Sb = w.Vb + (int64_t)d.mspace * d.stride;
          w.HD = w.Vb + 2 * (int64_t)d.mspace * d.stride;
          w.X = w.HD + d.stride;
          w.T = slot + sl.T;
          w.F = slot + sl.F;
          w.part = slot + sl.part;
          w.state = slot + sl.state;
          w.sc = slot + sl.sc;
          w.evict = m.evict ? m.evict + (i - m.first) : nullptr;
          w.mmax = d.mspace;
          shape = d;
        }
        // the copies read host memory kept alive until this call's work has
        // run (released by a later call or at plan destruction)
        const char* h_items = push_bytes(fl.host, items);
        HIP_TRY(hipMemcpyAsync(d_items, h_items, take * sizeof(WideItem), hipMemcpyHostToDevice, st), "upload");
        spans.push_back({mi, {(int)ptrs.size(), take}});
        for (int j = 0; j < take; ++j) {
          ptrs.push_back(d_items + j);
          pos.push_back((int32_t)(todo[mi][next[mi] + j] - m.first));
        }
        next[mi] += take;
        left -= take;
      }
      const int n = (int)ptrs.size();
      char* cbase;
      if (!group) {
        ifci_plan_s* P = members[0].P;
        cbase = P->ws + P->off_wide_ctl + ((int64_t)P->wide_cap * sizeof(WideItem) + 255) / 256 * 256;
      } else {
        const int64_t need = ctl_block_bytes(n);
        if (need > O->group_ctl_bytes) {
          // grow the owner's control block (its earlier work is done first)
          HIP_TRY(hipStreamSynchronize(st), "ifci_davidson_group");
          if (O->group_ctl) (void)hipFree(O->group_ctl);
          O->group_ctl = nullptr;
          O->group_ctl_bytes = 0;
          HIP_TRY(hipMalloc((void**)&O->group_ctl, need), "ifci_davidson_group control block");
          O->group_ctl_bytes = need;
        }
        cbase = O->group_ctl;
      }
      const CtlBlock cb = ctl_block(cbase, n);
      const char* h_ptrs = push_bytes(fl.host, ptrs);
      const char* h_pos = push_bytes(fl.host, pos);
      HIP_TRY(hipMemcpyAsync(cb.ptrs, h_ptrs, n * sizeof(WideItem*), hipMemcpyHostToDevice, st), "upload");
      HIP_TRY(hipMemcpyAsync(cb.pos, h_pos, n * sizeof(int32_t), hipMemcpyHostToDevice, st), "upload");
      WideRun R;
      R.items = cb.ptrs;
      R.n = n;
      R.ctl = cb.ctl;
      R.d = shape;
      R.k = shape.k;
      R.precision = O->opt.precision;
      R.max_iter = O->opt.max_iter;
      R.r_tol = O->opt.r_tol;
      R.r_tol_inner = O->opt.r_tol_inner;
      HIP_TRY(wide_setup(R, st), "ifci_davidson wide set-up");
      // one chunk of iterations, captured once and replayed
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIP_TRY(hipStreamBeginCapture(O->capture_stream, hipStreamCaptureModeThreadLocal), "capture");
      hipError_t ce = hipSuccess;
      for (int c = 0; c < kWideChunk && ce == hipSuccess; ++c) ce = wide_iteration(R, O->capture_stream);
      const hipError_t ee = hipStreamEndCapture(O->capture_stream, &graph);
      HIP_TRY(ce, "ifci_davidson wide capture");
      HIP_TRY(ee, "ifci_davidson wide capture");
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(ie, "ifci_davidson wide instantiate");
      fl.graphs.push_back(exec);
      const int n_chunks = (R.max_iter + kWideChunk) / kWideChunk;  // at least max_iter + 1 iterations
      for (int c = 0; c < n_chunks; ++c) {
        HIP_TRY(hipGraphLaunch(exec, st), "ifci_davidson wide launch");
        if (async) continue;
        HIP_TRY(hipMemcpyAsync(O->pinned + (c & 1), cb.ctl + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                "ifci_davidson live count");
        HIP_TRY(hipEventRecord(O->poll_event[c & 1], st), "ifci_davidson");
        if (c >= 1) {
          HIP_TRY(hipEventSynchronize(O->poll_event[(c - 1) & 1]), "ifci_davidson");
          if (O->pinned[(c - 1) & 1] == 0) break;
        }
      }
      for (auto& sp : spans) {
        const WideMember& m = members[sp.first];
        HIP_TRY(wide_finish(cb.ptrs + sp.second.first, sp.second.second, cb.pos + sp.second.first, m.P->e_const,
                            m.e_out, m.status_out, m.iters_out, m.resid_out, st),
                "ifci_davidson wide finish");
      }
    }
  }
  HIP_TRY(hipEventCreateWithFlags(&fl.done, hipEventDisableTiming), "event");
  HIP_TRY(hipEventRecord(fl.done, st), "event");
  O->in_flight.push_back(std::move(fl));
  // the members' regions are in use until that event: their next calls
  // wait for it through stream order; record it on them too for release
  return IFCI_OK;
}

// One launch of the on-chip batched solver over the increments `ids`
// (heaviest first) of plan p.
ifci_status launch_on_chip(ifci_plan_s* p, const std::vector<int32_t>& ids, int64_t first, double* e_out,
                           int32_t* status_out, const uint8_t* evict_mask, int32_t* iters_out, double* resid_out,
                           hipStream_t st) {
  if (ids.empty()) return IFCI_OK;
  if (ids != p->order_batch) {
    // a new work list: wait for any earlier upload from order_batch
    // before reusing its host memory (a repeated list is already there)
    HIP_TRY(hipStreamSynchronize(st), "ifci_davidson");
    p->order_batch = ids;
    HIP_TRY(hipMemcpyAsync(p->d_order, p->order_batch.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           st),
            "ifci_davidson upload");
  }
  SolveArgs A;
  A.inc = p->d_inc;
  A.order = p->d_order;
  A.count = (int32_t)ids.size();
  A.precision = p->opt.precision;
  A.max_iter = p->opt.max_iter;
  A.max_space = p->opt.max_space;
  A.n_guess = p->opt.n_guess;
  A.r_tol = p->opt.r_tol;
  A.r_tol_inner = p->opt.r_tol_inner;
  A.tables = p->d_tables;
  A.ints = p->ws_ints();
  A.dav = p->ws_dav();
  A.first = first;
  A.e_out = e_out;
  A.status_out = status_out;
  A.iters_out = iters_out;
  A.resid_out = resid_out;
  A.evict = evict_mask;
  A.e_const = p->e_const;
  A.phase = p->phase_counters;
  A.tune = p->tune;
  HIP_TRY(launch_batched(A, batch_lds(p, ids), st), "ifci_davidson batched");
  return IFCI_OK;
}

// Validated HBCI call on increment inc: the increment's description for
// the kernels, with the reference key from the host orbital lists.
ifci_status hbci_setup(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, void* work, int64_t work_bytes,
                       HbciInc* I) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !o) {
    set_error("HBCI: bad increment index or null options");
    return IFCI_ERR_ARG;
  }
  if (!(o->eps1 >= 0.0) || !(o->eps2 >= 0.0) || !std::isfinite(o->eps1) || !std::isfinite(o->eps2) ||
      o->max_iter < 1 || o->max_dav < 1 || o->m_max < 2 || o->m_max > 16 || !(o->r_tol > 0.0) || o->max_det < 2 ||
      o->max_det > ((int64_t)1 << 30) || o->max_nnz < 1 || o->max_ext < 1 || o->max_ext > ((int64_t)1 << 40)) {
    set_error("HBCI: options out of range (eps >= 0, max_iter, max_dav >= 1, 2 <= m_max <= 16, r_tol > 0, "
              "2 <= max_det <= 2^30, max_nnz, max_ext >= 1)");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  const IncDev& d = p->inc[inc];
  if (!work || ((uintptr_t)work & 255u) || work_bytes < hbci_work_bytes(d.k, *o)) {
    set_error("HBCI: work must be non-null, 256-byte aligned and at least ifci_hbci_work_bytes long");
    return IFCI_ERR_ARG;
  }
  uint32_t ref = 0;
  for (int i = 0; i < d.k; ++i) {
    const int orb = p->orbs[d.act_off + i];
    if (std::binary_search(p->ref_occ.begin(), p->ref_occ.end(), orb)) ref |= 1u << i;
  }
  I->h = p->h;
  I->eri = p->eri;
  I->n_orb = p->n_orb;
  I->act = p->d_orbs + d.act_off;
  I->k = d.k;
  I->core = p->d_orbs + d.core_off;
  I->n_core = d.n_core;
  I->ref = (uint64_t)ref | ((uint64_t)ref << 32);
  I->e_core = p->ws_ints() + d.int_off + int_block(d.k).misc;
  I->e_const = p->e_const;
  return IFCI_OK;
}

ifci_status hbci_space_args(const ifci_hbci_options* o, const uint64_t* dets, int64_t n, const double* c) {
  if (!dets || !c || n < 1 || n > o->max_det) {
    set_error("HBCI: need non-null dets and c and 1 <= n <= max_det");
    return IFCI_ERR_ARG;
  }
  return IFCI_OK;
}

}  // namespace

extern "C" {

int ifci_abi_version(void) { return IFCI_ABI_VERSION; }

void ifci_default_options(ifci_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = IFCI_FP64;
  o->solver = IFCI_SOLVER_BATCHED;
  o->r_tol = 1e-7;
  o->r_tol_inner = 1e-4;
  o->max_iter = 300;
  o->max_space = 12;
  o->flags = 0;
  o->n_guess = 64;
}

const char* ifci_status_string(ifci_status s) {
  switch (s) {
    case IFCI_OK: return "ok";
    case IFCI_ERR_ARG: return "invalid argument";
    case IFCI_ERR_UNSUPPORTED: return "unsupported";
    case IFCI_ERR_OOM: return "out of memory";
    case IFCI_ERR_DEVICE: return "device error";
    case IFCI_ERR_NOT_CONVERGED: return "not converged";
    case IFCI_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* ifci_last_error(void) { return g_error.c_str(); }

ifci_status ifci_tables(int32_t k, int32_t n_alpha, int32_t* strings, int32_t* link) {
  if (k < 1 || k > kMaxAct || n_alpha < 0 || n_alpha > k) {
    set_error("ifci_tables: need 1 <= k <= 16 and 0 <= n_alpha <= k");
    return IFCI_ERR_ARG;
  }
  fill_link_dump(k, n_alpha, strings, link);
  return IFCI_OK;
}

ifci_status ifci_plan_create(const ifci_problem* problem, const ifci_options* options, int hip_device,
                             ifci_plan_t* out) {
  if (!out) {
    set_error("null output pointer");
    return IFCI_ERR_ARG;
  }
  *out = nullptr;
  ifci_options opt;
  if (options)
    opt = *options;
  else
    ifci_default_options(&opt);
  ifci_plan_s* P = new (std::nothrow) ifci_plan_s();
  if (!P) return IFCI_ERR_OOM;
  P->device = hip_device;
  ifci_status s = plan_build(P, problem, &opt);
  if (s != IFCI_OK) {
    delete P;
    return s;
  }
  const int n_inc = (int)P->inc.size();
  // on-chip feasibility of each increment
  P->batched_ok.resize(n_inc);
  for (int i = 0; i < n_inc; ++i) {
    const IncDev& d = P->inc[i];
    P->batched_ok[i] = d.k <= 8 && batched_lds_bytes(d.k, d.n_str, d.n_link) <= kMaxLds;
  }
  // energy-assembly tables: the subsets of every increment (any order)
  std::map<std::vector<int>, int> index;
  for (int i = 0; i < n_inc; ++i) index[P->inc_bodies[i]] = i;
  std::vector<int32_t> sub_ptr(1, 0), sub_idx, inc_size(n_inc);
  for (int i = 0; i < n_inc; ++i) {
    const std::vector<int>& S = P->inc_bodies[i];
    const int sz = (int)S.size();
    inc_size[i] = sz;
    for (int k = 1; k <= sz; ++k) {
      std::vector<int> c(k);
      for (int j = 0; j < k; ++j) c[j] = j;
      while (true) {
        std::vector<int> T(k);
        for (int j = 0; j < k; ++j) T[j] = S[c[j]];
        sub_idx.push_back(index.at(T));
        int j = k - 1;
        while (j >= 0 && c[j] == sz - k + j) --j;
        if (j < 0) break;
        ++c[j];
        for (int l = j + 1; l < k; ++l) c[l] = c[l - 1] + 1;
      }
    }
    sub_ptr.push_back((int32_t)sub_idx.size());
  }
  // orbital roles per increment (and the reference as the last row)
  const int n = P->n_orb;
  std::vector<int8_t> loc((size_t)(n_inc + 1) * n, -2);
  for (int i = 0; i < n_inc; ++i) {
    const IncDev& d = P->inc[i];
    for (int a = 0; a < d.k; ++a) loc[(size_t)i * n + P->orbs[d.act_off + a]] = (int8_t)a;
    for (int c = 0; c < d.n_core; ++c) loc[(size_t)i * n + P->orbs[d.core_off + c]] = -1;
  }
  for (int o : P->ref_occ) loc[(size_t)n_inc * n + o] = -1;
  std::vector<double> w_inc(n_inc);
  for (int i = 0; i < n_inc; ++i) w_inc[i] = P->weights[inc_size[i] - 1];

  P->h_sub_ptr = std::move(sub_ptr);
  P->h_sub_idx = std::move(sub_idx);
  P->h_inc_size = std::move(inc_size);
  P->h_loc = std::move(loc);
  P->h_w_inc = std::move(w_inc);
  *out = P;
  return IFCI_OK;
}

ifci_status ifci_plan_destroy(ifci_plan_t p) {
  if (!p) return IFCI_OK;
  if (p->on_device) {
    DeviceGuard g(p->device);
    free_device(p);
  }
  delete p;
  return IFCI_OK;
}

ifci_status ifci_plan_info(ifci_plan_t p, int64_t* n_inc, int64_t* workspace_bytes, int64_t* max_ndet) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (n_inc) *n_inc = (int64_t)p->inc.size();
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  if (max_ndet) *max_ndet = p->max_ndet;
  return IFCI_OK;
}

ifci_status ifci_increment(ifci_plan_t p, int64_t idx, int32_t* bodies, int32_t* n_act, int32_t* n_alpha,
                           int64_t* n_det) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (idx < 0 || idx >= (int64_t)p->inc.size()) {
    set_error("increment index out of range");
    return IFCI_ERR_ARG;
  }
  const IncDev& d = p->inc[idx];
  if (bodies) {
    const std::vector<int>& S = p->inc_bodies[idx];
    for (int i = 0; i < p->order; ++i) bodies[i] = i < (int)S.size() ? S[i] : -1;
  }
  if (n_act) *n_act = d.k;
  if (n_alpha) *n_alpha = d.na;
  if (n_det) *n_det = d.n_det;
  return IFCI_OK;
}

ifci_status ifci_weights(ifci_plan_t p, double* w) {
  if (check_plan(p) != IFCI_OK || !w) {
    set_error("null argument");
    return IFCI_ERR_ARG;
  }
  for (int k = 0; k < p->order; ++k) w[k] = p->weights[k];
  return IFCI_OK;
}

ifci_status ifci_set_workspace(ifci_plan_t p, void* dev_ptr, int64_t bytes) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (!dev_ptr || bytes < p->ws_bytes || ((uintptr_t)dev_ptr & 255u)) {
    set_error("workspace must be non-null, 256-byte aligned and at least workspace_bytes long");
    return IFCI_ERR_ARG;
  }
  {
    DeviceGuard g(p->device);
    if (!g.ok) return dev_err(hipErrorInvalidDevice, "ifci_set_workspace");
    ifci_status s = ensure_device(p);
    if (s != IFCI_OK) return s;
  }
  p->ws = (char*)dev_ptr;
  p->integrals_set = false;
  std::fill(p->solved.begin(), p->solved.end(), 0);
  return IFCI_OK;
}

ifci_status ifci_set_integrals(ifci_plan_t p, const double* h, const double* eri, ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (!h || !eri) {
    set_error("null integral pointer");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ws(p);
  if (s != IFCI_OK) return s;
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_embed(p->d_inc, (int)p->inc.size(), p->d_orbs, h, eri, p->n_orb, p->ws_ints(),
                       p->d_orbs + p->ref_off, (int)p->ref_occ.size(), p->e_const, p->ws_misc(), st),
          "ifci_set_integrals");
  p->h = h;
  p->eri = eri;
  p->integrals_set = true;
  std::fill(p->solved.begin(), p->solved.end(), 0);
  return IFCI_OK;
}

ifci_status ifci_sigma(ifci_plan_t p, int64_t inc, const double* c, double* sigma, int32_t precision,
                       ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !c || !sigma || c == sigma ||
      (precision != IFCI_FP64 && precision != IFCI_MIXED)) {
    set_error("ifci_sigma: bad increment, pointer or precision");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  const IncDev& d = p->inc[inc];
  if (d.npair * d.n_det > p->E_doubles) {
    set_error("ifci_sigma: the general product of this increment needs npair x n_det scratch "
              "(use ifci_sigma_sector for symmetric vectors)");
    return IFCI_ERR_UNSUPPORTED;
  }
  DeviceGuard g(p->device);
  HIP_TRY(launch_sigma_wide(d, p->d_inc, (int)inc, p->ws_ints(), p->d_tables, c, sigma, p->ws_E(), precision, 0,
                            0.0, (hipStream_t)stream),
          "ifci_sigma");
  return IFCI_OK;
}

ifci_status ifci_sigma_noalloc(ifci_plan_t p, int64_t inc, const double* c, double* sigma, int32_t precision,
                               ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !c || !sigma || c == sigma ||
      (precision != IFCI_FP64 && precision != IFCI_MIXED)) {
    set_error("ifci_sigma_noalloc: bad increment, pointer or precision");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  const IncDev& d = p->inc[inc];
  const int64_t need = d.npair * d.n_det * (precision == IFCI_MIXED ? 4 : 8);
  if (need > kStaticScratchDoubles * 8) {
    set_error("ifci_sigma_noalloc: this increment's product needs " + std::to_string(need) +
              " bytes of scratch; the static scratch holds " + std::to_string(kStaticScratchDoubles * 8) +
              " (use ifci_sigma)");
    return IFCI_ERR_UNSUPPORTED;
  }
  DeviceGuard g(p->device);
  double* E = nullptr;
  HIP_TRY(static_scratch(&E), "ifci_sigma_noalloc");
  HIP_TRY(launch_sigma_wide(d, p->d_inc, (int)inc, p->ws_ints(), p->d_tables, c, sigma, E, precision, 0, 0.0,
                            (hipStream_t)stream),
          "ifci_sigma_noalloc");
  return IFCI_OK;
}

ifci_status ifci_sigma_sector(ifci_plan_t p, int64_t inc, const double* c, double* sigma, int32_t precision,
                              ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !c || !sigma || c == sigma ||
      (precision != IFCI_FP64 && precision != IFCI_MIXED)) {
    set_error("ifci_sigma_sector: bad increment, pointer or precision");
    return IFCI_ERR_ARG;
  }
  const IncDev& d = p->inc[inc];
  if (!p->batched_ok[inc] && !sigma_column_supported(d)) {
    set_error("ifci_sigma_sector: no symmetric-sector sigma for this increment shape");
    return IFCI_ERR_UNSUPPORTED;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  DeviceGuard g(p->device);
  if (!p->batched_ok[inc]) {
    HIP_TRY(launch_sigma_wide(d, p->d_inc, (int)inc, p->ws_ints(), p->d_tables, c, sigma, p->ws_E(), precision, 1,
                              0.0, (hipStream_t)stream),
            "ifci_sigma_sector");
    return IFCI_OK;
  }
  std::vector<int32_t> one(1, (int32_t)inc);
  HIP_TRY(launch_sigma_one(p->d_inc, (int)inc, p->ws_ints(), p->d_tables, c, sigma, precision, batch_lds(p, one),
                           (hipStream_t)stream),
          "ifci_sigma_sector");
  return IFCI_OK;
}

ifci_status ifci_davidson(ifci_plan_t p, int64_t first, int64_t count, double* e_out, int32_t* status_out,
                          const uint8_t* evict_mask, int32_t* iters_out, double* resid_out,
                          ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  const int64_t n_inc = (int64_t)p->inc.size();
  if (first < 0 || count < 0 || first + count > n_inc || !e_out || !status_out) {
    set_error("ifci_davidson: range outside the plan or null output");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  if (count == 0) return IFCI_OK;
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  const bool plain_only = p->opt.solver == IFCI_SOLVER_PLAIN;
  // batched part: heaviest first
  std::vector<int32_t> ids, rest;
  const bool screened = !p->keep.empty();
  bool any_dropped = false;
  for (int32_t i : p->order_all)
    if (i >= first && i < first + count) {
      if (screened && !p->keep[i]) {
        any_dropped = true;
        continue;
      }
      if (!plain_only && p->batched_ok[i])
        ids.push_back(i);
      else
        rest.push_back(i);
    }
  if (any_dropped)
    HIP_TRY(launch_mark_screened(p->d_keep, first, count, e_out, status_out, iters_out, resid_out, st),
            "ifci_davidson screened");
  s = launch_on_chip(p, ids, first, e_out, status_out, evict_mask, iters_out, resid_out, st);
  if (s != IFCI_OK) return s;
  if (!rest.empty() && !plain_only) {
    std::vector<WideMember> mem(1);
    mem[0] = WideMember{p, rest, first, e_out, status_out, iters_out, resid_out, evict_mask};
    s = run_wide(p, mem, st);
    if (s != IFCI_OK) return s;
  } else if (!rest.empty()) {
    std::vector<uint8_t> ev;
    if (evict_mask) {
      ev.resize(count);
      HIP_TRY(hipMemcpyAsync(ev.data(), evict_mask, count, hipMemcpyDeviceToHost, st), "ifci_davidson");
      HIP_TRY(hipStreamSynchronize(st), "ifci_davidson");
    }
    // one device-wide solve: slot scratch, its stream
    auto solve_one_plain = [&](int32_t i, int slot, hipStream_t sst) -> hipError_t {
      const IncDev& d = p->inc[i];
      PlainArgs A;
      A.d = d;
      A.d_inc = p->d_inc;
      A.inc = i;
      A.ints = p->ws_ints();
      A.tables = p->d_tables;
      A.dav = p->ws_dav() + d.vec_off;
      A.E = p->ws_E(slot);
      A.tmp = p->ws_tmp(slot);
      A.part = p->ws_part(slot);
      A.state = p->ws_state(slot);
      A.precision = p->opt.precision;
      A.max_iter = p->opt.max_iter;
      A.max_space = d.mspace;  // the block's subspace (12 where 3 selects the on-chip iteration)
      A.r_tol = p->opt.r_tol;
      A.r_tol_inner = p->opt.r_tol_inner;
      A.e_const = p->e_const;
      A.evict = evict_mask ? ev[i - first] != 0 : false;
      const int64_t o = i - first;
      return run_plain(A, e_out + o, status_out + o, iters_out ? iters_out + o : nullptr,
                       resid_out ? resid_out + o : nullptr, sst);
    };
    const int W = (int)std::min<size_t>((size_t)p->n_slots, rest.size());
    if (W <= 1) {
      for (int32_t i : rest) HIP_TRY(solve_one_plain(i, 0, st), "ifci_davidson plain");
    } else {
      // Several increments at once, each driven by a host thread on its own
      // stream with its own scratch slot (a device-wide solve waits on the
      // host every iteration; other solves fill the GPU meanwhile).  The
      // worker streams start after the work already queued on `st`, and
      // `st` continues after all of them.
      if ((int)p->slot_streams.size() < W) {
        if (!p->fork_event) HIP_TRY(hipEventCreateWithFlags(&p->fork_event, hipEventDisableTiming), "ifci_davidson");
        while ((int)p->slot_streams.size() < W) {
          hipStream_t ss;
          hipEvent_t se;
          HIP_TRY(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking), "ifci_davidson stream");
          HIP_TRY(hipEventCreateWithFlags(&se, hipEventDisableTiming), "ifci_davidson event");
          p->slot_streams.push_back(ss);
          p->slot_events.push_back(se);
        }
      }
      prepare_sigma_wide();
      HIP_TRY(hipEventRecord(p->fork_event, st), "ifci_davidson");
      for (int w = 0; w < W; ++w) HIP_TRY(hipStreamWaitEvent(p->slot_streams[w], p->fork_event, 0), "ifci_davidson");
      std::atomic<size_t> next(0);
      std::mutex err_mu;
      hipError_t first_err = hipSuccess;
      std::vector<std::thread> pool;
      pool.reserve(W);
      for (int w = 0; w < W; ++w)
        pool.emplace_back([&, w] {
          hipError_t e = hipSetDevice(p->device);
          while (e == hipSuccess) {
            const size_t j = next.fetch_add(1);
            if (j >= rest.size()) break;
            e = solve_one_plain(rest[j], w, p->slot_streams[w]);
          }
          if (e == hipSuccess) e = hipEventRecord(p->slot_events[w], p->slot_streams[w]);
          if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(err_mu);
            if (first_err == hipSuccess) first_err = e;
            next.store(rest.size());
          }
        });
      for (std::thread& t : pool) t.join();
      HIP_TRY(first_err, "ifci_davidson plain (concurrent)");
      for (int w = 0; w < W; ++w) HIP_TRY(hipStreamWaitEvent(st, p->slot_events[w], 0), "ifci_davidson");
    }
  }
  for (int64_t i = first; i < first + count; ++i) p->solved[i] = screened ? p->keep[i] : 1;
  return IFCI_OK;
}

ifci_status ifci_davidson_group(const ifci_plan_t* plans, int32_t n_plans, double* const* e_out,
                                int32_t* const* status_out, int32_t* const* iters_out, double* const* resid_out,
                                ifci_stream_t stream) {
  if (!plans || n_plans < 1 || !e_out || !status_out) {
    set_error("ifci_davidson_group: null plans or outputs");
    return IFCI_ERR_ARG;
  }
  ifci_plan_s* O = plans[0];
  for (int32_t j = 0; j < n_plans; ++j) {
    ifci_plan_s* p = plans[j];
    if (check_plan(p) != IFCI_OK || !e_out[j] || !status_out[j]) {
      set_error("ifci_davidson_group: null plan or output of plan " + std::to_string(j));
      return IFCI_ERR_ARG;
    }
    if (p->device != O->device || p->opt.precision != O->opt.precision || p->opt.solver != IFCI_SOLVER_BATCHED ||
        O->opt.solver != IFCI_SOLVER_BATCHED || p->opt.max_iter != O->opt.max_iter || p->opt.r_tol != O->opt.r_tol ||
        p->opt.r_tol_inner != O->opt.r_tol_inner || p->opt.max_space != O->opt.max_space ||
        p->opt.flags != O->opt.flags) {
      set_error("ifci_davidson_group: plans must share the device and the options, with the batched solver");
      return IFCI_ERR_ARG;
    }
    for (int32_t k = 0; k < j; ++k)
      if (plans[k] == p) {
        set_error("ifci_davidson_group: a plan is listed twice");
        return IFCI_ERR_ARG;
      }
    if (!p->keep.empty()) {
      set_error("ifci_davidson_group: plan " + std::to_string(j) + " carries a screening mask (use ifci_davidson)");
      return IFCI_ERR_UNSUPPORTED;
    }
  }
  for (int32_t j = 0; j < n_plans; ++j) {
    ifci_status s = need_ints(plans[j]);
    if (s != IFCI_OK) return s;
  }
  DeviceGuard g(O->device);
  hipStream_t st = (hipStream_t)stream;
  std::vector<WideMember> mem;
  for (int32_t j = 0; j < n_plans; ++j) {
    ifci_plan_s* p = plans[j];
    std::vector<int32_t> ids, rest;
    for (int32_t i : p->order_all) (p->batched_ok[i] ? ids : rest).push_back(i);
    int32_t* it = iters_out ? iters_out[j] : nullptr;
    double* rs = resid_out ? resid_out[j] : nullptr;
    ifci_status s = launch_on_chip(p, ids, 0, e_out[j], status_out[j], nullptr, it, rs, st);
    if (s != IFCI_OK) return s;
    if (!rest.empty()) mem.push_back(WideMember{p, rest, 0, e_out[j], status_out[j], it, rs, nullptr});
  }
  if (!mem.empty()) {
    ifci_status s = run_wide(O, mem, st);
    if (s != IFCI_OK) return s;
  }
  for (int32_t j = 0; j < n_plans; ++j) std::fill(plans[j]->solved.begin(), plans[j]->solved.end(), 1);
  return IFCI_OK;
}

ifci_status ifci_set_phase_counters(ifci_plan_t p, int64_t* counters, int64_t n) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (counters && n < (int64_t)p->inc.size() * kPhases) {
    set_error("ifci_set_phase_counters: need n_inc * 8 counters");
    return IFCI_ERR_ARG;
  }
  p->phase_counters = counters;
  return IFCI_OK;
}

ifci_status ifci_set_tuning(ifci_plan_t p, int32_t k, int32_t precision, int32_t ps_block, int32_t e_waves) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (k < 1 || k > ifci::kTuneK || (precision != IFCI_FP64 && precision != IFCI_MIXED) || ps_block < -1 ||
      ps_block > ifci::kPsMax || e_waves < 0 || e_waves > kBatchThreads / 64) {
    set_error("ifci_set_tuning: k 1..8, precision FP64 or MIXED, ps_block -1..64, e_waves 0..8");
    return IFCI_ERR_ARG;
  }
  const int pr = precision == IFCI_MIXED ? 1 : 0;
  p->tune.ps_block[k][pr] = (int8_t)ps_block;
  p->tune.e_waves[k][pr] = (int8_t)e_waves;
  return IFCI_OK;
}

ifci_status ifci_screen(ifci_plan_t p, const double* e_inc, double threshold, uint8_t* keep, int64_t* n_kept,
                        ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  const int n_inc = (int)p->inc.size();
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> w(n_inc);
  if (threshold < 0.0 || std::isnan(threshold)) {
    // no screening: the closed-form weights of eqs. 1-5
    p->keep.clear();
    for (int i = 0; i < n_inc; ++i) w[i] = p->weights[p->h_inc_size[i] - 1];
  } else {
    if (!e_inc) {
      set_error("ifci_screen: null e_inc");
      return IFCI_ERR_ARG;
    }
    // increments are ordered by size: the one- and two-body ones come first
    int n12 = 0;
    while (n12 < n_inc && p->h_inc_size[n12] <= 2) ++n12;
    std::vector<double> e(n12);
    double e_ref = 0.0;
    HIP_TRY(hipMemcpyAsync(e.data(), e_inc, sizeof(double) * n12, hipMemcpyDeviceToHost, st), "ifci_screen");
    HIP_TRY(hipMemcpyAsync(&e_ref, p->ws_misc(), sizeof(double), hipMemcpyDeviceToHost, st), "ifci_screen");
    HIP_TRY(hipStreamSynchronize(st), "ifci_screen");
    for (int i = 0; i < n12; ++i)
      if (!std::isfinite(e[i])) {
        set_error("ifci_screen: the energies of the one- and two-body increments are needed (solve them first)");
        return IFCI_ERR_ARG;
      }
    // eps_ij for every pair of bodies (eq. 3)
    const int nb = p->n_bodies;
    std::vector<double> e1(nb, 0.0);
    std::vector<uint8_t> link((size_t)nb * nb, 0);
    for (int i = 0; i < n12; ++i)
      if (p->h_inc_size[i] == 1) e1[p->inc_bodies[i][0]] = e[i] - e_ref;
    for (int i = 0; i < n12; ++i)
      if (p->h_inc_size[i] == 2) {
        const int a = p->inc_bodies[i][0], b = p->inc_bodies[i][1];
        const double eps = (e[i] - e_ref) - e1[a] - e1[b];
        link[(size_t)a * nb + b] = link[(size_t)b * nb + a] = std::fabs(eps) >= threshold;
      }
    // kept: one or two bodies, or a connected graph of bodies
    p->keep.assign(n_inc, 1);
    for (int i = n12; i < n_inc; ++i) {
      const std::vector<int>& S = p->inc_bodies[i];
      std::vector<uint8_t> seen(S.size(), 0);
      std::vector<int> todo(1, 0);
      seen[0] = 1;
      int reached = 1;
      while (!todo.empty()) {
        const int a = todo.back();
        todo.pop_back();
        for (size_t b = 0; b < S.size(); ++b)
          if (!seen[b] && link[(size_t)S[a] * nb + S[b]]) {
            seen[b] = 1;
            ++reached;
            todo.push_back((int)b);
          }
      }
      p->keep[i] = reached == (int)S.size();
    }
    // each kept increment's coefficient in the screened sum: eps_S written
    // as a combination of E_c(T) over the kept T (recursion of eqs. 2-5 with
    // the dropped increments at zero), summed over S
    std::vector<std::vector<std::pair<int, double>>> coef(n_inc);
    std::vector<double> dense(n_inc, 0.0);
    std::vector<uint8_t> mark(n_inc, 0);
    for (int i = 0; i < n_inc; ++i) {
      if (!p->keep[i]) continue;
      std::vector<int> touched(1, i);
      dense[i] = 1.0;
      mark[i] = 1;
      for (int t = p->h_sub_ptr[i]; t < p->h_sub_ptr[i + 1]; ++t) {
        const int T = p->h_sub_idx[t];
        if (T == i || !p->keep[T]) continue;
        for (const auto& uv : coef[T]) {
          if (!mark[uv.first]) {
            mark[uv.first] = 1;
            touched.push_back(uv.first);
          }
          dense[uv.first] -= uv.second;
        }
      }
      for (int u : touched) {
        if (dense[u] != 0.0) coef[i].push_back({u, dense[u]});
        dense[u] = 0.0;
        mark[u] = 0;
      }
    }
    std::fill(w.begin(), w.end(), 0.0);
    for (int i = 0; i < n_inc; ++i)
      for (const auto& uv : coef[i]) w[uv.first] += uv.second;
    free_one(p->d_keep);
    HIP_TRY(upload(&p->d_keep, p->keep), "ifci_screen");
  }
  p->h_w_inc = w;
  HIP_TRY(hipMemcpyAsync(p->d_w_inc, p->h_w_inc.data(), sizeof(double) * n_inc, hipMemcpyHostToDevice, st),
          "ifci_screen");
  HIP_TRY(hipStreamSynchronize(st), "ifci_screen");
  int64_t kept = 0;
  for (int i = 0; i < n_inc; ++i) {
    const uint8_t k = p->keep.empty() ? 1 : p->keep[i];
    kept += k;
    if (keep) keep[i] = k;
  }
  if (n_kept) *n_kept = kept;
  return IFCI_OK;
}

namespace {
// Every non-decreasing label sequence of length 1 .. order over n_groups
// labels, by length, then lexicographically.
std::vector<std::vector<int>> label_combinations(int n_groups, int order) {
  std::vector<std::vector<int>> out;
  for (int k = 1; k <= order; ++k) {
    std::vector<int> c(k, 0);
    while (true) {
      out.push_back(c);
      int j = k - 1;
      while (j >= 0 && c[j] == n_groups - 1) --j;
      if (j < 0) break;
      ++c[j];
      for (int l = j + 1; l < k; ++l) c[l] = c[j];
    }
  }
  return out;
}
}  // namespace

ifci_status ifci_group_count(ifci_plan_t p, int32_t n_groups, int64_t* n_combos) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (n_groups < 1 || n_groups > 64 || !n_combos) {
    set_error("ifci_group_count: n_groups 1..64 and an output");
    return IFCI_ERR_ARG;
  }
  // multisets of k labels from n_groups: C(n_groups + k - 1, k)
  int64_t n = 0;
  for (int k = 1; k <= p->order; ++k) {
    double c = 1.0;
    for (int j = 1; j <= k; ++j) c = c * (n_groups + k - j) / j;
    n += (int64_t)(c + 0.5);
  }
  *n_combos = n;
  return IFCI_OK;
}

ifci_status ifci_group_sums(ifci_plan_t p, const double* eps, const int32_t* group_of_body, int32_t n_groups,
                            double* sums, int32_t* combos, ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (!eps || !group_of_body || !sums || n_groups < 1 || n_groups > 64) {
    set_error("ifci_group_sums: null pointer or n_groups outside 1..64");
    return IFCI_ERR_ARG;
  }
  for (int b = 0; b < p->n_bodies; ++b)
    if (group_of_body[b] < 0 || group_of_body[b] >= n_groups) {
      set_error("ifci_group_sums: label of body " + std::to_string(b) + " out of range");
      return IFCI_ERR_ARG;
    }
  const int n_inc = (int)p->inc.size();
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> e(n_inc);
  HIP_TRY(hipMemcpyAsync(e.data(), eps, sizeof(double) * n_inc, hipMemcpyDeviceToHost, st), "ifci_group_sums");
  HIP_TRY(hipStreamSynchronize(st), "ifci_group_sums");
  const std::vector<std::vector<int>> all = label_combinations(n_groups, p->order);
  std::map<std::vector<int>, size_t> index;
  for (size_t c = 0; c < all.size(); ++c) index[all[c]] = c;
  std::vector<double> s(all.size(), 0.0), comp(all.size(), 0.0);
  for (int i = 0; i < n_inc; ++i) {
    std::vector<int> lab;
    for (int b : p->inc_bodies[i]) lab.push_back(group_of_body[b]);
    std::sort(lab.begin(), lab.end());
    const size_t c = index.at(lab);
    // Neumaier-compensated running sum
    const double x = e[i], t = s[c] + x;
    comp[c] += std::fabs(s[c]) >= std::fabs(x) ? (s[c] - t) + x : (x - t) + s[c];
    s[c] = t;
  }
  for (size_t c = 0; c < all.size(); ++c) {
    sums[c] = s[c] + comp[c];
    if (combos)
      for (int j = 0; j < p->order; ++j) combos[c * p->order + j] = j < (int)all[c].size() ? all[c][j] : -1;
  }
  return IFCI_OK;
}

ifci_status ifci_sno_orbitals(const double* gamma, int32_t n_orb, const int32_t* vir, int32_t n_vir,
                              const int32_t* inc_occ, int64_t n_inc, int32_t order, double eta, double* rot,
                              int32_t* n_keep, ifci_stream_t stream) {
  if (!gamma || !vir || !inc_occ || !rot || !n_keep || n_orb < 1 || n_orb > 64 || n_vir < 1 || n_vir > 16 ||
      n_inc < 1 || order < 1 || std::isnan(eta)) {
    set_error("ifci_sno_orbitals: null pointer, n_orb 1..64, n_vir 1..16, n_inc >= 1, order >= 1");
    return IFCI_ERR_ARG;
  }
  HIP_TRY(launch_sno_orbitals(gamma, n_orb, vir, n_vir, inc_occ, n_inc, order, std::pow(10.0, -eta), rot, n_keep,
                              (hipStream_t)stream),
          "ifci_sno_orbitals");
  return IFCI_OK;
}

ifci_status ifci_sno_transform(const double* h, const double* eri, int32_t n_orb, const int32_t* vir, int32_t n_vir,
                               const int32_t* col_orb, int32_t n_s, int32_t n_other, const double* rot,
                               int32_t n_keep, double* work, int64_t work_doubles, double* h_out, double* eri_out,
                               ifci_stream_t stream) {
  if (!h || !eri || !vir || !col_orb || !rot || !work || !h_out || !eri_out || n_orb < 1 || n_orb > 64 ||
      n_vir < 1 || n_vir > 16 || n_s < 1 || n_other < 0 || n_keep < 0 || n_keep > n_vir ||
      n_s + n_other + n_vir > n_orb) {
    set_error("ifci_sno_transform: null pointer or inconsistent sizes");
    return IFCI_ERR_ARG;
  }
  const int m = n_s + n_keep + n_other;
  const int64_t n3m = (int64_t)n_orb * n_orb * n_orb * m;
  if (work_doubles < (int64_t)n_orb * m + 2 * n3m) {
    set_error("ifci_sno_transform: work holds " + std::to_string(work_doubles) + " doubles, needs " +
              std::to_string((int64_t)n_orb * m + 2 * n3m));
    return IFCI_ERR_ARG;
  }
  double* C = work;
  double* b0 = work + (int64_t)n_orb * m;
  double* b1 = b0 + n3m;
  HIP_TRY(launch_sno_transform(h, eri, n_orb, vir, n_vir, col_orb, n_s, n_other, rot, n_keep, C, b0, b1, h_out,
                               eri_out, (hipStream_t)stream),
          "ifci_sno_transform");
  return IFCI_OK;
}

void ifci_hbci_default_options(ifci_hbci_options* o) {
  if (!o) return;
  o->eps1 = 1e-3;
  o->eps2 = 1e-6;
  o->max_iter = 32;
  o->max_dav = 200;
  o->m_max = 12;
  o->r_tol = 1e-6;
  o->max_det = (int64_t)1 << 20;
  o->max_nnz = (int64_t)1 << 28;
  o->max_ext = (int64_t)1 << 26;
}

ifci_status ifci_hbci_work_bytes(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, int64_t* bytes) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !o || !bytes || o->max_det < 2 || o->max_nnz < 1 ||
      o->max_ext < 1 || o->m_max < 2 || o->m_max > 16) {
    set_error("ifci_hbci_work_bytes: bad increment, options or pointer");
    return IFCI_ERR_ARG;
  }
  *bytes = hbci_work_bytes(p->inc[inc].k, *o);
  return IFCI_OK;
}

ifci_status ifci_hbci_solve(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, void* work, int64_t work_bytes,
                            double* result, uint64_t* dets_out, double* c_out, ifci_stream_t stream) {
  HbciInc I;
  ifci_status s = hbci_setup(p, inc, o, work, work_bytes, &I);
  if (s != IFCI_OK) return s;
  if (!result) {
    set_error("ifci_hbci_solve: null result");
    return IFCI_ERR_ARG;
  }
  DeviceGuard g(p->device);
  return hbci_solve(I, *o, work, result, dets_out, c_out, (hipStream_t)stream);
}

ifci_status ifci_hbci_solve_range(ifci_plan_t p, int64_t first, int64_t count, const ifci_hbci_options* o,
                                  void* const* works, int64_t work_bytes, int32_t n_workers, double* results) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (first < 0 || count < 0 || first + count > (int64_t)p->inc.size() || !o || !works || !results ||
      n_workers < 1 || n_workers > 64) {
    set_error("ifci_hbci_solve_range: bad range, null pointer or n_workers outside 1..64");
    return IFCI_ERR_ARG;
  }
  for (int w = 0; w < n_workers; ++w) {
    HbciInc I;
    for (int64_t i = first; i < first + count; ++i) {
      ifci_status s = hbci_setup(p, i, o, works[w], work_bytes, &I);
      if (s != IFCI_OK) return s;
    }
  }
  if (count == 0) return IFCI_OK;
  // largest first, so that the last increments to start are short
  std::vector<int64_t> order(count);
  for (int64_t j = 0; j < count; ++j) order[j] = first + j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return p->inc[a].n_det > p->inc[b].n_det; });
  std::atomic<int64_t> next(0);
  std::mutex mu;
  ifci_status first_status = IFCI_OK;
  std::string first_msg;
  std::vector<std::thread> pool;
  pool.reserve(n_workers);
  for (int w = 0; w < n_workers; ++w)
    pool.emplace_back([&, w] {
      ifci_status s = IFCI_OK;
      hipStream_t st = nullptr;
      if (hipSetDevice(p->device) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
        set_error("ifci_hbci_solve_range: no stream for a worker");
        s = IFCI_ERR_DEVICE;
      }
      while (s == IFCI_OK) {
        const int64_t j = next.fetch_add(1);
        if (j >= count) break;
        const int64_t i = order[j];
        HbciInc I;
        s = hbci_setup(p, i, o, works[w], work_bytes, &I);
        if (s == IFCI_OK) s = hbci_solve(I, *o, works[w], results + (i - first) * 8, nullptr, nullptr, st);
      }
      if (st) (void)hipStreamDestroy(st);
      if (s != IFCI_OK) {
        std::lock_guard<std::mutex> lk(mu);
        if (first_status == IFCI_OK) {
          first_status = s;
          first_msg = ifci_last_error();
        }
        next.store(count);
      }
    });
  for (std::thread& t : pool) t.join();
  if (first_status != IFCI_OK) set_error(first_msg);
  return first_status;
}

ifci_status ifci_hbci_sigma(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, void* work, int64_t work_bytes,
                            const uint64_t* dets, int64_t n, const double* c, double* sigma, ifci_stream_t stream) {
  HbciInc I;
  ifci_status s = hbci_setup(p, inc, o, work, work_bytes, &I);
  if (s != IFCI_OK) return s;
  if ((s = hbci_space_args(o, dets, n, c)) != IFCI_OK) return s;
  if (!sigma || sigma == c) {
    set_error("ifci_hbci_sigma: sigma must be non-null and distinct from c");
    return IFCI_ERR_ARG;
  }
  DeviceGuard g(p->device);
  return hbci_sigma(I, *o, work, dets, n, c, sigma, (hipStream_t)stream);
}

ifci_status ifci_hbci_select(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, void* work, int64_t work_bytes,
                             const uint64_t* dets, int64_t n, const double* c, double eps1, uint64_t* added,
                             int64_t* n_added, ifci_stream_t stream) {
  HbciInc I;
  ifci_status s = hbci_setup(p, inc, o, work, work_bytes, &I);
  if (s != IFCI_OK) return s;
  if ((s = hbci_space_args(o, dets, n, c)) != IFCI_OK) return s;
  if (!added || !n_added || !(eps1 >= 0.0)) {
    set_error("ifci_hbci_select: null output or eps1 < 0");
    return IFCI_ERR_ARG;
  }
  DeviceGuard g(p->device);
  return hbci_select(I, *o, work, dets, n, c, eps1, added, n_added, (hipStream_t)stream);
}

ifci_status ifci_hbci_pt2(ifci_plan_t p, int64_t inc, const ifci_hbci_options* o, void* work, int64_t work_bytes,
                          const uint64_t* dets, int64_t n, const double* c, double e_var, double eps2, double* e_pt2,
                          int64_t* n_ext, ifci_stream_t stream) {
  HbciInc I;
  ifci_status s = hbci_setup(p, inc, o, work, work_bytes, &I);
  if (s != IFCI_OK) return s;
  if ((s = hbci_space_args(o, dets, n, c)) != IFCI_OK) return s;
  if (!e_pt2 || !n_ext || !(eps2 >= 0.0) || !std::isfinite(e_var)) {
    set_error("ifci_hbci_pt2: null output, eps2 < 0 or e_var not finite");
    return IFCI_ERR_ARG;
  }
  DeviceGuard g(p->device);
  return hbci_pt2(I, *o, work, dets, n, c, e_var, eps2, e_pt2, n_ext, (hipStream_t)stream);
}

ifci_status ifci_vector(ifci_plan_t p, int64_t inc, double* c_out, ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (inc < 0 || inc >= (int64_t)p->inc.size() || !c_out) {
    set_error("ifci_vector: bad increment or pointer");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  if (!p->solved[inc]) {
    set_error("ifci_vector: increment not solved yet");
    return IFCI_ERR_STATE;
  }
  DeviceGuard g(p->device);
  const IncDev& d = p->inc[inc];
  const double* X = p->ws_dav() + d.vec_off + 2 * (int64_t)d.mspace * d.stride + d.stride;
  HIP_TRY(launch_expand(d, X, c_out, (hipStream_t)stream), "ifci_vector");
  return IFCI_OK;
}

ifci_status ifci_energy(ifci_plan_t p, const double* e_inc, const int32_t* status, double* eps, double* out,
                        ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (!e_inc || !out) {
    set_error("ifci_energy: null pointer");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  double* misc = p->ws_misc();
  double* dout = misc + 8;
  int32_t* bad = (int32_t*)(misc + 200);
  if (p->keep.empty())
    HIP_TRY(launch_energy(e_inc, status, p->d_sub_ptr, p->d_sub_idx, p->d_inc_size, (int)p->inc.size(), p->order,
                          misc, eps ? eps : p->ws_eps(), dout, bad, st),
            "ifci_energy");
  else
    HIP_TRY(launch_energy_screened(e_inc, status, p->d_sub_ptr, p->d_sub_idx, p->d_inc_size, p->d_keep,
                                   (int)p->inc.size(), p->order, misc, eps ? eps : p->ws_eps(), dout, bad, st),
            "ifci_energy");
  int32_t nbad = 0;
  HIP_TRY(hipMemcpyAsync(out, dout, sizeof(double) * (p->order + 2), hipMemcpyDeviceToHost, st), "ifci_energy");
  HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st), "ifci_energy");
  HIP_TRY(hipStreamSynchronize(st), "ifci_energy");
  if (status && nbad > 0) {
    set_error("ifci_energy: " + std::to_string(nbad) + " increments not converged");
    return IFCI_ERR_NOT_CONVERGED;
  }
  return IFCI_OK;
}

ifci_status ifci_rdm(ifci_plan_t p, const double* weights, double* dE_dh, double* dE_deri, ifci_stream_t stream) {
  if (check_plan(p) != IFCI_OK) return IFCI_ERR_ARG;
  if (!dE_dh) {
    set_error("ifci_rdm: null dE_dh");
    return IFCI_ERR_ARG;
  }
  ifci_status s = need_ints(p);
  if (s != IFCI_OK) return s;
  for (size_t i = 0; i < p->solved.size(); ++i)
    if (!p->solved[i] && (p->keep.empty() || p->keep[i])) {
      set_error("ifci_rdm: every increment must be solved first (ifci_davidson)");
      return IFCI_ERR_STATE;
    }
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_rdm(p->d_inc, p->inc.data(), (int)p->inc.size(), p->ws_dav(), p->d_tables, p->ws_rdm(),
                     p->d_rdm_off, p->opt.max_space, p->keep.empty() ? nullptr : p->d_keep, st),
          "ifci_rdm");
  HIP_TRY(launch_rdm_accumulate(p->d_inc, (int)p->inc.size(), p->d_orbs, (const int32_t*)p->d_loc, p->ws_rdm(),
                                p->d_rdm_off, weights ? weights : p->d_w_inc, p->d_orbs + p->ref_off,
                                (int)p->ref_occ.size(), p->n_orb, dE_dh, dE_deri, st),
          "ifci_rdm accumulate");
  return IFCI_OK;
}

}  // extern "C"
