// Host-side plan: problem validation, increment enumeration, string tables,
// workspace layout.  Internal to libifci.
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "ifci_internal.h"

struct ifci_plan_s {
  int device = 0;
  // problem
  int n_orb = 0;
  int n_bodies = 0;
  int order = 0;
  double e_const = 0.0;
  std::vector<std::vector<int>> bodies;
  std::vector<int> nocc;
  ifci_options opt{};
  ifci::Tuning tune;  // per-shape settings of the on-chip solvers (ifci_set_tuning)
  // increments
  std::vector<std::vector<int>> inc_bodies;
  std::vector<ifci::IncDev> inc;
  std::vector<int32_t> orbs;    // orbital blob
  std::vector<int32_t> tables;  // table blob
  std::vector<double> weights;  // w_k, k = 1..order
  std::vector<int> ref_occ;     // reference-occupied orbitals (sorted)
  // sizes
  int64_t ints_doubles = 0, dav_doubles = 0;
  int64_t max_ndet = 0, max_npair = 0, max_stride = 0;
  int64_t rdm_doubles = 0;
  std::vector<int64_t> rdm_off;  // per increment: active gamma (k^2) then Gamma (k^4)
  // workspace regions (byte offsets)
  int64_t off_ints = 0, off_dav = 0, off_E = 0, off_tmp = 0, off_part = 0, off_state = 0,
          off_rdm = 0, off_misc = 0, off_eps = 0, ws_bytes = 0;
  int64_t E_doubles = 0, tmp_doubles = 0, part_doubles = 0;
  // concurrent device-wide solves: each slot has its own E, tmp, part and
  // state scratch and (created on first use) its own stream and event
  int n_slots = 1;
  std::vector<hipStream_t> slot_streams;
  std::vector<hipEvent_t> slot_events;
  hipEvent_t fork_event = nullptr;
  // batched device-wide solver: region of wide_cap slots, control block,
  // and what the calls in flight keep alive (host copies of uploaded
  // arrays, graphs) until their work has run
  int64_t off_wide = 0, off_wide_ctl = 0, wide_slot_doubles = 0;
  int wide_cap = 0;
  hipStream_t capture_stream = nullptr;
  int32_t* pinned = nullptr;  // 2 ints of host memory the live counts are copied to
  hipEvent_t poll_event[2] = {nullptr, nullptr};
  struct InFlight {
    hipEvent_t done = nullptr;
    std::vector<hipGraphExec_t> graphs;
    std::vector<std::vector<char>> host;
  };
  std::vector<InFlight> in_flight;
  char* group_ctl = nullptr;  // control block of solves across several plans (grown on demand)
  int64_t group_ctl_bytes = 0;
  // device
  ifci::IncDev* d_inc = nullptr;
  int32_t* d_orbs = nullptr;
  int32_t* d_tables = nullptr;
  int32_t* d_order = nullptr;  // increments of the current batch, heaviest first
  std::vector<int32_t> order_all;
  std::vector<int32_t> order_batch;  // host copy kept alive for async uploads
  std::vector<uint8_t> batched_ok;   // increment fits the on-chip solver
  int32_t* d_sub_ptr = nullptr;      // energy assembly: subsets of each increment
  int32_t* d_sub_idx = nullptr;
  int32_t* d_inc_size = nullptr;
  int64_t* d_rdm_off = nullptr;
  int8_t* d_loc = nullptr;           // [n_inc + 1][n_orb] orbital roles
  double* d_w_inc = nullptr;         // expansion weight of every increment
  bool on_device = false;
  int64_t* phase_counters = nullptr;  // tracing: per-increment phase clocks
  std::vector<int32_t> h_sub_ptr, h_sub_idx, h_inc_size;
  // connected n-body screening (ifci_screen): mask (empty: none) and its
  // device copy
  std::vector<uint8_t> keep;
  uint8_t* d_keep = nullptr;
  std::vector<int8_t> h_loc;
  std::vector<double> h_w_inc;
  int64_t ref_off = 0;               // reference-occupied orbitals in the orbital blob
  char* ws = nullptr;
  const double* h = nullptr;
  const double* eri = nullptr;
  bool integrals_set = false;
  bool vectors_ready = false;
  std::vector<uint8_t> solved;  // host mirror: which increments have a vector

  double* ws_ints() const { return (double*)(ws + off_ints); }
  double* ws_dav() const { return (double*)(ws + off_dav); }
  double* ws_E(int slot = 0) const { return (double*)(ws + off_E) + (int64_t)slot * E_doubles; }
  double* ws_tmp(int slot = 0) const { return (double*)(ws + off_tmp) + (int64_t)slot * tmp_doubles; }
  double* ws_part(int slot = 0) const { return (double*)(ws + off_part) + (int64_t)slot * part_doubles; }
  double* ws_state(int slot = 0) const { return (double*)(ws + off_state) + (int64_t)slot * 4096; }
  double* ws_rdm() const { return (double*)(ws + off_rdm); }
  double* ws_misc() const { return (double*)(ws + off_misc); }
  double* ws_eps() const { return (double*)(ws + off_eps); }
};

namespace ifci {

void set_error(const std::string& msg);

// Tables of one (k, na) space, appended to `blob`.  Returns offsets.
struct ShapeTables {
  int k, na, n_str, npair, n_link;
  int64_t str_off, pair_off, link_off, ord_off, pairT_off;
};
ShapeTables build_shape(int k, int na, std::vector<int32_t>& blob);
int64_t binom(int n, int k);
void fill_link_dump(int k, int na, int32_t* strings, int32_t* link);

}  // namespace ifci

ifci_status plan_build(ifci_plan_s* P, const ifci_problem* pr, const ifci_options* op);

namespace ifci {
// bytes of slots the batched device-wide solver may take in a workspace
constexpr int64_t kWideBudget = (int64_t)32 << 30;
// doubles of one slot of that solver for increment d: preconditioned
// residual, string energies, partial sums, state, sigma scratch
int64_t wide_slot_doubles(const IncDev& d);
struct WideSlot {
  int64_t T, F, part, state, sc;
};
WideSlot wide_slot(const IncDev& d);
int64_t wide_ctl_bytes(int cap);
}  // namespace ifci
