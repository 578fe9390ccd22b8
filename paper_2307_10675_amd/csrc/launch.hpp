// Host-callable launchers of the libifci kernels.  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include "ifci_internal.h"

namespace ifci {

constexpr int kMaxLds = 163840;  // LDS per workgroup on gfx950

// Raise the dynamic-LDS limit of kernel `fn` to kMaxLds on the current
// device, once per (kernel, device); safe to call from several host threads.
hipError_t allow_max_lds(const void* fn);

hipError_t launch_embed(const IncDev* incs, int n_inc, const int32_t* orbs, const double* h,
                        const double* eri, int n, double* ints, const int32_t* ref_occ, int n_ref,
                        double e_const, double* misc, hipStream_t st);

int64_t batched_lds_bytes(int k, int n_str, int n_link);
int64_t batched_lds_want(int k, int n_str, int n_link);
hipError_t launch_batched(const SolveArgs& A, int lds_bytes, hipStream_t st);
hipError_t launch_sigma_one(const IncDev* incs, int inc, const double* ints, const int32_t* tables,
                            const double* c, double* sig, int precision, int lds_bytes,
                            hipStream_t st);

// Device-wide sigma for any increment.  mode 0: c and sigma full [n_det]
// vectors, any c (E materialised in the workspace).  mode 1: c and sigma
// packed scaled symmetric vectors; half-filled increments of 10, 12 or 14
// orbitals take the fused column kernel (sigma_column_supported), others the
// materialised E.
bool sigma_column_supported(const IncDev& d);
hipError_t prepare_sigma_wide();  // one-time kernel attributes, thread safe
int64_t sigma_column_ws_doubles(const IncDev& d);  // workspace of the column path
// The static scratch array (plain.hip): its device address on the current
// device (looked up once per device), kStaticScratchDoubles doubles.
constexpr int64_t kStaticScratchDoubles = (int64_t)4 << 20;  // 32 MiB
hipError_t static_scratch(double** out);
hipError_t launch_sigma_wide(const IncDev& d, const IncDev* d_inc_dev, int inc, const double* ints,
                             const int32_t* tables, const double* c, double* sig, double* E,
                             int precision, int mode, double shift, hipStream_t st);

// Host-driven Davidson over one increment with device-wide kernels.
struct PlainArgs {
  IncDev d;
  const IncDev* d_inc;
  int inc;
  const double* ints;
  const int32_t* tables;
  double* dav;     // Davidson block of this increment
  double* E;       // sigma scratch
  double* tmp;     // [>= 2 stride]
  double* part;    // partial sums
  double* state;   // device state block
  int precision, max_iter, max_space;
  double r_tol, r_tol_inner, e_const;
  bool evict;
};
hipError_t run_plain(const PlainArgs& A, double* e_out, int32_t* status_out, int32_t* iters_out,
                     double* resid_out, hipStream_t st);

hipError_t launch_expand(const IncDev& d, const double* X, double* c, hipStream_t st);

// ---------------------------------------------------------------- batched device-wide solver
// One increment of the batched device-wide Davidson (wide.hip).  Pointers
// are device addresses: the increment's integral block and tables, its
// Davidson block (basis, sigma, diagonal, Ritz vector), and its slot of the
// solver region (temporaries, partial sums, state, sigma scratch).
struct WideItem {
  IncDev d;
  const double* B;
  const int32_t* tabs;
  double* Vb;
  double* Sb;
  double* HD;
  double* X;
  double* T;
  double* F;
  double* part;
  double* state;          // a DavState
  double* sc;             // sigma scratch
  const uint8_t* evict;   // nonzero byte: stop after one iteration (EVICTED); may be null
  int32_t mmax;
  int32_t pad;
};

// One batch: n increments of one shape (d), their items (device array of
// pointers), a control block of wide_ctl_ints(n) ints (live counts and
// lists).
struct WideRun {
  WideItem* const* items;
  int n;
  int* ctl;
  IncDev d;
  int k;
  int precision, max_iter;
  double r_tol, r_tol_inner;
};
int64_t wide_sigma_scratch_doubles(const IncDev& d);
int64_t wide_part_doubles(const IncDev& d);
int wide_ctl_ints(int n);
hipError_t wide_prepare(int k);                          // kernel attributes (current device)
hipError_t wide_setup(const WideRun& R, hipStream_t s);      // diagonal, guess, state, fragments, lists
hipError_t wide_iteration(const WideRun& R, hipStream_t s);  // one iteration's launches (capturable)
hipError_t wide_finish(WideItem* const* items, int n, const int32_t* out_pos, double e_const, double* e_out,
                       int32_t* status_out, int32_t* iters_out, double* resid_out, hipStream_t s);

hipError_t launch_energy_screened(const double* e_inc, const int32_t* status, const int32_t* sub_ptr,
                                  const int32_t* sub_idx, const int32_t* inc_size, const uint8_t* keep, int n_inc,
                                  int order, const double* misc_in, double* eps, double* out, int32_t* bad,
                                  hipStream_t st);
hipError_t launch_mark_screened(const uint8_t* keep, int64_t first, int64_t count, double* e_out,
                                int32_t* status_out, int32_t* iters_out, double* resid_out, hipStream_t st);
hipError_t launch_sno_orbitals(const double* gamma, int n_orb, const int32_t* vir, int n_vir, const int32_t* inc_occ,
                               int64_t n_inc, int order, double thresh, double* rot, int32_t* n_keep,
                               hipStream_t st);
hipError_t launch_sno_transform(const double* h, const double* eri, int n_orb, const int32_t* vir, int n_vir,
                                const int32_t* col_orb, int n_s, int n_other, const double* rot, int n_keep,
                                double* C, double* buf0, double* buf1, double* h_out, double* eri_out,
                                hipStream_t st);
hipError_t launch_energy(const double* e_inc, const int32_t* status, const int32_t* sub_ptr,
                         const int32_t* sub_idx, const int32_t* inc_size, int n_inc, int order,
                         const double* misc_in, double* eps, double* out, int32_t* bad,
                         hipStream_t st);

hipError_t launch_rdm(const IncDev* incs, const IncDev* host_incs, int n_inc, const double* dav_base,
                      const int32_t* tables, double* rdm, const int64_t* rdm_off_dev, int mmax, const uint8_t* keep,
                      hipStream_t st);
hipError_t launch_rdm_accumulate(const IncDev* incs, int n_inc, const int32_t* orbs,
                                 const int32_t* loc, const double* rdm, const int64_t* rdm_off_dev,
                                 const double* w, const int32_t* ref_occ, int n_ref, int n,
                                 double* dh, double* deri, hipStream_t st);

// Heat-bath selected CI of one increment (hbci.hip).  The integrals are the
// full h and eri with the increment's sorted active and core orbital lists
// (device); ref is the reference determinant's key; e_core points at the
// increment's frozen-core energy on the device; e_const is the problem's
// constant.  Each call synchronises the stream.
struct HbciInc {
  const double* h;
  const double* eri;
  int n_orb;
  const int32_t* act;
  int k;
  const int32_t* core;
  int n_core;
  uint64_t ref;
  const double* e_core;
  double e_const;
};
int64_t hbci_work_bytes(int k, const ifci_hbci_options& o);
ifci_status hbci_solve(const HbciInc& I, const ifci_hbci_options& o, void* work, double* result, uint64_t* dets_out,
                       double* c_out, hipStream_t st);
ifci_status hbci_sigma(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                       const double* c, double* sigma, hipStream_t st);
ifci_status hbci_select(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                        const double* c, double eps1, uint64_t* added, int64_t* n_added, hipStream_t st);
ifci_status hbci_pt2(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                     const double* c, double e_var, double eps2, double* e_pt2, int64_t* n_ext, hipStream_t st);

}  // namespace ifci
