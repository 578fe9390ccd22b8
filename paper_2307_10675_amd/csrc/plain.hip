// Device-wide sigma and a host-driven Davidson for one increment of any
// supported size (up to 16 active orbitals): sigma of arbitrary
// (non-symmetric) vectors, the symmetric-sector sigma of one increment, and
// the unfused per-increment path (one launch per step, the host reading the
// solver state every iteration) that the batched solvers are compared with.
// The kernel bodies live in sigma_wide.hpp and davidson_ops.hpp.
#include <map>
#include <mutex>
#include <set>
#include <utility>

#include "davidson_ops.hpp"
#include "device_common.hpp"
#include "sigma_wide.hpp"
#include "launch.hpp"

namespace ifci {

__global__ void __launch_bounds__(256) sym_combine_kernel(IncDev d, const double* __restrict__ Sm,
                                                          double* __restrict__ sig) {
  sym_combine_body(d, Sm, sig, blockIdx.x, gridDim.x);
}

bool sigma_column_supported(const IncDev& d) {
  return d.na * 2 == d.k && (d.k == 10 || d.k == 12 || d.k == 14 || d.k == 16);
}

// Workspace doubles of the column path (full C of either precision, S, the
// fragment image, with 256-byte alignment of each).
int64_t sigma_column_ws_doubles(const IncDev& d) {
  const int64_t n = d.n_str;
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  const int64_t np = (int64_t)d.k * (d.k + 1) / 2, mt = (np + 15) / 16, ks = (np + 3) / 4;
  return up((n + 1) * n + 16) + up(n * n) + up(mt * (ks + 1) * 64) + 64;
}

template <typename T, int K>
static hipError_t launch_column_k(const IncDev& d, const double* V, const int32_t* ptab, const int16_t* ptabT,
                                  const double* c, double* sig, double* ws, double shift, hipStream_t st) {
  typedef ColShape<T, K> SH;
  static_assert(SH::lds <= kMaxLds, "column sigma LDS");
  const int n = d.n_str;
  // workspace (256-byte aligned): full C, then S, then the fragment image,
  // each starting on a 256-byte boundary
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  T* cf = (T*)ws;
  const int64_t cf_elems = (int64_t)(n + 1) * n + 16;
  const int64_t off_s = up((cf_elems * (int64_t)sizeof(T) + 7) / 8);
  double* Sm = ws + off_s;
  T* vfg = (T*)(ws + up(off_s + (int64_t)n * n));
  const int nfrag = (int)(SH::vf_bytes / sizeof(T));
  hipLaunchKernelGGL((col_frag_kernel<T, K>), dim3((nfrag + 255) / 256), dim3(256), 0, st, V, shift, 2.0 * d.na,
                     vfg);
  hipLaunchKernelGGL((expand_sym_kernel<T>), dim3(2048), dim3(256), 0, st, d, c, cf);
  hipLaunchKernelGGL((sigma_column_kernel<T, K>), dim3(n), dim3(col_threads<T>()), (unsigned)SH::lds, st, d, V, ptab,
                     ptabT, (const T*)cf, (const T*)vfg, Sm);
  hipLaunchKernelGGL(sym_combine_kernel, dim3(4096), dim3(256), 0, st, d, Sm, sig);
  return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch_column_split(const IncDev& d, const double* V, const int32_t* ptab, const int16_t* ptabT,
                                      const double* c, double* sig, double* ws, double shift, hipStream_t st) {
  typedef ColSplit<T, K> SH;
  const int n = d.n_str;
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  T* cf = (T*)ws;
  const int64_t cf_elems = (int64_t)(n + 1) * n + 16;
  const int64_t off_s = up((cf_elems * (int64_t)sizeof(T) + 7) / 8);
  double* Sm = ws + off_s;
  T* vfg = (T*)(ws + up(off_s + (int64_t)n * n));
  const int nfrag = (int)((int64_t)SH::MT * SH::KSP * 64);
  hipLaunchKernelGGL((col_frag_kernel<T, K>), dim3((nfrag + 255) / 256), dim3(256), 0, st, V, shift, 2.0 * d.na,
                     vfg);
  hipLaunchKernelGGL((expand_sym_kernel<T>), dim3(4096), dim3(256), 0, st, d, c, cf);
  hipLaunchKernelGGL((sigma_column_split_kernel<T, K>), dim3(n), dim3(split_threads<T>()), (unsigned)SH::lds, st, d,
                     ptab, ptabT, (const T*)cf, (const T*)vfg, Sm);
  hipLaunchKernelGGL(sym_combine_kernel, dim3(4096), dim3(256), 0, st, d, Sm, sig);
  return hipGetLastError();
}

hipError_t allow_max_lds(const void* fn) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count({fn, dev})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
  if (e == hipSuccess) done.insert({fn, dev});
  return e;
}

// Set-up of the column kernels on the current device (their LDS exceeds the
// default limit); safe to call from several host threads.
hipError_t prepare_sigma_wide() {
  const void* fns[] = {(const void*)sigma_column_kernel<float, 10>, (const void*)sigma_column_kernel<double, 10>,
                       (const void*)sigma_column_kernel<float, 12>, (const void*)sigma_column_kernel<double, 12>,
                       (const void*)sigma_column_kernel<float, 14>, (const void*)sigma_column_kernel<double, 14>,
                       (const void*)sigma_column_split_kernel<float, 16>,
                       (const void*)sigma_column_split_kernel<double, 16>};
  for (const void* f : fns) {
    const hipError_t e = allow_max_lds(f);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t launch_sigma_column(const IncDev& d, const double* V, const int32_t* ptab, const int16_t* ptabT,
                                      const double* c, double* sig, double* ws, int precision, double shift,
                                      hipStream_t st) {
  if (prepare_sigma_wide() != hipSuccess) return hipErrorInvalidValue;
  const bool f32 = precision == IFCI_MIXED;
  switch (d.k) {
    case 10: return f32 ? launch_column_k<float, 10>(d, V, ptab, ptabT, c, sig, ws, shift, st)
                        : launch_column_k<double, 10>(d, V, ptab, ptabT, c, sig, ws, shift, st);
    case 12: return f32 ? launch_column_k<float, 12>(d, V, ptab, ptabT, c, sig, ws, shift, st)
                        : launch_column_k<double, 12>(d, V, ptab, ptabT, c, sig, ws, shift, st);
    case 14: return f32 ? launch_column_k<float, 14>(d, V, ptab, ptabT, c, sig, ws, shift, st)
                        : launch_column_k<double, 14>(d, V, ptab, ptabT, c, sig, ws, shift, st);
    case 16: return f32 ? launch_column_split<float, 16>(d, V, ptab, ptabT, c, sig, ws, shift, st)
                        : launch_column_split<double, 16>(d, V, ptab, ptabT, c, sig, ws, shift, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- static scratch
// E of the general product for callers that cannot allocate
// (ifci_sigma_noalloc): a fixed array of kStaticScratchDoubles doubles on
// every device the library runs on, held until the process ends.  Host code
// never uses the array's name as an address: it uses the device address
// hipGetSymbolAddress gives for the current device, looked up once per
// device.  Every call on a device shares that device's array.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double** out) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, p).first;
  }
  if (out) *out = it->second;
  return hipSuccess;
}

hipError_t launch_sigma_wide(const IncDev& d, const IncDev*, int, const double* ints, const int32_t* tables,
                             const double* c, double* sig, double* E, int precision, int mode, double shift,
                             hipStream_t st) {
  const double* V = ints + d.int_off + int_block(d.k).V;
  const int32_t* ptab = tables + d.pair_off;
  const int32_t* links = tables + d.link_off;
  if (mode == 1 && sigma_column_supported(d))
    return launch_sigma_column(d, V, ptab, (const int16_t*)(tables + d.pairT_off), c, sig, E, precision, shift, st);
  const int64_t tiles = (d.n_det + 63) / 64;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g1((unsigned)tiles), blk(kWideThreads);
  const int64_t nout = mode == 0 ? d.n_det : d.n_sym;
  const dim3 g2((unsigned)((nout + kWideThreads - 1) / kWideThreads));
  if (precision == IFCI_MIXED) {
    float* Ef = (float*)E;
    if (mode == 0) {
      hipLaunchKernelGGL((contract_kernel<float, 0>), g1, blk, 0, st, d, V, ptab, c, Ef, shift);
      hipLaunchKernelGGL((gather_full_kernel<float>), g2, blk, 0, st, d, links, Ef, sig);
    } else {
      hipLaunchKernelGGL((contract_kernel<float, 1>), g1, blk, 0, st, d, V, ptab, c, Ef, shift);
      hipLaunchKernelGGL((gather_sym_kernel<float>), g2, blk, 0, st, d, links, Ef, sig);
    }
  } else {
    if (mode == 0) {
      hipLaunchKernelGGL((contract_kernel<double, 0>), g1, blk, 0, st, d, V, ptab, c, E, shift);
      hipLaunchKernelGGL((gather_full_kernel<double>), g2, blk, 0, st, d, links, E, sig);
    } else {
      hipLaunchKernelGGL((contract_kernel<double, 1>), g1, blk, 0, st, d, V, ptab, c, E, shift);
      hipLaunchKernelGGL((gather_sym_kernel<double>), g2, blk, 0, st, d, links, E, sig);
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ Davidson
// The per-increment loop: the steps of davidson_ops.hpp, one launch each,
// with the host reading the state after the residual test.

__global__ void string_energy_kernel(IncDev d, const int32_t* __restrict__ strs, const double* __restrict__ B,
                                     double* __restrict__ F) {
  string_energy_body(d, strs, B, F, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) hdiag_kernel(IncDev d, const int32_t* __restrict__ strs,
                                                    const double* __restrict__ B, const double* __restrict__ F,
                                                    double* __restrict__ HD, double* part) {
  hdiag_body(d, strs, B, F, HD, nullptr, part + 2 * blockIdx.x, blockIdx.x, gridDim.x);
}

__global__ void init_state_kernel(DavState* S, const double* part, int nblk, double* V0, int64_t ns,
                                  double ecore, int phase) {
  __shared__ int64_t g;
  __shared__ double e0;
  if (threadIdx.x == 0) {
    double b = part[0];
    double ix = part[1];
    for (int i = 1; i < nblk; ++i)
      if (part[2 * i] < b || (part[2 * i] == b && part[2 * i + 1] < ix)) b = part[2 * i], ix = part[2 * i + 1];
    g = (int64_t)ix;
    e0 = b;
    S->E0 = b;
    S->guess = (int)ix;
    S->m = 0;
    S->phase = phase;
    S->iters = 0;
    S->status = IFCI_INC_NOT_CONVERGED;
    S->action = 0;
    S->ecore = ecore;
    S->keep = 0;
    S->theta = 0.0;
    S->resid = 1e300;
  }
  for (int i = threadIdx.x; i < 256; i += blockDim.x) S->G[i] = 0.0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) V0[i] = (i == g) ? 1.0 : 0.0;
  (void)e0;
}

__global__ void __launch_bounds__(256) dots_kernel(const double* __restrict__ Vb, int64_t st, int m,
                                                   const double* __restrict__ s, int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  op_dots(Vb, st, m, s, ns, part + blockIdx.x * kNV, blockIdx.x, gridDim.x, red);
}

__global__ void __launch_bounds__(64) small_G_kernel(DavState* S, const double* part, int nblk, int mmax) {
  __shared__ double g[kNV];
  small_G(S, part, nblk, mmax, g);
}

__global__ void __launch_bounds__(256) passA_kernel(const DavState* __restrict__ S, double* Vb, double* Sb,
                                                    int64_t st, const double* __restrict__ HD,
                                                    double* __restrict__ X, double* __restrict__ T,
                                                    int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double y[16];
  op_passA(S, Vb, Sb, st, HD, X, T, ns, part + blockIdx.x * kNV, blockIdx.x, gridDim.x, red, y);
}

__global__ void __launch_bounds__(64) small_A_kernel(DavState* S, const double* part, int nblk, double tol32,
                                                     double tol64, int max_iter, int evict) {
  __shared__ double v[kNV];
  small_A(S, part, nblk, tol32, tol64, max_iter, evict, v);
}

__global__ void __launch_bounds__(256) restart_kernel(const DavState* __restrict__ S, double* Vb, double* Sb,
                                                      int64_t st, int64_t ns) {
  __shared__ double q[kMaxSpace * kKeep];
  op_restart(S, Vb, Sb, st, ns, blockIdx.x, gridDim.x, q);
}

__global__ void small_R_kernel(DavState* S) { small_R(S); }

__global__ void __launch_bounds__(256) switch_kernel(DavState* S, double* Vb, const double* X, int64_t ns) {
  op_switch(S, Vb, X, ns, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) passB_kernel(const DavState* __restrict__ S, const double* __restrict__ Vb,
                                                    int64_t st, double* __restrict__ T, int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double cf[16];
  op_passB(S, Vb, st, T, ns, part + blockIdx.x * kNV, blockIdx.x, gridDim.x, red, cf);
}

__global__ void __launch_bounds__(64) small_B_kernel(DavState* S, const double* part, int nblk) {
  __shared__ double v[kNV];
  small_B(S, part, nblk, v);
}

__global__ void __launch_bounds__(256) passC_kernel(const DavState* __restrict__ S, const double* __restrict__ Vb,
                                                    int64_t st, double* __restrict__ T, int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double c2[16];
  if (!S->reorth) return;
  op_passC(S, Vb, st, T, ns, part + blockIdx.x * kNV, blockIdx.x, gridDim.x, red, c2);
}

__global__ void __launch_bounds__(64) small_C_kernel(DavState* S, const double* part, int nblk) {
  if (!S->reorth) return;
  __shared__ double v[kNV];
  small_C(S, part, nblk, v);
}

__global__ void __launch_bounds__(256) normalize_kernel(DavState* S, double* Vb, int64_t st,
                                                        const double* __restrict__ T, int64_t ns) {
  op_normalize(S, Vb, st, T, ns, blockIdx.x, gridDim.x);
}

__global__ void set_m_kernel(DavState* S) {
  if (threadIdx.x == 0) S->m = S->mb + 1;
}

__global__ void finish_kernel(const DavState* S, double e_const, double* e_out, int32_t* status_out,
                              int32_t* iters_out, double* resid_out) {
  if (threadIdx.x != 0) return;
  if (e_out) *e_out = S->theta + S->E0 + S->ecore + e_const;
  if (status_out) *status_out = S->status;
  if (iters_out) *iters_out = S->iters;
  if (resid_out) *resid_out = S->resid;
}

static inline unsigned nblocks(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > kPartBlocks) b = kPartBlocks;
  return (unsigned)b;
}

hipError_t run_plain(const PlainArgs& A, double* e_out, int32_t* status_out, int32_t* iters_out,
                     double* resid_out, hipStream_t st) {
  static_assert(sizeof(DavState) <= 4096 * 8, "state block too small");
  const IncDev& d = A.d;
  const int64_t ns = d.n_sym, sd = d.stride;
  const int mmax = A.max_space;
  double* Vb = A.dav;
  double* Sb = A.dav + mmax * sd;
  double* HD = A.dav + 2 * mmax * sd;
  double* X = HD + sd;
  double* T = A.tmp;
  double* F = A.tmp + sd;
  DavState* S = (DavState*)A.state;
  const double* B = A.ints + d.int_off;
  const int32_t* strs = A.tables + d.str_off;
  const unsigned nb = nblocks(ns, 256);
  hipError_t e;
  DavState hs;
  double ecore = 0.0;
  e = hipMemcpyAsync(&ecore, B + int_block(d.k).misc, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(string_energy_kernel, dim3((d.n_str + 255) / 256), dim3(256), 0, st, d, strs, B, F);
  hipLaunchKernelGGL(hdiag_kernel, dim3(nb), dim3(256), 0, st, d, strs, B, F, HD, A.part);
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(256), 0, st, S, A.part, (int)nb, Vb, ns, ecore,
                     A.precision == IFCI_MIXED ? 32 : 64);
  int m = 0, phase = A.precision == IFCI_MIXED ? 32 : 64;
  double shift = 0.0;
  if ((e = hipMemcpyAsync(&hs, S, sizeof(DavState), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  shift = hs.E0;
  while (true) {
    e = launch_sigma_wide(d, A.d_inc, A.inc, A.ints, A.tables, Vb + m * sd, Sb + m * sd, A.E,
                          phase == 32 ? IFCI_MIXED : IFCI_FP64, 1, shift, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(256), 0, st, Vb, sd, m, Sb + m * sd, ns, A.part);
    hipLaunchKernelGGL(small_G_kernel, dim3(1), dim3(64), 0, st, S, A.part, (int)nb, mmax);
    hipLaunchKernelGGL(passA_kernel, dim3(nb), dim3(256), 0, st, S, Vb, Sb, sd, HD, X, T, ns, A.part);
    hipLaunchKernelGGL(small_A_kernel, dim3(1), dim3(64), 0, st, S, A.part, (int)nb, A.r_tol_inner, A.r_tol,
                       A.max_iter, A.evict ? 1 : 0);
    if ((e = hipMemcpyAsync(&hs, S, sizeof(DavState), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (hs.action == 1 || hs.action == 3 || hs.action == 4) break;
    if (hs.action == 2) {
      hipLaunchKernelGGL(switch_kernel, dim3(nb), dim3(256), 0, st, S, Vb, X, ns);
      m = 0;
      phase = 64;
      continue;
    }
    if (hs.restart) {
      hipLaunchKernelGGL(restart_kernel, dim3(nb), dim3(256), 0, st, S, Vb, Sb, sd, ns);
      hipLaunchKernelGGL(small_R_kernel, dim3(1), dim3(64), 0, st, S);
      if ((e = hipMemcpyAsync(&hs, S, sizeof(DavState), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(passB_kernel, dim3(nb), dim3(256), 0, st, S, Vb, sd, T, ns, A.part);
    hipLaunchKernelGGL(small_B_kernel, dim3(1), dim3(64), 0, st, S, A.part, (int)nb);
    hipLaunchKernelGGL(passC_kernel, dim3(nb), dim3(256), 0, st, S, Vb, sd, T, ns, A.part);
    hipLaunchKernelGGL(small_C_kernel, dim3(1), dim3(64), 0, st, S, A.part, (int)nb);
    hipLaunchKernelGGL(normalize_kernel, dim3(nb), dim3(256), 0, st, S, Vb, sd, T, ns);
    hipLaunchKernelGGL(set_m_kernel, dim3(1), dim3(64), 0, st, S);
    m = hs.mb + 1;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, st, S, A.e_const, e_out, status_out, iters_out,
                     resid_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ vectors
__global__ void expand_kernel(IncDev d, const double* __restrict__ X, double* __restrict__ c) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n_det) return;
  const int n = d.n_str;
  const int a = (int)(j / n), b = (int)(j % n);
  const double v = X[packed(a, b)];
  c[j] = (a == b) ? v : v * kRSqrt2;
}

hipError_t launch_expand(const IncDev& d, const double* X, double* c, hipStream_t st) {
  hipLaunchKernelGGL(expand_kernel, dim3((unsigned)((d.n_det + 255) / 256)), dim3(256), 0, st, d, X, c);
  return hipGetLastError();
}

}  // namespace ifci
