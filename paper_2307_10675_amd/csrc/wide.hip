// Batched device-wide Davidson: every increment too large for the on-chip
// solver (more than 8 active orbitals) runs in the same launches as every
// other increment of its shape, with the control of the iteration on the
// device.
//
// Each increment (an "item") keeps its solver state (DavState), its partial
// sums, temporaries and sigma scratch in device memory.  One iteration is a
// fixed list of launches; every kernel runs a fixed, persistent grid that
// strides over the work units (increment, block) of the increments still
// live, read from device-side lists that a compaction kernel rebuilds at the
// end of every iteration.  The decisions the per-increment loop takes on the
// host -- thick restart, the switch from the FP32 to the FP64 stage, the stop
// -- are flags in each state that the kernels of the next steps read.  So
// the launch list never changes, it can be captured once as a graph and
// replayed, and an iteration after every increment has stopped costs only
// the launches themselves.
//
// Steps and arithmetic are those of davidson_ops.hpp and sigma_wide.hpp
// (Davidson's method with a diagonal preconditioner and thick restart;
// Knowles-Handy sigma), as in the per-increment loop.
#include <hip/hip_runtime.h>

#include <vector>

#include "davidson_ops.hpp"
#include "device_common.hpp"
#include "launch.hpp"
#include "sigma_wide.hpp"

namespace ifci {

namespace {

constexpr int kVecThreads = 256;
constexpr int kVecGrid = 1024;    // persistent grid of the vector steps
constexpr int kSmallGrid = 512;   // persistent grid of the one-wave steps
constexpr int kCompactThreads = 1024;

__host__ __device__ inline int vec_blocks(int64_t ns) {
  const int64_t b = (ns + kVecThreads - 1) / kVecThreads;
  return (int)(b < 1 ? 1 : (b > kPartBlocks ? kPartBlocks : b));
}

// live lists in the control block: ctl[1 + which] is the count, the list
// starts at ctl + 8 + which * cap (which: 0 all, 1 FP32 stage, 2 FP64 stage)
__device__ __forceinline__ int live_count(const int* ctl, int which) { return ctl[1 + which]; }
__device__ __forceinline__ const int* live_list(const int* ctl, int cap, int which) { return ctl + 8 + which * cap; }

__device__ __forceinline__ DavState* st(const WideItem* w) { return (DavState*)w->state; }

// sigma scratch of a column-path item (doubles from w->sc): full C (T),
// S (FP64), FP32 fragment image, FP64 fragment image
struct ColScratch {
  int64_t cf, sm, vf32, vf64, total;
};
__host__ __device__ inline ColScratch col_scratch(const IncDev& d) {
  auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
  const int64_t n = d.n_str, np = (int64_t)d.k * (d.k + 1) / 2;
  const int64_t mt = (np + 15) / 16, ks = (np + 3) / 4, ks2 = (ks + 1) / 2;
  ColScratch c;
  c.cf = 0;
  c.sm = up((n + 1) * n + 16);
  c.vf32 = c.sm + up(n * n);
  c.vf64 = c.vf32 + up((mt * 2 * ks2 * 64 + 1) / 2);
  c.total = c.vf64 + up(mt * ks * 64);
  return c;
}

// ------------------------------------------------------------------ set-up
__global__ void __launch_bounds__(kVecThreads) wb_string_energy_kernel(WideItem* const* it, int n) {
  const int per = (it[0]->d.n_str + kVecThreads - 1) / kVecThreads;
  for (int u = blockIdx.x; u < n * per; u += gridDim.x) {
    const WideItem* w = it[u / per];
    string_energy_body(w->d, w->tabs + w->d.str_off, w->B, w->F, (u % per) * kVecThreads + threadIdx.x);
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_hdiag_kernel(WideItem* const* it, int n) {
  const int nb = vec_blocks(it[0]->d.n_sym);
  for (int u = blockIdx.x; u < n * nb; u += gridDim.x) {
    const WideItem* w = it[u / nb];
    const int blk = u % nb;
    hdiag_body(w->d, w->tabs + w->d.str_off, w->B, w->F, w->HD, w->Vb, w->part + 2 * blk, blk, nb);
  }
}

// Lowest diagonal entry (the guess) from the block partials, initial state,
// V0 = that unit vector (hdiag zeroed the rest).  One wave per increment.
__global__ void __launch_bounds__(64) wb_init_kernel(WideItem* const* it, int n, int precision) {
  for (int u = blockIdx.x; u < n; u += gridDim.x) {
    const WideItem* w = it[u];
    DavState* S = st(w);
    const int nb = vec_blocks(w->d.n_sym);
    const int lane = threadIdx.x;
    double best = 1e300, bi = 1e300;
    for (int b = lane; b < nb; b += 64) {
      const double v = w->part[2 * b], ix = w->part[2 * b + 1];
      if (v < best || (v == best && ix < bi)) best = v, bi = ix;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64), oi = __shfl_xor(bi, o, 64);
      if (ov < best || (ov == best && oi < bi)) best = ov, bi = oi;
    }
    for (int i = lane; i < 256; i += 64) S->G[i] = 0.0;
    if (lane == 0) {
      S->E0 = best;
      S->guess = (int)bi;
      S->m = 0;
      S->phase = precision == IFCI_MIXED ? 32 : 64;
      S->iters = 0;
      S->status = IFCI_INC_NOT_CONVERGED;
      S->action = kActContinue;
      S->ecore = w->B[int_block(w->d.k).misc];
      S->keep = 0;
      S->theta = 0.0;
      S->resid = 1e300;
      S->alive = 1;
      w->Vb[(int64_t)bi] = 1.0;
    }
    __syncthreads();
  }
}

// A-fragment images of V (with the diagonal-pair shift E0 of each
// increment) for the column sigma, built once per solve.
template <typename T, int K>
__global__ void __launch_bounds__(kVecThreads) wb_frag_kernel(WideItem* const* it, int n) {
  const int64_t np = (int64_t)K * (K + 1) / 2, mt = (np + 15) / 16, ks = (np + 3) / 4, ks2 = (ks + 1) / 2;
  const int nfrag = (int)(mt * (sizeof(T) == 4 ? 2 * ks2 : ks) * 64);
  const int per = (nfrag + kVecThreads - 1) / kVecThreads;
  for (int u = blockIdx.x; u < n * per; u += gridDim.x) {
    const WideItem* w = it[u / per];
    const ColScratch cs = col_scratch(w->d);
    T* vf = (T*)(w->sc + (sizeof(T) == 4 ? cs.vf32 : cs.vf64));
    const double* V = w->B + int_block(K).V;
    col_frag_body<T, K>(V, st(w)->E0, 2.0 * w->d.na, vf, (u % per) * kVecThreads + threadIdx.x);
  }
}

// Rebuild the live lists: an increment stops at the residual test's
// done / out-of-iterations / evicted; the others are listed by stage.
__global__ void __launch_bounds__(kCompactThreads) wb_compact_kernel(WideItem* const* it, int n, int* ctl, int cap) {
  __shared__ int wsum[3][kCompactThreads / 64];
  __shared__ int base[3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (threadIdx.x < 3) base[threadIdx.x] = 0;
  __syncthreads();
  int* lists[3] = {ctl + 8, ctl + 8 + cap, ctl + 8 + 2 * cap};
  for (int c0 = 0; c0 < n; c0 += blockDim.x) {
    const int j = c0 + threadIdx.x;
    int f[3] = {0, 0, 0};
    if (j < n) {
      DavState* S = st(it[j]);
      if (S->alive) {
        const int a = S->action;
        if (a == kActDone || a == kActMaxIter || a == kActEvicted) {
          S->alive = 0;
        } else {
          f[0] = 1;
          f[1] = S->phase == 32;
          f[2] = !f[1];
        }
      }
    }
    int pos[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint64_t m = __ballot(f[q]);
      pos[q] = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[q][wave] = __popcll(m);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      int off = base[q];
      for (int w2 = 0; w2 < wave; ++w2) off += wsum[q][w2];
      if (f[q]) lists[q][off + pos[q]] = j;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      int t = 0;
      for (int w2 = 0; w2 < nw; ++w2) t += wsum[threadIdx.x][w2];
      base[threadIdx.x] += t;
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) ctl[1 + threadIdx.x] = base[threadIdx.x];
}

// ------------------------------------------------------------------ sigma
template <typename T>
__global__ void __launch_bounds__(kVecThreads) wb_expand_kernel(WideItem* const* it, const int* ctl, int cap,
                                                                int which) {
  const int nl = live_count(ctl, which);
  const int* lst = live_list(ctl, cap, which);
  const int per = kVecGrid;  // blocks per increment, grid-strided inside over 32 x 32 tiles
  const int n = it[0]->d.n_str;
  const int64_t nb = (int64_t)((n + 32) / 32) * ((n + 31) / 32);
  const int units = nb < per ? (int)nb : per;
  for (int u = blockIdx.x; u < nl * units; u += gridDim.x) {
    const WideItem* w = it[lst[u / units]];
    const DavState* S = st(w);
    expand_sym_body<T>(w->d.n_str, w->Vb + (int64_t)S->m * w->d.stride, (T*)(w->sc + col_scratch(w->d).cf),
                       u % units, units);
  }
}

// Workgroup shape of the batched column kernel.  A 10-orbital column has 16
// tiles of 16 strings: 4 waves take them in 4 equal rounds (12 waves would
// leave 8 idle in the second), and 4 (FP32) or 3 (FP64) such workgroups share
// a CU; larger columns keep the 12 waves of the single-increment kernel.
template <typename T, int K>
constexpr int wide_col_threads() { return K <= 10 ? 256 : col_threads<T>(); }
template <typename T, int K>
constexpr int wide_col_waves() { return K <= 10 ? (sizeof(T) == 4 ? 4 : 3) : 3; }  // per SIMD

// Column sigma over (increment, beta string) units: each workgroup takes a
// contiguous range of units, so it reloads the fragment image only where its
// range crosses into the next increment.
template <typename T, int K>
__global__ void __launch_bounds__((wide_col_threads<T, K>()), (wide_col_waves<T, K>())) wb_column_kernel(WideItem* const* it, const int* ctl, int cap,
                                                                     int which) {
  extern __shared__ __align__(16) char lds[];
  const int nl = live_count(ctl, which);
  const int* lst = live_list(ctl, cap, which);
  const int n = it[0]->d.n_str;
  const int64_t W = (int64_t)nl * n;
  const int64_t lo = W * blockIdx.x / gridDim.x, hi = W * (blockIdx.x + 1) / gridDim.x;
  int prev = -1;
  for (int64_t u = lo; u < hi; ++u) {
    const int item = lst[u / n];
    const int b = (int)(u % n);
    const WideItem* w = it[item];
    const ColScratch cs = col_scratch(w->d);
    column_body<T, K>(w->tabs + w->d.pair_off, (const int16_t*)(w->tabs + w->d.pairT_off), (const T*)(w->sc + cs.cf),
                      (const T*)(w->sc + (sizeof(T) == 4 ? cs.vf32 : cs.vf64)), w->sc + cs.sm, b, lds,
                      item != prev);
    prev = item;
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(split_threads<T>()) wb_column_split_kernel(WideItem* const* it, const int* ctl,
                                                                             int cap, int which) {
  extern __shared__ __align__(16) char lds[];
  const int nl = live_count(ctl, which);
  const int* lst = live_list(ctl, cap, which);
  const int n = it[0]->d.n_str;
  const int64_t W = (int64_t)nl * n;
  const int64_t lo = W * blockIdx.x / gridDim.x, hi = W * (blockIdx.x + 1) / gridDim.x;
  for (int64_t u = lo; u < hi; ++u) {
    const WideItem* w = it[lst[u / n]];
    const ColScratch cs = col_scratch(w->d);
    column_split_body<T, K>(w->tabs + w->d.pair_off, (const int16_t*)(w->tabs + w->d.pairT_off),
                            (const T*)(w->sc + cs.cf), (const T*)(w->sc + (sizeof(T) == 4 ? cs.vf32 : cs.vf64)),
                            w->sc + cs.sm, (int)(u % n), lds);
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_combine_kernel(WideItem* const* it, const int* ctl, int cap) {
  const int nl = live_count(ctl, 0);
  const int* lst = live_list(ctl, cap, 0);
  const int64_t nt = sym_combine_tiles(it[0]->d.n_str);
  const int per = nt < kVecGrid ? (int)nt : kVecGrid;  // blocks per increment, grid-strided inside
  for (int64_t u = blockIdx.x; u < (int64_t)nl * per; u += gridDim.x) {
    const WideItem* w = it[lst[u / per]];
    const DavState* S = st(w);
    sym_combine_body(w->d, w->sc + col_scratch(w->d).sm, w->Sb + (int64_t)S->m * w->d.stride, u % per, per);
  }
}

// general product (E materialised per increment in its scratch)
template <typename T>
__global__ void __launch_bounds__(kWideThreads) wb_contract_kernel(WideItem* const* it, const int* ctl, int cap,
                                                                   int which) {
  const int nl = live_count(ctl, which);
  const int* lst = live_list(ctl, cap, which);
  const int64_t per = (it[0]->d.n_det + 63) / 64;
  for (int64_t u = blockIdx.x; u < (int64_t)nl * per; u += gridDim.x) {
    const WideItem* w = it[lst[u / per]];
    const DavState* S = st(w);
    contract_body<T, 1>(w->d, w->B + int_block(w->d.k).V, w->tabs + w->d.pair_off,
                        w->Vb + (int64_t)S->m * w->d.stride, (T*)w->sc, S->E0, u % per);
  }
}

template <typename T>
__global__ void __launch_bounds__(kWideThreads) wb_gather_kernel(WideItem* const* it, const int* ctl, int cap,
                                                                 int which) {
  const int nl = live_count(ctl, which);
  const int* lst = live_list(ctl, cap, which);
  const int64_t per = (it[0]->d.n_sym + kWideThreads - 1) / kWideThreads;
  for (int64_t u = blockIdx.x; u < (int64_t)nl * per; u += gridDim.x) {
    const WideItem* w = it[lst[u / per]];
    const DavState* S = st(w);
    gather_sym_body<T>(w->d, w->tabs + w->d.link_off, (const T*)w->sc, w->Sb + (int64_t)S->m * w->d.stride,
                       (u % per) * kWideThreads + threadIdx.x);
  }
}

// ------------------------------------------------------------------ vector and small steps
// Each takes the live increments, optionally only those whose state passes
// `want` (evaluated once per unit from the state, the same for every thread).
enum Want { kAll = 0, kCont, kContRestart, kContReorth, kSwitching };

__device__ __forceinline__ bool wanted(const DavState* S, int want) {
  switch (want) {
    case kCont: return S->action == kActContinue;
    case kContRestart: return S->action == kActContinue && S->restart;
    case kContReorth: return S->action == kActContinue && S->reorth;
    case kSwitching: return S->action == kActSwitch;
    default: return true;
  }
}

#define WB_VEC_LOOP(want)                                                  \
  const int nl = live_count(ctl, 0);                                       \
  const int* lst = live_list(ctl, cap, 0);                                 \
  const int nb = vec_blocks(it[0]->d.n_sym);                               \
  for (int u = blockIdx.x; u < nl * nb; u += gridDim.x) {                  \
    WideItem* w = it[lst[u / nb]];                                         \
    DavState* S = st(w);                                                   \
    const int blk = u % nb;                                                \
    if (!wanted(S, want)) continue;                                        \
    const int64_t sd = w->d.stride, ns = w->d.n_sym;                       \
    (void)sd;                                                              \
    (void)ns;

#define WB_SMALL_LOOP(want)                                                \
  const int nl = live_count(ctl, 0);                                       \
  const int* lst = live_list(ctl, cap, 0);                                 \
  const int nb = vec_blocks(it[0]->d.n_sym);                               \
  (void)nb;                                                                \
  for (int u = blockIdx.x; u < nl; u += gridDim.x) {                       \
    WideItem* w = it[lst[u]];                                              \
    DavState* S = st(w);                                                   \
    if (!wanted(S, want)) continue;

__global__ void __launch_bounds__(kVecThreads) wb_dots_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double red[4 * kNV];
  WB_VEC_LOOP(kAll)
  const int m = S->m;
  op_dots(w->Vb, sd, m, w->Sb + (int64_t)m * sd, ns, w->part + blk * kNV, blk, nb, red);
  }
}

__global__ void __launch_bounds__(64) wb_small_G_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double g[kNV];
  WB_SMALL_LOOP(kAll)
  small_G(S, w->part, nb, w->mmax, g);
  __syncthreads();
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_passA_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double red[4 * kNV];
  __shared__ double y[16];
  WB_VEC_LOOP(kAll)
  op_passA(S, w->Vb, w->Sb, sd, w->HD, w->X, w->T, ns, w->part + blk * kNV, blk, nb, red, y);
  }
}

__global__ void __launch_bounds__(64) wb_small_A_kernel(WideItem* const* it, const int* ctl, int cap, double tol32,
                                                        double tol64, int max_iter) {
  __shared__ double v[kNV];
  WB_SMALL_LOOP(kAll)
  small_A(S, w->part, nb, tol32, tol64, max_iter, w->evict ? (int)(*w->evict != 0) : 0, v);
  __syncthreads();
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_switch_kernel(WideItem* const* it, const int* ctl, int cap) {
  WB_VEC_LOOP(kSwitching)
  op_switch(S, w->Vb, w->X, ns, blk, nb);
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_restart_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double q[kMaxSpace * kKeep];
  WB_VEC_LOOP(kContRestart)
  op_restart(S, w->Vb, w->Sb, sd, ns, blk, nb, q);
  }
}

__global__ void __launch_bounds__(64) wb_small_R_kernel(WideItem* const* it, const int* ctl, int cap) {
  WB_SMALL_LOOP(kContRestart)
  small_R(S);
  __syncthreads();
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_passB_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double red[4 * kNV];
  __shared__ double cf[16];
  WB_VEC_LOOP(kCont)
  op_passB(S, w->Vb, sd, w->T, ns, w->part + blk * kNV, blk, nb, red, cf);
  }
}

__global__ void __launch_bounds__(64) wb_small_B_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double v[kNV];
  WB_SMALL_LOOP(kCont)
  small_B(S, w->part, nb, v);
  __syncthreads();
  }
}

__global__ void __launch_bounds__(kVecThreads) wb_passC_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double red[4 * kNV];
  __shared__ double c2[16];
  WB_VEC_LOOP(kContReorth)
  op_passC(S, w->Vb, sd, w->T, ns, w->part + blk * kNV, blk, nb, red, c2);
  }
}

__global__ void __launch_bounds__(64) wb_small_C_kernel(WideItem* const* it, const int* ctl, int cap) {
  __shared__ double v[kNV];
  WB_SMALL_LOOP(kContReorth)
  small_C(S, w->part, nb, v);
  __syncthreads();
  }
}

// V[mb + 1] <- t / ||t||; the first block also advances m (normalize reads
// only mb, so no block of the same launch reads m)
__global__ void __launch_bounds__(kVecThreads) wb_normalize_kernel(WideItem* const* it, const int* ctl, int cap) {
  WB_VEC_LOOP(kCont)
  op_normalize(S, w->Vb, sd, w->T, ns, blk, nb);
  if (blk == 0 && threadIdx.x == 0) S->m = S->mb + 1;
  }
}

// Outputs of items [0, n): position out_pos[j] of the caller's arrays.
__global__ void wb_finish_kernel(WideItem* const* it, int n, const int32_t* out_pos, double e_const, double* e_out,
                                 int32_t* status_out, int32_t* iters_out, double* resid_out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const DavState* S = st(it[j]);
    const int o = out_pos[j];
    e_out[o] = S->theta + S->E0 + S->ecore + e_const;
    status_out[o] = S->status;
    if (iters_out) iters_out[o] = S->iters;
    if (resid_out) resid_out[o] = S->resid;
  }
}

inline unsigned grid_for(int64_t units, int cap) {
  return (unsigned)(units < 1 ? 1 : (units > cap ? cap : units));
}

template <typename T, int K>
hipError_t column_sigma(const WideRun& R, int which, hipStream_t s) {
  const int n = R.n;
  hipLaunchKernelGGL((wb_expand_kernel<T>), dim3(kVecGrid), dim3(kVecThreads), 0, s, R.items, R.ctl, n, which);
  if constexpr (K <= 14) {
    typedef ColShape<T, K> SH;
    static_assert(SH::lds <= kMaxLds, "column sigma LDS");
    constexpr int kThreads = wide_col_threads<T, K>();
    // workgroups per CU: at 10 orbitals the resident count (by waves, 4 SIMDs
    // x waves each, and by LDS), else two where the LDS would hold two
    constexpr int by_waves = 4 * wide_col_waves<T, K>() / (kThreads / 64);
    constexpr int by_lds = (int)(kMaxLds / SH::lds);
    constexpr int per_cu = K <= 10 ? (by_waves < by_lds ? by_waves : by_lds) : (SH::lds <= kMaxLds / 2 ? 2 : 1);
    static_assert(per_cu >= 1, "column sigma residency");
    hipLaunchKernelGGL((wb_column_kernel<T, K>), dim3(256 * per_cu), dim3(kThreads), (unsigned)SH::lds, s, R.items,
                       R.ctl, n, which);
  } else {
    typedef ColSplit<T, K> SH;
    hipLaunchKernelGGL((wb_column_split_kernel<T, K>), dim3(256), dim3(split_threads<T>()), (unsigned)SH::lds, s,
                       R.items, R.ctl, n, which);
  }
  return hipSuccess;
}

template <typename T>
hipError_t column_sigma_k(const WideRun& R, int which, hipStream_t s) {
  switch (R.k) {
    case 10: return column_sigma<T, 10>(R, which, s);
    case 12: return column_sigma<T, 12>(R, which, s);
    case 14: return column_sigma<T, 14>(R, which, s);
    case 16: return column_sigma<T, 16>(R, which, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int K>
hipError_t frag_k(const WideRun& R, hipStream_t s) {
  hipLaunchKernelGGL((wb_frag_kernel<T, K>), dim3(kVecGrid), dim3(kVecThreads), 0, s, R.items, R.n);
  return hipSuccess;
}

template <typename T>
hipError_t frags(const WideRun& R, hipStream_t s) {
  switch (R.k) {
    case 10: return frag_k<T, 10>(R, s);
    case 12: return frag_k<T, 12>(R, s);
    case 14: return frag_k<T, 14>(R, s);
    case 16: return frag_k<T, 16>(R, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int64_t wide_sigma_scratch_doubles(const IncDev& d) {
  if (sigma_column_supported(d)) return col_scratch(d).total;
  return ((int64_t)d.npair * d.n_det + 31) / 32 * 32;
}

int64_t wide_part_doubles(const IncDev& d) { return (int64_t)vec_blocks(d.n_sym) * kNV; }

int wide_ctl_ints(int n) { return 8 + 3 * n; }

hipError_t wide_prepare(int k) {
  hipError_t e = prepare_sigma_wide();
  if (e != hipSuccess) return e;
  const void* fns[] = {(const void*)wb_column_kernel<float, 10>, (const void*)wb_column_kernel<double, 10>,
                       (const void*)wb_column_kernel<float, 12>, (const void*)wb_column_kernel<double, 12>,
                       (const void*)wb_column_kernel<float, 14>, (const void*)wb_column_kernel<double, 14>,
                       (const void*)wb_column_split_kernel<float, 16>,
                       (const void*)wb_column_split_kernel<double, 16>};
  (void)k;
  for (const void* f : fns) {
    e = allow_max_lds(f);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t wide_setup(const WideRun& R, hipStream_t s) {
  const IncDev& d = R.d;
  const int n = R.n;
  hipLaunchKernelGGL(wb_string_energy_kernel, dim3(grid_for((int64_t)n * ((d.n_str + 255) / 256), kVecGrid)),
                     dim3(kVecThreads), 0, s, R.items, n);
  hipLaunchKernelGGL(wb_hdiag_kernel, dim3(grid_for((int64_t)n * vec_blocks(d.n_sym), kVecGrid)), dim3(kVecThreads), 0,
                     s, R.items, n);
  hipLaunchKernelGGL(wb_init_kernel, dim3(grid_for(n, kSmallGrid)), dim3(64), 0, s, R.items, n, R.precision);
  if (sigma_column_supported(d)) {
    hipError_t e = R.precision == IFCI_MIXED ? frags<float>(R, s) : hipSuccess;
    if (e == hipSuccess) e = frags<double>(R, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(wb_compact_kernel, dim3(1), dim3(kCompactThreads), 0, s, R.items, n, R.ctl, n);
  return hipGetLastError();
}

hipError_t wide_iteration(const WideRun& R, hipStream_t s) {
  const int n = R.n;
  const bool col = sigma_column_supported(R.d);
  // sigma of V[m] into S[m]: FP32 increments, then FP64 ones
  if (col) {
    hipError_t e = R.precision == IFCI_MIXED ? column_sigma_k<float>(R, 1, s) : hipSuccess;
    if (e == hipSuccess) e = column_sigma_k<double>(R, 2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wb_combine_kernel, dim3(kVecGrid), dim3(kVecThreads), 0, s, R.items, R.ctl, n);
  } else {
    if (R.precision == IFCI_MIXED) {
      hipLaunchKernelGGL((wb_contract_kernel<float>), dim3(kVecGrid), dim3(kWideThreads), 0, s, R.items, R.ctl, n, 1);
      hipLaunchKernelGGL((wb_gather_kernel<float>), dim3(kVecGrid), dim3(kWideThreads), 0, s, R.items, R.ctl, n, 1);
    }
    hipLaunchKernelGGL((wb_contract_kernel<double>), dim3(kVecGrid), dim3(kWideThreads), 0, s, R.items, R.ctl, n, 2);
    hipLaunchKernelGGL((wb_gather_kernel<double>), dim3(kVecGrid), dim3(kWideThreads), 0, s, R.items, R.ctl, n, 2);
  }
  const dim3 gv(kVecGrid), bv(kVecThreads), gs(grid_for(n, kSmallGrid)), bs(64);
  hipLaunchKernelGGL(wb_dots_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_small_G_kernel, gs, bs, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_passA_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_small_A_kernel, gs, bs, 0, s, R.items, R.ctl, n, R.r_tol_inner, R.r_tol, R.max_iter);
  if (R.precision == IFCI_MIXED) hipLaunchKernelGGL(wb_switch_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_restart_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_small_R_kernel, gs, bs, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_passB_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_small_B_kernel, gs, bs, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_passC_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_small_C_kernel, gs, bs, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_normalize_kernel, gv, bv, 0, s, R.items, R.ctl, n);
  hipLaunchKernelGGL(wb_compact_kernel, dim3(1), dim3(kCompactThreads), 0, s, R.items, n, R.ctl, n);
  return hipGetLastError();
}

hipError_t wide_finish(WideItem* const* items, int n, const int32_t* out_pos, double e_const, double* e_out,
                       int32_t* status_out, int32_t* iters_out, double* resid_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(wb_finish_kernel, dim3(grid_for((n + 255) / 256, 64)), dim3(256), 0, s, items, n, out_pos,
                     e_const, e_out, status_out, iters_out, resid_out);
  return hipGetLastError();
}

}  // namespace ifci
