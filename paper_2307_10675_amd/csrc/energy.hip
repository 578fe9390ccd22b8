// Energy assembly of the incremental expansion (paper, iFCI section, eqs. 1-5),
// with or without connected n-body screening (the CnB paragraph).
//
// eqs. 2-5 define eps_S = E_c(S) - sum over proper non-empty subsets T of
// eps_T.  Unrolling that recursion gives the equivalent closed form
// (Moebius inversion on the lattice of subsets)
//   eps_S = sum over non-empty T subset of S of (-1)^(|S| - |T|) E_c(T),
// with E_c(T) = E(T) - E_ref.  Each increment's sum runs in a fixed order with
// Neumaier compensation; the order sums E_c^(k) = sum_{|S| = k} eps_S run in
// the canonical increment order, so results are bitwise reproducible.
#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

struct Neumaier {
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

__global__ void eps_kernel(const double* __restrict__ e_inc, const int32_t* __restrict__ sub_ptr,
                           const int32_t* __restrict__ sub_idx, const int32_t* __restrict__ inc_size,
                           int n_inc, const double* __restrict__ misc, double* __restrict__ eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inc) return;
  const double eref = misc[0];
  const int sz = inc_size[i];
  Neumaier acc;
  for (int t = sub_ptr[i]; t < sub_ptr[i + 1]; ++t) {
    const int T = sub_idx[t];
    const double ec = e_inc[T] - eref;
    acc.add(((sz - inc_size[T]) & 1) ? -ec : ec);
  }
  eps[i] = acc.value();
}

// Compensated pair (s, c): value s + c.  Two pairs combine with an exact
// two-sum of the leading parts, so the tree below keeps the compensation.
__device__ inline void two_sum_merge(double& s, double& c, double s2, double c2) {
  const double t = s + s2;
  const double bp = t - s;
  const double err = (s - (t - bp)) + (s2 - bp);
  s = t;
  c = c + c2 + err;
}

// out[0] = E_total, out[1] = E_ref, out[1 + k] = E_c^(k); bad = number of
// increments whose status is not DONE.  Increments are sorted by size, so
// order k is one contiguous range; each thread sums a contiguous chunk of it
// (Neumaier) and the block merges the chunks in a fixed tree.
constexpr int kSumThreads = 256;
__global__ void __launch_bounds__(kSumThreads)
    order_sum_kernel(const double* __restrict__ eps, const int32_t* __restrict__ inc_size, int n_inc, int order,
                     const double* __restrict__ misc, const int32_t* __restrict__ status,
                     double* __restrict__ out, int32_t* __restrict__ bad) {
  __shared__ double ss[kSumThreads], sc[kSumThreads];
  __shared__ int sb[kSumThreads];
  const int t = threadIdx.x;
  Neumaier tot;
  if (t == 0) tot.add(misc[0]);
  for (int k = 1; k <= order; ++k) {
    // first index with size >= k and first with size > k
    int lo = 0, hi = n_inc;
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (inc_size[m] < k) lo = m + 1; else hi = m;
    }
    int lo2 = lo, hi2 = n_inc;
    while (lo2 < hi2) {
      const int m = (lo2 + hi2) >> 1;
      if (inc_size[m] <= k) lo2 = m + 1; else hi2 = m;
    }
    const int cnt = lo2 - lo, chunk = (cnt + kSumThreads - 1) / kSumThreads;
    Neumaier acc;
    for (int i = lo + t * chunk; i < lo + min(cnt, (t + 1) * chunk); ++i) acc.add(eps[i]);
    ss[t] = acc.s;
    sc[t] = acc.c;
    __syncthreads();
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
      if (t < w) {
        double a = ss[t], c = sc[t];
        two_sum_merge(a, c, ss[t + w], sc[t + w]);
        ss[t] = a;
        sc[t] = c;
      }
      __syncthreads();
    }
    if (t == 0) {
      const double v = ss[0] + sc[0];
      out[1 + k] = v;
      tot.add(v);
    }
    __syncthreads();
  }
  int nb = 0;
  if (status)
    for (int i = t; i < n_inc; i += kSumThreads) nb += (status[i] != IFCI_INC_DONE && status[i] != IFCI_INC_SCREENED);
  sb[t] = nb;
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if (t < w) sb[t] += sb[t + w];
    __syncthreads();
  }
  if (t == 0) {
    out[0] = tot.value();
    out[1] = misc[0];
    *bad = sb[0];
  }
}

// Screened expansion, one size level at a time (levels ascending): a kept
// increment's eps_S = E_c(S) - sum over its proper subsets of eps_T (the
// dropped ones hold 0), a dropped one's eps_S = 0.
__global__ void eps_screened_kernel(const double* __restrict__ e_inc, const int32_t* __restrict__ sub_ptr,
                                    const int32_t* __restrict__ sub_idx, const int32_t* __restrict__ inc_size,
                                    const uint8_t* __restrict__ keep, int n_inc, int level,
                                    const double* __restrict__ misc, double* __restrict__ eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inc || inc_size[i] != level) return;
  if (!keep[i]) {
    eps[i] = 0.0;
    return;
  }
  Neumaier acc;
  acc.add(e_inc[i] - misc[0]);
  for (int t = sub_ptr[i]; t < sub_ptr[i + 1]; ++t) {
    const int T = sub_idx[t];
    if (T != i) acc.add(-eps[T]);
  }
  eps[i] = acc.value();
}

hipError_t launch_energy_screened(const double* e_inc, const int32_t* status, const int32_t* sub_ptr,
                                  const int32_t* sub_idx, const int32_t* inc_size, const uint8_t* keep, int n_inc,
                                  int order, const double* misc_in, double* eps, double* out, int32_t* bad,
                                  hipStream_t st) {
  for (int level = 1; level <= order; ++level)
    hipLaunchKernelGGL(eps_screened_kernel, dim3((n_inc + 255) / 256), dim3(256), 0, st, e_inc, sub_ptr, sub_idx,
                       inc_size, keep, n_inc, level, misc_in, eps);
  hipLaunchKernelGGL(order_sum_kernel, dim3(1), dim3(kSumThreads), 0, st, eps, inc_size, n_inc, order, misc_in,
                     status, out, bad);
  return hipGetLastError();
}

// Outputs of the dropped increments of [first, first + count): energy and
// residual NaN, status IFCI_INC_SCREENED, no iterations.
__global__ void mark_screened_kernel(const uint8_t* __restrict__ keep, int64_t first, int64_t count,
                                     double* __restrict__ e_out, int32_t* __restrict__ status_out,
                                     int32_t* __restrict__ iters_out, double* __restrict__ resid_out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= count || keep[first + o]) return;
  e_out[o] = __builtin_nan("");
  status_out[o] = IFCI_INC_SCREENED;
  if (iters_out) iters_out[o] = 0;
  if (resid_out) resid_out[o] = __builtin_nan("");
}

hipError_t launch_mark_screened(const uint8_t* keep, int64_t first, int64_t count, double* e_out,
                                int32_t* status_out, int32_t* iters_out, double* resid_out, hipStream_t st) {
  hipLaunchKernelGGL(mark_screened_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, keep, first,
                     count, e_out, status_out, iters_out, resid_out);
  return hipGetLastError();
}

hipError_t launch_energy(const double* e_inc, const int32_t* status, const int32_t* sub_ptr,
                         const int32_t* sub_idx, const int32_t* inc_size, int n_inc, int order,
                         const double* misc_in, double* eps, double* out, int32_t* bad,
                         hipStream_t st) {
  hipLaunchKernelGGL(eps_kernel, dim3((n_inc + 255) / 256), dim3(256), 0, st, e_inc, sub_ptr, sub_idx,
                     inc_size, n_inc, misc_in, eps);
  hipLaunchKernelGGL(order_sum_kernel, dim3(1), dim3(kSumThreads), 0, st, eps, inc_size, n_inc, order, misc_in,
                     status, out, bad);
  return hipGetLastError();
}

}  // namespace ifci
