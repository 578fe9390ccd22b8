// Energy assembly of the incremental expansion (paper, iFCI section, eqs. 1-5).
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

// out[0] = E_total, out[1] = E_ref, out[1 + k] = E_c^(k); bad = number of
// increments whose status is not DONE.
__global__ void order_sum_kernel(const double* __restrict__ eps, const int32_t* __restrict__ inc_size,
                                 int n_inc, int order, const double* __restrict__ misc,
                                 const int32_t* __restrict__ status, double* __restrict__ out,
                                 int32_t* __restrict__ bad) {
  __shared__ double sums[64];
  const int k = threadIdx.x + 1;
  if (k <= order) {
    Neumaier acc;
    for (int i = 0; i < n_inc; ++i)
      if (inc_size[i] == k) acc.add(eps[i]);
    sums[k - 1] = acc.value();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Neumaier tot;
    tot.add(misc[0]);
    for (int j = 0; j < order; ++j) tot.add(sums[j]);
    out[0] = tot.value();
    out[1] = misc[0];
    for (int j = 0; j < order; ++j) out[2 + j] = sums[j];
    int nb = 0;
    if (status)
      for (int i = 0; i < n_inc; ++i) nb += (status[i] != IFCI_INC_DONE);
    *bad = nb;
  }
}

hipError_t launch_energy(const double* e_inc, const int32_t* status, const int32_t* sub_ptr,
                         const int32_t* sub_idx, const int32_t* inc_size, int n_inc, int order,
                         const double* misc_in, double* eps, double* out, int32_t* bad,
                         hipStream_t st) {
  hipLaunchKernelGGL(eps_kernel, dim3((n_inc + 255) / 256), dim3(256), 0, st, e_inc, sub_ptr, sub_idx,
                     inc_size, n_inc, misc_in, eps);
  hipLaunchKernelGGL(order_sum_kernel, dim3(1), dim3(64), 0, st, eps, inc_size, n_inc, order, misc_in,
                     status, out, bad);
  return hipGetLastError();
}

}  // namespace ifci
