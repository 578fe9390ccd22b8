// Frozen-core embedding of every increment and the reference energy.
//
// An increment S correlates the orbitals of its bodies (active space A);
// the reference-occupied orbitals of the other bodies form a closed-shell
// core C and their virtual orbitals are dropped (the reading of "including
// only the occupied orbitals" of the paper's iFCI section).  With the core
// doubly occupied the full-space Hamiltonian restricted to the space of S is
//   E_core + sum_pq h'_pq E_pq + 1/2 sum_pqrs (pq|rs)(E_pq E_rs - delta_qr E_ps)
// over p, q, r, s in A, where (standard closed-shell frozen-core algebra)
//   E_core = sum_c 2 h_cc + sum_cd [2 (cc|dd) - (cd|dc)],
//   h'_pq  = h_pq + sum_c [2 (pq|cc) - (pc|cq)].
// The kernels use the equivalent form sum_pq k_pq E_pq + 1/2 sum (pq|rs) E_pq E_rs
// with k_pq = h'_pq - 1/2 sum_r (pr|rq), and contract over unordered pairs
// P = (i >= j): V[P][Q] = 1/2 (ij|kl) + [Q = (mm)] k_ij / N, which also
// carries the one-electron term because sum_m E_mm = N in an N-electron space.
#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

__device__ __forceinline__ double g4(const double* eri, int n, int p, int q, int r, int s) {
  return eri[(((int64_t)p * n + q) * n + r) * n + s];
}

__global__ void __launch_bounds__(256) embed_kernel(const IncDev* __restrict__ incs, int n_inc,
                                                    const int32_t* __restrict__ orbs,
                                                    const double* __restrict__ h,
                                                    const double* __restrict__ eri, int n,
                                                    double* __restrict__ ints,
                                                    const int32_t* __restrict__ ref_occ, int n_ref,
                                                    double e_const, double* __restrict__ misc) {
  __shared__ double heff[kMaxAct * kMaxAct];
  __shared__ double keff[kMaxAct * kMaxAct];
  __shared__ double red[8];
  __shared__ int act[kMaxAct];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  if (blockIdx.x == n_inc) {
    // reference energy: closed-shell determinant over every reference-occupied orbital
    double s = 0.0;
    for (int64_t t = tid; t < (int64_t)n_ref * n_ref; t += blockDim.x) {
      int i = ref_occ[t / n_ref], j = ref_occ[t % n_ref];
      s += 2.0 * g4(eri, n, i, i, j, j) - g4(eri, n, i, j, j, i);
    }
    for (int t = tid; t < n_ref; t += blockDim.x) s += 2.0 * h[(int64_t)ref_occ[t] * n + ref_occ[t]];
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double e = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) e += red[w];
      misc[0] = e + e_const;
    }
    return;
  }

  const IncDev d = incs[blockIdx.x];
  const int k = d.k, np = d.npair, nc = d.n_core;
  const int32_t* core = orbs + d.core_off;
  if (tid < k) act[tid] = orbs[d.act_off + tid];
  __syncthreads();
  double* B = ints + d.int_off;
  const IntBlock L = int_block(k);

  for (int t = tid; t < k * k; t += blockDim.x) {
    const int p = act[t / k], q = act[t % k];
    double s = h[(int64_t)p * n + q];
    for (int ic = 0; ic < nc; ++ic) {
      const int c = core[ic];
      s += 2.0 * g4(eri, n, p, q, c, c) - g4(eri, n, p, c, c, q);
    }
    heff[t] = s;
  }
  __syncthreads();
  for (int t = tid; t < k * k; t += blockDim.x) {
    const int i = t / k, j = t % k;
    const int p = act[i], q = act[j];
    double s = heff[t];
    for (int r = 0; r < k; ++r) s -= 0.5 * g4(eri, n, p, act[r], act[r], q);
    keff[t] = s;
    B[L.keff + t] = s;
    B[L.J + t] = g4(eri, n, p, p, q, q);
    B[L.K + t] = g4(eri, n, p, q, q, p);
    if (i == j) B[L.hd + i] = heff[t];
  }
  __syncthreads();
  const double nel = 2.0 * d.na;
  for (int t = tid; t < np * np; t += blockDim.x) {
    const int P = t / np, Q = t % np;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= P) ++i;
    const int j = P - i * (i + 1) / 2;
    int kk = 0;
    while ((kk + 1) * (kk + 2) / 2 <= Q) ++kk;
    const int l = Q - kk * (kk + 1) / 2;
    double v = 0.5 * g4(eri, n, act[i], act[j], act[kk], act[l]);
    if (kk == l && nel > 0.0) v += keff[i * k + j] / nel;
    B[L.V + t] = v;
  }
  // frozen-core energy
  double s = 0.0;
  for (int64_t t = tid; t < (int64_t)nc * nc; t += blockDim.x) {
    const int c = core[t / nc], e = core[t % nc];
    s += 2.0 * g4(eri, n, c, c, e, e) - g4(eri, n, c, e, e, c);
  }
  for (int t = tid; t < nc; t += blockDim.x) s += 2.0 * h[(int64_t)core[t] * n + core[t]];
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) {
    double e = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) e += red[w];
    B[L.misc + 0] = e;
    B[L.misc + 1] = nel;
  }
}

hipError_t launch_embed(const IncDev* incs, int n_inc, const int32_t* orbs, const double* h,
                        const double* eri, int n, double* ints, const int32_t* ref_occ, int n_ref,
                        double e_const, double* misc, hipStream_t st) {
  hipLaunchKernelGGL(embed_kernel, dim3(n_inc + 1), dim3(256), 0, st, incs, n_inc, orbs, h, eri, n,
                     ints, ref_occ, n_ref, e_const, misc);
  return hipGetLastError();
}

}  // namespace ifci
