// Density matrices of the converged increments and the analytic gradient of
// the iFCI energy.
//
// For a normalised state Psi:  gamma_pq = <Psi|E_pq|Psi>,
//   Gamma_pqrs = <Psi|E_pq E_rs|Psi> - delta_qr gamma_ps = <E_qp Psi|E_rs Psi> - delta_qr gamma_ps,
// so with D[pq][I] = (E_pq c)_I the product M = D D^T (a dense contraction over
// determinants, MFMA) gives Gamma and gamma_pq = sum_I c_I D[pq][I].
// (E_pq c)_I = sum_J <J|E_qp|I> c_J is gathered through the ordered
// single-replacement table (E_qp on the alpha string and on the beta string).
//
// Hellmann-Feynman: every eigenvalue E(S) satisfies dE/dh_pq = gamma_pq and
// dE/d(pq|rs) = Gamma_pqrs / 2 for full-space h and (pq|rs) taken entry by
// entry.  The full-space densities of an increment follow from its active
// ones and a doubly occupied core c, d (closed-shell algebra):
//   gamma_cc = 2;  Gamma_ccdd = 4 - 2 delta_cd;  Gamma_cddc = -2 (c != d);
//   Gamma_ccpq = Gamma_pqcc = 2 gamma_pq;  Gamma_cpqc = -gamma_qp;
//   Gamma_pccq = -gamma_pq  (p, q active); every other mixed entry is zero.
// The truncated expansion E = E_ref + sum_S w_|S| (E(S) - E_ref) then has
// gradient (1 - sum w) dE_ref + sum_S w_S dE(S).
#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

constexpr int kRdmThreads = 512;
constexpr int kRdmChunk = 32;       // determinants staged per step
constexpr int kTilesPerWave = 8;    // output tiles per wave (per group of 64)

// grid: (increment, tile group).  Output for increment i at rdm + rdm_off[i]:
// gamma [k*k] then Gamma [k^4].
__global__ void __launch_bounds__(kRdmThreads) rdm_kernel(const IncDev* __restrict__ incs,
                                                          const double* __restrict__ dav,
                                                          const int32_t* __restrict__ tables,
                                                          double* __restrict__ rdm,
                                                          const int64_t* __restrict__ rdm_off, int mmax,
                                                          const uint8_t* __restrict__ keep) {
  extern __shared__ __align__(16) char lds[];
  if (keep && !keep[blockIdx.x]) return;  // dropped by the screening: no vector
  const IncDev d = incs[blockIdx.x];
  const int k = d.k, k2 = k * k, n = d.n_str;
  const int nt = (k2 + 15) / 16;          // tiles per side
  const int ntiles = nt * nt;
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t0 = blockIdx.y * nw * kTilesPerWave;
  if (t0 >= ntiles) return;
  const double* X = dav + d.vec_off + 2 * (int64_t)d.mspace * d.stride + d.stride;
  (void)mmax;
  const int32_t* ord = tables + d.ord_off;
  double* Dc = (double*)lds;                       // [k2p][kRdmChunk]
  const int k2p = nt * 16;
  double* cc = Dc + (size_t)k2p * kRdmChunk;       // [kRdmChunk]
  double acc_g = 0.0;
  d4 acc[kTilesPerWave];
#pragma unroll
  for (int t = 0; t < kTilesPerWave; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nd = d.n_det;
  // determinant j = a n + b of the chunk: (a0, b0) of its first entry once per
  // chunk, then one 32-bit division by n per entry (t = b0 + jj < n + 32)
  int a0 = 0, b0 = 0;
  for (int64_t base = 0; base < nd; base += kRdmChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < k2p * kRdmChunk; e += blockDim.x) {
      const int x = e / kRdmChunk, jj = e % kRdmChunk;
      const int64_t j = base + jj;
      double v = 0.0;
      if (x < k2 && j < nd) {
        const int t = b0 + jj, ta = t / n;
        const int a = a0 + ta, b = t - ta * n;
        const int p = x / k, q = x % k;
        const int ea = ord[a * k2 + q * k + p];  // E_qp |a>
        if (ea >= 0) {
          const int J = ea >> 1;
          double cv = X[packed(J, b)];
          if (J != b) cv *= kRSqrt2;
          v = (ea & 1) ? -cv : cv;
        }
        const int eb = ord[b * k2 + q * k + p];
        if (eb >= 0) {
          const int J = eb >> 1;
          double cv = X[packed(a, J)];
          if (a != J) cv *= kRSqrt2;
          v += (eb & 1) ? -cv : cv;
        }
      }
      Dc[x * kRdmChunk + jj] = v;
    }
    for (int jj = threadIdx.x; jj < kRdmChunk; jj += blockDim.x) {
      const int64_t j = base + jj;
      double v = 0.0;
      if (j < nd) {
        const int t = b0 + jj, ta = t / n;
        const int a = a0 + ta, b = t - ta * n;
        v = X[packed(a, b)];
        if (a != b) v *= kRSqrt2;
      }
      cc[jj] = v;
    }
    b0 += kRdmChunk;  // advance to the next chunk's first entry
    a0 += b0 / n;
    b0 %= n;
    __syncthreads();
    if (blockIdx.y == 0 && (int)threadIdx.x < k2) {
      double s = 0.0;
      for (int jj = 0; jj < kRdmChunk; ++jj) s += cc[jj] * Dc[threadIdx.x * kRdmChunk + jj];
      acc_g += s;
    }
    // M[x][y] += sum_j D[x][j] D[y][j]
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
      const int tile = t0 + wave * kTilesPerWave + t;
      if (tile < ntiles) {
        const int tx = tile / nt, ty = tile % nt;
        for (int s = 0; s < kRdmChunk / 4; ++s) {
          const int jj = 4 * s + (lane >> 4);
          const double av = Dc[(tx * 16 + (lane & 15)) * kRdmChunk + jj];
          const double bv = Dc[(ty * 16 + (lane & 15)) * kRdmChunk + jj];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
  }
  double* out = rdm + rdm_off[blockIdx.x];
  __syncthreads();
  // group 0 writes gamma; the delta_qr gamma_ps term is applied by a second kernel
  if (blockIdx.y == 0 && (int)threadIdx.x < k2) out[threadIdx.x] = acc_g;
#pragma unroll
  for (int t = 0; t < kTilesPerWave; ++t) {
    const int tile = t0 + wave * kTilesPerWave + t;
    if (tile < ntiles) {
      const int tx = tile / nt, ty = tile % nt;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = tx * 16 + Mfma<double>::row(lane >> 4, r), y = ty * 16 + (lane & 15);
        if (x < k2 && y < k2) {
          // x = (q, p) of E_qp, y = (r, s): Gamma'_pqrs = M[(q,p)][(r,s)]
          const int q = x / k, p = x % k;
          out[k2 + (int64_t)(p * k + q) * k2 + y] = acc[t][r];
        }
      }
    }
  }
}

// Gamma_pqrs -= delta_qr gamma_ps, one thread per (p, q, s)
__global__ void rdm_delta_kernel(const IncDev* __restrict__ incs, double* __restrict__ rdm,
                                 const int64_t* __restrict__ rdm_off, const uint8_t* __restrict__ keep) {
  if (keep && !keep[blockIdx.x]) return;
  const IncDev d = incs[blockIdx.x];
  const int k = d.k, k2 = k * k;
  double* out = rdm + rdm_off[blockIdx.x];
  for (int e = threadIdx.x; e < k * k2; e += blockDim.x) {
    const int p = e / k2, q = (e / k) % k, s = e % k;
    out[k2 + ((int64_t)(p * k + q) * k + q) * k + s] -= out[p * k + s];
  }
}

hipError_t launch_rdm(const IncDev* incs, const IncDev* host_incs, int n_inc, const double* dav_base,
                      const int32_t* tables, double* rdm, const int64_t* rdm_off_dev, int mmax, const uint8_t* keep,
                      hipStream_t st) {
  const hipError_t e = allow_max_lds((const void*)rdm_kernel);
  if (e != hipSuccess) return e;
  int kmax = 0;
  for (int i = 0; i < n_inc; ++i) kmax = host_incs[i].k > kmax ? host_incs[i].k : kmax;
  const int nt = (kmax * kmax + 15) / 16;
  const int groups = (nt * nt + (kRdmThreads / 64) * kTilesPerWave - 1) / ((kRdmThreads / 64) * kTilesPerWave);
  const size_t lds = (size_t)(nt * 16) * kRdmChunk * 8 + kRdmChunk * 8 + (size_t)kmax * kmax * 8 + 64;
  if (lds > (size_t)kMaxLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rdm_kernel, dim3(n_inc, groups), dim3(kRdmThreads), lds, st, incs, dav_base, tables, rdm,
                     rdm_off_dev, mmax, keep);
  hipLaunchKernelGGL(rdm_delta_kernel, dim3(n_inc), dim3(256), 0, st, incs, rdm, rdm_off_dev, keep);
  return hipGetLastError();
}

// One thread per full-space entry: dh (n*n entries) then deri (n^4 entries).
// loc[i * n + o]: local active index of orbital o in increment i, -1 core,
// -2 removed.  Row n_inc describes the reference determinant.
__global__ void rdm_accumulate_kernel(const IncDev* __restrict__ incs, int n_inc, const int8_t* __restrict__ loc,
                                      const double* __restrict__ rdm, const int64_t* __restrict__ rdm_off,
                                      const double* __restrict__ w, int n, double* __restrict__ dh,
                                      double* __restrict__ deri) {
  const int64_t n2 = (int64_t)n * n, n4 = n2 * n2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 + (deri ? n4 : 0)) return;
  const bool one = e < n2;
  int o0, o1, o2 = 0, o3 = 0;
  if (one) {
    o0 = (int)(e / n);
    o1 = (int)(e % n);
  } else {
    const int64_t f = e - n2;
    o0 = (int)(f / (n2 * n));
    o1 = (int)((f / n2) % n);
    o2 = (int)((f / n) % n);
    o3 = (int)(f % n);
  }
  double wsum = 0.0;
  double acc = 0.0;
  for (int i = 0; i <= n_inc; ++i) {
    double wi;
    if (i < n_inc) {
      wi = w[i];
      wsum += wi;
    } else {
      wi = 1.0 - wsum;
    }
    if (wi == 0.0) continue;
    const int8_t* L = loc + (int64_t)i * n;
    const int l0 = L[o0], l1 = L[o1];
    const int k = (i < n_inc) ? incs[i].k : 0;
    const double* g = (i < n_inc) ? rdm + rdm_off[i] : nullptr;
    double v = 0.0;
    if (one) {
      if (l0 >= 0 && l1 >= 0)
        v = g[l0 * k + l1];
      else if (l0 == -1 && o0 == o1)
        v = 2.0;
    } else {
      const int l2 = L[o2], l3 = L[o3];
      const int na = (l0 >= 0) + (l1 >= 0) + (l2 >= 0) + (l3 >= 0);
      const int nc = (l0 == -1) + (l1 == -1) + (l2 == -1) + (l3 == -1);
      if (na == 4) {
        v = g[k * k + ((int64_t)(l0 * k + l1) * k + l2) * k + l3];
      } else if (nc == 4) {
        if (o0 == o1 && o2 == o3)
          v = (o0 == o2) ? 2.0 : 4.0;
        else if (o0 == o3 && o1 == o2)
          v = -2.0;
      } else if (na == 2 && nc == 2) {
        if (l0 == -1 && l1 == -1 && o0 == o1)
          v = 2.0 * g[l2 * k + l3];
        else if (l2 == -1 && l3 == -1 && o2 == o3)
          v = 2.0 * g[l0 * k + l1];
        else if (l0 == -1 && l3 == -1 && o0 == o3)
          v = -g[l2 * k + l1];
        else if (l1 == -1 && l2 == -1 && o1 == o2)
          v = -g[l0 * k + l3];
      }
      v *= 0.5;
    }
    acc += wi * v;
  }
  if (one)
    dh[e] = acc;
  else
    deri[e - n2] = acc;
}

hipError_t launch_rdm_accumulate(const IncDev* incs, int n_inc, const int32_t*, const int32_t* loc,
                                 const double* rdm, const int64_t* rdm_off_dev, const double* w,
                                 const int32_t*, int, int n, double* dh, double* deri, hipStream_t st) {
  const int64_t n2 = (int64_t)n * n;
  const int64_t tot = n2 + (deri ? n2 * n2 : 0);
  hipLaunchKernelGGL(rdm_accumulate_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, incs, n_inc,
                     (const int8_t*)loc, rdm, rdm_off_dev, w, n, dh, deri);
  return hipGetLastError();
}

}  // namespace ifci
