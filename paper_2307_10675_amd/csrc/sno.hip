// Summation natural orbitals (paper, Methods, iFCI section, the SNO
// paragraph, eq. 6): the virtual space of each increment.
//
// Each occupied orbital i is a body; every body shares the virtual orbitals
// V.  rho_i is the block over V of the one-particle density of the FCI of
// i's two electrons in {i} + V (exact CISD for two electrons; the caller
// solves those problems with the ordinary solver and takes their densities
// from the RDM adjoint).  For an increment S, rho_S = sum over i in S of
// rho_i; its eigenvectors are the natural orbitals, and those of occupation
// at least 10^-eta span the increment's virtual space.  The increment is
// then an ordinary problem in a rotated basis: S's occupied orbitals, the
// kept natural orbitals (largest occupation first), the other occupied
// orbitals frozen; its integrals are the full ones transformed by the
// matrix C whose columns are those orbitals.
#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

// One wavefront per increment: rho_S into LDS, its eigen-decomposition by
// the one-wave Jacobi, the kept natural orbitals as the first columns of
// rot (largest occupation first, the rest zero), their count in n_keep.
__global__ void __launch_bounds__(64) sno_orbitals_kernel(const double* __restrict__ gamma, int n_orb,
                                                          const int32_t* __restrict__ vir, int n_vir,
                                                          const int32_t* __restrict__ inc_occ, int order,
                                                          double thresh, double* __restrict__ rot,
                                                          int32_t* __restrict__ n_keep) {
  __shared__ double A[256], Q[256], y[16], ev[16], theta[1];
  __shared__ int perm[16];
  const int inc = blockIdx.x, lane = threadIdx.x;
  for (int t = lane; t < 256; t += 64) {
    const int a = t >> 4, b = t & 15;
    double v = 0.0;
    if (a < n_vir && b < n_vir)
      for (int m = 0; m < order; ++m) {
        const int i = inc_occ[(int64_t)inc * order + m];
        if (i >= 0) v += gamma[((int64_t)i * n_orb + vir[a]) * n_orb + vir[b]];
      }
    A[t] = v;
    Q[t] = (a == b) ? 1.0 : 0.0;
  }
  __builtin_amdgcn_wave_barrier();
  jacobi_warm(A, Q, n_vir, theta, y, ev, perm);
  // ev ascending: the k-th largest occupation is ev[n_vir - 1 - k]
  int kept = 0;
  for (int k = 0; k < n_vir; ++k)
    if (ev[n_vir - 1 - k] >= thresh) kept = k + 1;
  double* R = rot + (int64_t)inc * n_vir * n_vir;
  for (int t = lane; t < n_vir * n_vir; t += 64) {
    const int a = t / n_vir, k = t - a * n_vir;
    R[t] = k < kept ? Q[a * 16 + perm[n_vir - 1 - k]] : 0.0;
  }
  if (lane == 0) n_keep[inc] = kept;
}

// out[b][c][d][j] = sum_a C[a][j] in[a][b][c][d]: contracts the first index
// (n_in) with C (n_in x m) and appends the result as the last one, so four
// applications take (p q r s) to (i j k l).
__global__ void sno_quarter_kernel(const double* __restrict__ in, double* __restrict__ out,
                                   const double* __restrict__ C, int n_in, int64_t rest, int m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rest * m) return;
  const int64_t r = e / m;
  const int j = (int)(e - r * m);
  double s = 0.0;
  for (int a = 0; a < n_in; ++a) s += C[(int64_t)a * m + j] * in[(int64_t)a * rest + r];
  out[e] = s;
}

// C (n_orb x m): S's occupied orbitals, the kept natural orbitals over V,
// the other occupied orbitals; then h' = C^T h C.
__global__ void sno_basis_kernel(const double* __restrict__ rot, int n_vir, int n_keep,
                                 const int32_t* __restrict__ col_orb, int n_s, int n_other, int n_orb,
                                 const int32_t* __restrict__ vir, double* __restrict__ C) {
  const int m = n_s + n_keep + n_other;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_orb * m; t += gridDim.x * blockDim.x) {
    const int p = t / m, j = t - p * m;
    double v = 0.0;
    if (j < n_s) {
      v = (p == col_orb[j]) ? 1.0 : 0.0;
    } else if (j < n_s + n_keep) {
      const int k = j - n_s;
      for (int a = 0; a < n_vir; ++a)
        if (vir[a] == p) v = rot[(int64_t)a * n_vir + k];
    } else {
      v = (p == col_orb[n_s + (j - n_s - n_keep)]) ? 1.0 : 0.0;
    }
    C[t] = v;
  }
}

__global__ void sno_h_kernel(const double* __restrict__ h, const double* __restrict__ C, int n_orb, int m,
                             double* __restrict__ h_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * m) return;
  const int i = t / m, j = t - i * m;
  double s = 0.0;
  for (int p = 0; p < n_orb; ++p) {
    double u = 0.0;
    for (int q = 0; q < n_orb; ++q) u += h[p * n_orb + q] * C[q * m + j];
    s += C[p * m + i] * u;
  }
  h_out[t] = s;
}

hipError_t launch_sno_orbitals(const double* gamma, int n_orb, const int32_t* vir, int n_vir, const int32_t* inc_occ,
                               int64_t n_inc, int order, double thresh, double* rot, int32_t* n_keep,
                               hipStream_t st) {
  hipLaunchKernelGGL(sno_orbitals_kernel, dim3((unsigned)n_inc), dim3(64), 0, st, gamma, n_orb, vir, n_vir, inc_occ,
                     order, thresh, rot, n_keep);
  return hipGetLastError();
}

hipError_t launch_sno_transform(const double* h, const double* eri, int n_orb, const int32_t* vir, int n_vir,
                                const int32_t* col_orb, int n_s, int n_other, const double* rot, int n_keep,
                                double* C, double* buf0, double* buf1, double* h_out, double* eri_out,
                                hipStream_t st) {
  const int m = n_s + n_keep + n_other;
  hipLaunchKernelGGL(sno_basis_kernel, dim3((n_orb * m + 255) / 256), dim3(256), 0, st, rot, n_vir, n_keep, col_orb,
                     n_s, n_other, n_orb, vir, C);
  hipLaunchKernelGGL(sno_h_kernel, dim3((m * m + 255) / 256), dim3(256), 0, st, h, C, n_orb, m, h_out);
  // four quarter transformations, each contracting the leading index (of
  // extent n_orb) against C: input [n_orb][rest], rest = n_orb^(3 - q) m^q
  const double* in = eri;
  double* outs[4] = {buf0, buf1, buf0, eri_out};
  for (int q = 0; q < 4; ++q) {
    int64_t rest = 1;
    for (int t = 0; t < 3 - q; ++t) rest *= n_orb;
    for (int t = 0; t < q; ++t) rest *= m;
    const int64_t tot = rest * m;
    hipLaunchKernelGGL(sno_quarter_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, in, outs[q], C,
                       n_orb, rest, m);
    in = outs[q];
  }
  return hipGetLastError();
}

}  // namespace ifci
