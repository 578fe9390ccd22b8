// Device-wide sigma and a host-driven Davidson for one increment of any
// supported size (up to 16 active orbitals).  Used for increments whose CI
// vector does not fit on chip, for sigma of arbitrary (non-symmetric)
// vectors, and as the unfused per-increment path the batched solver is
// compared with.
//
// sigma = H c in three steps (Knowles-Handy determinant FCI):
//   contract:  E[P][I] = sum_Q V[P][Q] D[Q][I], with D[Q][I] = (E_Q c)_I built
//              on the fly from c through the pair tables of the alpha and
//              beta strings of I (MFMA 16x16x4 tiles, E written to HBM);
//   gather:    sigma_I = sum over links of alpha(I) of sign E[Q][(J, beta)]
//                      + sum over links of beta(I) of sign E[Q][(alpha, J)].
// For symmetric c, E is symmetric in its two string indices and the beta
// gather is the transpose of the alpha gather.
#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

constexpr int kWideThreads = 256;
constexpr int kMaxMT = 9;  // 136 pairs -> 9 tiles of 16

template <int SRC>
__device__ __forceinline__ double cval(const double* __restrict__ c, int n, int x, int y) {
  if (SRC == 0) return c[(int64_t)x * n + y];
  const double v = c[packed(x, y)];
  return x == y ? v : v * kRSqrt2;
}

// E[P][I] for a tile of 64 determinants per workgroup (one 16-wide tile per wave).
template <typename T, int SRC>
__global__ void __launch_bounds__(kWideThreads) contract_kernel(IncDev d, const double* __restrict__ V,
                                                                const int32_t* __restrict__ ptab,
                                                                const double* __restrict__ c,
                                                                T* __restrict__ E, double shift) {
  typedef Mfma<T> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = d.n_str, NP = d.npair;
  const int MT = (NP + 15) / 16, KS = (NP + 3) / 4;
  const int64_t ndet = d.n_det;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (j0 >= ndet) return;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t j = j0 + col;
  const bool valid = j < ndet;
  const int a = valid ? (int)(j / n) : 0, b = valid ? (int)(j % n) : 0;
  const double nel = 2.0 * d.na;
  const double sh = nel > 0.0 ? shift / (nel * nel) : 0.0;
  typename M::acc acc[kMaxMT];
#pragma unroll
  for (int m = 0; m < kMaxMT; ++m) acc[m] = M::zero();
  for (int s = 0; s < KS; ++s) {
    const int Q = 4 * s + kq;
    double bv = 0.0;
    if (valid && Q < NP) {
      const int e1 = ptab[a * NP + Q];
      if (e1 >= 0) {
        const double v = cval<SRC>(c, n, e1 >> 1, b);
        bv = (e1 & 1) ? -v : v;
      }
      const int e2 = ptab[b * NP + Q];
      if (e2 >= 0) {
        const double v = cval<SRC>(c, n, a, e2 >> 1);
        bv += (e2 & 1) ? -v : v;
      }
    }
    const T bt = (T)bv;
    const int Qa = 4 * s + kq;
    int qi = -1;
    for (int i = 0; i < d.k; ++i)
      if (Qa == i * (i + 3) / 2) qi = i;
#pragma unroll
    for (int m = 0; m < kMaxMT; ++m) {
      if (m < MT) {
        const int P = 16 * m + col;
        double av = 0.0;
        if (P < NP && Qa < NP) {
          av = V[P * NP + Qa];
          if (qi >= 0) {
            bool pd = false;
            for (int i = 0; i < d.k; ++i) pd |= (P == i * (i + 3) / 2);
            if (pd) av -= sh;
          }
        }
        acc[m] = M::mma((T)av, bt, acc[m]);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kMaxMT; ++m) {
    if (m < MT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = 16 * m + M::row(kq, r);
        if (P < NP && valid) E[(int64_t)P * ndet + j] = acc[m][r];
      }
    }
  }
}

// General gather: sigma[(a,b)] over the full determinant list.
template <typename T>
__global__ void __launch_bounds__(kWideThreads) gather_full_kernel(IncDev d, const int32_t* __restrict__ links,
                                                                   const T* __restrict__ E,
                                                                   double* __restrict__ sig) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n_det) return;
  const int n = d.n_str, nl = d.n_link;
  const int a = (int)(j / n), b = (int)(j % n);
  const int64_t nd = d.n_det;
  T s = (T)0;
  for (int l = 0; l < nl; ++l) {
    const int code = links[a * nl + l];
    const int Q = code >> 17, J = (code >> 1) & 0xFFFF;
    const T v = E[(int64_t)Q * nd + (int64_t)J * n + b];
    s += (code & 1) ? -v : v;
  }
  for (int l = 0; l < nl; ++l) {
    const int code = links[b * nl + l];
    const int Q = code >> 17, J = (code >> 1) & 0xFFFF;
    const T v = E[(int64_t)Q * nd + (int64_t)a * n + J];
    s += (code & 1) ? -v : v;
  }
  sig[j] = (double)s;
}

// Symmetric gather into a packed scaled vector: sigma = S + S^T.
template <typename T>
__global__ void __launch_bounds__(kWideThreads) gather_sym_kernel(IncDev d, const int32_t* __restrict__ links,
                                                                  const T* __restrict__ E,
                                                                  double* __restrict__ sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n_sym) return;
  int a, b;
  unpack(i, &a, &b);
  const int n = d.n_str, nl = d.n_link;
  const int64_t nd = d.n_det;
  T s1 = (T)0, s2 = (T)0;
  for (int l = 0; l < nl; ++l) {
    const int code = links[a * nl + l];
    const int Q = code >> 17, J = (code >> 1) & 0xFFFF;
    const T v = E[(int64_t)Q * nd + (int64_t)b * n + J];
    s1 += (code & 1) ? -v : v;
  }
  if (a == b) {
    sig[i] = 2.0 * (double)s1;
    return;
  }
  for (int l = 0; l < nl; ++l) {
    const int code = links[b * nl + l];
    const int Q = code >> 17, J = (code >> 1) & 0xFFFF;
    const T v = E[(int64_t)Q * nd + (int64_t)a * n + J];
    s2 += (code & 1) ? -v : v;
  }
  sig[i] = kSqrt2 * ((double)s1 + (double)s2);
}

hipError_t launch_sigma_wide(const IncDev& d, const IncDev*, int, const double* ints, const int32_t* tables,
                             const double* c, double* sig, double* E, int precision, int mode, double shift,
                             hipStream_t st) {
  const double* V = ints + d.int_off + int_block(d.k).V;
  const int32_t* ptab = tables + d.pair_off;
  const int32_t* links = tables + d.link_off;
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
struct DavState {
  double G[256];
  double Gs[256];
  double Q[256];
  double y[16];
  double cf[16];
  double c2[16];
  double ev[16];
  double theta, E0, resid, tt0, tt, dx, inv, ecore;
  int m, phase, iters, status, restart, action, mb, reorth;
  int guess, keep, pad[6];
  int perm[16];
};

constexpr int kPartBlocks = 1024;
constexpr int kNV = kMaxSpace + 3;

// partial sums of NV values per block into part[block][kNV]
__device__ inline void block_partial(double (&v)[kNV], int nv, double* part, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < kNV; ++j)
    if (j < nv) v[j] = wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < kNV; ++j)
      if (j < nv) red[wave * kNV + j] = v[j];
  __syncthreads();
  if (threadIdx.x < nv) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * kNV + threadIdx.x];
    part[blockIdx.x * kNV + threadIdx.x] = s;
  }
}

__device__ inline void reduce_parts(const double* part, int nblk, int nv, double* out) {
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b * kNV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ void string_energy_kernel(IncDev d, const int32_t* __restrict__ strs, const double* __restrict__ B,
                                     double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n_str) return;
  const IntBlock ib = int_block(d.k);
  const int k = d.k;
  const uint32_t s = (uint32_t)strs[i];
  double f = 0.0;
  for (int p = 0; p < k; ++p) {
    if (!(s >> p & 1u)) continue;
    f += B[ib.hd + p];
    for (int q = 0; q < k; ++q)
      if (s >> q & 1u) f += 0.5 * (B[ib.J + p * k + q] - B[ib.K + p * k + q]);
  }
  F[i] = f;
}

__global__ void __launch_bounds__(256) hdiag_kernel(IncDev d, const int32_t* __restrict__ strs,
                                                    const double* __restrict__ B, const double* __restrict__ F,
                                                    double* __restrict__ HD, double* part) {
  __shared__ double red[16];
  __shared__ int64_t redi[16];
  const IntBlock ib = int_block(d.k);
  const int k = d.k;
  double best = 1e300;
  int64_t bi = 0x7fffffffffffffffLL;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n_sym; i += (int64_t)gridDim.x * blockDim.x) {
    int a, b;
    unpack(i, &a, &b);
    const uint32_t sa = (uint32_t)strs[a], sb = (uint32_t)strs[b];
    double v = F[a] + F[b];
    for (int p = 0; p < k; ++p) {
      if (!(sa >> p & 1u)) continue;
      for (int q = 0; q < k; ++q)
        if (sb >> q & 1u) v += B[ib.J + p * k + q];
    }
    HD[i] = v;
    if (v < best) best = v, bi = i;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ov < best || (ov == best && oi < bi)) best = ov, bi = oi;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = best, redi[wave] = bi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (red[w] < red[0] || (red[w] == red[0] && redi[w] < redi[0])) red[0] = red[w], redi[0] = redi[w];
    part[blockIdx.x * 2] = red[0];
    part[blockIdx.x * 2 + 1] = (double)redi[0];
  }
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
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    const double si = s[i];
#pragma unroll
    for (int j = 0; j < kMaxSpace; ++j)
      if (j <= m) acc[j] += Vb[j * st + i] * si;
  }
  block_partial(acc, m + 1, part, red);
}

__global__ void __launch_bounds__(64) small_G_kernel(DavState* S, const double* part, int nblk, int mmax) {
  const int m = S->m;
  __shared__ double g[kNV];
  reduce_parts(part, nblk, m + 1, g);
  if (threadIdx.x <= (unsigned)m) {
    S->G[threadIdx.x * 16 + m] = g[threadIdx.x];
    S->G[m * 16 + threadIdx.x] = g[threadIdx.x];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += 64) S->Gs[i] = S->G[i];
  __syncthreads();
  jacobi_lowest(S->Gs, S->Q, m + 1, &S->theta, S->y, S->ev, S->perm);
  if (threadIdx.x == 0) {
    S->restart = (m + 1 == mmax);
    S->keep = mmax / 2 < kKeep ? mmax / 2 : kKeep;
    S->iters += 1;
  }
}

__global__ void __launch_bounds__(256) passA_kernel(const DavState* __restrict__ S, double* Vb, double* Sb,
                                                    int64_t st, const double* __restrict__ HD,
                                                    double* __restrict__ X, double* __restrict__ T,
                                                    int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double y[16];
  const int m = S->m;
  const double theta = S->theta, E0 = S->E0;
  if (threadIdx.x < 16) y[threadIdx.x] = S->y[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    double x = 0.0, sx = 0.0;
    for (int j = 0; j <= m; ++j) {
      x += y[j] * Vb[j * st + i];
      sx += y[j] * Sb[j * st + i];
    }
    const double r = sx - theta * x;
    double den = theta - (HD[i] - E0);
    if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
    const double t = r / den;
    acc[kMaxSpace] += r * r;
    acc[kMaxSpace + 1] += t * t;
    acc[kMaxSpace + 2] += x * t;
#pragma unroll
    for (int j = 0; j < kMaxSpace; ++j)
      if (j <= m) acc[j] += Vb[j * st + i] * t;
    T[i] = t;
    X[i] = x;
  }
  // pack: dots in [0, m], then rr, tt0, dx at m+1..m+3
  double out[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) out[j] = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxSpace; ++j)
    if (j <= m) out[j] = acc[j];
#pragma unroll
  for (int j = 0; j < kNV; ++j) {
    if (j == m + 1) out[j] = acc[kMaxSpace];
    if (j == m + 2) out[j] = acc[kMaxSpace + 1];
    if (j == m + 3) out[j] = acc[kMaxSpace + 2];
  }
  block_partial(out, m + 4, part, red);
}

// action: 0 continue, 1 done, 2 switch to FP64 refinement, 3 out of
// iterations, 4 evicted
__global__ void __launch_bounds__(64) small_A_kernel(DavState* S, const double* part, int nblk, double tol32,
                                                     double tol64, int max_iter, int evict) {
  const int m = S->m;
  __shared__ double v[kNV];
  reduce_parts(part, nblk, m + 4, v);
  if (threadIdx.x == 0) {
    const double rr = v[m + 1];
    S->resid = sqrt(rr);
    S->tt0 = v[m + 2];
    S->dx = v[m + 3];
    for (int j = 0; j < 16; ++j) S->cf[j] = (j <= m) ? v[j] : 0.0;
    S->mb = m;
    const double tol = S->phase == 32 ? tol32 : tol64;
    int action = 0;
    if (evict) {
      action = 4;
      S->status = IFCI_INC_EVICTED;
    } else if (S->resid <= tol) {
      if (S->phase == 32) {
        action = (S->iters >= max_iter) ? 3 : 2;
      } else {
        action = 1;
        S->status = IFCI_INC_DONE;
      }
    } else if (S->iters >= max_iter) {
      action = 3;
    }
    S->action = action;
  }
}

// Thick restart, device-wide: V[k] <- sum_j Q[j][perm k] V[j] for the keep
// lowest Ritz vectors, same for S.
__global__ void __launch_bounds__(256) restart_kernel(const DavState* __restrict__ S, double* Vb, double* Sb,
                                                      int64_t st, int64_t ns) {
  __shared__ double q[kMaxSpace * kKeep];
  const int m = S->m, keep = S->keep;
  for (int t = threadIdx.x; t < kMaxSpace * kKeep; t += blockDim.x) {
    const int j = t / kKeep, kk = t % kKeep;
    q[t] = (j <= m && kk < keep) ? S->Q[j * 16 + S->perm[kk]] : 0.0;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    for (int pass = 0; pass < 2; ++pass) {
      double* B = pass == 0 ? Vb : Sb;
      double vv[kMaxSpace];
#pragma unroll
      for (int j = 0; j < kMaxSpace; ++j) vv[j] = (j <= m) ? B[j * st + i] : 0.0;
#pragma unroll
      for (int kk = 0; kk < kKeep; ++kk) {
        if (kk < keep) {
          double v = 0.0;
#pragma unroll
          for (int j = 0; j < kMaxSpace; ++j) v += q[j * kKeep + kk] * vv[j];
          B[kk * st + i] = v;
        }
      }
    }
  }
}

__global__ void small_R_kernel(DavState* S) {
  if (threadIdx.x != 0) return;
  const int m = S->m, keep = S->keep;
  double cn[kKeep];
  for (int kk = 0; kk < keep; ++kk) {
    double c = 0.0;
    for (int j = 0; j <= m; ++j) c += S->Q[j * 16 + S->perm[kk]] * S->cf[j];
    cn[kk] = c;
  }
  for (int j = 0; j < 16; ++j) S->cf[j] = j < keep ? cn[j] : 0.0;
  for (int i = 0; i < 256; ++i) S->G[i] = 0.0;
  for (int kk = 0; kk < keep; ++kk) S->G[kk * 16 + kk] = S->ev[kk];
  S->mb = keep - 1;
}

__global__ void __launch_bounds__(256) switch_kernel(DavState* S, double* Vb, const double* X, int64_t ns) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x)
    Vb[i] = X[i];
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) S->G[i] = 0.0;
    if (threadIdx.x == 0) {
      S->phase = 64;
      S->m = 0;
    }
  }
}

__global__ void __launch_bounds__(256) passB_kernel(const DavState* __restrict__ S, const double* __restrict__ Vb,
                                                    int64_t st, double* __restrict__ T, int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double cf[16];
  const int mb = S->mb;
  if (threadIdx.x < 16) cf[threadIdx.x] = S->cf[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    double t = T[i];
    for (int j = 0; j <= mb; ++j) t -= cf[j] * Vb[j * st + i];
    T[i] = t;
    acc[kMaxSpace] += t * t;
#pragma unroll
    for (int j = 0; j < kMaxSpace; ++j)
      if (j <= mb) acc[j] += Vb[j * st + i] * t;
  }
  double out[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) out[j] = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxSpace; ++j)
    if (j <= mb) out[j] = acc[j];
#pragma unroll
  for (int j = 0; j < kNV; ++j)
    if (j == mb + 1) out[j] = acc[kMaxSpace];
  block_partial(out, mb + 2, part, red);
}

__global__ void __launch_bounds__(64) small_B_kernel(DavState* S, const double* part, int nblk) {
  const int mb = S->mb;
  __shared__ double v[kNV];
  reduce_parts(part, nblk, mb + 2, v);
  if (threadIdx.x == 0) {
    const double tt = v[mb + 1];
    S->tt = tt;
    S->reorth = tt < 0.5 * S->tt0;
    for (int j = 0; j < 16; ++j) S->c2[j] = (j <= mb) ? v[j] : 0.0;
    S->inv = tt > 0.0 ? 1.0 / sqrt(tt) : 0.0;
  }
}

__global__ void __launch_bounds__(256) passC_kernel(const DavState* __restrict__ S, const double* __restrict__ Vb,
                                                    int64_t st, double* __restrict__ T, int64_t ns, double* part) {
  __shared__ double red[4 * kNV];
  __shared__ double c2[16];
  if (!S->reorth) return;
  const int mb = S->mb;
  if (threadIdx.x < 16) c2[threadIdx.x] = S->c2[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    double t = T[i];
    for (int j = 0; j <= mb; ++j) t -= c2[j] * Vb[j * st + i];
    T[i] = t;
    acc[0] += t * t;
  }
  block_partial(acc, 1, part, red);
}

__global__ void __launch_bounds__(64) small_C_kernel(DavState* S, const double* part, int nblk) {
  if (!S->reorth) return;
  __shared__ double v[kNV];
  reduce_parts(part, nblk, 1, v);
  if (threadIdx.x == 0) {
    S->tt = v[0];
    S->inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
  }
}

__global__ void __launch_bounds__(256) normalize_kernel(DavState* S, double* Vb, int64_t st,
                                                        const double* __restrict__ T, int64_t ns) {
  const double inv = S->inv;
  const int mn = S->mb + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x)
    Vb[mn * st + i] = T[i] * inv;
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
