// Bodies of the device-wide sigma steps and of the H diagonal, shared by the
// per-increment launches (plain.hip) and the batched solver (wide.hip).
// Internal.
//
// sigma = H c in three steps (Knowles-Handy determinant FCI):
//   contract:  E[P][I] = sum_Q V[P][Q] D[Q][I], with D[Q][I] = (E_Q c)_I built
//              on the fly from c through the pair tables of the alpha and
//              beta strings of I (MFMA 16x16x4 tiles, E written to HBM);
//   gather:    sigma_I = sum over links of alpha(I) of sign E[Q][(J, beta)]
//                      + sum over links of beta(I) of sign E[Q][(alpha, J)].
// For symmetric c, E is symmetric in its two string indices and the beta
// gather is the transpose of the alpha gather.  Half-filled increments of 10
// to 16 orbitals take the fused column form below instead.
#pragma once

#include <type_traits>

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
__device__ __forceinline__ void contract_body(const IncDev& d, const double* __restrict__ V,
                                              const int32_t* __restrict__ ptab, const double* __restrict__ c,
                                              T* __restrict__ E, double shift, int64_t tile) {
  typedef Mfma<T> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = d.n_str, NP = d.npair;
  const int MT = (NP + 15) / 16, KS = (NP + 3) / 4;
  const int64_t ndet = d.n_det;
  const int64_t j0 = (tile * 4 + wave) * 16;
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

template <typename T, int SRC>
__global__ void __launch_bounds__(kWideThreads) contract_kernel(IncDev d, const double* __restrict__ V,
                                                                const int32_t* __restrict__ ptab,
                                                                const double* __restrict__ c,
                                                                T* __restrict__ E, double shift) {
  contract_body<T, SRC>(d, V, ptab, c, E, shift, blockIdx.x);
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
__device__ __forceinline__ void gather_sym_body(const IncDev& d, const int32_t* __restrict__ links,
                                                const T* __restrict__ E, double* __restrict__ sig, int64_t i) {
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

template <typename T>
__global__ void __launch_bounds__(kWideThreads) gather_sym_kernel(IncDev d, const int32_t* __restrict__ links,
                                                                  const T* __restrict__ E,
                                                                  double* __restrict__ sig) {
  gather_sym_body<T>(d, links, E, sig, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------- fused column sigma (k 10..14)
// Symmetric vectors of increments too large for the on-chip solver, one
// workgroup per beta string b (a column of C).  With the pair table of
// string J, (J1, s1) = E_Q J (read pair-major, 16 strings a row segment),
// the column is
//   D[Q][J] = s1 C[J1][b] + s2 C[J][J2]      ((J2, s2) = E_Q b),
//   E[P][J] = sum_Q V[P][Q] D[Q][J]           (MFMA, 16-string tiles),
//   S[E_P J][b] += s E[P][J]                  (scatter, LDS FP64 atomics),
// the scatter form of the alpha gather (E_P is symmetric, so the pair table
// is its own inverse).  sigma = S + S^T follows in a separate pass.  The
// column copy of C, the A fragments of V and the FP64 accumulator S[:, b]
// live in LDS; C (full, unscaled, in the contraction precision) and the
// table rows come from L2.  Where LDS allows, the column copy is stored with
// its negation and S with a negated twin, so one table index J + neg (n + 1)
// addresses both the signed C value and the signed accumulator slot (S is
// the first half minus the second).  FP64 sums of the FP32 products make S
// practically independent of the atomic order.
// Both precisions run three waves per SIMD (more waves hide the loads and
// VALU work beside the MFMAs; four leave too few registers; FP64 with three
// instead of two: 14o14e 5.50 -> 5.29 ms).
template <typename T>
constexpr int col_threads() { return 768; }

template <typename T, int K>
struct ColShape {
  static constexpr int NP = K * (K + 1) / 2;
  static constexpr int MT = (NP + 15) / 16;
  static constexpr int KS = (NP + 3) / 4;
  static constexpr int KS2 = (KS + 1) / 2;  // FP32: two k-steps per LDS read
  static constexpr int N = max_strings(K);
  static constexpr int64_t vf_bytes = (int64_t)MT * (sizeof(T) == 4 ? 2 * KS2 : KS) * 64 * sizeof(T);
  static constexpr int64_t brow_bytes = 32 * (int64_t)KS;  // [KS][4] uint32 row offsets + [KS][4] T signs
  static constexpr bool kNeg =
      vf_bytes + 2 * (int64_t)(N + 1) * sizeof(T) + 16 + 16 * (int64_t)(N + 1) + brow_bytes <= kMaxLds;
  static constexpr int64_t col_bytes = (kNeg ? 2 : 1) * (int64_t)(N + 1) * sizeof(T);
  static constexpr int64_t s_bytes = (kNeg ? 16 : 8) * (int64_t)(N + 1);
  static constexpr int64_t lds = vf_bytes + ((col_bytes + 15) / 16) * 16 + s_bytes + brow_bytes;
};

// Packed scaled symmetric c -> full unscaled C [(n + 1) x n] of T (row n and
// a tail of 16 entries zero), in 32 x 32 tiles, grid-strided over the tiles
// blk, blk + nblk, ...  (256 threads).  Entry (r, cc) is c[tri(cc) + r] above
// the diagonal and c[tri(r) + cc] on and below it; tiles wholly above the
// diagonal are read along r into LDS and written along cc, so both the reads
// of c and the writes of C are coalesced.
template <typename T>
__device__ __forceinline__ void expand_sym_body(int n, const double* __restrict__ c, T* __restrict__ cf, int blk,
                                                int nblk) {
  __shared__ double tl[32][33];
  const int tc = (n + 31) / 32;
  const int64_t nt = (int64_t)((n + 32) / 32) * tc;  // (n + 1) rows
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (blk == 0 && threadIdx.x < 16) cf[(int64_t)(n + 1) * n + threadIdx.x] = (T)0;
  for (int64_t t = blk; t < nt; t += nblk) {
    const int r0 = (int)(t / tc) * 32, c0 = (int)(t % tc) * 32;
    if (r0 + 32 <= c0) {
      for (int k = ty; k < 32; k += 8) {
        const int cc = c0 + k;
        tl[k][tx] = cc < n ? c[tri(cc) + r0 + tx] : 0.0;
      }
      __syncthreads();
      for (int k = ty; k < 32; k += 8) {
        const int cc = c0 + tx;
        if (cc < n) cf[(int64_t)(r0 + k) * n + cc] = (T)(tl[tx][k] * kRSqrt2);
      }
      __syncthreads();
    } else {
      for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, cc = c0 + tx;
        if (r > n || cc >= n) continue;
        double v = 0.0;
        if (r < n) {
          v = c[packed(r, cc)];
          if (r != cc) v *= kRSqrt2;
        }
        cf[(int64_t)r * n + cc] = (T)v;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) expand_sym_kernel(IncDev d, const double* __restrict__ c, T* __restrict__ cf) {
  expand_sym_body<T>(d.n_str, c, cf, blockIdx.x, gridDim.x);
}

// A fragments of V for the column kernel, in its LDS image, with the
// diagonal-pair shift.  The rows of each 16-row tile are ordered so that
// accumulator register r of lane L holds pair 16 m + 4 r + L / 16: the
// pair-table entry of k-step 4 m + r that the lane loaded for D, which the
// scatter reuses.  (FP64 MFMA rows already come in that order; FP32 rows come
// as 4 (L / 16) + r, so fragment row rho takes pair 4 (rho % 4) + rho / 4.)
// FP32 fragments are stored two k-steps per lane and entry (one 64-bit LDS
// read per row tile and two k-steps).
template <typename T, int K>
__device__ __forceinline__ void col_frag_body(const double* __restrict__ V, double shift, double nel,
                                              T* __restrict__ vf, int i) {
  typedef ColShape<T, K> SH;
  constexpr int NP = SH::NP, KS = SH::KS;
  constexpr int KP = sizeof(T) == 4 ? 2 * SH::KS2 : KS;  // k-steps stored per row tile (FP32: padded to pairs)
  const double sh = nel > 0.0 ? shift / (nel * nel) : 0.0;
  if (i >= SH::MT * KP * 64) return;
  const int L = i & 63, ms = i >> 6;
  const int m = ms / KP, s = ms - m * KP;
  const int rho = L & 15;
  const int P = 16 * m + (sizeof(T) == 4 ? 4 * (rho & 3) + (rho >> 2) : rho), Q = 4 * s + (L >> 4);
  double v = 0.0;
  if (P < NP && Q < NP && s < KS) {
    v = V[P * NP + Q];
    // diagonal pairs are P = i (i + 3) / 2
    auto diag = [](int x) {
      const int r = (int)((__builtin_sqrt(8.0 * x + 9.0) - 3.0) * 0.5 + 0.5);
      return r * (r + 3) / 2 == x;
    };
    if (diag(P) && diag(Q)) v -= sh;
  }
  if (sizeof(T) == 4)
    vf[((m * SH::KS2 + (s >> 1)) * 64 + L) * 2 + (s & 1)] = (T)v;
  else
    vf[i] = (T)v;
}

template <typename T, int K>
__global__ void __launch_bounds__(256) col_frag_kernel(const double* __restrict__ V, double shift, double nel,
                                                       T* __restrict__ vf) {
  col_frag_body<T, K>(V, shift, nel, vf, blockIdx.x * blockDim.x + threadIdx.x);
}

// Column b of the product (see above); `lds` is the workgroup's dynamic
// LDS.  load_frag: copy the A-fragment image vfg into LDS first (it stays
// there for later columns of the same increment).  Ends with a barrier, so
// the next column may reuse the LDS at once.
template <typename T, int K>
__device__ __forceinline__ void column_body(const int32_t* __restrict__ ptab, const int16_t* __restrict__ ptabT,
                                            const T* __restrict__ cf, const T* __restrict__ vfg,
                                            double* __restrict__ Sm, int b, char* lds, bool load_frag) {
  typedef ColShape<T, K> SH;
  typedef Mfma<T> M;
  constexpr int NP = SH::NP, MT = SH::MT, KS = SH::KS, N = SH::N;
  constexpr bool kNeg = SH::kNeg;
  T* Vf = (T*)lds;
  T* ccol = (T*)(lds + SH::vf_bytes);
  double* S = (double*)(lds + SH::vf_bytes + ((SH::col_bytes + 15) / 16) * 16);
  uint32_t* browl = (uint32_t*)((char*)S + SH::s_bytes);
  T* bsgl = (T*)(browl + 4 * KS);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // the A-fragment image of V (built once per sigma or solve by col_frag_body)
  if (load_frag)
    for (int i = threadIdx.x; i < (int)(SH::vf_bytes / 16); i += blockDim.x)
      ((float4*)Vf)[i] = ((const float4*)vfg)[i];
  // column b of C (row b: C is symmetric), its negation, and S = 0
  for (int j = threadIdx.x; j <= N; j += blockDim.x) {
    const T v = j < N ? cf[(int64_t)b * N + j] : (T)0;
    ccol[j] = v;
    if (kNeg) ccol[N + 1 + j] = -v;
  }
  for (int j = threadIdx.x; j < (kNeg ? 2 : 1) * (N + 1); j += blockDim.x) S[j] = 0.0;
  // beta part of k-step s for lanes with L / 16 = kq: browl[4 s + kq] the
  // offset of row J2 of C (J2 = N, the zero row, for no link), bsgl the sign
  for (int i = threadIdx.x; i < 4 * KS; i += blockDim.x) {
    const int e = i < NP ? ptab[b * NP + i] : -1;
    browl[i] = (uint32_t)((e < 0 ? N : (e >> 1)) * N);
    bsgl[i] = (e >= 0 && (e & 1)) ? (T)-1 : (T)1;
  }
  __syncthreads();

  const int kq = lane >> 4, col = lane & 15;
  const int ntile = (N + 15) / 16;
  for (int t = wave; t < ntile; t += nw) {
    const int jr = 16 * t + col;
    const bool jv = jr < N;
    const int J = jv ? jr : N - 1;
    // pair-table entries of this lane's k-steps (J1 << 1 | neg, J1 = N for
    // no link) and the beta values, all issued first
    // (beta loads run kBD k-steps ahead of their use)
    constexpr int kBD = 8;
    int32_t ent[KS];
    T vb[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int Q = 4 * s + kq;
      ent[s] = Q < NP ? (int)ptabT[Q * N + J] : N;
    }
    auto beta = [&](int s) -> T { return cf[(int64_t)browl[4 * s + kq] + jr]; };
#pragma unroll
    for (int s = 0; s < kBD && s < KS; ++s) vb[s] = beta(s);
    typename M::acc acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = M::zero();
    auto alpha = [&](int s) -> T {
      const int e = ent[s];
      if (kNeg) return ccol[e];
      const bool ng = e > N;
      const T v = ccol[ng ? e - (N + 1) : e];
      return ng ? -v : v;
    };
    T va = alpha(0);
    float2 af[MT];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const T bop = fma_t(bsgl[4 * s + kq], vb[s], va);
      if (s + 1 < KS) va = alpha(s + 1);
      if (s + kBD < KS) vb[s + kBD] = beta(s + kBD);
      if constexpr (sizeof(T) == 4) {
        if ((s & 1) == 0) {
#pragma unroll
          for (int m = 0; m < MT; ++m) af[m] = ((const float2*)Vf)[(m * SH::KS2 + (s >> 1)) * 64 + lane];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        T a;
        if constexpr (sizeof(T) == 4)
          a = (s & 1) == 0 ? af[m].x : af[m].y;
        else
          a = Vf[(m * KS + s) * 64 + lane];
        acc[m] = M::mma(a, bop, acc[m]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // scatter: register r of row tile m holds pair 4 (4 m + r) + kq, whose
    // table entry is ent[4 m + r]; S[E_P J] += s E[P][J]
    if (jv) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int sp = 4 * m + r;
          if (sp < KS && 4 * sp + kq < NP) {
            const int e = ent[sp];
            if (kNeg) {
              if (e != N) lds_add(&S[e], (double)acc[m][r]);
            } else if (e != N) {
              const bool ng = e > N;
              lds_add(&S[ng ? e - (N + 1) : e], ng ? -(double)acc[m][r] : (double)acc[m][r]);
            }
          }
        }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x) Sm[(int64_t)b * N + j] = kNeg ? S[j] - S[N + 1 + j] : S[j];
  __syncthreads();
}

template <typename T, int K>
__global__ void __launch_bounds__(col_threads<T>()) sigma_column_kernel(IncDev d, const double* __restrict__ V,
                                                                   const int32_t* __restrict__ ptab,
                                                                   const int16_t* __restrict__ ptabT,
                                                                   const T* __restrict__ cf,
                                                                   const T* __restrict__ vfg,
                                                                   double* __restrict__ Sm) {
  extern __shared__ __align__(16) char lds[];
  column_body<T, K>(ptab, ptabT, cf, vfg, Sm, blockIdx.x, lds, true);
}

// 16 orbitals (12,870 strings, 136 pairs) do not fit that LDS layout.  The
// split variant keeps the same scheme with the column copy left in L2 (the
// alpha values are read from C, kBD k-steps ahead like the beta values).
// Both precisions keep an FP64 accumulator (103 KB) and take the fragments in
// passes of MTP row tiles (each pass sweeps every tile of the column and
// rebuilds D; the MFMA work is not repeated): FP32 in two passes of 5 + 4
// tiles, FP64 in three of 3.  An FP32 accumulator would leave room for all
// nine FP32 tiles in one pass, but its LDS atomics (ds_add_f32) cost more
// than the second pass: 16o16e FP32 95.5 ms in one pass against 85.8 ms in
// two with ds_add_f64 (waves waiting to issue LDS instructions: 20 % of wave
// time against under 1 %).
template <typename T, int K>
struct ColSplit {
  static constexpr int NP = K * (K + 1) / 2;
  static constexpr int MT = (NP + 15) / 16;
  static constexpr int KS = (NP + 3) / 4;
  static constexpr int KS2 = (KS + 1) / 2;
  static constexpr int N = max_strings(K);
  static constexpr bool kF32 = sizeof(T) == 4;
  static constexpr int MTP = kF32 ? 5 : 3;                // row tiles per pass
  static constexpr int NPASS = (MT + MTP - 1) / MTP;
  static constexpr int KSP = kF32 ? 2 * KS2 : KS;         // k-steps stored per row tile
  typedef double SA;  // accumulator
  static constexpr int64_t vf_bytes = (int64_t)MTP * KSP * 64 * sizeof(T);
  static constexpr int64_t col_bytes = 0;
  static constexpr int64_t s_bytes = ((int64_t)N * sizeof(SA) + 15) / 16 * 16;
  static constexpr int64_t brow_bytes = (int64_t)4 * KS * (4 + sizeof(T));
  static constexpr int64_t lds = vf_bytes + col_bytes + s_bytes + brow_bytes;
};

// Three waves per SIMD in both precisions; FP32 with a shorter load
// lookahead.  FP64 with three waves instead of two: 16o16e 155 -> 140 ms.
template <typename T>
constexpr int split_threads() { return 768; }

// Column b of the split product; ends with a barrier.
template <typename T, int K>
__device__ __forceinline__ void column_split_body(const int32_t* __restrict__ ptab,
                                                  const int16_t* __restrict__ ptabT, const T* __restrict__ cf,
                                                  const T* __restrict__ vfg, double* __restrict__ Sm, int b,
                                                  char* lds) {
  typedef ColSplit<T, K> SH;
  typedef Mfma<T> M;
  typedef typename SH::SA SA;
  constexpr int NP = SH::NP, MT = SH::MT, KS = SH::KS, N = SH::N, MTP = SH::MTP;
  constexpr bool kF32 = SH::kF32;
  static_assert(SH::lds <= kMaxLds, "split column sigma LDS");
  T* Vf = (T*)lds;
  SA* S = (SA*)(lds + SH::vf_bytes + SH::col_bytes);
  uint32_t* browl = (uint32_t*)(lds + SH::vf_bytes + SH::col_bytes + SH::s_bytes);
  T* bsgl = (T*)(browl + 4 * KS);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const T* crow = cf + (int64_t)b * N;  // column b of C (= row b)
  for (int j = threadIdx.x; j < N; j += blockDim.x) S[j] = (SA)0;
  for (int i = threadIdx.x; i < 4 * KS; i += blockDim.x) {
    const int e = i < NP ? ptab[b * NP + i] : -1;
    browl[i] = (uint32_t)((e < 0 ? N : (e >> 1)) * N);
    bsgl[i] = (e >= 0 && (e & 1)) ? (T)-1 : (T)1;
  }
  const int kq = lane >> 4, col = lane & 15;
  const int ntile = (N + 15) / 16;
  static_for<0, SH::NPASS>([&](auto pp) {
    constexpr int m0 = decltype(pp)::value * MTP;
    constexpr int MP = (MT - m0) < MTP ? (MT - m0) : MTP;  // row tiles of this pass
    __syncthreads();  // the previous pass is done with Vf
    for (int i = threadIdx.x; i < (int)((int64_t)MP * SH::KSP * 64 * sizeof(T) / 16); i += blockDim.x)
      ((float4*)Vf)[i] = ((const float4*)(vfg + (int64_t)m0 * SH::KSP * 64))[i];
    __syncthreads();
    for (int t = wave; t < ntile; t += nw) {
      const int jr = 16 * t + col;
      const bool jv = jr < N;
      const int J = jv ? jr : N - 1;
      constexpr int kBD = sizeof(T) == 4 ? 6 : 8;  // loads run kBD k-steps ahead of their use
      // table entries (J + neg (N + 1) <= 2 N < 2^16), two k-steps per register
      constexpr int KE = (KS + 1) / 2;
      uint32_t entp[KE];
      T vb[KS], vaq[KS];
#pragma unroll
      for (int h = 0; h < KE; ++h) {
        const int Q0 = 8 * h + kq, Q1 = Q0 + 4;
        const uint32_t e0 = Q0 < NP ? (uint16_t)ptabT[Q0 * N + J] : (uint32_t)N;
        const uint32_t e1 = Q1 < NP ? (uint16_t)ptabT[Q1 * N + J] : (uint32_t)N;
        entp[h] = e0 | (e1 << 16);
      }
      auto ent = [&](int s) -> int { return (int)((entp[s >> 1] >> (16 * (s & 1))) & 0xffffu); };
      auto beta = [&](int s) -> T { return cf[(int64_t)browl[4 * s + kq] + jr]; };
      // alpha value C[J1][b] (J1 + neg (N + 1) = ent, N: no link), loaded
      // unconditionally (from entry 0 where there is no link) and used times
      // afac(s) = +-1 or 0 at its k-step, so that no branch splits the stream
      // of loads and the waits can count them exactly
      auto alpha = [&](int s) -> T {
        const int e = ent(s);
        const int j1 = e > N ? e - (N + 1) : e;
        return crow[j1 < N ? j1 : 0];
      };
      auto afac = [&](int s) -> T {
        const int e = ent(s);
        const bool ng = e > N;
        return (ng ? e - (N + 1) : e) < N ? (ng ? (T)-1 : (T)1) : (T)0;
      };
#pragma unroll
      for (int s = 0; s < kBD && s < KS; ++s) {
        vb[s] = beta(s);
        vaq[s] = alpha(s);
      }
      typename M::acc acc[MP];
#pragma unroll
      for (int m = 0; m < MP; ++m) acc[m] = M::zero();
      float2 af[MP];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const T bop = fma_t(bsgl[4 * s + kq], vb[s], vaq[s] * afac(s));
        if (s + kBD < KS) {
          vb[s + kBD] = beta(s + kBD);
          vaq[s + kBD] = alpha(s + kBD);
        }
        if constexpr (kF32) {
          if ((s & 1) == 0) {
#pragma unroll
            for (int m = 0; m < MP; ++m) af[m] = ((const float2*)Vf)[(m * SH::KS2 + (s >> 1)) * 64 + lane];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < MP; ++m) {
          T a;
          if constexpr (kF32)
            a = (s & 1) == 0 ? af[m].x : af[m].y;
          else
            a = Vf[(m * KS + s) * 64 + lane];
          acc[m] = M::mma(a, bop, acc[m]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // scatter: register r of row tile m0 + m holds pair 4 (4 (m0 + m) + r)
      // + kq, whose table entry is ent[4 (m0 + m) + r]
      if (jv) {
#pragma unroll
        for (int m = 0; m < MP; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int sp = 4 * (m0 + m) + r;
            if (sp < KS && 4 * sp + kq < NP) {
              const int e = ent(sp);
              if (e != N) {
                const bool ng = e > N;
                const SA v = (SA)acc[m][r];
                lds_add(&S[ng ? e - (N + 1) : e], ng ? -v : v);
              }
            }
          }
      }
    }
  });
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x) Sm[(int64_t)b * N + j] = (double)S[j];
  __syncthreads();
}

template <typename T, int K>
__global__ void __launch_bounds__(split_threads<T>()) sigma_column_split_kernel(
    IncDev d, const int32_t* __restrict__ ptab, const int16_t* __restrict__ ptabT, const T* __restrict__ cf,
    const T* __restrict__ vfg, double* __restrict__ Sm) {
  extern __shared__ __align__(16) char lds[];
  column_split_body<T, K>(ptab, ptabT, cf, vfg, Sm, blockIdx.x, lds);
}

// sigma (packed scaled) = S + S^T from Sm[b][a] = S[a][b], in 32 x 32 tiles
// (ta <= tb) of the upper triangle, grid-strided over the tiles blk, blk +
// nblk, ...  (256 threads).  Sm[a][b] is read along b into LDS; Sm[b][a] and
// sigma[tri(b) + a] along a.
__device__ __forceinline__ int64_t sym_combine_tiles(int n) {
  const int64_t t = (n + 31) / 32;
  return t * (t + 1) / 2;
}
__device__ __forceinline__ void sym_combine_body(const IncDev& d, const double* __restrict__ Sm,
                                                 double* __restrict__ sig, int64_t blk, int64_t nblk) {
  __shared__ double tl[32][33];
  const int n = d.n_str;
  const int64_t nt = sym_combine_tiles(n);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t t = blk; t < nt; t += nblk) {
    int ta, tb;
    unpack(t, &ta, &tb);
    const int a0 = 32 * ta, b0 = 32 * tb;
    for (int k = ty; k < 32; k += 8) {
      const int a = a0 + k, b = b0 + tx;
      tl[k][tx] = (a < n && b < n) ? Sm[(int64_t)a * n + b] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int a = a0 + tx, b = b0 + k;
      if (a <= b && b < n) {
        const double y = Sm[(int64_t)b * n + a];
        sig[tri(b) + a] = a == b ? 2.0 * y : kSqrt2 * (y + tl[tx][k]);
      }
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------- H diagonal
// F(a) = sum_{p in a} h'_pp + 1/2 sum_{p, q in a} (J_pq - K_pq): the energy of
// one spin string; H_(a,b) = F(a) + F(b) + sum_{p in a, q in b} J_pq.
__device__ __forceinline__ void string_energy_body(const IncDev& d, const int32_t* __restrict__ strs,
                                                   const double* __restrict__ B, double* __restrict__ F, int i) {
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

// Packed diagonal HD over the elements blk * blockDim + tid (+ k nblk
// blockDim), the lowest entry of the block (lowest index on ties) in
// part_row[0] (value) and part_row[1] (index); V0, if given, is zeroed over
// the same elements.  Ends with a barrier.
__device__ inline void hdiag_body(const IncDev& d, const int32_t* __restrict__ strs, const double* __restrict__ B,
                                  const double* __restrict__ F, double* __restrict__ HD, double* __restrict__ V0,
                                  double* part_row, int blk, int nblk) {
  __shared__ double red[16];
  __shared__ int64_t redi[16];
  const IntBlock ib = int_block(d.k);
  const int k = d.k;
  double best = 1e300;
  int64_t bi = 0x7fffffffffffffffLL;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < d.n_sym; i += (int64_t)nblk * blockDim.x) {
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
    if (V0) V0[i] = 0.0;
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
    part_row[0] = red[0];
    part_row[1] = (double)redi[0];
  }
  __syncthreads();
}

}  // namespace ifci
