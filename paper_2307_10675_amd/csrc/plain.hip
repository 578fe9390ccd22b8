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
#include <mutex>
#include <set>
#include <utility>

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
// a tail of 16 entries zero).
template <typename T>
__global__ void __launch_bounds__(256) expand_sym_kernel(IncDev d, const double* __restrict__ c, T* __restrict__ cf) {
  const int n = d.n_str;
  const int64_t total = (int64_t)(n + 1) * n + 16;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n;
    const int cc = (int)(i - r * n);
    double v = 0.0;
    if (r < n) {
      const int a = (int)r;
      v = c[packed(a, cc)];
      if (a != cc) v *= kRSqrt2;
    }
    cf[i] = (T)v;
  }
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
__global__ void __launch_bounds__(256) col_frag_kernel(const double* __restrict__ V, double shift, double nel,
                                                       T* __restrict__ vf) {
  typedef ColShape<T, K> SH;
  constexpr int NP = SH::NP, KS = SH::KS;
  constexpr int KP = sizeof(T) == 4 ? 2 * SH::KS2 : KS;  // k-steps stored per row tile (FP32: padded to pairs)
  const double sh = nel > 0.0 ? shift / (nel * nel) : 0.0;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(col_threads<T>()) sigma_column_kernel(IncDev d, const double* __restrict__ V,
                                                                   const int32_t* __restrict__ ptab,
                                                                   const int16_t* __restrict__ ptabT,
                                                                   const T* __restrict__ cf,
                                                                   const T* __restrict__ vfg,
                                                                   double* __restrict__ Sm) {
  typedef ColShape<T, K> SH;
  typedef Mfma<T> M;
  constexpr int NP = SH::NP, MT = SH::MT, KS = SH::KS, N = SH::N;
  constexpr bool kNeg = SH::kNeg;
  extern __shared__ __align__(16) char lds[];
  T* Vf = (T*)lds;
  T* ccol = (T*)(lds + SH::vf_bytes);
  double* S = (double*)(lds + SH::vf_bytes + ((SH::col_bytes + 15) / 16) * 16);
  uint32_t* browl = (uint32_t*)((char*)S + SH::s_bytes);
  T* bsgl = (T*)(browl + 4 * KS);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int b = blockIdx.x;
  // the A-fragment image of V (built once per sigma by col_frag_kernel)
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
}

// 16 orbitals (12,870 strings, 136 pairs) do not fit that LDS layout.  The
// split variant keeps the same scheme with the column copy left in L2 (the
// alpha values are read from C, kBD k-steps ahead like the beta values).
// FP32 keeps all A fragments in LDS (one pass) with an FP32 accumulator (its
// atomic order is not fixed: repeated products agree to FP32 rounding); FP64
// keeps an FP64 accumulator and takes the fragments in passes of MTP row
// tiles (each pass sweeps every tile of the column and rebuilds D; the MFMA
// work is not repeated).
template <typename T, int K>
struct ColSplit {
  static constexpr int NP = K * (K + 1) / 2;
  static constexpr int MT = (NP + 15) / 16;
  static constexpr int KS = (NP + 3) / 4;
  static constexpr int KS2 = (KS + 1) / 2;
  static constexpr int N = max_strings(K);
  static constexpr bool kF32 = sizeof(T) == 4;
  static constexpr int MTP = kF32 ? MT : 3;                // row tiles per pass
  static constexpr int NPASS = (MT + MTP - 1) / MTP;
  static constexpr int KSP = kF32 ? 2 * KS2 : KS;         // k-steps stored per row tile
  typedef typename std::conditional<kF32, float, double>::type SA;  // accumulator
  static constexpr int64_t vf_bytes = (int64_t)MTP * KSP * 64 * sizeof(T);
  static constexpr int64_t col_bytes = 0;
  static constexpr int64_t s_bytes = ((int64_t)N * sizeof(SA) + 15) / 16 * 16;
  static constexpr int64_t brow_bytes = (int64_t)4 * KS * (4 + sizeof(T));
  static constexpr int64_t lds = vf_bytes + col_bytes + s_bytes + brow_bytes;
};

// Three waves per SIMD in both precisions; FP32 with a shorter load
// lookahead (fits the registers of its single pass).  FP64 with three waves
// instead of two: 16o16e 155 -> 140 ms.
template <typename T>
constexpr int split_threads() { return 768; }

template <typename T, int K>
__global__ void __launch_bounds__(split_threads<T>()) sigma_column_split_kernel(
    IncDev d, const int32_t* __restrict__ ptab, const int16_t* __restrict__ ptabT, const T* __restrict__ cf,
    const T* __restrict__ vfg, double* __restrict__ Sm) {
  typedef ColSplit<T, K> SH;
  typedef Mfma<T> M;
  typedef typename SH::SA SA;
  constexpr int NP = SH::NP, MT = SH::MT, KS = SH::KS, N = SH::N, MTP = SH::MTP;
  constexpr bool kF32 = SH::kF32;
  static_assert(SH::lds <= kMaxLds, "split column sigma LDS");
  extern __shared__ __align__(16) char lds[];
  T* Vf = (T*)lds;
  SA* S = (SA*)(lds + SH::vf_bytes + SH::col_bytes);
  uint32_t* browl = (uint32_t*)(lds + SH::vf_bytes + SH::col_bytes + SH::s_bytes);
  T* bsgl = (T*)(browl + 4 * KS);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int b = blockIdx.x;
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
      int32_t ent[KS];
      T vb[KS], vaq[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int Q = 4 * s + kq;
        ent[s] = Q < NP ? (int)ptabT[Q * N + J] : N;
      }
      auto beta = [&](int s) -> T { return cf[(int64_t)browl[4 * s + kq] + jr]; };
      // alpha value C[J1][b] signed, J1 + neg (N + 1) = ent (N: no link)
      auto alpha = [&](int s) -> T {
        const int e = ent[s];
        const bool ng = e > N;
        const int j1 = ng ? e - (N + 1) : e;
        const T v = j1 < N ? crow[j1] : (T)0;
        return ng ? -v : v;
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
        const T bop = fma_t(bsgl[4 * s + kq], vb[s], vaq[s]);
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
              const int e = ent[sp];
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
}

// sigma (packed scaled) = S + S^T from Sm[b][a] = S[a][b].
__global__ void __launch_bounds__(256) sym_combine_kernel(IncDev d, const double* __restrict__ Sm,
                                                          double* __restrict__ sig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n_sym) return;
  int a, b;
  unpack(i, &a, &b);
  const int64_t n = d.n_str;
  sig[i] = a == b ? 2.0 * Sm[(int64_t)a * n + a] : kSqrt2 * (Sm[(int64_t)b * n + a] + Sm[(int64_t)a * n + b]);
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
  hipLaunchKernelGGL(sym_combine_kernel, dim3((unsigned)((d.n_sym + 255) / 256)), dim3(256), 0, st, d, Sm, sig);
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
  hipLaunchKernelGGL(sym_combine_kernel, dim3((unsigned)((d.n_sym + 255) / 256)), dim3(256), 0, st, d, Sm, sig);
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
