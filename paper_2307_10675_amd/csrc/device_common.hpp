// Device helpers shared by the libifci kernels: MFMA wrappers, wavefront and
// workgroup reductions, packed-index arithmetic and the small symmetric
// eigensolver of the Davidson subspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ifci_internal.h"

namespace ifci {

// f(std::integral_constant<int, i>) for i = B .. E-1, unrolled at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// C(k, k/2): the most strings a k-orbital increment can have
__host__ __device__ constexpr int max_strings(int k) {
  int c = 1;
  for (int i = 1; i <= k / 2; ++i) c = c * (k - k / 2 + i) / i;
  return c;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// 16x16x4 tiles.  Lane L holds A[L % 16][L / 16] and B[L / 16][L % 16];
// accumulator register r of lane L holds column L % 16 and row row(L / 16, r):
// 4 r + L / 16 for FP64 (v_mfma_f64_16x16x4f64), 4 (L / 16) + r for FP32
// (v_mfma_f32_16x16x4f32), as measured on gfx950.
template <>
struct Mfma<double> {
  typedef d4 acc;
  static constexpr __host__ __device__ int row(int lane_hi, int r) { return 4 * r + lane_hi; }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef f4 acc;
  static constexpr __host__ __device__ int row(int lane_hi, int r) { return 4 * lane_hi + r; }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV values over the workgroup; every thread gets the totals in out[].
// Deterministic: fixed butterfly inside each wave, waves added in order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) red[wave * NV + j] = v[j];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Same sums with one barrier: every thread adds the per-wave partials itself
// (in the same fixed order) and gets the totals back in v[].  `red` holds two
// buffers of 128 doubles (8 waves x NV <= 16) used alternately (`parity`
// flips each call), so a call never overwrites partials that a slower
// thread may still be reading from the call before.
template <int NV>
__device__ __forceinline__ void block_sum_1b(double (&v)[NV], double* red, int& parity) {
  static_assert(NV <= 16, "two buffers of 8 waves x 16 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* buf = red + parity * 128;
  parity ^= 1;
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) buf[wave * NV + j] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += buf[w * NV + j];
    v[j] = s;
  }
}

// Packed upper-triangle index: entry (a, b), a <= b, lives at b (b + 1) / 2 + a.
__device__ __forceinline__ int64_t packed(int64_t a, int64_t b) {
  return a <= b ? tri(b) + a : tri(a) + b;
}
// 32-bit variant for indices below 2^24 (single-precision square root, then
// an exact integer correction).
__device__ __forceinline__ void unpack32(int i, int* a, int* b) {
  int c = (int)((__builtin_sqrtf(8.0f * (float)i + 1.0f) - 1.0f) * 0.5f);
  if (((c + 1) * (c + 2)) / 2 <= i) ++c;
  if ((c * (c + 1)) / 2 > i) --c;
  *b = c;
  *a = i - (c * (c + 1)) / 2;
}
__device__ __forceinline__ void unpack(int64_t i, int* a, int* b) {
  int64_t c = (int64_t)((sqrt(8.0 * (double)i + 1.0) - 1.0) * 0.5);
  while (tri(c + 1) <= i) ++c;
  while (tri(c) > i) --c;
  *b = (int)c;
  *a = (int)(i - tri(c));
}

// Atomic add into LDS (ds_add_f64).  The pointer must point into LDS.
typedef __attribute__((address_space(3))) double lds_double;
__device__ __forceinline__ void lds_add(double* p, double v) {
  __atomic_fetch_add((lds_double*)p, v, __ATOMIC_RELAXED);
}

constexpr double kSqrt2 = 1.4142135623730950488;
constexpr double kRSqrt2 = 0.70710678118654752440;

// Eigen-decomposition of the symmetric n x n matrix A (row stride 16,
// n <= 16) by parallel cyclic Jacobi (Golub & Van Loan, symmetric Schur
// rotations in the Brent-Luk circle ordering), accumulating the rotations
// into Q (stride 16), which the caller initialises (identity, or
// eigenvectors of a previous nearby matrix to warm start).  An odd n is
// padded with a decoupled index whose diagonal entry lies far above the
// spectrum (its row and column of A and Q are overwritten).  Each round
// rotates N / 2 disjoint planes at once: lanes below N / 2 compute the
// planes' rotations and pass them on by shuffles, lane L updates the 2 x 2
// block (L / 8, L % 8) of A and rows L / 8 and L / 8 + 8 of Q in plane L % 8.
// Pivots below 1e-15 ||A||_F are not rotated (FP64 rounding keeps
// regenerating off-diagonal noise near 1e-16 ||A||); sweeps stop after one
// whose squared pivots sum below 1e-24 ||A||_F^2 (the quadratic convergence
// of the cyclic method leaves the off-diagonal part at rounding level after
// such a sweep).  Executed by one
// full wavefront, which orders its own LDS accesses, so no workgroup
// barrier is needed.  Returns the sorted eigenvalues in evals, their
// columns of Q in perm, and the lowest pair in theta / y.
__device__ inline void jacobi_warm(double* A, double* Q, int n, double* theta, double* y, double* evals,
                                   int* perm) {
  const int lane = threadIdx.x & 63;
  const int N = n + (n & 1), H = N >> 1, m = N - 1;
  __builtin_amdgcn_wave_barrier();
  double f2 = 0.0;
  if (lane < n)
    for (int j = 0; j < n; ++j) f2 += A[lane * 16 + j] * A[lane * 16 + j];
  f2 = wave_sum(f2);
  if (n & 1) {
    // decoupled padding index n
    const double big = 1e3 * (1.0 + sqrt(f2));
    if (lane < 16) {
      A[lane * 16 + n] = (lane == n) ? big : 0.0;
      A[n * 16 + lane] = (lane == n) ? big : 0.0;
      Q[lane * 16 + n] = (lane == n) ? 1.0 : 0.0;
      Q[n * 16 + lane] = (lane == n) ? 1.0 : 0.0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  const double tol = 1e-15 * sqrt(f2);
  const int kr = lane >> 3, kc = lane & 7;
  const bool blk = kr < H && kc < H;
  for (int sweep = 0; sweep < 12 && N > 1; ++sweep) {
    double piv2 = 0.0;
    for (int s = 0; s < m; ++s) {
      // plane k of round s: (P - 1, s) for k = 0, else (s + k, s - k) mod (N - 1)
      auto plane = [&](int k, int* p, int* q) {
        int x, yv;
        if (k == 0) {
          x = m;
          yv = s;
        } else {
          x = s + k;
          if (x >= m) x -= m;
          yv = s - k + m;
          if (yv >= m) yv -= m;
        }
        *p = x < yv ? x : yv;
        *q = x < yv ? yv : x;
      };
      double c = 1.0, sn = 0.0;
      if (lane < H) {
        int p, q;
        plane(lane, &p, &q);
        const double apq = A[p * 16 + q];
        piv2 += apq * apq;
        if (fabs(apq) > tol) {
          const double tau = (A[q * 16 + q] - A[p * 16 + p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
        }
      }
      const double c1 = __shfl(c, kr & 7, 64), s1 = __shfl(sn, kr & 7, 64);
      const double c2 = __shfl(c, kc, 64), s2 = __shfl(sn, kc, 64);
      __builtin_amdgcn_wave_barrier();
      if (blk) {
        int p1, q1, p2, q2;
        plane(kr, &p1, &q1);
        plane(kc, &p2, &q2);
        const double a = A[p1 * 16 + p2], b = A[p1 * 16 + q2], e = A[q1 * 16 + p2], f = A[q1 * 16 + q2];
        const double a1 = c2 * a - s2 * b, b1 = s2 * a + c2 * b;
        const double e1 = c2 * e - s2 * f, f1 = s2 * e + c2 * f;
        A[p1 * 16 + p2] = c1 * a1 - s1 * e1;
        A[q1 * 16 + p2] = s1 * a1 + c1 * e1;
        A[p1 * 16 + q2] = c1 * b1 - s1 * f1;
        A[q1 * 16 + q2] = s1 * b1 + c1 * f1;
      }
      if (kc < H) {
        int p, q;
        plane(kc, &p, &q);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = kr + 8 * h;
          if (i < N) {
            const double vp = Q[i * 16 + p], vq = Q[i * 16 + q];
            Q[i * 16 + p] = c2 * vp - s2 * vq;
            Q[i * 16 + q] = s2 * vp + c2 * vq;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    piv2 = wave_sum(piv2);
    if (!(piv2 > 1e-24 * f2)) break;
  }
  __builtin_amdgcn_wave_barrier();
  // eigenvalues in increasing order (ties by index): perm[i] is the column
  // of Q holding the i-th lowest; lane j finds the rank of eigenvalue j
  if (lane < n) {
    const double vj = A[lane * 16 + lane];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double vi = A[i * 16 + i];
      rank += (vi < vj || (vi == vj && i < lane)) ? 1 : 0;
    }
    perm[rank] = lane;
    evals[rank] = vj;
    if (rank == 0) *theta = vj;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < n) y[lane] = Q[lane * 16 + perm[0]];
  __builtin_amdgcn_wave_barrier();
}

// Cold-start variant: Q = I, then jacobi_warm.
__device__ inline void jacobi_lowest(double* A, double* Q, int n, double* theta, double* y, double* evals,
                                     int* perm) {
  const int lane = threadIdx.x & 63;
  if (lane < 16)
    for (int j = 0; j < 16; ++j) Q[lane * 16 + j] = (lane == j) ? 1.0 : 0.0;
  jacobi_warm(A, Q, n, theta, y, evals, perm);
}

}  // namespace ifci
