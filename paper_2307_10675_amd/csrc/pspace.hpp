// P-space preconditioner and initial guess of the on-chip three-vector
// solver.  Internal.
//
// The P determinants of the symmetric sector with the lowest diagonal
// entries span a block H_PP of the Hamiltonian that carries most of the
// coupling among the low-energy configurations.  It is built once per
// increment from the Slater-Condon rules over the embedded active-space
// integrals and diagonalised, H_PP - E0 = U diag(lam) U^T.  Its lowest
// eigenvector is the initial guess, and each iteration the correction on
// those P entries is the exact inverse of the shifted block,
// t_P = U diag(1 / (theta - lam)) U^T r_P, while every other entry keeps
// the diagonal correction r_I / (theta - (H_II - E0)).  This is the block
// preconditioner of Davidson-type CI solvers (the diagonal one with a
// small exactly treated subspace); it changes how fast the iteration
// converges, not what it converges to.
#pragma once

#include "device_common.hpp"
#include "ifci_internal.h"

namespace ifci {

// Active-space integrals as the on-chip solver holds them: V[P][Q] =
// (pq|rs) / 2 + [r = s] k_pq / N over unordered pairs, k = h' - 1/2 sum_r
// (pr|rq), h'_pq the frozen-core one-electron operator (hp, computed once),
// J_pq = (pp|qq), K_pq = (pq|qp).
struct ActInts {
  const double* V;     // [np][np]
  const double* keff;  // [k][k]
  const double* hp;    // [k][k]
  const double* Jm;
  const double* Km;
  int k, np;
  double inv_nel;  // 1 / N (0 for an empty space)
};

__device__ __forceinline__ int pair_index(int p, int q) {
  return p >= q ? ((p * (p + 1)) >> 1) + q : ((q * (q + 1)) >> 1) + p;
}

// (pq|rs) of the active space
__device__ __forceinline__ double aeri(const ActInts& I, int p, int q, int r, int s) {
  double v = I.V[pair_index(p, q) * I.np + pair_index(r, s)];
  if (r == s) v -= I.keff[p * I.k + q] * I.inv_nel;
  return 2.0 * v;
}

// (-1)^(occupied orbitals of s strictly between p and q): the sign of E_pq
// on a string holding q (and not p)
__device__ __forceinline__ double e_sign(uint32_t s, int p, int q) {
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  const uint32_t m = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
  return (__popc(s & m) & 1) ? -1.0 : 1.0;
}

// One-electron-like part of a single replacement q -> p in one spin whose
// string (before) is s, with the other spin's string o:
// h'_pq + sum_{r in s, r != q} [(pq|rr) - (pr|rq)] + sum_{r in o} (pq|rr).
__device__ inline double single_value(const ActInts& I, uint32_t s, uint32_t o, int p, int q) {
  double v = I.hp[p * I.k + q];
  for (int r = 0; r < I.k; ++r) {
    if ((s >> r & 1u) && r != q) v += aeri(I, p, q, r, r) - aeri(I, p, r, r, q);
    if (o >> r & 1u) v += aeri(I, p, q, r, r);
  }
  return v;
}

// Same-spin double replacement (q1, q2) -> (p1, p2) of string s:
// sign x [(p1 q1|p2 q2) - (p1 q2|p2 q1)], the sign that of E_p1q1 E_p2q2 on s.
__device__ inline double double_value(const ActInts& I, uint32_t s, uint32_t t) {
  const uint32_t an = s & ~t, cr = t & ~s;
  const int q1 = __ffs(an) - 1, q2 = 31 - __clz(an);
  const int p1 = __ffs(cr) - 1, p2 = 31 - __clz(cr);
  const double s1 = e_sign(s, p2, q2);
  const uint32_t s2str = (s & ~(1u << q2)) | (1u << p2);
  const double s2 = e_sign(s2str, p1, q1);
  return s1 * s2 * (aeri(I, p1, q1, p2, q2) - aeri(I, p1, q2, p2, q1));
}

// <C,D|H|A,B> (active-space H without the frozen-core energy) between the
// determinants (alpha string, beta string) = (C, D) and (A, B), given as
// indices into the string list; F holds the string energies, so the
// diagonal is F(a) + F(b) + sum_{p in a, q in b} J_pq.
__device__ inline double det_element(const ActInts& I, const int32_t* strs, const double* F, int ci, int di,
                                     int ai, int bi) {
  const uint32_t A = (uint32_t)strs[ai], B = (uint32_t)strs[bi], C = (uint32_t)strs[ci], D = (uint32_t)strs[di];
  const int na = __popc(A ^ C) >> 1, nb = __popc(B ^ D) >> 1;
  if (na + nb > 2) return 0.0;
  if (na + nb == 0) {
    double v = F[ai] + F[bi];
    for (int p = 0; p < I.k; ++p) {
      if (!(A >> p & 1u)) continue;
      for (int q = 0; q < I.k; ++q)
        if (B >> q & 1u) v += I.Jm[p * I.k + q];
    }
    return v;
  }
  if (na == 1 && nb == 0) {
    const int q = __ffs(A & ~C) - 1, p = __ffs(C & ~A) - 1;
    return e_sign(A, p, q) * single_value(I, A, B, p, q);
  }
  if (na == 0 && nb == 1) {
    const int q = __ffs(B & ~D) - 1, p = __ffs(D & ~B) - 1;
    return e_sign(B, p, q) * single_value(I, B, A, p, q);
  }
  if (na == 2) return double_value(I, A, C);
  if (nb == 2) return double_value(I, B, D);
  // one alpha and one beta replacement: (pq|rs) with the two string signs
  const int q = __ffs(A & ~C) - 1, p = __ffs(C & ~A) - 1;
  const int s = __ffs(B & ~D) - 1, r = __ffs(D & ~B) - 1;
  return e_sign(A, p, q) * e_sign(B, r, s) * aeri(I, p, q, r, s);
}

// <i|H|j> between the orthonormal symmetric-sector states of packed entries
// i = (a <= b) and j = (c <= d): |a,a>, or (|a,b> + |b,a>) / sqrt 2.  With
// the alpha-beta exchange symmetry of H (<b,a|H|d,c> = <a,b|H|c,d> for equal
// alpha and beta counts) the four terms fold into two.
__device__ inline double sector_element(const ActInts& I, const int32_t* strs, const double* F, int i, int j) {
  int a, b, c, d;
  unpack32(i, &a, &b);
  unpack32(j, &c, &d);
  if (a == b && c == d) return det_element(I, strs, F, a, a, c, c);
  if (a == b) return kSqrt2 * det_element(I, strs, F, a, a, c, d);
  if (c == d) return kSqrt2 * det_element(I, strs, F, a, b, c, c);
  return det_element(I, strs, F, a, b, c, d) + det_element(I, strs, F, a, b, d, c);
}

// Pair k of round s of the circle schedule over P (even) indices: every
// pair appears once in P - 1 rounds and the P / 2 pairs of a round are
// disjoint.  Pair 0 holds P - 1 and s; pair k > 0 holds (s + k) and
// (s - k) mod (P - 1).  Returned as p < q.
__device__ __forceinline__ void round_pair(int P, int s, int k, int* p, int* q) {
  const int m = P - 1;
  int x, y;
  if (k == 0) {
    x = m;
    y = s;
  } else {
    x = s + k;
    if (x >= m) x -= m;
    y = s - k + m;
    if (y >= m) y -= m;
  }
  *p = x < y ? x : y;
  *q = x < y ? y : x;
}

// Rotation (c, s) of the Jacobi step that zeroes a_pq of the 2 x 2 block
// [[a_pp, a_pq], [a_pq, a_qq]] (Golub & Van Loan, the symmetric Schur
// decomposition): t = tan of the angle, the smaller root of
// t^2 + 2 tau t - 1 = 0 with tau = (a_qq - a_pp) / (2 a_pq).
__device__ __forceinline__ void schur_rotation(float app, float aqq, float apq, float* c, float* s) {
  if (apq == 0.0f) {
    *c = 1.0f;
    *s = 0.0f;
    return;
  }
  const float tau = (aqq - app) / (2.0f * apq);
  const float at = fabsf(tau);
  const float t = (tau >= 0.0f ? 1.0f : -1.0f) / (at > 1e15f ? 2.0f * at : at + sqrtf(1.0f + tau * tau));
  *c = 1.0f / sqrtf(1.0f + t * t);
  *s = t * *c;
}

// Eigen-decomposition of the symmetric P x P matrix A (LDS, row-major, FP32,
// P even, at most 64) by parallel cyclic Jacobi: rounds of the circle
// schedule rotate P / 2 disjoint planes at once, U (LDS, starts as I)
// accumulates the rotations, and a sweep of P - 1 rounds visits every
// plane once.  Sweeps stop when the squared off-diagonal part falls below
// tol2 of the squared norm of A, or after 12 sweeps.  On return A[j][j]
// are the eigenvalues and column j of U the eigenvectors.
//
// A round: the first P / 2 threads compute the planes' rotations into cs
// and their index pairs into pq; a barrier; every thread updates the 2 x 2
// blocks of A and the (row, plane) entries of U it owns for the whole call
// (at most two blocks and four entries at 512 threads); a barrier.
// cs: LDS [2 P] floats, pq: LDS [P] ints; red, parity: the reduction buffer
// of block_sum_1b and its parity.
__device__ inline void block_jacobi(float* A, float* U, int P, float* cs, int* pq, double* red, int& parity,
                                    double tol2) {
  constexpr int kBlk = 2, kRow = 4;
  static_assert(kBlk * kBatchThreads >= (kPsMax / 2) * (kPsMax / 2) && kRow * kBatchThreads >= kPsMax * kPsMax / 2,
                "every block and U entry has an owner");
  const int tid = threadIdx.x, nt = kBatchThreads, H = P / 2;
  int br[kBlk], bc[kBlk], ui[kRow], uk[kRow];
#pragma unroll
  for (int j = 0; j < kBlk; ++j) {
    const int t = tid + j * nt;
    br[j] = t < H * H ? t / H : -1;
    bc[j] = t < H * H ? t - (t / H) * H : 0;
  }
#pragma unroll
  for (int j = 0; j < kRow; ++j) {
    const int t = tid + j * nt;
    ui[j] = t < P * H ? t / H : -1;
    uk[j] = t < P * H ? t - (t / H) * H : 0;
  }
  for (int t = tid; t < P * P; t += nt) U[t] = (t / P == t % P) ? 1.0f : 0.0f;
  __syncthreads();
  for (int sweep = 0; sweep < 12; ++sweep) {
    double acc[2] = {0.0, 0.0};
    for (int t = tid; t < P * P; t += nt) {
      const double v = (double)A[t];
      acc[0] += (t / P == t % P) ? 0.0 : v * v;
      acc[1] += v * v;
    }
    block_sum_1b<2>(acc, red, parity);
    if (!(acc[0] > tol2 * acc[1])) break;
    for (int s = 0; s < P - 1; ++s) {
      if (tid < H) {
        int p, q;
        round_pair(P, s, tid, &p, &q);
        float c, sn;
        schur_rotation(A[p * P + p], A[q * P + q], A[p * P + q], &c, &sn);
        cs[2 * tid] = c;
        cs[2 * tid + 1] = sn;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kBlk; ++j) {
        if (br[j] < 0) continue;
        const int kr = br[j], kc = bc[j];
        const int p1 = pq[2 * kr], q1 = pq[2 * kr + 1], p2 = pq[2 * kc], q2 = pq[2 * kc + 1];
        const float c1 = cs[2 * kr], s1 = cs[2 * kr + 1], c2 = cs[2 * kc], s2 = cs[2 * kc + 1];
        const float a = A[p1 * P + p2], b = A[p1 * P + q2], e = A[q1 * P + p2], f = A[q1 * P + q2];
        // columns (p2, q2), then rows (p1, q1)
        const float a1 = c2 * a - s2 * b, b1 = s2 * a + c2 * b;
        const float e1 = c2 * e - s2 * f, f1 = s2 * e + c2 * f;
        A[p1 * P + p2] = c1 * a1 - s1 * e1;
        A[q1 * P + p2] = s1 * a1 + c1 * e1;
        A[p1 * P + q2] = c1 * b1 - s1 * f1;
        A[q1 * P + q2] = s1 * b1 + c1 * f1;
      }
#pragma unroll
      for (int j = 0; j < kRow; ++j) {
        if (ui[j] < 0) continue;
        const int i = ui[j], k = uk[j];
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const float c = cs[2 * k], sn = cs[2 * k + 1];
        const float up = U[i * P + p], uq = U[i * P + q];
        U[i * P + p] = c * up - sn * uq;
        U[i * P + q] = sn * up + c * uq;
      }
      __syncthreads();
    }
  }
}

}  // namespace ifci
