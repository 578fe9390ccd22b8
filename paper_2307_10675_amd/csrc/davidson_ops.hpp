// Steps of the device-wide Davidson iteration (Davidson, J. Comput. Phys. 17,
// 87, 1975; thick restart, DGKS re-orthogonalisation), written once and used
// by the per-increment host-driven loop and by the batched solver that runs
// many increments per launch with device-side control.  Internal.
//
// Vector steps work on packed scaled symmetric vectors of length ns (entry
// (a <= b) at b (b + 1) / 2 + a, off-diagonals times sqrt 2, so plain dot
// products are those of the full vectors).  A step covers the elements
// blk * blockDim + tid + k * nblk * blockDim of one increment and writes its
// partial sums to part[blk][kNV]; the small steps then reduce the nblk
// partials in a fixed order, so results do not depend on how the blocks of a
// launch are scheduled.
#pragma once

#include "device_common.hpp"

namespace ifci {

// Solver state of one increment (device memory, one block of 4096 doubles).
struct DavState {
  double G[256];   // Rayleigh matrix V^T H V (stride 16)
  double Gs[256];  // its copy, diagonalised in place
  double Q[256];   // eigenvectors of Gs
  double y[16];    // lowest Ritz vector in the subspace basis
  double cf[16];   // V^T t (first orthogonalisation pass)
  double c2[16];   // V^T t (second pass)
  double ev[16];   // Ritz values, increasing
  double theta, E0, resid, tt0, tt, dx, inv, ecore;
  int m, phase, iters, status, restart, action, mb, reorth;
  int guess, keep, alive, pad[5];
  int perm[16];
};

// action codes written by the residual test (small_A)
enum { kActContinue = 0, kActDone = 1, kActSwitch = 2, kActMaxIter = 3, kActEvicted = 4 };

constexpr int kPartBlocks = 1024;
constexpr int kNV = kMaxSpace + 3;

// Partial sums of nv values of this block into part_row[0..nv).  Ends with a
// barrier, so `red` may be reused right away.
__device__ inline void block_partial_row(double (&v)[kNV], int nv, double* part_row, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < kNV; ++j)
    if (j < nv) v[j] = wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < kNV; ++j)
      if (j < nv) red[wave * kNV + j] = v[j];
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * kNV + threadIdx.x];
    part_row[threadIdx.x] = s;
  }
  __syncthreads();
}

// Sum of nblk partial rows, value j in out[j] (LDS) for j < nv.  Run by
// one wavefront: lane t adds the rows t, t + 64, ... in order, then a fixed
// butterfly adds the lanes, so the result does not depend on scheduling and
// the row loads of a lane are independent of each other.
__device__ inline void reduce_parts(const double* part, int nblk, int nv, double* out) {
  const int lane = threadIdx.x & 63;
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int b = lane; b < nblk; b += 64)
#pragma unroll
    for (int j = 0; j < kNV; ++j)
      if (j < nv) acc[j] += part[b * kNV + j];
#pragma unroll
  for (int j = 0; j < kNV; ++j)
    if (j < nv) acc[j] = wave_sum(acc[j]);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < kNV; ++j)
      if (j < nv) out[j] = acc[j];
  __syncthreads();
}

// ---------------------------------------------------------------- vector steps
// part_row[j] = V_j . s for j <= m
__device__ inline void op_dots(const double* __restrict__ Vb, int64_t st, int m, const double* __restrict__ s,
                               int64_t ns, double* part_row, int blk, int nblk, double* red) {
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) {
    const double si = s[i];
#pragma unroll
    for (int j = 0; j < kMaxSpace; ++j)
      if (j <= m) acc[j] += Vb[j * st + i] * si;
  }
  block_partial_row(acc, m + 1, part_row, red);
}

// Ritz vector x = V y, residual r = S y - theta x, preconditioned
// t = r / (theta - (H_II - E0)) (denominator clamped at 1e-8); stores x and
// t; partials: V_j . t (j <= m), then r.r, t.t, x.t.  `ysh` is 16 doubles of
// LDS.
__device__ inline void op_passA(const DavState* __restrict__ S, const double* __restrict__ Vb,
                                const double* __restrict__ Sb, int64_t st, const double* __restrict__ HD,
                                double* __restrict__ X, double* __restrict__ T, int64_t ns, double* part_row,
                                int blk, int nblk, double* red, double* ysh) {
  const int m = S->m;
  const double theta = S->theta, E0 = S->E0;
  if (threadIdx.x < 16) ysh[threadIdx.x] = S->y[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) {
    double x = 0.0, sx = 0.0;
    for (int j = 0; j <= m; ++j) {
      x += ysh[j] * Vb[j * st + i];
      sx += ysh[j] * Sb[j * st + i];
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
  block_partial_row(out, m + 4, part_row, red);
}

// Thick restart: V[k] <- sum_j Q[j][perm k] V[j] for the `keep` lowest Ritz
// vectors, the same for S.  `qsh` is kMaxSpace * kKeep doubles of LDS.
__device__ inline void op_restart(const DavState* __restrict__ S, double* Vb, double* Sb, int64_t st, int64_t ns,
                                  int blk, int nblk, double* qsh) {
  const int m = S->m, keep = S->keep;
  for (int t = threadIdx.x; t < kMaxSpace * kKeep; t += blockDim.x) {
    const int j = t / kKeep, kk = t % kKeep;
    qsh[t] = (j <= m && kk < keep) ? S->Q[j * 16 + S->perm[kk]] : 0.0;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) {
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
          for (int j = 0; j < kMaxSpace; ++j) v += qsh[j * kKeep + kk] * vv[j];
          B[kk * st + i] = v;
        }
      }
    }
  }
  __syncthreads();
}

// Start of the FP64 stage: V[0] <- x; block 0 clears G and sets phase 64, m 0.
__device__ inline void op_switch(DavState* S, double* Vb, const double* X, int64_t ns, int blk, int nblk) {
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) Vb[i] = X[i];
  if (blk == 0) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) S->G[i] = 0.0;
    if (threadIdx.x == 0) {
      S->phase = 64;
      S->m = 0;
    }
  }
}

// First orthogonalisation pass: t -= sum_{j <= mb} cf[j] V_j; partials
// V_j . t (j <= mb) and t.t.  `csh` is 16 doubles of LDS.
__device__ inline void op_passB(const DavState* __restrict__ S, const double* __restrict__ Vb, int64_t st,
                                double* __restrict__ T, int64_t ns, double* part_row, int blk, int nblk, double* red,
                                double* csh) {
  const int mb = S->mb;
  if (threadIdx.x < 16) csh[threadIdx.x] = S->cf[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) {
    double t = T[i];
    for (int j = 0; j <= mb; ++j) t -= csh[j] * Vb[j * st + i];
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
  block_partial_row(out, mb + 2, part_row, red);
}

// Second (DGKS) pass, run when the first lost more than half the norm:
// t -= sum c2[j] V_j; partial t.t.
__device__ inline void op_passC(const DavState* __restrict__ S, const double* __restrict__ Vb, int64_t st,
                                double* __restrict__ T, int64_t ns, double* part_row, int blk, int nblk, double* red,
                                double* csh) {
  const int mb = S->mb;
  if (threadIdx.x < 16) csh[threadIdx.x] = S->c2[threadIdx.x];
  __syncthreads();
  double acc[kNV];
#pragma unroll
  for (int j = 0; j < kNV; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x) {
    double t = T[i];
    for (int j = 0; j <= mb; ++j) t -= csh[j] * Vb[j * st + i];
    T[i] = t;
    acc[0] += t * t;
  }
  block_partial_row(acc, 1, part_row, red);
}

// V[mb + 1] <- t / ||t||
__device__ inline void op_normalize(const DavState* __restrict__ S, double* Vb, int64_t st,
                                    const double* __restrict__ T, int64_t ns, int blk, int nblk) {
  const double inv = S->inv;
  const int mn = S->mb + 1;
  for (int64_t i = (int64_t)blk * blockDim.x + threadIdx.x; i < ns; i += (int64_t)nblk * blockDim.x)
    Vb[mn * st + i] = T[i] * inv;
}

// ---------------------------------------------------------------- small steps
// One wavefront (64 threads) per increment.  `sh` is kNV doubles of LDS.

// New column of the Rayleigh matrix from the partials of op_dots, then its
// lowest eigenpair (cyclic Jacobi); counts the iteration and decides whether
// the next orthogonalisation is preceded by a thick restart.
__device__ inline void small_G(DavState* S, const double* part, int nblk, int mmax, double* g) {
  const int m = S->m;
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

// Residual test on the partials of op_passA: decides the action (continue,
// done, switch to the FP64 stage, out of iterations, evicted).
__device__ inline void small_A(DavState* S, const double* part, int nblk, double tol32, double tol64, int max_iter,
                               int evict, double* v) {
  const int m = S->m;
  reduce_parts(part, nblk, m + 4, v);
  if (threadIdx.x == 0) {
    const double rr = v[m + 1];
    S->resid = sqrt(rr);
    S->tt0 = v[m + 2];
    S->dx = v[m + 3];
    for (int j = 0; j < 16; ++j) S->cf[j] = (j <= m) ? v[j] : 0.0;
    S->mb = m;
    const double tol = S->phase == 32 ? tol32 : tol64;
    int action = kActContinue;
    if (evict) {
      action = kActEvicted;
      S->status = IFCI_INC_EVICTED;
    } else if (S->resid <= tol) {
      if (S->phase == 32) {
        action = (S->iters >= max_iter) ? kActMaxIter : kActSwitch;
      } else {
        action = kActDone;
        S->status = IFCI_INC_DONE;
      }
    } else if (S->iters >= max_iter) {
      action = kActMaxIter;
    }
    S->action = action;
  }
}

// After a thick restart: the kept Ritz vectors are the new basis, their
// Ritz values the diagonal of G, and cf is re-expressed in that basis.
__device__ inline void small_R(DavState* S) {
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

__device__ inline void small_B(DavState* S, const double* part, int nblk, double* v) {
  const int mb = S->mb;
  reduce_parts(part, nblk, mb + 2, v);
  if (threadIdx.x == 0) {
    const double tt = v[mb + 1];
    S->tt = tt;
    S->reorth = tt < 0.5 * S->tt0;
    for (int j = 0; j < 16; ++j) S->c2[j] = (j <= mb) ? v[j] : 0.0;
    S->inv = tt > 0.0 ? 1.0 / sqrt(tt) : 0.0;
  }
}

__device__ inline void small_C(DavState* S, const double* part, int nblk, double* v) {
  reduce_parts(part, nblk, 1, v);
  if (threadIdx.x == 0) {
    S->tt = v[0];
    S->inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
  }
}

}  // namespace ifci
