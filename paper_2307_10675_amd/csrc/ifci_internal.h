// Internal structures shared by the host plan and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ifci.h"

namespace ifci {

constexpr int kMaxAct = 16;      // largest active space (orbitals)
constexpr int kMaxSpace = 16;    // largest Davidson subspace
constexpr int kKeep = 4;         // Ritz vectors kept at a thick restart
constexpr int kBatchThreads = 512;

// Device-side description of one increment.  Offsets count elements of the
// blob they index (int32 for tables/orbitals, double for workspace regions).
struct IncDev {
  int32_t k;       // active orbitals
  int32_t na;      // alpha (= beta) electrons
  int32_t n_str;   // C(k, na)
  int32_t npair;   // k (k + 1) / 2
  int32_t n_link;  // na (k - na + 1)
  int32_t n_core;
  int32_t id;      // canonical increment index
  int32_t mspace;  // subspace vectors of this increment's Davidson block
  int64_t n_det;   // n_str^2
  int64_t n_sym;   // n_str (n_str + 1) / 2
  int64_t stride;  // padded n_sym used for packed vectors
  int64_t act_off;   // int32 offset into the orbital blob (k active orbitals)
  int64_t core_off;  // int32 offset into the orbital blob (n_core core orbitals)
  int64_t str_off;   // int32 offset into the table blob: strings [n_str]
  int64_t pair_off;  // int32 offset: pair table [n_str][npair], (J << 1 | neg) or -1
  int64_t link_off;  // int32 offset: compact links [n_str][n_link], (Q << 17 | J << 1 | neg)
  int64_t ord_off;   // int32 offset: ordered table [n_str][k*k]: E_pq|I> -> (J << 1 | neg) or -1
  int64_t pairT_off; // int32 offset: pair table pair-major, int16 [npair][n_str], J + neg (n_str + 1), n_str: none
  int64_t int_off;   // double offset into the integral region
  int64_t vec_off;   // double offset into the Davidson region
};

// Layout of one increment's embedded-integral block (doubles from int_off).
__host__ __device__ inline int64_t int_block_size(int k) {
  int64_t np = (int64_t)k * (k + 1) / 2;
  int64_t s = np * np + 3 * (int64_t)k * k + k + 4;
  return (s + 7) & ~int64_t(7);
}
struct IntBlock {
  int64_t V, keff, J, K, hd, misc;  // misc[0] = E_core, misc[1] = N electrons
};
__host__ __device__ inline IntBlock int_block(int k) {
  int64_t np = (int64_t)k * (k + 1) / 2;
  IntBlock b;
  b.V = 0;
  b.keff = np * np;
  b.J = b.keff + (int64_t)k * k;
  b.K = b.J + (int64_t)k * k;
  b.hd = b.K + (int64_t)k * k;
  b.misc = b.hd + k;
  return b;
}

// Largest P-space block of the on-chip three-vector solver.
constexpr int kPsMax = 64;

// Davidson storage of one increment (doubles from vec_off): basis V[mmax],
// sigma S[mmax], diagonal, converged vector X, each `stride` long; then the
// FP32 eigenvector image of the P-space block (kPsMax^2 floats).
__host__ __device__ inline int64_t vec_block_size(int64_t stride, int mmax) {
  return (2 * (int64_t)mmax + 2) * stride + kPsMax * kPsMax / 2;
}
__host__ __device__ inline int64_t ps_image_offset(int64_t stride, int mmax) {
  return (2 * (int64_t)mmax + 2) * stride;
}

// Per-shape settings of the on-chip solvers (k = active orbitals 1..8,
// precision 0 = FP64 sigma, 1 = FP32 sigma), chosen by a tuner and handed
// over through ifci_set_tuning; -1 / 0 keep the built-in choice.
constexpr int kTuneK = 8;
struct Tuning {
  int8_t ps_block[kTuneK + 1][2];  // P-space block size (-1: n_guess)
  int8_t e_waves[kTuneK + 1][2];   // waves contracting E slices (0: all that fit)
};

struct SolveArgs {
  const IncDev* inc;
  const int32_t* order;   // which increments, heaviest first
  int32_t count;
  int32_t precision;
  int32_t max_iter;
  int32_t max_space;
  int32_t n_guess;        // P-space block of the three-vector solver (0 or 1: none)
  double r_tol;
  double r_tol_inner;
  const int32_t* tables;
  double* ints;
  double* dav;
  // outputs indexed by position in the caller's [first, first+count) range
  int64_t first;
  double* e_out;
  int32_t* status_out;
  int32_t* iters_out;
  double* resid_out;
  const uint8_t* evict;
  double e_const;
  int64_t* phase;   // optional [n_inc][kPhases] clock counters (tracing)
  Tuning tune;
};

// Phases recorded by the tracing counters of the batched solver.
enum Phase { kPhPrologue = 0, kPhSigma, kPhSubspace, kPhPassA, kPhRestart, kPhOrtho, kPhIters, kPhTotal, kPhases };

__host__ __device__ inline int64_t tri(int64_t b) { return b * (b + 1) / 2; }

}  // namespace ifci
