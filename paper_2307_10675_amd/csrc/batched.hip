// Batched iFCI increment solver: one workgroup owns one increment and runs
// its whole Davidson solve with the CI vector, the sigma accumulator and the
// string tables resident in LDS (increments whose C fits on chip, up to
// 8 active orbitals at half filling).  Increments are dispatched heaviest
// first, so the hardware workgroup dispatcher acts as the work queue over
// the uneven sizes.
//
// Sigma (Knowles-Handy determinant FCI, restricted to symmetric C):
//   D[Q][(a,b)] = (E_Q c)(a,b)  for unordered pairs Q, E_Q = E_kl + E_lk (or E_kk),
//                 gathered through the pair table of string a (alpha part)
//                 and of string b (beta part);
//   E[P][(a,b)] = sum_Q V[P][Q] D[Q][(a,b)]         (MFMA, the dense contraction);
//   S[a][b]     = sum over the links of a of sign * E[Q][(J,b)];
//   sigma       = S + S^T     (the beta part of sigma is the transpose of the
//                              alpha part when C = C^T).
// The MFMA rows P run over the off-diagonal pairs only.  A diagonal pair pp
// links string a to itself when orbital p is occupied, so the diagonal rows
// enter S[a][b] only as sum over p in a of E[pp][(a,b)] = sum_Q w_Q(a)
// D[Q][(a,b)] with w_Q(a) = sum over p in a of V[pp][Q]: a per-string dot
// product over the B operands already formed for the MFMA (one FMA per
// operand), which at 8 orbitals saves the third 16-row tile (28 off-diagonal
// pairs of 36).
// Each wavefront owns one beta column b at a time: it computes E for the
// whole column in its private LDS slice (stored transposed, E[a][P]) and
// gathers S[:, b] from it, so no workgroup barrier sits inside the column
// loop.  The MFMA B operand is built without dependent loads: the alpha
// part reads a per-wave copy of column b (and its negation) at offsets held
// in registers for the whole sigma, the beta part reads C at a per-column
// row offset plus a compile-time tile offset.  The packed sigma slot of
// (a, b) receives exactly two contributions (from column b and column a),
// added to zero with LDS atomics; two-term sums are order independent, so
// the result is deterministic.
//
// Vectors are stored packed and scaled: entry (a <= b) holds C[a][b] times
// sqrt(2) when a != b, so that plain dot products of packed vectors equal
// full-space dot products.
//
// LDS holds a persistent part (tables, subspace matrix and its eigenvectors,
// the CI vector and the sigma accumulator) and a transient part (working
// vector, eigensolver scratch, reduction buffers) that the per-wave E slices
// overlay while sigma runs.  The end of the transient region, beyond both,
// holds the diagonal-pair weights and (FP32) the A fragments of V, which the
// solvers build once per increment and precision.
#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"
#include "pspace.hpp"

namespace ifci {

struct Lds {
  char* root;      // start of the dynamic LDS (byte offsets below are from here)
  // persistent
  char* colb;      // per sigma wave: column b of C and its negation, [2 (n_str + 1)] of T
  int32_t* ptab;   // int16 [n_str + 1][npair_pad] decoded pair table J | neg << 15, with
                   // J = n_str for no link (and for the sentinel last row and the
                   // padding pairs)
  int32_t* links;  // [n_str][n_link]  (o << 17 | J << 1 | neg), off-diagonal pairs o first
  int32_t* strs;   // [n_str]
  double* F;       // [n_str] string energies
  double* Jm;      // [k*k] (pp|qq)
  double* Km;      // [k*k] (pq|qp)
  double* hd;      // [k] h'_pp
  double* G;       // [16*16] subspace matrix
  double* Qp;      // [16*16] eigenvectors of the previous subspace matrix
  double* Lam;     // [16] its eigenvalues
  int* pidx;       // [kPsMax] packed entries of the P-space block (three-vector solver)
  double* plam;    // [kPsMax + 2] eigenvalues of that block, minus E0; [kPsMax]: the
                   // largest diagonal entry of the block (with pidx[P - 1] it bounds
                   // the block in (H_II, I) order)
  double* cp;      // CI vector, full (n+1) x (n+1) of T with a zero last row and column
  double* sp;      // [n_sym] sigma accumulator, packed scaled
  // transient (overlaid by the E slices during sigma)
  double* tv;      // [n_sym] working vector, packed scaled
  double* Gs;      // [16*16]
  double* Qv;      // [16*16]
  double* y;       // [16]
  double* cf;      // [16] projection coefficients
  double* ev;      // [16] sorted eigenvalues
  int* perm;       // [16]
  double* scal;    // [32]
  int* iscal;      // [16]
  double* red;     // [16 waves * 24]
  char* et;        // E slices (start of the transient part)
  int et_total;    // bytes from et to the end of LDS
};

__host__ __device__ inline int64_t a16(int64_t x) { return (x + 15) & ~int64_t(15); }

// CI vector in LDS: FP64 packed with a zero tail of n+1 entries, or FP32
// full (n+1) x (n+1) with a zero last row and column.
__host__ __device__ inline int64_t cp_bytes(int n_str) {
  const int64_t a = 8 * (tri(n_str) + n_str + 1), b = 4 * (int64_t)(n_str + 1) * (n_str + 1);
  return a16(a > b ? a : b);
}
// pair count padded to the MFMA k-step
__host__ __device__ inline int npair_pad(int k) { return (k * (k + 1) / 2 + 3) / 4 * 4; }
// int16 table of (n+1) x npair_pad entries
__host__ __device__ inline int64_t ptab_bytes(int k, int n_str) {
  return a16(2 * (int64_t)(n_str + 1) * npair_pad(k));
}
// column copies: eight waves of floats, or of doubles when that stays small
__host__ __device__ inline int64_t colb_bytes(int n_str) {
  const int64_t e = 2 * (int64_t)(n_str + 1);
  return a16(n_str <= 64 ? 8 * 8 * e : 8 * 4 * e);
}
__host__ __device__ inline int64_t persistent_bytes(int k, int n_str, int n_link) {
  const int64_t ns = tri(n_str);
  return colb_bytes(n_str) + ptab_bytes(k, n_str) + a16(4 * (int64_t)n_str * n_link) + a16(4 * n_str) +
         a16(8 * n_str) + a16(8 * (2 * k * k + k)) + 8 * (256 + 256 + 16) + 12 * kPsMax + 16 + cp_bytes(n_str) +
         a16(8 * ns);
}
__host__ __device__ inline int64_t transient_bytes(int n_str) {
  return a16(8 * tri(n_str)) + 8 * (256 + 256 + 16 + 16 + 16) + 4 * 16 + 8 * 32 + 4 * 16 + 16 + 8 * 16 * 24;
}
// E slice of one wave, transposed: E[a][o] for one column and the
// off-diagonal pairs o, 16-string tiles of the longest column by an odd row
// stride of at least 17 (n_off | 1), and a spare tail for the padding rows of
// the last MFMA tile.  With a stride of at least 16 the padding rows
// o >= n_off of the last row tile reach only into the first 16 (MT - 1)
// entries of the next string's row.
__host__ __device__ constexpr int slice_rows(int k) { return (max_strings(k) + 15) / 16 * 16; }
__host__ __device__ constexpr int slice_stride(int k) {
  return ((k * (k - 1) / 2) | 1) > 17 ? ((k * (k - 1) / 2) | 1) : 17;
}
// Row stride of the diagonal-pair weight table w[Q][a] (the strings of the
// longest column): 16 mod 32, so the 32 lanes of a half wave (16 strings x 2
// pairs) read distinct banks.
__host__ __device__ constexpr int wt_stride(int k) { return slice_rows(k) | 16; }
// Weight table w[npair_pad][wt_stride] and the diagonal rows u[k][npair_pad]
// of V it is summed from, of T, at the start of the sigma scratch (ahead of
// the E slices).
// FP32 A fragments of the off-diagonal rows of V in lane order,
// [MT][KS][64] floats (FP64 reads its fragments from V for each sigma: the
// FP64 copy would cost an E slice at 8 orbitals).
__host__ __device__ inline int64_t afr_bytes(int k, int elem) {
  const int mt = (k * (k - 1) / 2 + 15) / 16;
  return elem == 4 ? a16((int64_t)(mt > 0 ? mt : 1) * (npair_pad(k) / 4) * 64 * elem) : 0;
}
__host__ __device__ inline int64_t wt_bytes(int k, int elem) {
  return a16((int64_t)npair_pad(k) * wt_stride(k) * elem) + a16((int64_t)k * npair_pad(k) * elem) +
         afr_bytes(k, elem);
}
// Entry rows * stride + 16 is kept zero: absent links read it.
__host__ __device__ inline int64_t et_slice_bytes(int k, int, int elem) {
  return a16(((int64_t)slice_rows(k) * slice_stride(k) + 17) * elem);
}

__device__ inline Lds carve(char* base, const IncDev& d, int lds_bytes) {
  Lds L;
  char* p = base;
  const int n = d.n_str, np = d.npair, k = d.k;
  L.root = base;
  L.colb = p;
  p += colb_bytes(n);
  L.ptab = (int32_t*)p;
  p += ptab_bytes(k, n);
  (void)np;
  L.links = (int32_t*)p;
  p += a16(4 * n * d.n_link);
  L.strs = (int32_t*)p;
  p += a16(4 * n);
  L.F = (double*)p;
  p += a16(8 * n);
  L.Jm = (double*)p;
  L.Km = L.Jm + k * k;
  L.hd = L.Km + k * k;
  p += a16(8 * (2 * k * k + k));
  L.G = (double*)p;
  p += 8 * 256;
  L.Qp = (double*)p;
  p += 8 * 256;
  L.Lam = (double*)p;
  p += 8 * 16;
  L.plam = (double*)p;
  p += 8 * (kPsMax + 2);
  L.pidx = (int*)p;
  p += 4 * kPsMax;
  L.cp = (double*)p;
  p += cp_bytes(n);
  L.sp = (double*)p;
  p += a16(8 * d.n_sym);
  // transient
  L.et = p;
  L.et_total = (int)((base + lds_bytes) - p);
  L.tv = (double*)p;
  p += a16(8 * d.n_sym);
  L.Gs = (double*)p;
  p += 8 * 256;
  L.Qv = (double*)p;
  p += 8 * 256;
  L.y = (double*)p;
  p += 8 * 16;
  L.cf = (double*)p;
  p += 8 * 16;
  L.ev = (double*)p;
  p += 8 * 16;
  L.perm = (int*)p;
  p += 4 * 16;
  L.scal = (double*)p;
  p += 8 * 32;
  L.iscal = (int*)p;
  p += 4 * 16;
  p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
  L.red = (double*)p;
  return L;
}

// Byte offset from L.et of the diagonal-pair weight table of element size
// elem: the last wt_bytes of the scratch region (16-byte aligned).
__device__ inline int64_t wt_offset(const Lds& L, int k, int elem) {
  return ((int64_t)L.et_total - wt_bytes(k, elem)) & ~(int64_t)15;
}

// 32-bit packed index of (x, y) in the upper triangle (at most 70 strings here).
__device__ __forceinline__ int pk32(int x, int y) {
  return x <= y ? ((y * (y + 1)) >> 1) + x : ((x * (x + 1)) >> 1) + y;
}

// ---------------------------------------------------------------------------
// Sigma of the CI vector in L.cp (unscaled; FP32 full (n+1) x (n+1) with a
// zero last row and column, FP64 packed with a zero tail), accumulated into
// L.sp (packed, scaled, must be zero).
// V holds the pair contraction matrix; shift is subtracted from its
// (diagonal pair, diagonal pair) block, which subtracts shift * N / N^2 * N
// = shift from the operator.
template <typename T, int K>
__device__ __forceinline__ void sigma_sector(const IncDev& d, const Lds& L, const double* __restrict__ V,
                                             double shift, int et_waves, bool build_w) {
  constexpr int NP = K * (K + 1) / 2;
  constexpr int NO = K * (K - 1) / 2;       // off-diagonal pairs: the MFMA rows
  constexpr int MT = (NO + 15) / 16;        // 0 at one orbital
  constexpr int MTA = MT > 0 ? MT : 1;      // array extent
  constexpr int KS = (NP + 3) / 4;
  typedef Mfma<T> M;
  // bit P set for the diagonal pairs P = i (i + 3) / 2 (the pair (i, i))
  constexpr uint64_t kDiagPairs = [] {
    uint64_t m = 0;
    for (int i = 0; i < K; ++i) m |= 1ull << (i * (i + 3) / 2);
    return m;
  }();
  static_assert(NP <= 64, "pair mask holds 64 pairs");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = d.n_str, nlink = d.n_link - d.na;  // off-diagonal links per string
  const int lstride = d.n_link;                     // row stride of the link table
  const T* cp = (const T*)L.cp;
  const double nel = 2.0 * d.na;
  const double sh = nel > 0.0 ? shift / (nel * nel) : 0.0;
  constexpr int NPp = 4 * KS;
  constexpr int WS = wt_stride(K);

  // Diagonal-pair weights w[Q][a] = sum over the orbitals p of string a of
  // V[pp][Q] (shifted in the diagonal block), summed in a fixed order from
  // the rows u[p][Q]; zero for padding pairs and strings a >= n.  They sit
  // at the end of the scratch region, which neither the E slices nor the
  // solver's transient data reach, so a caller that keeps V, the shift and
  // T builds them once (build_w) and reuses them for later sigmas.
  T* const wt = (T*)(L.et + wt_offset(L, K, (int)sizeof(T)));
  T* const ut = (T*)((char*)wt + a16((int64_t)NPp * WS * (int64_t)sizeof(T)));
  // A fragments: V[P(16 m + lane % 16)][4 s + lane / 16] for the off-diagonal
  // pair P(o) = o + p of row o (p the larger orbital of the pair); FP32
  // stores them in lane order beside the weights, built with them
  constexpr bool kAfrLds = sizeof(T) == 4;
  T* const afl = (T*)((char*)ut + a16((int64_t)K * NPp * (int64_t)sizeof(T)));
  auto afr_value = [&](int m, int sq, int ln) -> T {
    const int o = 16 * m + (ln & 15), Q = 4 * sq + (ln >> 4);
    double v = 0.0;
    if (m < MT && o < NO && Q < NP) {
      int p = 1;
      while (p * (p + 1) / 2 <= o) ++p;
      v = V[(o + p) * NP + Q];
    }
    return (T)v;
  };
  if (build_w) {
  for (int i = threadIdx.x; kAfrLds && i < MTA * KS * 64; i += blockDim.x) {
    const int ms = i >> 6, m = ms / KS;
    afl[i] = afr_value(m, ms - m * KS, i & 63);
  }
  for (int i = threadIdx.x; i < K * NPp; i += blockDim.x) {
    const int p = i / NPp, Q = i - p * NPp;
    double v = 0.0;
    if (Q < NP) {
      v = V[(p * (p + 3) / 2) * NP + Q];
      if ((kDiagPairs >> Q) & 1) v -= sh;
    }
    ut[i] = (T)v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NPp * WS; i += blockDim.x) {
    const int Q = i / WS, a = i - Q * WS;
    T v = (T)0;
    if (a < n && Q < NP) {
      uint32_t occ = (uint32_t)L.strs[a];
      while (occ) {
        const int p = __builtin_ctz(occ);
        occ &= occ - 1u;
        v += ut[p * NPp + Q];
      }
    }
    wt[i] = v;
  }
  __syncthreads();
  }

  if (wave >= et_waves) return;
  T afr[MTA][KS];
#pragma unroll
  for (int m = 0; m < MTA; ++m)
#pragma unroll
    for (int s = 0; s < KS; ++s) afr[m][s] = kAfrLds ? afl[(m * KS + s) * 64 + lane] : afr_value(m, s, lane);
  constexpr int NTM = slice_rows(K) / 16;  // 16-string tiles of the longest column
  constexpr int NS = slice_stride(K);      // E slice row stride (odd, >= 17)
  static_assert(NS >= 16 && 16 * MT - NS <= NS, "padding rows must stay within the next row's first tiles");
  constexpr bool kFull = sizeof(T) == 4;   // FP32: full layout, FP64: packed
  const int nt_count = (n + 15) / 16;
  const int kq = lane >> 4, col = lane & 15;
  const int ld = n + 1;
  T* et = (T*)(L.et + (size_t)wave * et_slice_bytes(K, n, (int)sizeof(T)));
  const T* const wl = wt + kq * WS + col;  // this lane's w[4 s + kq][16 t + col] at compile-time offsets
  const int16_t* pt = (const int16_t*)L.ptab;  // [a][Q]: J | neg << 15, J = n: none
  T* colb = (T*)L.colb + (size_t)wave * 2 * ld;
  const uint32_t colb_off = (uint32_t)((const char*)colb - L.root);
  const uint32_t cp_off = (uint32_t)((const char*)cp - L.root);

  // B operand of the MFMA step s of tile t for this lane (a = 16 t + col,
  // Q = 4 s + kq):  D[Q][(a, b)] = sign1 C[J1][b] + sign2 C[a][J2].
  // The alpha part reads the wave's copy of column b and of its negation
  // (colb[J1 + neg (n+1)]); its LDS byte offsets depend on (a, Q) only, so
  // they are computed once per sigma and kept in registers, two 16-bit
  // offsets a register.  A missing link, a padding pair and a string a >= n
  // address colb[n] = 0.  The beta part reads C[a][J2] = C[J2][a] with the
  // sign of (b, Q) applied in a fused multiply-add; J2 = n (no link) reads
  // the zero row (FP32) or the zero tail (FP64).  No load depends on another.
  constexpr int NA = NTM * KS;
  uint32_t ia[(NA + 1) / 2];
#pragma unroll
  for (int i = 0; i < (NA + 1) / 2; ++i) ia[i] = 0;
#pragma unroll
  for (int t = 0; t < NTM; ++t)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int a = min(16 * t + col, n);
      const int e = (int)(uint16_t)pt[a * NPp + 4 * s + kq];
      const int J = e & 0x7FFF;
      const int j = J >= n ? n : J + (e >> 15) * ld;
      const int i = t * KS + s;
      ia[i >> 1] |= (colb_off + (uint32_t)j * (uint32_t)sizeof(T)) << (16 * (i & 1));
    }

  // Alpha-gather link codes, two 16-bit codes per register: the E-slice
  // offset J NS + Q (below 2^15) with bit 15 = negative sign; an absent link
  // reads the slice's zero entry.  Pass 0: string a = lane, all its links.
  // Pass 1 (more than 64 strings, 8 orbitals): strings 64 + lane / 8, three
  // links per lane, summed over the 8 lanes of a string in a fixed tree.
  // FP32 keeps the codes in registers for every column; FP64 has no
  // registers to spare and decodes them per column.
  constexpr int LM = (K / 2) * ((K + 1) / 2);  // max of na (K - na): off-diagonal links
  constexpr int LP = LM > 0 ? (LM + 1) / 2 : 1;
  constexpr bool kTwoPass = max_strings(K) > 64;
  static_assert(!kTwoPass || (LM <= 24 && max_strings(K) <= 64 + 8), "pass 1 covers 8 strings of 24 links");
  constexpr int ZI = slice_rows(K) * NS + 16;  // zero entry of the slice
  constexpr bool kLinkRegs = kFull;
  auto code_of = [&](int a, int l) -> uint32_t {
    if (a < n && l < nlink) {
      const int code = L.links[a * lstride + l];
      return (uint32_t)(((code >> 1) & 0xFFFF) * NS + (code >> 17)) | ((uint32_t)(code & 1) << 15);
    }
    return (uint32_t)ZI;
  };
  const int a1 = 64 + (lane >> 3);  // pass-1 string of this lane
  auto link_codes = [&](uint32_t (&lk0)[LP], uint32_t (&lk1)[2]) {
#pragma unroll
    for (int i = 0; i < LP; ++i) lk0[i] = code_of(lane, 2 * i) | (code_of(lane, 2 * i + 1) << 16);
    if (kTwoPass) {
      const int l1 = 3 * (lane & 7);
      lk1[0] = code_of(a1, l1) | (code_of(a1, l1 + 1) << 16);
      lk1[1] = code_of(a1, l1 + 2);
    }
  };
  uint32_t lk0_keep[LP], lk1_keep[2];
  if (kLinkRegs) link_codes(lk0_keep, lk1_keep);
  if (lane == 0) et[ZI] = (T)0;

  // MFMA output row of (lane, r) within a 16-row tile, and the lane's store
  // base in the transposed slice: E[a][P] at et[a NS + P]
  T* const ebase = et + col * NS + M::row(kq, 0);
  constexpr int RSTEP = M::row(0, 1) - M::row(0, 0);  // row step between accumulator registers

  // per column: the wave's copy of column b and its negation (row n / the
  // tail is zero), and the beta part (one entry per k-step of this lane).
  // The next column's are prepared while the current one is gathered.
  int j2[KS];
  T sg[KS];
  uint32_t r2[KS];  // FP32: byte offset of C[J2][col]
  auto column_setup = [&](int bb) {
    for (int j = lane; j < ld; j += 64) {
      const T v = kFull ? cp[j * ld + bb] : cp[pk32(j, bb)];
      colb[j] = v;
      colb[ld + j] = -v;
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int e = (int)(uint16_t)pt[bb * NPp + 4 * s + kq];
      j2[s] = e & 0x7FFF;
      sg[s] = (e & 0x8000) ? (T)-1 : (T)1;
      r2[s] = cp_off + (uint32_t)((j2[s] * ld + col) * (int)sizeof(T));
    }
  };
  if (wave < n) column_setup(wave);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  for (int b = wave; b < n; b += et_waves) {
    // diagonal-pair part of S[:, b]: string lane (pass 0), string 64 + lane / 8 (pass 1)
    T dext0 = (T)0, dext1 = (T)0;
    // Keep the packed offsets packed: without this the compiler unpacks
    // them once before the loop into twice as many registers and spills.
#pragma unroll
    for (int i = 0; i < (NA + 1) / 2; ++i) asm volatile("" : "+v"(ia[i]));
    if (kLinkRegs) {
#pragma unroll
      for (int i = 0; i < LP; ++i) asm volatile("" : "+v"(lk0_keep[i]));
    }

    auto beta = [&](int t, int s) -> T {
      if (kFull) return *(const T*)(L.root + r2[s] + 16 * t * sizeof(T));
      const int a = min(16 * t + col, n);  // a = n: the zero tail
      return cp[pk32(a, j2[s])];
    };
    // E[:, (a, b)] for C consecutive 16-string tiles from tile t on (C
    // independent MFMA chains per row tile), stored transposed into the
    // wave's slice.  Rows a >= n of the slice are padding.  The last MFMA
    // row tile holds rows o >= n_off (zero) that spill into the next
    // string's row: it is stored first, so the other tiles overwrite what it
    // spilled.  Beside the MFMAs each lane accumulates w[Q][a] D[Q][(a, b)]
    // over its pairs Q = 4 s + kq: the diagonal-pair part of S[a][b] once
    // summed over the four k-lanes.
    auto tiles = [&](auto tt, auto cnt) {
      constexpr int t = decltype(tt)::value;
      constexpr int C = decltype(cnt)::value;
      typename M::acc acc[C][MTA];
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int m = 0; m < MTA; ++m) acc[c][m] = M::zero();
      auto alpha = [&](int tt2, int s) -> T {
        const int i = tt2 * KS + s;
        return *(const T*)(L.root + ((ia[i >> 1] >> (16 * (i & 1))) & 0xFFFFu));
      };
      // loads of step s + 1 are issued ahead of the MFMAs of step s
      T va[C], vb[C], wv[C], dsum[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        va[c] = alpha(t + c, 0);
        vb[c] = beta(t + c, 0);
        wv[c] = wl[16 * (t + c)];
        dsum[c] = (T)0;
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        T bo[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          bo[c] = fma_t(sg[s], vb[c], va[c]);
          dsum[c] = fma_t(wv[c], bo[c], dsum[c]);
        }
        if (s + 1 < KS) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            va[c] = alpha(t + c, s + 1);
            vb[c] = beta(t + c, s + 1);
            wv[c] = wl[4 * (s + 1) * WS + 16 * (t + c)];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c][m] = M::mma(afr[m][s], bo[c], acc[c][m]);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the diagonal-pair sums of string 16 (t + c) + col, summed over the
      // k-lanes, to the gather lane of that string
#pragma unroll
      for (int c = 0; c < C; ++c) {
        T v = dsum[c];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (t + c < 4) {
          if ((lane >> 4) == t + c) dext0 = v;
        } else {
          dext1 = __shfl(v, lane >> 3);
        }
      }
#pragma unroll
      for (int mm = 0; mm < MT; ++mm) {
        const int m = (mm + MT - 1) % MT;  // last row tile first
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < C; ++c) ebase[16 * (t + c) * NS + 16 * m + RSTEP * r] = acc[c][m][r];
        // the overlap is between lanes, which the compiler does not see:
        // keep the spilling stores ahead of the others
        if (mm == 0) asm volatile("" ::: "memory");
      }
    };
    // FP32 columns of full length run all their tiles in one pass (one
    // accumulator drain per column, MT x NTM independent MFMAs per k-step);
    // otherwise pairs of tiles
    if (kFull && nt_count == NTM) {
      tiles(std::integral_constant<int, 0>{}, std::integral_constant<int, NTM>{});
    } else {
      static_for<0, (NTM + 1) / 2>([&](auto hp) {
        constexpr int t = 2 * decltype(hp)::value;
        if (t + 1 < nt_count)
          tiles(std::integral_constant<int, t>{}, std::integral_constant<int, 2>{});
        else if (t < nt_count)
          tiles(std::integral_constant<int, t>{}, std::integral_constant<int, 1>{});
      });
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the next column's copy and beta part (colb and r2 are free again)
    if (b + et_waves < n) column_setup(b + et_waves);
    // S[a][b] = sum over the links (a -> J, pair Q) of sign E[(J, b)][Q]
    uint32_t lk0_col[LP], lk1_col[2];
    if (!kLinkRegs) link_codes(lk0_col, lk1_col);
    const uint32_t(&lk0)[LP] = kLinkRegs ? lk0_keep : lk0_col;
    const uint32_t(&lk1)[2] = kLinkRegs ? lk1_keep : lk1_col;
    {
      T v[2 * LP];
#pragma unroll
      for (int i = 0; i < LP; ++i) {
        v[2 * i] = et[lk0[i] & 0x7FFFu];
        v[2 * i + 1] = et[(lk0[i] >> 16) & 0x7FFFu];
      }
      // all loads in flight before the first use (left alone, the compiler
      // trades them for registers and waits on each load in turn)
      __builtin_amdgcn_sched_barrier(0);
      T sum = dext0;
#pragma unroll
      for (int l = 0; l < 2 * LP; ++l) sum += ((lk0[l >> 1] >> (16 * (l & 1))) & 0x8000u) ? -v[l] : v[l];
      if (lane < n) lds_add(&L.sp[pk32(lane, b)], (lane == b ? 2.0 : kSqrt2) * (double)sum);
    }
    if (kTwoPass && n > 64) {
      const T u0 = et[lk1[0] & 0x7FFFu], u1 = et[(lk1[0] >> 16) & 0x7FFFu], u2 = et[lk1[1] & 0x7FFFu];
      __builtin_amdgcn_sched_barrier(0);
      T sum = ((lk1[0] & 0x8000u) ? -u0 : u0) + ((lk1[0] & 0x80000000u) ? -u1 : u1);
      sum += (lk1[1] & 0x8000u) ? -u2 : u2;
      sum += __shfl_down(sum, 4);
      sum += __shfl_down(sum, 2);
      sum += __shfl_down(sum, 1);
      sum += dext1;  // one lane of the eight: the lane the sum lands on
      if ((lane & 7) == 0 && a1 < n) lds_add(&L.sp[pk32(a1, b)], (a1 == b ? 2.0 : kSqrt2) * (double)sum);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Pair table (decoded, see Lds::ptab), strings and link lists into LDS.
__device__ inline void load_tables(const IncDev& d, const Lds& L, const int32_t* __restrict__ tables) {
  const int n = d.n_str, np = d.npair;
  const int npp = npair_pad(d.k);
  int16_t* pt = (int16_t*)L.ptab;
  for (int i = threadIdx.x; i < (n + 1) * npp; i += blockDim.x) {
    const int a = i / npp, Q = i - a * npp;
    const int e = (a < n && Q < np) ? tables[d.pair_off + a * np + Q] : -1;
    const int J = e < 0 ? n : (e >> 1), neg = e < 0 ? 0 : (e & 1);
    pt[i] = (int16_t)(J | (neg << 15));
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) L.strs[i] = tables[d.str_off + i];
  // links of each string without its diagonal pairs (carried by the
  // per-string dot product of sigma_sector), the pair Q = p (p + 1) / 2 + q
  // (p > q) renumbered to its off-diagonal index o = Q - p; the na(k - na)
  // entries first, the rest unused
  const int nl = d.n_link;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    int m = 0;
    for (int l = 0; l < nl; ++l) {
      const int code = tables[d.link_off + a * nl + l];
      const int Q = code >> 17;
      int p = 0;
      while ((p + 1) * (p + 2) / 2 <= Q) ++p;
      if (Q - p * (p + 1) / 2 == p) continue;
      L.links[a * nl + m++] = ((Q - p) << 17) | (code & 0x1FFFF);
    }
    for (; m < nl; ++m) L.links[a * nl + m] = 0;
  }
}

// Expand the packed scaled vector tv into the unscaled cp of type T (FP32
// full with a zero last row and column, FP64 packed with a zero tail) and
// clear sp.
template <typename T>
__device__ inline void prepare_sigma(const IncDev& d, const Lds& L) {
  T* cp = (T*)L.cp;
  const int n = d.n_str, ld = n + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (sizeof(T) == 4) {
    for (int a = wave; a < ld; a += nw)
      for (int b = lane; b < ld; b += 64) {
        double v = 0.0;
        if (a < n && b < n) {
          v = L.tv[pk32(a, b)];
          if (a != b) v *= kRSqrt2;
        }
        cp[a * ld + b] = (T)v;
      }
  } else {
    for (int b = wave; b < n; b += nw)
      for (int a = lane; a <= b; a += 64) {
        const int i = ((b * (b + 1)) >> 1) + a;
        const double v = L.tv[i];
        cp[i] = (T)(a == b ? v : v * kRSqrt2);
      }
    for (int i = threadIdx.x; i <= n; i += blockDim.x) cp[d.n_sym + i] = (T)0;  // zero tail
  }
  for (int64_t i = threadIdx.x; i < d.n_sym; i += blockDim.x) L.sp[i] = 0.0;
  __syncthreads();
}

// Entry i = (a, b) of the packed scaled vector, value v, into cp in the
// layout of T, and the sigma accumulator slot cleared: the per-entry part of
// prepare_sigma, for callers that produce the vector entry by entry.
template <typename T>
__device__ __forceinline__ void stage_entry(const IncDev& d, const Lds& L, int i, double v) {
  int a, b;
  unpack32(i, &a, &b);
  T* cp = (T*)L.cp;
  const T c = (T)(a == b ? v : v * kRSqrt2);
  if (sizeof(T) == 4) {
    const int ld = d.n_str + 1;
    cp[a * ld + b] = c;
    cp[b * ld + a] = c;
  } else {
    cp[i] = c;
  }
  L.sp[i] = 0.0;
}

// staged: the caller already wrote cp and cleared sp (stage_entry) and
// synchronised; otherwise they are built here from L.tv.
template <typename T, int K>
__device__ inline void sigma_phase(const IncDev& d, const Lds& L, const double* V, double shift,
                                   int et_waves, bool staged = false, bool build_w = true, bool sync = true) {
  if (!staged) prepare_sigma<T>(d, L);
  sigma_sector<T, K>(d, L, V, shift, et_waves, build_w);
  if (sync) __syncthreads();
}

template <typename T, int K>
__device__ inline int et_waves_for(const IncDev& d, const Lds& L) {
  const int64_t slice = et_slice_bytes(K, d.n_str, (int)sizeof(T));
  int w = (int)(wt_offset(L, K, (int)sizeof(T)) / slice);
  const int wc = (int)(colb_bytes(d.n_str) / (2 * (int64_t)(d.n_str + 1) * (int64_t)sizeof(T)));
  w = w < wc ? w : wc;
  const int nw = blockDim.x >> 6;
  return w > nw ? nw : w;
}

// The tuned number of contracting waves, never above what LDS holds.
__device__ __forceinline__ int tuned_waves(int fit, int tuned) { return tuned > 0 && tuned < fit ? tuned : fit; }

// Load the increment's tables and diagonal data and write the diagonal to HD.
__device__ inline void load_increment(const IncDev& d, const Lds& L, const int32_t* __restrict__ tables,
                                      const double* __restrict__ B, double* __restrict__ HD) {
  const int n = d.n_str, np = d.npair, k = d.k;
  const IntBlock ib = int_block(k);
  load_tables(d, L, tables);
  for (int i = threadIdx.x; i < k * k; i += blockDim.x) {
    L.Jm[i] = B[ib.J + i];
    L.Km[i] = B[ib.K + i];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) L.hd[i] = B[ib.hd + i];
  __syncthreads();
  // string energies F(s) = sum_{p in s} h'_pp + 1/2 sum_{p,q in s} [(pp|qq) - (pq|qp)]
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t s = (uint32_t)L.strs[i];
    double f = 0.0;
    for (int p = 0; p < k; ++p) {
      if (!(s >> p & 1u)) continue;
      f += L.hd[p];
      for (int q = 0; q < k; ++q)
        if (s >> q & 1u) f += 0.5 * (L.Jm[p * k + q] - L.Km[p * k + q]);
    }
    L.F[i] = f;
  }
  __syncthreads();
  // H_(a,b),(a,b) = F(a) + F(b) + sum_{p in a, q in b} (pp|qq)
  for (int64_t i = threadIdx.x; i < d.n_sym; i += blockDim.x) {
    int a, b;
    unpack(i, &a, &b);
    const uint32_t sa = (uint32_t)L.strs[a], sb = (uint32_t)L.strs[b];
    double v = L.F[a] + L.F[b];
    for (int p = 0; p < k; ++p) {
      if (!(sa >> p & 1u)) continue;
      for (int q = 0; q < k; ++q)
        if (sb >> q & 1u) v += L.Jm[p * k + q];
    }
    HD[i] = v;
  }
  __syncthreads();
}

__device__ inline void argmin_block(const double* __restrict__ HD, int64_t ns, const Lds& L) {
  double best = 1e300;
  int64_t bi = 0x7fffffff;
  for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) {
    const double v = HD[i];
    if (v < best) best = v, bi = i;
  }
  // wave argmin with ties to the lower index
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ov < best || (ov == best && oi < bi)) best = ov, bi = oi;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    L.red[2 * wave] = best;
    L.red[2 * wave + 1] = (double)bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = L.red[0];
    double ix = L.red[1];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (L.red[2 * w] < b || (L.red[2 * w] == b && L.red[2 * w + 1] < ix)) b = L.red[2 * w], ix = L.red[2 * w + 1];
    L.scal[0] = b;
    L.iscal[0] = (int)ix;
  }
  __syncthreads();
}

// Subspace eigenproblem of the (m+1)-dimensional matrix G, warm started:
// with the previous block's eigenpairs (Lam, Qp), G is first rotated to
// [[diag(Lam), Qp^T g], [., g_mm]] (g = the new column), and Jacobi only
// has to resolve that arrowhead.  Leaves Lam/Qp for the next call, the
// sorted eigenvalues in ev/perm and the lowest pair in scal[20] / y.
__device__ inline void subspace_solve(const Lds& L, int m) {
  const int tid = threadIdx.x, n = m + 1;
  if (tid < 256) {
    const int i = tid >> 4, j = tid & 15;
    double gs = 0.0, q = 0.0;
    if (i < n && j < n) {
      if (i < m && j < m) {
        gs = (i == j) ? L.Lam[i] : 0.0;
        q = L.Qp[i * 16 + j];
      } else if (i == m && j == m) {
        gs = L.G[m * 16 + m];
        q = 1.0;
      } else {
        const int r = (i == m) ? j : i;  // entry r of Qp^T g
        double s = 0.0;
        for (int l = 0; l < m; ++l) s += L.Qp[l * 16 + r] * L.G[l * 16 + m];
        gs = s;
        q = 0.0;
      }
    }
    L.Gs[tid] = gs;
    L.Qv[tid] = q;
  }
  __syncthreads();
  if (tid < 64) jacobi_warm(L.Gs, L.Qv, n, &L.scal[20], L.y, L.ev, L.perm);
  __syncthreads();
  if (tid < 256) {
    const int i = tid >> 4;
    L.Qp[tid] = L.Qv[tid];
    if ((tid & 15) == 0 && i < n) L.Lam[i] = L.Gs[i * 16 + i];
  }
  __syncthreads();
}


// Lowest eigenpair of a symmetric 3 x 3 matrix g (g[2][2] = 1e30 with a
// zero third row and column marks a 2 x 2 problem).  2 x 2: closed form.
// 3 x 3: Newton on the characteristic polynomial from below the Gershgorin
// bound (monotone convergence to the lowest root), then the eigenvector as
// the largest cross product of two rows of g - theta I.  Every thread of the
// workgroup computes the same values.
__device__ inline void small_eig3(const double g[3][3], double* theta, double z[3]) {
  const double a = g[0][0], b = g[0][1], c = g[1][1];
  if (g[2][2] >= 1e29) {
    const double m = 0.5 * (a + c), h = 0.5 * (a - c);
    const double l = m - sqrt(h * h + b * b);
    double v0, v1;
    if (fabs(a - l) >= fabs(c - l)) {
      v0 = b;
      v1 = l - a;
    } else {
      v0 = l - c;
      v1 = b;
    }
    if (v0 == 0.0 && v1 == 0.0) v0 = 1.0;
    const double nr = 1.0 / sqrt(v0 * v0 + v1 * v1);
    *theta = l;
    z[0] = v0 * nr;
    z[1] = v1 * nr;
    z[2] = 0.0;
    return;
  }
  const double d = g[0][2], e = g[1][2], f = g[2][2];
  // det(l I - g) = l^3 + c2 l^2 + c1 l + c0
  const double c2 = -(a + c + f);
  const double c1 = a * c + a * f + c * f - b * b - d * d - e * e;
  const double c0 = -(a * (c * f - e * e) - b * (b * f - e * d) + d * (b * e - c * d));
  double l = fmin(a - fabs(b) - fabs(d), fmin(c - fabs(b) - fabs(e), f - fabs(d) - fabs(e)));
  const double scale = 1.0 + fabs(a) + fabs(c) + fabs(f);
#pragma unroll 1
  for (int it = 0; it < 64; ++it) {
    const double pv = ((l + c2) * l + c1) * l + c0;
    const double dv = (3.0 * l + 2.0 * c2) * l + c1;
    if (!(dv > 0.0)) break;
    // the hardware reciprocal is accurate enough for a Newton step (the
    // iteration still ends at the root) and shortens the dependent chain
    const double step = pv * __builtin_amdgcn_rcp(dv);
    l -= step;
    if (fabs(step) <= 1e-15 * scale) break;
  }
  const double r0[3] = {a - l, b, d}, r1[3] = {b, c - l, e}, r2[3] = {d, e, f - l};
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double w01[3], w02[3], w12[3];
  cross(r0, r1, w01);
  cross(r0, r2, w02);
  cross(r1, r2, w12);
  const double n01 = w01[0] * w01[0] + w01[1] * w01[1] + w01[2] * w01[2];
  const double n02 = w02[0] * w02[0] + w02[1] * w02[1] + w02[2] * w02[2];
  const double n12 = w12[0] * w12[0] + w12[1] * w12[1] + w12[2] * w12[2];
  const double* w = w01;
  double nn = n01;
  if (n02 > nn) {
    w = w02;
    nn = n02;
  }
  if (n12 > nn) {
    w = w12;
    nn = n12;
  }
  const double nr = 1.0 / sqrt(nn);
  z[0] = w[0] * nr;
  z[1] = w[1] * nr;
  z[2] = w[2] * nr;
  // Rayleigh quotient of the unit vector: the eigenvalue to rounding
  double gz[3];
  for (int i = 0; i < 3; ++i) gz[i] = g[i][0] * z[0] + g[i][1] * z[1] + g[i][2] * z[2];
  *theta = z[0] * gz[0] + z[1] * gz[1] + z[2] * gz[2];
}

// ---------------------------------------------------------------------------
// P-space block of the three-vector solver (pspace.hpp): size, set-up, and
// the per-iteration correction.

// Byte offset from L.et of the P-space scratch: past the transient arrays.
__device__ inline int64_t ps_scratch_offset(const IncDev& d) { return a16(transient_bytes(d.n_str)); }

// P-space scratch from L.et + ps_scratch_offset: U [P][P] FP32 (where the
// FP32 image is kept during iterations), A [P][P] FP32, the Jacobi
// rotations (2 P floats) and planes (P ints) in 1 KB, h' [K][K] and a copy
// of the pair matrix V [np][np] and k [K][K] of the increment (FP64) for
// the Slater-Condon elements.
__device__ inline int64_t ps_scratch_bytes(int P, int K) {
  const int64_t np = K * (K + 1) / 2;
  return 8LL * P * P + 1024 + 8LL * (2 * K * K + np * np) + 64;
}

// Block size for this increment: even, at most n_guess, kPsMax and an
// eighth of the sector dimension, with room in LDS for the set-up (A, U,
// h', the rotations) and, across iterations, for the FP32 U image below the
// diagonal-pair weights of both precisions.  The eighth: a block that
// covers most of the sector makes the preconditioner nearly the exact
// shifted inverse, whose correction is nearly parallel to the vector
// itself, and an iteration started from the block's lowest eigenvector can
// then settle on an excited state next to it (seen in mixed precision on a
// 4o4e increment, 20 of 21 entries in the block).
template <int K>
__device__ inline int ps_size(const IncDev& d, const Lds& L, int n_guess) {
  int P = n_guess < kPsMax ? n_guess : kPsMax;
  if (P > (int)d.n_sym / 8) P = (int)d.n_sym / 8;
  P &= ~1;
  const int64_t off = ps_scratch_offset(d);
  const int64_t wt = wt_offset(L, K, 4) < wt_offset(L, K, 8) ? wt_offset(L, K, 4) : wt_offset(L, K, 8);
  while (P >= 2 && (off + ps_scratch_bytes(P, K) > L.et_total || off + 4LL * P * P > wt)) P -= 2;
  return P >= 2 ? P : 0;
}

// Block position of this thread's entry e, packed 7 bits per entry in a
// 64-bit word (0x7f: not in the block): kept compact because it stays live
// across every sigma.
__device__ __forceinline__ int ps_pos(uint64_t pk, int e) { return (int)((pk >> (7 * e)) & 0x7f); }

// First half of the set-up: the P lowest diagonal entries (ties to the
// lower index) in L.pidx, the largest of their diagonal values in
// L.plam[kPsMax], their block positions for this thread's entries in pk
// (ps_pos), and H_PP - E0 from the Slater-Condon rules in the scratch
// matrix A.  An entry I is in the block exactly when (H_II, I) <=
// (L.plam[kPsMax], L.pidx[P - 1]) in lexicographic order.
template <int K, int NE>
__device__ __forceinline__ void ps_build(const IncDev& d, const Lds& L, const double* __restrict__ B,
                                                   const double* HD, double E0, int P, uint64_t& pk, int& parity) {
  static_assert(NE <= 9, "seven bits per entry in 64");
  const int tid = threadIdx.x, nsi = (int)d.n_sym;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const IntBlock ib = int_block(K);
  double hv[NE];
  unsigned avail = 0;
  pk = ~0ull;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int i = tid + e * kBatchThreads;
    hv[e] = 1e300;
    if (i < nsi) {
      hv[e] = HD[i];
      avail |= 1u << e;
    }
  }
  // selection: P rounds of a block argmin over the entries not yet taken
  for (int j = 0; j < P; ++j) {
    double best = 1e300;
    int bi = 0x7fffffff;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tid + e * kBatchThreads;
      if ((avail >> e & 1u) && (hv[e] < best || (hv[e] == best && i < bi))) best = hv[e], bi = i;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov < best || (ov == best && oi < bi)) best = ov, bi = oi;
    }
    double* buf = L.red + parity * 128;
    parity ^= 1;
    if (lane == 0) {
      buf[2 * wave] = best;
      buf[2 * wave + 1] = (double)bi;
    }
    __syncthreads();
    double wb = buf[0];
    int wi = (int)buf[1];
    for (int w = 1; w < nw; ++w) {
      const double v = buf[2 * w];
      const int ix = (int)buf[2 * w + 1];
      if (v < wb || (v == wb && ix < wi)) wb = v, wi = ix;
    }
    if ((wi & (kBatchThreads - 1)) == tid) {
      const int e = wi / kBatchThreads;
#pragma unroll
      for (int q = 0; q < NE; ++q)
        if (q == e) {
          avail &= ~(1u << q);
          pk = (pk & ~(0x7full << (7 * q))) | ((uint64_t)j << (7 * q));
        }
    }
    if (tid == 0) {
      L.pidx[j] = wi;
      L.plam[kPsMax] = wb;
    }
  }
  float* Am = (float*)(L.et + ps_scratch_offset(d)) + P * P;
  double* hp = (double*)(Am + P * P + 256);
  double* kl = hp + K * K;
  double* Vl = kl + K * K;
  constexpr int NP = K * (K + 1) / 2;
  for (int t = tid; t < NP * NP; t += blockDim.x) Vl[t] = B[ib.V + t];
  for (int t = tid; t < K * K; t += blockDim.x) kl[t] = B[ib.keff + t];
  __syncthreads();
  ActInts I;
  I.V = Vl;
  I.keff = kl;
  I.hp = hp;
  I.Jm = L.Jm;
  I.Km = L.Km;
  I.k = K;
  I.np = K * (K + 1) / 2;
  I.inv_nel = d.na > 0 ? 1.0 / (2.0 * d.na) : 0.0;
  // h'_pq = k_pq + 1/2 sum_r (pr|rq)
  for (int t = tid; t < K * K; t += blockDim.x) {
    const int p = t / K, q = t - p * K;
    double v = I.keff[t];
    for (int r = 0; r < K; ++r) v += 0.5 * aeri(I, p, r, r, q);
    hp[t] = v;
  }
  __syncthreads();
  for (int t = tid; t < P * P; t += blockDim.x) {
    const int r = t / P, c = t - r * P;
    if (c < r) continue;
    double v = sector_element(I, L.strs, L.F, L.pidx[r], L.pidx[c]);
    if (r == c) v -= E0;
    Am[r * P + c] = (float)v;
    Am[c * P + r] = (float)v;
  }
  __syncthreads();
}

// Second half: the eigenpairs of A in FP32 (eigenvalues in L.plam, U
// [l][j] in the scratch and in Ug) and the lowest eigenvector as the
// initial vector in x (global) and L.tv.  FP32 holds the eigenvalues of
// the shifted block to about 1e-7 of its norm: ample for a preconditioner
// and a starting vector, neither of which sets the converged energy.
template <int K, int NE>
__device__ __forceinline__ void ps_eigen(const IncDev& d, const Lds& L, int P, uint64_t pk, float* Ug, double* xv,
                                         int& parity) {
  const int tid = threadIdx.x, nsi = (int)d.n_sym;
  float* Um = (float*)(L.et + ps_scratch_offset(d));
  float* Am = Um + P * P;
  float* cs = Am + P * P;
  int* pq = (int*)(cs + 2 * kPsMax);
  // stop at a squared off-diagonal part of 1e-2 of the squared norm (an
  // off-diagonal part near 10% of the matrix): the block only gives the
  // starting vector and a preconditioner, and on the 2,516 increments of the
  // 16-body workload the mean iteration count stayed at 34.3 from 1e-5 to
  // 1e-2 (34.9 at 5e-2) while the sweeps saved took 6% of the launch
  block_jacobi(Am, Um, P, cs, pq, L.red, parity, 1e-2);
  // eigenvalues and the lowest one (ties to the lower index)
  for (int j = tid; j < P; j += blockDim.x) L.plam[j] = (double)Am[j * P + j];
  int j0 = 0;
  float l0 = Am[0];
  for (int j = 1; j < P; ++j)
    if (Am[j * P + j] < l0) l0 = Am[j * P + j], j0 = j;
  for (int t = tid; t < P * P / 4; t += blockDim.x) ((float4*)Ug)[t] = ((const float4*)Um)[t];
  // the initial vector: column j0 of U on the block's entries, normalised
  // in FP64
  double acc[1] = {0.0};
  double xe[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int j = ps_pos(pk, e);
    xe[e] = j != 0x7f ? (double)Um[j * P + j0] : 0.0;
    acc[0] += xe[e] * xe[e];
  }
  block_sum_1b<1>(acc, L.red, parity);
  const double inv = 1.0 / sqrt(acc[0]);
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int i = tid + e * kBatchThreads;
    if (i < nsi) {
      xv[i] = xe[e] * inv;
      L.tv[i] = xe[e] * inv;
    }
  }
  __syncthreads();
}

// t_P = U diag(1 / (theta - lam)) U^T r_P with U the FP32 image in LDS (Us,
// [l][j]), r_P gathered from the full residual in v (LDS, every entry
// written by its owner before the call) and t_P scattered back into v over
// the block's entries; zP: LDS [kPsMax] doubles.  Each wave handles eight
// rows (eight lanes per row, eight terms each, summed by a fixed
// butterfly).  Three barriers.
__device__ inline void ps_apply(const float* Us, int P, double theta, const double* plam, const int* pidx,
                                double* v, double* zP) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = wave * 8 + (lane >> 3), part = lane & 7;
  __syncthreads();
  {
    // z_j = (sum_l U[l][j] r_l) / (theta - lam_j)
    double y = 0.0;
    if (row < P)
      for (int l = part * 8; l < part * 8 + 8 && l < P; ++l) y += (double)Us[l * P + row] * v[pidx[l]];
    y += __shfl_xor(y, 1, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 4, 64);
    if (row < P && part == 0) {
      double den = theta - plam[row];
      if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
      zP[row] = y / den;
    }
  }
  __syncthreads();
  {
    // t_l = sum_j U[l][j] z_j
    double t = 0.0;
    if (row < P)
      for (int j = part * 8; j < part * 8 + 8 && j < P; ++j) t += (double)Us[row * P + j] * zP[j];
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 4, 64);
    if (row < P && part == 0) v[pidx[row]] = t;
  }
  __syncthreads();
}

// Locally optimal block-free iteration (Davidson restarted every step to the
// three vectors {x, w, p}: the Ritz vector, its preconditioned residual and
// the previous search direction; LOBPCG with block size one).  The basis is
// kept orthonormal: w is orthogonalised against x and p (classical
// Gram-Schmidt, repeated when the norm drops by more than 1/sqrt(2)), and the
// new direction p is built from the Rayleigh-Ritz coefficients already
// orthogonal to the new x.  Vectors: x, w, p in V[0..2], their sigmas in
// S[0..2], w also in LDS for the next sigma.
template <int K>
__device__ __forceinline__ void solve_lobpcg(const SolveArgs& A, int pos, char* lds, int lds_bytes) {
  const int id = A.order[pos];
  const IncDev d = A.inc[id];
  Lds L = carve(lds, d, lds_bytes);
  const double* B = A.ints + d.int_off;
  const IntBlock ib = int_block(d.k);
  const double* Vm = B + ib.V;
  const int64_t ns = d.n_sym, st = d.stride;
  double* base = A.dav + d.vec_off;
  const int mmax = A.max_space;
  double* xv = base;
  double* wv = base + st;
  double* pv = base + 2 * st;
  double* ax = base + mmax * st;
  double* ap = ax + 2 * st;
  double* HD = base + 2 * mmax * st;
  double* X = HD + st;
  const int tid = threadIdx.x;
  int64_t ph[kPhases];
#pragma unroll
  for (int q = 0; q < kPhases; ++q) ph[q] = 0;
  const bool trace = A.phase != nullptr;
  int64_t t_start = trace ? clock64() : 0, t_mark = t_start;
#define IFCI_MARK(PH)                      \
  if (trace) {                             \
    const int64_t now_ = clock64();        \
    ph[PH] += now_ - t_mark;               \
    t_mark = now_;                         \
  }

  load_increment(d, L, A.tables, B, HD);
  argmin_block(HD, ns, L);
  const double E0 = L.scal[0];
  const int64_t guess = L.iscal[0];
  // vector entries per thread: the packed sector of the largest K-orbital shape
  constexpr int NE = (max_strings(K) * (max_strings(K) + 1) / 2 + kBatchThreads - 1) / kBatchThreads;
  int bsp = 0;  // buffer parity of block_sum_1b
  // P-space block: initial vector and block preconditioner (or the lowest
  // determinant and the diagonal preconditioner)
  float* Ug = (float*)(base + ps_image_offset(st, mmax));
  // P-space block: n_guess, capped per shape by the tuning table
  const int tp = A.tune.ps_block[K][A.precision == IFCI_MIXED ? 1 : 0];
  const int ng = tp >= 0 && tp < A.n_guess ? tp : A.n_guess;
  const int P = ng > 1 ? ps_size<K>(d, L, ng) : 0;
  float* Us = (float*)(L.et + ps_scratch_offset(d));
  double* zP = L.Gs;
  if (P > 0) {
    uint64_t pk;  // block positions of this thread's entries (ps_pos)
    ps_build<K, NE>(d, L, B, HD, E0, P, pk, bsp);
    IFCI_MARK(kPhPrologue);
    ps_eigen<K, NE>(d, L, P, pk, Ug, xv, bsp);
    IFCI_MARK(kPhRestart);
  } else {
    for (int64_t i = tid; i < ns; i += blockDim.x) {
      const double v = (i == guess) ? 1.0 : 0.0;
      L.tv[i] = v;
      xv[i] = v;
    }
    __syncthreads();
  }
  IFCI_MARK(kPhPrologue);

  // every vector of the increment addressed from `base` by a 32-bit offset
  const int nsi = (int)ns, sti = (int)st, mst = mmax * (int)st;
  const int ew64 = tuned_waves(et_waves_for<double, K>(d, L), A.tune.e_waves[K][0]);
  const int ew32 = tuned_waves(et_waves_for<float, K>(d, L), A.tune.e_waves[K][1]);
  int phase = (A.precision == IFCI_MIXED) ? 32 : 64;
  int iters = 0, status = IFCI_INC_NOT_CONVERGED;
  double theta = 0.0, resid = 1e300;
  const int64_t o = (int64_t)id - A.first;
  const bool evict = A.evict && A.evict[o] != 0;
  bool staged = false;   // cp / sp already hold the next sigma's input
  bool fresh = true;     // x has no sigma yet (start or precision switch)
  bool have_p = false;
  bool w_built = false;  // the diagonal-pair weights of the current precision are in LDS
  double xap = 0.0, pap = 0.0;  // x.Ap and p.Ap of the current basis

  while (true) {
    // ---- sigma of the vector in L.tv (x when fresh, else w)
    if (phase == 32)
      sigma_phase<float, K>(d, L, Vm, E0, ew32, staged, !w_built, false);
    else
      sigma_phase<double, K>(d, L, Vm, E0, ew64, staged, !w_built, false);
    w_built = true;
    staged = false;
    ++iters;
    // ---- this thread's NE entries of x, w, p, Ax, Ap and the diagonal, in
    // registers for the whole non-sigma part of the iteration (one round of
    // loads; sigma(w) is read from L.sp)
    // (32-bit indices clamped into range: every load is unconditional and
    // addressed from a uniform base; entries past ns are zeroed after)
    double rx[NE], rw[NE], rp[NE], rax[NE], rap[NE], rhd[NE], rs[NE];
    const bool use_w = !fresh, use_p = !fresh && have_p;
    // an opaque copy of the thread index: the element addresses are then
    // formed here, not hoisted out of the iteration loop into (spilled)
    // registers
    int tix = tid;
    asm volatile("" : "+v"(tix));
    // (issued before the barrier that ends sigma: a wave that has finished
    // its columns loads while the others still contract; each thread reads
    // only entries it wrote itself)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = min(tix + e * kBatchThreads, nsi - 1);
      rx[e] = base[i];
      rw[e] = base[sti + i];
      rp[e] = base[2 * sti + i];
      rax[e] = base[mst + i];
      rap[e] = base[mst + 2 * sti + i];
      rhd[e] = base[2 * mst + i];
    }
    __syncthreads();
    IFCI_MARK(kPhSigma);
    // the FP32 eigenvectors of the P-space block back into LDS (the E slices
    // of every sigma overwrite them); read before the correction needs them
    if (P > 0)
      for (int u = tix; u < P * P / 4; u += kBatchThreads) ((float4*)Us)[u] = ((const float4*)Ug)[u];
#pragma unroll
    for (int e = 0; e < NE; ++e) rs[e] = L.sp[min(tix + e * kBatchThreads, nsi - 1)];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const bool in = tid + e * kBatchThreads < nsi;
      if (!in) rx[e] = rs[e] = rhd[e] = 0.0;
      if (!in || !use_w) rw[e] = rax[e] = 0.0;
      if (!in || !use_p) rp[e] = rap[e] = 0.0;
    }
    double gxw = 0.0, gww = 0.0, gpw = 0.0;
    if (fresh) {
      // Ax = sigma(x), theta = x.Ax
      double acc[1] = {0.0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        rax[e] = rs[e];
        acc[0] += rx[e] * rs[e];
      }
      block_sum_1b<1>(acc, L.red, bsp);
      theta = acc[0];
      have_p = false;
    } else {
      // the new column of the 3 x 3 Rayleigh-Ritz matrix
      double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        acc[0] += rx[e] * rs[e];
        acc[1] += rw[e] * rs[e];
        acc[2] += rp[e] * rs[e];
      }
      block_sum_1b<3>(acc, L.red, bsp);
      gxw = acc[0];
      gww = acc[1];
      gpw = have_p ? acc[2] : 0.0;
    }
    IFCI_MARK(kPhSubspace);
    // ---- Rayleigh-Ritz on span{x, w, p}
    double cx[3] = {1.0, 0.0, 0.0}, cpv[3] = {0.0, 0.0, 0.0};
    bool new_p = false;
    if (!fresh) {
      // (without p the third basis vector is decoupled and placed far above)
      const double big = 1e30;
      double g[3][3] = {{theta, gxw, have_p ? xap : 0.0},
                        {gxw, gww, have_p ? gpw : 0.0},
                        {have_p ? xap : 0.0, have_p ? gpw : 0.0, have_p ? pap : big}};
      double z[3];
      double th;
      small_eig3(g, &th, z);
      if (!have_p) z[2] = 0.0;
      if (z[0] < 0.0) {
        z[0] = -z[0];
        z[1] = -z[1];
        z[2] = -z[2];
      }
      // new x and the direction p'' = (z1 w + z2 p) orthogonalised against x'
      const double rho = z[1] * z[1] + z[2] * z[2];
      cx[0] = z[0];
      cx[1] = z[1];
      cx[2] = z[2];
      const double pn = z[0] * sqrt(rho);
      if (pn > 1e-14) {
        cpv[0] = -rho * z[0] / pn;
        cpv[1] = z[0] * z[0] * z[1] / pn;
        cpv[2] = z[0] * z[0] * z[2] / pn;
        new_p = true;
      }
      // x'.Ap'' and p''.Ap'' from the 3 x 3 matrix (g was overwritten)
      const double G3[3][3] = {{theta, gxw, xap}, {gxw, gww, gpw}, {xap, gpw, pap}};
      double gp[3];
      for (int i = 0; i < 3; ++i) {
        gp[i] = 0.0;
        for (int j = 0; j < 3; ++j) gp[i] += G3[i][j] * cpv[j];
      }
      double nxap = 0.0, npap = 0.0;
      for (int i = 0; i < 3; ++i) {
        nxap += cx[i] * gp[i];
        npap += cpv[i] * gp[i];
      }
      theta = th;
      xap = nxap;
      pap = npap;
    }
    // ---- update x, Ax, p, Ap in registers; residual r = Ax - theta x and
    // correction t = r / (theta - (H_II - E0)) -- on the P-space entries the
    // block's exact inverse -- with its overlaps
    double rt[NE];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      double x = rx[e], sx = rax[e];
      if (!fresh) {
        const double w = rw[e], sw = rs[e], pp = rp[e], sp = rap[e];
        x = cx[0] * rx[e] + cx[1] * w + cx[2] * pp;
        sx = cx[0] * rax[e] + cx[1] * sw + cx[2] * sp;
        const double pnew = cpv[0] * rx[e] + cpv[1] * w + cpv[2] * pp;
        const double apnew = cpv[0] * rax[e] + cpv[1] * sw + cpv[2] * sp;
        if (new_p) {
          rp[e] = pnew;
          rap[e] = apnew;
        }
        rx[e] = x;
        rax[e] = sx;
      }
      const bool in = tid + e * kBatchThreads < nsi;
      const double r = in ? sx - theta * x : 0.0;
      rt[e] = r;
      acc[0] += r * r;
      if (P > 0 && in) L.tv[tix + e * kBatchThreads] = r;
    }
    // the block's entries: (H_II, I) up to its last one
    const double ps_h = P > 0 ? L.plam[kPsMax] : -1e300;
    const int ps_i = P > 0 ? L.pidx[P - 1] : -1;
    if (P > 0) ps_apply(Us, P, theta, L.plam, L.pidx, L.tv, zP);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tix + e * kBatchThreads;
      double den = theta - (rhd[e] - E0);
      if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
      const bool in_p = i < nsi && (rhd[e] < ps_h || (rhd[e] == ps_h && i <= ps_i));
      const double t = in_p ? L.tv[i] : rt[e] / den;
      rt[e] = t;
      acc[1] += t * t;
      acc[2] += rx[e] * t;
      acc[3] += (new_p ? rp[e] : 0.0) * t;
    }
    block_sum_1b<4>(acc, L.red, bsp);
    resid = sqrt(acc[0]);
    const double tt0 = acc[1];
    const double dxw = acc[2];
    const double dpw = new_p ? acc[3] : 0.0;
    const bool was_fresh = fresh;
    have_p = new_p || (have_p && fresh);
    if (fresh) have_p = false;
    fresh = false;
    // x, Ax (and p, Ap) back to memory
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tix + e * kBatchThreads;
      if (i < nsi) {
        base[i] = rx[e];
        base[mst + i] = rax[e];
        if (new_p) {
          base[2 * sti + i] = rp[e];
          base[mst + 2 * sti + i] = rap[e];
        }
      }
    }
    (void)was_fresh;
    IFCI_MARK(kPhPassA);

    const double tol = (phase == 32) ? A.r_tol_inner : A.r_tol;
    if (evict) {
      status = IFCI_INC_EVICTED;
      break;
    }
    if (resid <= tol) {
      if (phase == 32) {
        // FP64 refinement: sigma of x in FP64, then continue in FP64
        phase = 64;
        w_built = false;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          const int i = tix + e * kBatchThreads;
          if (i < nsi) L.tv[i] = rx[e];
        }
        fresh = true;
        __syncthreads();
        if (iters >= A.max_iter) break;
        continue;
      }
      status = IFCI_INC_DONE;
      break;
    }
    if (iters >= A.max_iter) break;
    // ---- orthogonalise t against x and p (twice if it cancels), normalise:
    // the next w
    double acc2[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      double t = rt[e] - dxw * rx[e];
      if (have_p) t -= dpw * rp[e];
      rt[e] = t;
      acc2[0] += t * t;
      acc2[1] += rx[e] * t;
      acc2[2] += (have_p ? rp[e] : 0.0) * t;
    }
    block_sum_1b<3>(acc2, L.red, bsp);
    double tt = acc2[0];
    if (tt < 0.5 * tt0) {
      const double c0 = acc2[1], c1 = have_p ? acc2[2] : 0.0;
      double acc3[1] = {0.0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        double t = rt[e] - c0 * rx[e];
        if (have_p) t -= c1 * rp[e];
        rt[e] = t;
        acc3[0] += t * t;
      }
      block_sum_1b<1>(acc3, L.red, bsp);
      tt = acc3[0];
    }
    if (!(tt > 1e-28)) break;  // no new direction: stagnated
    const double inv = 1.0 / sqrt(tt);
    // w to memory and, in the layout of the next sigma, straight into cp
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tix + e * kBatchThreads;
      if (i < nsi) {
        const double t = rt[e] * inv;
        base[sti + i] = t;
        if (phase == 32)
          stage_entry<float>(d, L, i, t);
        else
          stage_entry<double>(d, L, i, t);
      }
    }
    staged = true;
    __syncthreads();
    IFCI_MARK(kPhOrtho);
  }
  for (int64_t i = tid; i < ns; i += blockDim.x) X[i] = xv[i];
  if (trace && tid == 0) {
    ph[kPhIters] = iters;
    ph[kPhTotal] = clock64() - t_start;
#pragma unroll
    for (int q = 0; q < kPhases; ++q) A.phase[(int64_t)id * kPhases + q] = ph[q];
  }
#undef IFCI_MARK
  if (tid == 0) {
    const double e = theta + E0 + B[ib.misc + 0] + A.e_const;
    if (A.e_out) A.e_out[o] = e;
    if (A.status_out) A.status_out[o] = status;
    if (A.iters_out) A.iters_out[o] = iters;
    if (A.resid_out) A.resid_out[o] = resid;
  }
}

// One kernel per solver so that each gets its own register allocation.
// Thick-restart Davidson with the vector work of the three-vector solver:
// every thread owns NE entries of each vector, and the basis V and its
// sigmas S (mmax vectors each, global memory) are streamed in passes, each
// over the basis index with the entries unrolled: (A) x = V y, Ax = S y,
// the residual and the preconditioned correction t (with the P-space block
// when there is one); (B) the overlaps c_j = V_j.t and d_j = S_j.t, summed
// per wave as they are formed; at a restart (R) the kept Ritz vectors and
// their sigmas, written over the first slots; (C) classical Gram-Schmidt
// of t against the basis, repeated when its norm drops by more than
// 1/sqrt 2.  The new column of the subspace matrix needs no further pass:
// with t' = t - sum_k c_k B_k, S_j.t' = d_j - sum_k c_k G[k][j]; only its
// diagonal entry waits for the new sigma (one dot product).  The residual
// is formed from the stored vectors, so the convergence test does not
// depend on the subspace matrix being exact.  Nothing but scalars stays in
// registers across a sigma.
template <int K>
__device__ __forceinline__ void solve_dav(const SolveArgs& A, int pos, char* lds, int lds_bytes) {
  const int id = A.order[pos];
  const IncDev d = A.inc[id];
  Lds L = carve(lds, d, lds_bytes);
  const double* B = A.ints + d.int_off;
  const IntBlock ib = int_block(d.k);
  const double* Vm = B + ib.V;
  const int64_t ns = d.n_sym, st = d.stride;
  double* base = A.dav + d.vec_off;
  const int mmax = A.max_space;
  double* HD = base + 2 * mmax * st;
  double* X = HD + st;
  const int tid = threadIdx.x;
  int64_t ph[kPhases];
#pragma unroll
  for (int q = 0; q < kPhases; ++q) ph[q] = 0;
  const bool trace = A.phase != nullptr;
  int64_t t_start = trace ? clock64() : 0, t_mark = t_start;
#define IFCI_MARK(PH)                      \
  if (trace) {                             \
    const int64_t now_ = clock64();        \
    ph[PH] += now_ - t_mark;               \
    t_mark = now_;                         \
  }

  load_increment(d, L, A.tables, B, HD);
  argmin_block(HD, ns, L);
  const double E0 = L.scal[0];
  const int64_t guess = L.iscal[0];
  constexpr int NE = (max_strings(K) * (max_strings(K) + 1) / 2 + kBatchThreads - 1) / kBatchThreads;
  int bsp = 0;
  float* Ug = (float*)(base + ps_image_offset(st, mmax));
  // P-space block: n_guess, capped per shape by the tuning table
  const int tp = A.tune.ps_block[K][A.precision == IFCI_MIXED ? 1 : 0];
  const int ng = tp >= 0 && tp < A.n_guess ? tp : A.n_guess;
  const int P = ng > 1 ? ps_size<K>(d, L, ng) : 0;
  float* Us = (float*)(L.et + ps_scratch_offset(d));
  if (P > 0) {
    uint64_t pk;
    ps_build<K, NE>(d, L, B, HD, E0, P, pk, bsp);
    IFCI_MARK(kPhPrologue);
    ps_eigen<K, NE>(d, L, P, pk, Ug, base, bsp);
    IFCI_MARK(kPhRestart);
  } else {
    for (int64_t i = tid; i < ns; i += blockDim.x) {
      const double v = (i == guess) ? 1.0 : 0.0;
      L.tv[i] = v;
      base[i] = v;
    }
  }
  for (int i = tid; i < 256; i += blockDim.x) L.G[i] = 0.0;
  __syncthreads();
  IFCI_MARK(kPhPrologue);

  const int nsi = (int)ns, sti = (int)st, mst = mmax * (int)st;
  const int lane = tid & 63, wave = tid >> 6, nw = kBatchThreads >> 6;
  const int ew64 = tuned_waves(et_waves_for<double, K>(d, L), A.tune.e_waves[K][0]);
  const int ew32 = tuned_waves(et_waves_for<float, K>(d, L), A.tune.e_waves[K][1]);
  int phase = (A.precision == IFCI_MIXED) ? 32 : 64;
  int m = 0, iters = 0, status = IFCI_INC_NOT_CONVERGED;
  double theta = 0.0, resid = 1e300;
  const int64_t o = (int64_t)id - A.first;
  const bool evict = A.evict && A.evict[o] != 0;
  const int keep = mmax / 2 < kKeep ? mmax / 2 : kKeep;
  bool staged = false;
  bool w_built = false;
  // per-wave partial overlaps [kMaxSpace][2][8]: the eigenvector scratch of
  // subspace_solve, free once it returns
  double* wpart = L.Qv;

  while (true) {
    // ---- sigma of v_m -> S_m, and G[m][m]
    if (phase == 32)
      sigma_phase<float, K>(d, L, Vm, E0, ew32, staged, !w_built);
    else
      sigma_phase<double, K>(d, L, Vm, E0, ew64, staged, !w_built);
    w_built = true;
    staged = false;
    ++iters;
    int tix = tid;
    asm volatile("" : "+v"(tix));
    {
      double acc[1] = {0.0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = tix + e * kBatchThreads;
        if (i < nsi) {
          const double sv = L.sp[i];
          acc[0] += base[m * sti + i] * sv;
          base[mst + m * sti + i] = sv;
        }
      }
      block_sum_1b<1>(acc, L.red, bsp);
      if (tid == 0) L.G[m * 16 + m] = acc[0];
    }
    // the FP32 eigenvectors of the P-space block back into LDS
    if (P > 0)
      for (int u = tix; u < P * P / 4; u += kBatchThreads) ((float4*)Us)[u] = ((const float4*)Ug)[u];
    __syncthreads();
    IFCI_MARK(kPhSigma);
    subspace_solve(L, m);
    theta = L.scal[20];
    IFCI_MARK(kPhSubspace);
    const bool restart = (m + 1 == mmax);
    // ---- pass A: x = V y, Ax = S y, r, t
    double rx[NE], rax[NE], rt[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) rx[e] = rax[e] = 0.0;
#pragma unroll 4
    for (int j = 0; j <= m; ++j) {
      const double yj = L.y[j];
      const double* vj = base + j * sti;
      const double* sj = base + mst + j * sti;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = min(tix + e * kBatchThreads, nsi - 1);
        rx[e] += yj * vj[i];
        rax[e] += yj * sj[i];
      }
    }
    double accr = 0.0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const bool in = tix + e * kBatchThreads < nsi;
      const double r = in ? rax[e] - theta * rx[e] : 0.0;
      rt[e] = r;
      accr += r * r;
      if (P > 0 && in) L.tv[tix + e * kBatchThreads] = r;
    }
    const double ps_h = P > 0 ? L.plam[kPsMax] : -1e300;
    const int ps_i = P > 0 ? L.pidx[P - 1] : -1;
    if (P > 0) ps_apply(Us, P, theta, L.plam, L.pidx, L.tv, L.Gs);
    double acct = 0.0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tix + e * kBatchThreads;
      const double hd = HD[min(i, nsi - 1)];
      double den = theta - (hd - E0);
      if (fabs(den) < 1e-8) den = (den < 0.0) ? -1e-8 : 1e-8;
      const bool in_p = i < nsi && (hd < ps_h || (hd == ps_h && i <= ps_i));
      const double t = in_p ? L.tv[i] : rt[e] / den;
      rt[e] = i < nsi ? t : 0.0;
      acct += rt[e] * rt[e];
    }
    IFCI_MARK(kPhPassA);
    // ---- pass B: c_j = V_j.t, d_j = S_j.t (j <= m), wave sums into wpart
#pragma unroll 4
    for (int j = 0; j <= m; ++j) {
      const double* vj = base + j * sti;
      const double* sj = base + mst + j * sti;
      double c = 0.0, dd = 0.0;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = min(tix + e * kBatchThreads, nsi - 1);
        c += vj[i] * rt[e];
        dd += sj[i] * rt[e];
      }
      c = wave_sum(c);
      dd = wave_sum(dd);
      if (lane == 0) {
        wpart[(2 * j) * 8 + wave] = c;
        wpart[(2 * j + 1) * 8 + wave] = dd;
      }
    }
    double tt0;
    {
      double a2[2] = {accr, acct};
      block_sum_1b<2>(a2, L.red, bsp);
      resid = sqrt(a2[0]);
      tt0 = a2[1];
      // Gs [0, 16) c, [16, 32) d: the wave partials in a fixed order
      if (tid < 2 * (m + 1)) {
        const int j = tid >> 1, w = tid & 1;
        double sum = 0.0;
        for (int q = 0; q < nw; ++q) sum += wpart[(2 * j + w) * 8 + q];
        L.Gs[w * kMaxSpace + j] = sum;
      }
    }
    IFCI_MARK(kPhRestart);

    const double tol = (phase == 32) ? A.r_tol_inner : A.r_tol;
    bool done = false;
    if (evict) {
      status = IFCI_INC_EVICTED;
      done = true;
    } else if (resid <= tol && phase == 64) {
      status = IFCI_INC_DONE;
      done = true;
    } else if (iters >= A.max_iter) {
      done = true;
    }
    if (done) {
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = tix + e * kBatchThreads;
        if (i < nsi) X[i] = rx[e];
      }
      break;
    }
    if (resid <= tol) {
      // FP64 refinement: restart from x with FP64 sigma
      phase = 64;
      w_built = false;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = tix + e * kBatchThreads;
        if (i < nsi) {
          L.tv[i] = rx[e];
          base[i] = rx[e];
        }
      }
      for (int i = tid; i < 256; i += blockDim.x) L.G[i] = 0.0;
      m = 0;
      __syncthreads();
      continue;
    }
    __syncthreads();
    // ---- restart: the keep lowest Ritz vectors and their sigmas over slots
    // 0 .. keep-1 (slot 0: x and Ax from pass A), each entry read in full
    // before it is written
    if (restart) {
      int qc[kKeep];
#pragma unroll
      for (int k = 0; k < kKeep; ++k) qc[k] = L.perm[k < keep ? k : 0];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = min(tix + e * kBatchThreads, nsi - 1);
        const bool in = tix + e * kBatchThreads < nsi;
        double nv[kKeep], nsg[kKeep];
#pragma unroll
        for (int k = 0; k < kKeep; ++k) nv[k] = nsg[k] = 0.0;
        for (int j = 0; j <= m; ++j) {
          const double v = base[j * sti + i], sv = base[mst + j * sti + i];
#pragma unroll
          for (int k = 1; k < kKeep; ++k) {
            const double q = L.Qp[j * 16 + qc[k]];
            nv[k] += q * v;
            nsg[k] += q * sv;
          }
        }
        if (in) {
          base[i] = rx[e];
          base[mst + i] = rax[e];
#pragma unroll
          for (int k = 1; k < kKeep; ++k)
            if (k < keep) {
              base[k * sti + i] = nv[k];
              base[mst + k * sti + i] = nsg[k];
            }
        }
      }
    }
    // overlaps with the basis t is orthogonalised against, into Gs [64, 80)
    // (c) and [96, 112) (d): after a restart the kept Ritz vectors, c' = Q^T c
    // and d' = Q^T d, and the subspace matrix becomes diag of their values
    const int mb = restart ? keep - 1 : m;
    if (tid < kMaxSpace) {
      double c = 0.0, dd = 0.0;
      if (restart) {
        if (tid < keep) {
          const int q = L.perm[tid];
          for (int j = 0; j <= m; ++j) {
            c += L.Qp[j * 16 + q] * L.Gs[j];
            dd += L.Qp[j * 16 + q] * L.Gs[kMaxSpace + j];
          }
        }
      } else if (tid <= m) {
        c = L.Gs[tid];
        dd = L.Gs[kMaxSpace + tid];
      }
      L.Gs[64 + tid] = c;
      L.Gs[96 + tid] = dd;
    }
    __syncthreads();
    if (restart) {
      for (int i = tid; i < 256; i += blockDim.x) {
        L.G[i] = 0.0;
        L.Qp[i] = ((i >> 4) == (i & 15)) ? 1.0 : 0.0;
      }
      __syncthreads();
      if (tid < keep) {
        L.G[tid * 16 + tid] = L.ev[tid];
        L.Lam[tid] = L.ev[tid];
      }
    }
    // ---- pass C: t -= sum_j c_j B_j; if its norm dropped below half,
    // the overlaps with t' and a second subtraction
    double tt = 0.0;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll 2
      for (int j = 0; j <= mb; ++j) {
        const double c = L.Gs[(pass == 0 ? 64 : 0) + j];
        const double* bj = base + j * sti;
#pragma unroll
        for (int e = 0; e < NE; ++e) rt[e] -= c * bj[min(tix + e * kBatchThreads, nsi - 1)];
      }
      double a1[1] = {0.0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        rt[e] = tix + e * kBatchThreads < nsi ? rt[e] : 0.0;
        a1[0] += rt[e] * rt[e];
      }
      block_sum_1b<1>(a1, L.red, bsp);
      tt = a1[0];
      if (pass == 1 || !(tt < 0.5 * tt0)) break;
      // overlaps B_j.t' into Gs [0, 16), accumulated into c
#pragma unroll 2
      for (int j = 0; j <= mb; ++j) {
        const double* bj = base + j * sti;
        double c = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e) c += bj[min(tix + e * kBatchThreads, nsi - 1)] * rt[e];
        c = wave_sum(c);
        if (lane == 0) wpart[j * 8 + wave] = c;
      }
      __syncthreads();
      if (tid <= mb) {
        double sum = 0.0;
        for (int q = 0; q < nw; ++q) sum += wpart[tid * 8 + q];
        L.Gs[tid] = sum;
        L.Gs[64 + tid] += sum;
      }
      __syncthreads();
    }
    if (!(tt > 1e-28)) {  // no new direction: stagnated
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int i = tix + e * kBatchThreads;
        if (i < nsi) X[i] = rx[e];
      }
      break;
    }
    const double inv = 1.0 / sqrt(tt);
    // new column of the subspace matrix: S_j.t' / |t'| with
    // S_j.t' = d_j - sum_k c_k G[k][j] (c accumulated over both passes)
    const int mn = mb + 1;
    if (tid <= mb) {
      double g = L.Gs[96 + tid];
      for (int k = 0; k <= mb; ++k) g -= L.Gs[64 + k] * L.G[k * 16 + tid];
      g *= inv;
      L.G[tid * 16 + mn] = g;
      L.G[mn * 16 + tid] = g;
    }
    // the new basis vector: global slot mn and the next sigma's input
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int i = tix + e * kBatchThreads;
      const double t = rt[e] * inv;
      if (i < nsi) {
        base[mn * sti + i] = t;
        if (phase == 32)
          stage_entry<float>(d, L, i, t);
        else
          stage_entry<double>(d, L, i, t);
      }
    }
    m = mn;
    staged = true;
    __syncthreads();
    IFCI_MARK(kPhOrtho);
  }
  if (trace && tid == 0) {
    ph[kPhIters] = iters;
    ph[kPhTotal] = clock64() - t_start;
#pragma unroll
    for (int q = 0; q < kPhases; ++q) A.phase[(int64_t)id * kPhases + q] = ph[q];
  }
#undef IFCI_MARK
  if (tid == 0) {
    const double e = theta + E0 + B[ib.misc + 0] + A.e_const;
    if (A.e_out) A.e_out[o] = e;
    if (A.status_out) A.status_out[o] = status;
    if (A.iters_out) A.iters_out[o] = iters;
    if (A.resid_out) A.resid_out[o] = resid;
  }
}

__global__ void __launch_bounds__(kBatchThreads) batched_kernel(SolveArgs A, int lds_bytes) {
  extern __shared__ __align__(16) char lds[];
  const int pos = blockIdx.x;
  if (pos >= A.count) return;
  const int k = A.inc[A.order[pos]].k;
  switch (k) {
    case 1: solve_dav<1>(A, pos, lds, lds_bytes); break;
    case 2: solve_dav<2>(A, pos, lds, lds_bytes); break;
    case 3: solve_dav<3>(A, pos, lds, lds_bytes); break;
    case 4: solve_dav<4>(A, pos, lds, lds_bytes); break;
    case 5: solve_dav<5>(A, pos, lds, lds_bytes); break;
    case 6: solve_dav<6>(A, pos, lds, lds_bytes); break;
    case 7: solve_dav<7>(A, pos, lds, lds_bytes); break;
    case 8: solve_dav<8>(A, pos, lds, lds_bytes); break;
    default: break;
  }
}

__global__ void __launch_bounds__(kBatchThreads) batched_lobpcg_kernel(SolveArgs A, int lds_bytes) {
  extern __shared__ __align__(16) char lds[];
  const int pos = blockIdx.x;
  if (pos >= A.count) return;
  const int k = A.inc[A.order[pos]].k;
  switch (k) {
    case 1: solve_lobpcg<1>(A, pos, lds, lds_bytes); break;
    case 2: solve_lobpcg<2>(A, pos, lds, lds_bytes); break;
    case 3: solve_lobpcg<3>(A, pos, lds, lds_bytes); break;
    case 4: solve_lobpcg<4>(A, pos, lds, lds_bytes); break;
    case 5: solve_lobpcg<5>(A, pos, lds, lds_bytes); break;
    case 6: solve_lobpcg<6>(A, pos, lds, lds_bytes); break;
    case 7: solve_lobpcg<7>(A, pos, lds, lds_bytes); break;
    case 8: solve_lobpcg<8>(A, pos, lds, lds_bytes); break;
    default: break;
  }
}

// Single sigma through the on-chip path (for checking it): full symmetric c
// in, full sigma out, both [n_det] FP64.
template <int K>
__device__ void sigma_one(const IncDev d, const double* __restrict__ ints, const int32_t* __restrict__ tables,
                          const double* __restrict__ c, double* __restrict__ sig, int precision,
                          char* lds, int lds_bytes) {
  Lds L = carve(lds, d, lds_bytes);
  const int n = d.n_str;
  load_tables(d, L, tables);
  for (int64_t i = threadIdx.x; i < d.n_sym; i += blockDim.x) {
    int a, b;
    unpack(i, &a, &b);
    const double v = c[(int64_t)a * n + b];
    L.tv[i] = (a == b) ? v : v * kSqrt2;
  }
  __syncthreads();
  const double* Vm = ints + d.int_off + int_block(d.k).V;
  if (precision == IFCI_MIXED)
    sigma_phase<float, K>(d, L, Vm, 0.0, et_waves_for<float, K>(d, L));
  else
    sigma_phase<double, K>(d, L, Vm, 0.0, et_waves_for<double, K>(d, L));
  for (int64_t i = threadIdx.x; i < d.n_sym; i += blockDim.x) {
    int a, b;
    unpack(i, &a, &b);
    const double v = (a == b) ? L.sp[i] : L.sp[i] * kRSqrt2;
    sig[(int64_t)a * n + b] = v;
    sig[(int64_t)b * n + a] = v;
  }
}

__global__ void __launch_bounds__(kBatchThreads) sigma_one_kernel(const IncDev* __restrict__ incs, int inc,
                                                                  const double* __restrict__ ints,
                                                                  const int32_t* __restrict__ tables,
                                                                  const double* c, double* sig,
                                                                  int precision, int lds_bytes) {
  extern __shared__ __align__(16) char lds[];
  const IncDev d = incs[inc];
  switch (d.k) {
    case 1: sigma_one<1>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 2: sigma_one<2>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 3: sigma_one<3>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 4: sigma_one<4>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 5: sigma_one<5>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 6: sigma_one<6>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 7: sigma_one<7>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    case 8: sigma_one<8>(d, ints, tables, c, sig, precision, lds, lds_bytes); break;
    default: break;
  }
}

// LDS the batched solver needs for an increment: the persistent part plus
// the larger of the transient part and one FP64 E slice.
int64_t batched_lds_bytes(int k, int n_str, int n_link) {
  const int64_t tr = transient_bytes(n_str), sl = et_slice_bytes(k, n_str, 8);
  return persistent_bytes(k, n_str, n_link) + (tr > sl ? tr : sl) + wt_bytes(k, 8) + 16;
}
// LDS that gives every wave of the workgroup its FP64 E slice.
int64_t batched_lds_want(int k, int n_str, int n_link) {
  const int64_t tr = transient_bytes(n_str), sl = (kBatchThreads / 64) * et_slice_bytes(k, n_str, 8);
  return persistent_bytes(k, n_str, n_link) + (tr > sl ? tr : sl) + wt_bytes(k, 8) + 16;
}

hipError_t launch_batched(const SolveArgs& A, int lds_bytes, hipStream_t st) {
  hipError_t e = allow_max_lds((const void*)batched_kernel);
  if (e == hipSuccess) e = allow_max_lds((const void*)batched_lobpcg_kernel);
  if (e != hipSuccess) return e;
  if (A.max_space == 3)
    hipLaunchKernelGGL(batched_lobpcg_kernel, dim3(A.count), dim3(kBatchThreads), lds_bytes, st, A, lds_bytes);
  else
    hipLaunchKernelGGL(batched_kernel, dim3(A.count), dim3(kBatchThreads), lds_bytes, st, A, lds_bytes);
  return hipGetLastError();
}

hipError_t launch_sigma_one(const IncDev* incs, int inc, const double* ints, const int32_t* tables,
                            const double* c, double* sig, int precision, int lds_bytes, hipStream_t st) {
  const hipError_t e = allow_max_lds((const void*)sigma_one_kernel);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sigma_one_kernel, dim3(1), dim3(kBatchThreads), lds_bytes, st, incs, inc, ints, tables,
                     c, sig, precision, lds_bytes);
  return hipGetLastError();
}

}  // namespace ifci
