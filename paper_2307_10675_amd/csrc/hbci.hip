// Heat-bath selected CI with a second-order Epstein-Nesbet correction for
// one increment (paper, Methods, iFCI subsection, the HBCI paragraph: the
// paper's increment solver; the method of Holmes, Tubman and Umrigar,
// J. Chem. Theory Comput. 12, 3674 (2016)).
//
// Determinants are 64-bit keys over the increment's k active orbitals: bit
// p is orbital p with spin alpha, bit 32 + p the same orbital with spin beta.
// The core's operators stand first, then alpha, then beta, each ascending, so
// the matrix elements are those of the active Hamiltonian
//   sum_pq h'_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps)
// with h' the frozen-core one-electron operator (Slater-Condon rules in that
// determinant convention); the constant E_core + e_const is added only to the
// energies handed back.
//
// Device data, all in the caller's work buffer:
//  * the variational space V: keys in insertion order, an open-addressing
//    hash table key -> index (linear probing, MurmurHash3's 64-bit
//    finaliser), every key's spin-flipped partner, the diagonal;
//  * H over V without its diagonal as CSR, rebuilt after every selection;
//  * the Davidson basis and sigma vectors;
//  * the PT2 external space: a second hash table key -> N_a.
// Kernels that walk the excitations of a determinant give it one wavefront;
// the lanes share its occupied/empty orbital lists in LDS and stride over
// the flat list of its single and double replacements.  The integrals sit
// in LDS: h' (k x k) and (pq|rs) packed over pairs of orbital pairs (at
// most 9316 doubles for k = 16).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "launch.hpp"

namespace ifci {

void set_error(const std::string& msg);

namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kNB = 512;        // workgroups of the vector kernels
// Waves per workgroup of the kernels that hold the integrals in LDS: at 16
// orbitals (77 KB) two workgroups fit a CU, so 16 waves each keep 32 waves
// of table probes in flight per CU.
constexpr int kWaves = 16;
constexpr int kMaxM = 16;       // largest Davidson subspace
constexpr int kParts = kMaxM + 1;
constexpr int kKeepRitz = 4;    // Ritz vectors kept at a Davidson restart

enum : unsigned { kFlagDetCap = 1u, kFlagExtCap = 2u, kFlagDuplicate = 4u, kFlagNoPartner = 8u };

struct HbciCtl {
  unsigned long long n_det;  // keys in V
  unsigned long long n_ext;  // keys in the external table
  unsigned int flags;
  unsigned int pad;
  double e_core;
  long long nnz;
};

struct Coef {
  double v[kMaxM];
};

struct CoefKeep {
  double v[kMaxM][kKeepRitz];
};

__device__ __forceinline__ uint64_t hmix(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__host__ __device__ __forceinline__ int tri2(int a, int b) { return a >= b ? (a * (a + 1) >> 1) + b : (b * (b + 1) >> 1) + a; }

__device__ __forceinline__ double G(const double* g, int p, int q, int r, int s) {
  return g[tri2(tri2(p, q), tri2(r, s))];
}

// (-1)^(occupied orbitals of s strictly between x and y)
__device__ __forceinline__ double phase(uint32_t s, int x, int y) {
  const int lo = x < y ? x : y, hi = x < y ? y : x;
  const uint32_t m = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
  return (__popc(s & m) & 1) ? -1.0 : 1.0;
}

__host__ __device__ __forceinline__ uint64_t flip_key(uint64_t key) { return (key >> 32) | (key << 32); }

// A flip pair's representative: the smaller of a key and its partner.  In
// the solve path vectors are flip-symmetric (c_a = c_flip(a), and H commutes
// with the flip), so only representatives are walked: a row of H, a
// selection source or a PT2 source stands for its partner too.
__device__ __forceinline__ bool canonical(uint64_t key) { return key <= flip_key(key); }

// ---------------------------------------------------------------- hash tables

__device__ __forceinline__ int32_t ht_find(const uint64_t* keys, const int32_t* vals, uint64_t mask, uint64_t key) {
  uint64_t h = hmix(key) & mask;
  for (uint64_t n = 0; n <= mask; ++n) {
    const uint64_t kk = keys[h];
    if (kk == key) return vals[h];
    if (kk == kEmpty) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

// Slot of key, inserting it when absent (*fresh then true); -1 when the
// probe went round the whole table.  A plain load may still see EMPTY where
// another wave has just claimed the slot; the compare-and-swap settles it.
__device__ __forceinline__ int64_t ht_insert(uint64_t* keys, uint64_t mask, uint64_t key, bool* fresh) {
  uint64_t h = hmix(key) & mask;
  for (uint64_t n = 0; n <= mask; ++n) {
    uint64_t kk = keys[h];
    if (kk == kEmpty)
      kk = atomicCAS((unsigned long long*)(keys + h), (unsigned long long)kEmpty, (unsigned long long)key);
    if (kk == kEmpty) {
      *fresh = true;
      return (int64_t)h;
    }
    if (kk == key) {
      *fresh = false;
      return (int64_t)h;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

struct Space {
  uint64_t* dets;
  uint64_t* keys;
  int32_t* vals;
  uint64_t mask;
  int64_t cap;
  HbciCtl* ctl;
};

__device__ __forceinline__ void add_det(const Space& V, uint64_t key) {
  bool fresh = false;
  const int64_t h = ht_insert(V.keys, V.mask, key, &fresh);
  if (h < 0) {
    atomicOr(&V.ctl->flags, kFlagDetCap);
    return;
  }
  if (!fresh) return;
  const unsigned long long idx = atomicAdd(&V.ctl->n_det, 1ull);
  if ((int64_t)idx < V.cap) {
    V.dets[idx] = key;
    V.vals[h] = (int32_t)idx;
  } else {
    V.vals[h] = -1;
    atomicOr(&V.ctl->flags, kFlagDetCap);
  }
}

// A slot of the external table: the key and its N_a side by side, so that a
// probe and the atomic update that follows touch one cache line.
struct alignas(16) ExtSlot {
  uint64_t key;
  double val;
};

// (each slot taken is listed in elist, so that the final sum visits the
// filled slots only)
__device__ __forceinline__ void ext_add(ExtSlot* et, int64_t* elist, uint64_t emask, int64_t cap, uint64_t key,
                                        double v, HbciCtl* ctl) {
  uint64_t h = hmix(key) & emask;
  for (uint64_t n = 0; n <= emask; ++n) {
    uint64_t kk = et[h].key;
    if (kk == kEmpty) {
      kk = atomicCAS((unsigned long long*)&et[h].key, (unsigned long long)kEmpty, (unsigned long long)key);
      if (kk == kEmpty) {
        const int64_t at = (int64_t)atomicAdd(&ctl->n_ext, 1ull);
        if (at < cap)
          elist[at] = (int64_t)h;
        else
          atomicOr(&ctl->flags, kFlagExtCap);
        atomicAdd(&et[h].val, v);
        return;
      }
    }
    if (kk == key) {
      atomicAdd(&et[h].val, v);
      return;
    }
    h = (h + 1) & emask;
  }
  atomicOr(&ctl->flags, kFlagExtCap);
}

// ------------------------------------------------------ integrals in LDS

struct Lds {
  double* h1;      // [k][k]
  double* g;       // packed (pq|rs)
  uint8_t* lo;     // pair decode: u = hi (hi - 1) / 2 + lo, lo < hi < 16
  uint8_t* hi;
  uint8_t* lists;  // per wave: occ alpha, empty alpha, occ beta, empty beta (16 each)
};

__host__ __device__ inline int packed_count(int k) {
  const int np = k * (k + 1) / 2;
  return np * (np + 1) / 2;
}

__host__ inline int lds_bytes_for(int k) { return (k * k + packed_count(k)) * 8 + 256 + kWaves * 64; }

__device__ Lds load_lds(const double* ints, int k) {
  extern __shared__ __align__(16) unsigned char smem[];
  Lds s;
  const int nint = k * k + packed_count(k);
  s.h1 = (double*)smem;
  s.g = s.h1 + k * k;
  s.lo = smem + nint * 8;
  s.hi = s.lo + 128;
  s.lists = s.lo + 256;
  for (int t = threadIdx.x; t < nint; t += blockDim.x) s.h1[t] = ints[t];
  for (int t = threadIdx.x; t < 120; t += blockDim.x) {
    int j = 1;
    while ((j + 1) * j / 2 <= t) ++j;
    s.lo[t] = (uint8_t)(t - j * (j - 1) / 2);
    s.hi[t] = (uint8_t)j;
  }
  __syncthreads();
  return s;
}

// --------------------------------------------------------- matrix elements

__device__ double diag_val(const Lds& s, int k, uint32_t A, uint32_t B) {
  double e = 0.0;
  for (uint32_t m = A; m; m &= m - 1) {
    const int p = __builtin_ctz(m);
    e += s.h1[p * k + p];
    for (uint32_t n = A; n; n &= n - 1) {
      const int q = __builtin_ctz(n);
      e += 0.5 * (G(s.g, p, p, q, q) - G(s.g, p, q, q, p));
    }
    for (uint32_t n = B; n; n &= n - 1) e += G(s.g, p, p, __builtin_ctz(n), __builtin_ctz(n));
  }
  for (uint32_t m = B; m; m &= m - 1) {
    const int p = __builtin_ctz(m);
    e += s.h1[p * k + p];
    for (uint32_t n = B; n; n &= n - 1) {
      const int q = __builtin_ctz(n);
      e += 0.5 * (G(s.g, p, p, q, q) - G(s.g, p, q, q, p));
    }
  }
  return e;
}

// <D'|H|D> for D' = a+_r a_p D within string S (the other string O)
__device__ double single_val(const Lds& s, int k, uint32_t S, uint32_t O, int p, int r) {
  double v = s.h1[r * k + p];
  for (uint32_t m = S; m; m &= m - 1) {
    const int q = __builtin_ctz(m);
    v += G(s.g, r, p, q, q) - G(s.g, r, q, q, p);
  }
  for (uint32_t m = O; m; m &= m - 1) {
    const int q = __builtin_ctz(m);
    v += G(s.g, r, p, q, q);
  }
  return phase(S, p, r) * v;
}

// D' = a+_r a+_s a_q a_p D = a+_r a_p (a+_s a_q D) within one string S:
// <D'|H|D> = sign ((rp|sq) - (rq|sp))
__device__ __forceinline__ double double_same(const double* g, uint32_t S, int p, int q, int r, int s) {
  const uint32_t S1 = S ^ (1u << q) ^ (1u << s);
  return phase(S, q, s) * phase(S1, p, r) * (G(g, r, p, s, q) - G(g, r, q, s, p));
}

// A determinant's replacements, one flat index t over: alpha singles, beta
// singles, alpha-alpha doubles, beta-beta doubles, alpha-beta doubles.
struct Det {
  uint32_t A, B;
  int na, nb, va, vb, ca2, cb2;
  int sa, sb, daa, dbb, total;
  const uint8_t* L;
};

__device__ __forceinline__ Det make_det(uint64_t key, int k, uint8_t* L, int lane) {
  Det d;
  d.A = (uint32_t)key;
  d.B = (uint32_t)(key >> 32);
  __builtin_amdgcn_wave_barrier();
  if (lane < k) {
    const int below = __popc(d.A & ((1u << lane) - 1u));
    if (d.A >> lane & 1u)
      L[below] = (uint8_t)lane;
    else
      L[16 + lane - below] = (uint8_t)lane;
  } else if (lane >= 32 && lane < 32 + k) {
    const int p = lane - 32;
    const int below = __popc(d.B & ((1u << p) - 1u));
    if (d.B >> p & 1u)
      L[32 + below] = (uint8_t)p;
    else
      L[48 + p - below] = (uint8_t)p;
  }
  __builtin_amdgcn_wave_barrier();
  d.L = L;
  d.na = __popc(d.A);
  d.nb = __popc(d.B);
  d.va = k - d.na;
  d.vb = k - d.nb;
  d.ca2 = d.va * (d.va - 1) / 2;
  d.cb2 = d.vb * (d.vb - 1) / 2;
  d.sa = d.na * d.va;
  d.sb = d.nb * d.vb;
  d.daa = d.na * (d.na - 1) / 2 * d.ca2;
  d.dbb = d.nb * (d.nb - 1) / 2 * d.cb2;
  d.total = d.sa + d.sb + d.daa + d.dbb + d.sa * d.sb;
  return d;
}

// Target key of replacement t; its matrix element into *val when VAL.
template <bool VAL>
__device__ __forceinline__ uint64_t replacement(const Det& d, int t, const Lds& s, int k, double* val) {
  const uint8_t* L = d.L;
  uint32_t A = d.A, B = d.B;
  if (t < d.sa) {
    const int p = L[t / d.va], r = L[16 + t % d.va];
    A ^= (1u << p) | (1u << r);
    if (VAL) *val = single_val(s, k, d.A, d.B, p, r);
  } else if ((t -= d.sa) < d.sb) {
    const int p = L[32 + t / d.vb], r = L[48 + t % d.vb];
    B ^= (1u << p) | (1u << r);
    if (VAL) *val = single_val(s, k, d.B, d.A, p, r);
  } else if ((t -= d.sb) < d.daa) {
    const int u = t / d.ca2, v = t - u * d.ca2;
    const int p = L[s.lo[u]], q = L[s.hi[u]], r = L[16 + s.lo[v]], w = L[16 + s.hi[v]];
    A ^= (1u << p) | (1u << q) | (1u << r) | (1u << w);
    if (VAL) *val = double_same(s.g, d.A, p, q, r, w);
  } else if ((t -= d.daa) < d.dbb) {
    const int u = t / d.cb2, v = t - u * d.cb2;
    const int p = L[32 + s.lo[u]], q = L[32 + s.hi[u]], r = L[48 + s.lo[v]], w = L[48 + s.hi[v]];
    B ^= (1u << p) | (1u << q) | (1u << r) | (1u << w);
    if (VAL) *val = double_same(s.g, d.B, p, q, r, w);
  } else {
    t -= d.dbb;
    const int u = t / d.sb, v = t - u * d.sb;
    const int p = L[u / d.va], r = L[16 + u % d.va];
    const int q = L[32 + v / d.vb], w = L[48 + v % d.vb];
    A ^= (1u << p) | (1u << r);
    B ^= (1u << q) | (1u << w);
    if (VAL) *val = phase(d.A, p, r) * phase(d.B, q, w) * G(s.g, r, p, w, q);
  }
  return (uint64_t)A | ((uint64_t)B << 32);
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup (256 threads); the result in thread 0.
__device__ __forceinline__ double group_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// ------------------------------------------------------------------ kernels

// h' and the packed (pq|rs) of the active orbitals, and the core energy.
__global__ void hbci_prep_kernel(const double* __restrict__ h, const double* __restrict__ eri, int n,
                                 const int32_t* __restrict__ act, int k, const int32_t* __restrict__ core, int nc,
                                 const double* __restrict__ e_core, double* __restrict__ ints, HbciCtl* ctl) {
  auto E4 = [&](int p, int q, int r, int s) { return eri[(((int64_t)p * n + q) * n + r) * n + s]; };
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int p = act[t / k], q = act[t % k];
    double v = h[(int64_t)p * n + q];
    for (int c = 0; c < nc; ++c) v += 2.0 * E4(p, q, core[c], core[c]) - E4(p, core[c], core[c], q);
    ints[t] = v;
  }
  const int npp = packed_count(k);
  for (int t = threadIdx.x; t < npp; t += blockDim.x) {
    int P = 0;
    while ((P + 1) * (P + 2) / 2 <= t) ++P;
    const int Q = t - P * (P + 1) / 2;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= P) ++i;
    const int j = P - i * (i + 1) / 2;
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= Q) ++a;
    const int b = Q - a * (a + 1) / 2;
    ints[k * k + t] = E4(act[i], act[j], act[a], act[b]);
  }
  if (threadIdx.x == 0) {
    ctl->n_det = 0;
    ctl->n_ext = 0;
    ctl->flags = 0;
    ctl->e_core = *e_core;
    ctl->nnz = 0;
  }
}

__global__ void fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_slots_kernel(ExtSlot* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = ExtSlot{kEmpty, 0.0};
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// V := the caller's keys (or the reference and its partner), in order.
__global__ void hbci_load_kernel(const uint64_t* __restrict__ in, int64_t n, uint64_t ref, Space V) {
  if (!in) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      add_det(V, ref);
      if (flip_key(ref) != ref) add_det(V, flip_key(ref));
    }
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = in[i];
    V.dets[i] = key;
    bool fresh = false;
    const int64_t h = ht_insert(V.keys, V.mask, key, &fresh);
    if (h < 0)
      atomicOr(&V.ctl->flags, kFlagDetCap);
    else if (!fresh)
      atomicOr(&V.ctl->flags, kFlagDuplicate);
    else
      V.vals[h] = (int32_t)i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) V.ctl->n_det = (unsigned long long)n;
}

// One selection step: every replacement a of a determinant i < n_src with
// |H_ai c_i| > eps joins V, with its flip partner.
__global__ void __launch_bounds__(64 * kWaves) hbci_select_kernel(const double* __restrict__ ints, int k,
                                                                  const double* __restrict__ c, int64_t n_src,
                                                                  double eps, Space V, int half) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < n_src; i += (int64_t)gridDim.x * kWaves) {
    const double ci = c[i];
    const uint64_t key = V.dets[i];
    if (ci == 0.0 || (half && !canonical(key))) continue;
    const Det d = make_det(key, k, L, lane);
    for (int t = lane; t < d.total; t += 64) {
      double v;
      const uint64_t a = replacement<true>(d, t, s, k, &v);
      if (fabs(v * ci) > eps) {
        add_det(V, a);
        if (flip_key(a) != a) add_det(V, flip_key(a));
      }
    }
  }
}

// The diagonal (and, with partners, each key's flip partner) of rows lo..n-1.
__global__ void __launch_bounds__(64 * kWaves) hbci_diag_kernel(const double* __restrict__ ints, int k, const Space V,
                                                        int64_t lo, int64_t n, int partners, double* __restrict__ diag,
                                                        int32_t* __restrict__ flip) {
  const Lds s = load_lds(ints, k);
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = V.dets[i];
    diag[i] = diag_val(s, k, (uint32_t)key, (uint32_t)(key >> 32));
    if (partners) {
      const int32_t f = ht_find(V.keys, V.vals, V.mask, flip_key(key));
      flip[i] = f;
      if (f < 0) atomicOr(&V.ctl->flags, kFlagNoPartner);
    }
  }
}

// Nonzeros of each row of H over V (replacements that land in V).
__global__ void __launch_bounds__(64 * kWaves) hbci_count_kernel(const double* __restrict__ ints, int k, const Space V,
                                                                 int64_t n, int half, int32_t* __restrict__ cnt) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  for (int64_t a = (int64_t)blockIdx.x * kWaves + wave; a < n; a += (int64_t)gridDim.x * kWaves) {
    const uint64_t key = V.dets[a];
    if (half && !canonical(key)) {
      if (lane == 0) cnt[a] = 0;
      continue;
    }
    const Det d = make_det(key, k, L, lane);
    int c = 0;
    for (int t = lane; t < d.total; t += 64) {
      double v;
      const uint64_t key = replacement<false>(d, t, s, k, &v);
      c += ht_find(V.keys, V.vals, V.mask, key) >= 0;
    }
    c = wave_sum_int(c);
    if (lane == 0) cnt[a] = c;
  }
}

// Exclusive prefix sum of cnt[0..n) into ptr[0..n]: blocks of 1024 rows,
// then the block totals, then the carry.
__global__ void __launch_bounds__(1024) scan_block_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                          int64_t* __restrict__ ptr, int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  sh[threadIdx.x] = i < n ? cnt[i] : 0;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  if (i < n) ptr[i + 1] = sh[threadIdx.x];
  if (threadIdx.x == 1023) bsum[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024) scan_top_kernel(int64_t* __restrict__ bsum, int64_t nb, HbciCtl* ctl) {
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t own = i < nb ? bsum[i] : 0;
    sh[threadIdx.x] = own;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t v = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - own;  // exclusive
    __syncthreads();
    if (threadIdx.x == 0) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) ctl->nnz = carry;
}

__global__ void scan_add_kernel(int64_t* __restrict__ ptr, int64_t n, const int64_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ptr[i + 1] += bsum[i / 1024];
  if (i == 0) ptr[0] = 0;
}

// Column indices and values of each row, in replacement order.
__global__ void __launch_bounds__(64 * kWaves) hbci_fill_kernel(const double* __restrict__ ints, int k, const Space V,
                                                                int64_t n, int half, const int64_t* __restrict__ ptr,
                                                                int32_t* __restrict__ col, double* __restrict__ val) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t a = (int64_t)blockIdx.x * kWaves + wave; a < n; a += (int64_t)gridDim.x * kWaves) {
    const uint64_t key = V.dets[a];
    if (half && !canonical(key)) continue;
    const Det d = make_det(key, k, L, lane);
    int64_t base = ptr[a];
    for (int t0 = 0; t0 < d.total; t0 += 64) {
      const int t = t0 + lane;
      int32_t j = -1;
      double v = 0.0;
      if (t < d.total) {
        const uint64_t key = replacement<false>(d, t, s, k, &v);
        j = ht_find(V.keys, V.vals, V.mask, key);
        if (j >= 0) replacement<true>(d, t, s, k, &v);
      }
      const uint64_t m = __ballot(j >= 0);
      if (j >= 0) {
        const int64_t at = base + __popcll(m & below);
        col[at] = j;
        val[at] = v;
      }
      base += __popcll(m);
    }
  }
}

// The rows of the determinants lo..n-1 added by a selection step, in a
// space of representatives (flip-symmetric vectors): each such row is
// counted from scratch, and each of its nonzeros (r, b) with b older than lo
// also counts the entries it implies in the old rows, which H's symmetry and
// its commuting with the flip fix: (b, r) when b is a representative, and
// (flip b, flip r) when r is not flip-invariant and flip b is a
// representative (for a flip-invariant r that entry is (flip b, r), reached
// from r's own nonzero (r, flip b)).
__global__ void __launch_bounds__(64 * kWaves) hbci_count_new_kernel(const double* __restrict__ ints, int k,
                                                                     const Space V, int64_t lo, int64_t n,
                                                                     const int32_t* __restrict__ flip,
                                                                     int32_t* __restrict__ cnt,
                                                                     int32_t* __restrict__ addc) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  for (int64_t r = lo + (int64_t)blockIdx.x * kWaves + wave; r < n; r += (int64_t)gridDim.x * kWaves) {
    const uint64_t key = V.dets[r];
    if (!canonical(key)) {
      if (lane == 0) cnt[r] = 0;
      continue;
    }
    const bool self = flip_key(key) == key;
    const Det d = make_det(key, k, L, lane);
    int c = 0;
    for (int t = lane; t < d.total; t += 64) {
      double v;
      const int32_t j = ht_find(V.keys, V.vals, V.mask, replacement<false>(d, t, s, k, &v));
      if (j < 0) continue;
      ++c;
      if (j < lo) {
        const uint64_t kb = V.dets[j];
        if (canonical(kb)) atomicAdd(addc + j, 1);
        if (!self && canonical(flip_key(kb))) atomicAdd(addc + flip[j], 1);
      }
    }
    c = wave_sum_int(c);
    if (lane == 0) cnt[r] = c;
  }
}

// cnt[a] = the old row's length plus its new entries, a < lo
__global__ void hbci_rowlen_kernel(const int64_t* __restrict__ ptr_old, int64_t lo, const int32_t* __restrict__ addc,
                                   int32_t* __restrict__ cnt) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < lo; a += (int64_t)gridDim.x * blockDim.x)
    cnt[a] = (int32_t)(ptr_old[a + 1] - ptr_old[a]) + addc[a];
}

// The old rows' entries to the front of their new rows (one wave per row).
__global__ void __launch_bounds__(256) hbci_copy_rows_kernel(const int64_t* __restrict__ ptr_old,
                                                             const int32_t* __restrict__ col_old,
                                                             const double* __restrict__ val_old, int64_t lo,
                                                             const int64_t* __restrict__ ptr_new,
                                                             int32_t* __restrict__ col_new,
                                                             double* __restrict__ val_new) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t a = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; a < lo; a += nw) {
    const int64_t b = ptr_old[a], len = ptr_old[a + 1] - b, to = ptr_new[a];
    for (int64_t e = lane; e < len; e += 64) {
      col_new[to + e] = col_old[b + e];
      val_new[to + e] = val_old[b + e];
    }
  }
}

// The new rows in full (replacement order) and their implied entries in
// the old rows, after the copied ones (in no fixed order).
__global__ void __launch_bounds__(64 * kWaves) hbci_fill_new_kernel(const double* __restrict__ ints, int k,
                                                                    const Space V, int64_t lo, int64_t n,
                                                                    const int32_t* __restrict__ flip,
                                                                    const int64_t* __restrict__ ptr_old,
                                                                    const int64_t* __restrict__ ptr,
                                                                    int32_t* __restrict__ pos, int32_t* __restrict__ col,
                                                                    double* __restrict__ val) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t r = lo + (int64_t)blockIdx.x * kWaves + wave; r < n; r += (int64_t)gridDim.x * kWaves) {
    const uint64_t key = V.dets[r];
    if (!canonical(key)) continue;
    const bool self = flip_key(key) == key;
    const int32_t fr = flip[r];
    const Det d = make_det(key, k, L, lane);
    int64_t base = ptr[r];
    for (int t0 = 0; t0 < d.total; t0 += 64) {
      const int t = t0 + lane;
      int32_t j = -1;
      double v = 0.0;
      if (t < d.total) {
        j = ht_find(V.keys, V.vals, V.mask, replacement<false>(d, t, s, k, &v));
        if (j >= 0) replacement<true>(d, t, s, k, &v);
      }
      const uint64_t m = __ballot(j >= 0);
      if (j >= 0) {
        const int64_t at = base + __popcll(m & below);
        col[at] = j;
        val[at] = v;
        if (j < lo) {
          const uint64_t kb = V.dets[j];
          if (canonical(kb)) {
            const int64_t e = ptr[j] + (ptr_old[j + 1] - ptr_old[j]) + atomicAdd(pos + j, 1);
            col[e] = (int32_t)r;
            val[e] = v;
          }
          if (!self && canonical(flip_key(kb))) {
            const int32_t f = flip[j];
            const int64_t e = ptr[f] + (ptr_old[f + 1] - ptr_old[f]) + atomicAdd(pos + f, 1);
            col[e] = fr;
            val[e] = v;
          }
        }
      }
      base += __popcll(m);
    }
  }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// y = H x over V: the diagonal plus the CSR rows (one wave per row).  With
// flip (flip-symmetric x, rows only for representatives) each row's value
// is written to the row and to its partner.
__global__ void __launch_bounds__(256) hbci_spmv_kernel(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, const double* __restrict__ diag,
                                                        const uint64_t* __restrict__ dets,
                                                        const int32_t* __restrict__ flip, const double* __restrict__ x,
                                                        double* __restrict__ y, int64_t n) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t a = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; a < n; a += nw) {
    if (flip && !canonical(dets[a])) continue;
    // four entries per lane in flight: their column and value loads, then
    // the four gathers, are independent of each other
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int64_t end = ptr[a + 1];
    int64_t e = ptr[a] + lane;
    for (; e + 192 < end; e += 256) {
      const int32_t c0 = col[e], c1 = col[e + 64], c2 = col[e + 128], c3 = col[e + 192];
      const double v0 = val[e], v1 = val[e + 64], v2 = val[e + 128], v3 = val[e + 192];
      s0 += v0 * x[c0];
      s1 += v1 * x[c1];
      s2 += v2 * x[c2];
      s3 += v3 * x[c3];
    }
    for (; e < end; e += 64) s0 += val[e] * x[col[e]];
    double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) {
      const double ya = s + diag[a] * x[a];
      y[a] = ya;
      if (flip) y[flip[a]] = ya;
    }
  }
}

// part[j][block] = partial of B_j . v, j < m
// part[row0 + j][block] = partial of B_j . v, j < m; with self, row
// row0 + m holds the partial of v . v
__global__ void __launch_bounds__(256) hbci_dots_kernel(const double* __restrict__ B, int64_t ld, int m,
                                                        const double* __restrict__ v, int64_t n,
                                                        double* __restrict__ part, int row0, int self) {
  __shared__ double red[4];
  for (int j = 0; j < m + self; ++j) {
    const double* b = j < m ? B + j * ld : v;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      s += b[i] * v[i];
    s = group_sum(s, red);
    if (threadIdx.x == 0) part[(row0 + j) * kNB + blockIdx.x] = s;
  }
}

// x = sum_j y_j V_j, w = sum_j y_j S_j, r = w - theta x; part = partial |r|^2
__global__ void __launch_bounds__(256) hbci_ritz_kernel(const double* __restrict__ Vb, const double* __restrict__ Sb,
                                                        int64_t ld, int m, Coef y, double theta, double* __restrict__ x,
                                                        double* __restrict__ w, double* __restrict__ r, int64_t n,
                                                        double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double xi = 0.0, wi = 0.0;
    for (int j = 0; j < m; ++j) {
      xi += y.v[j] * Vb[j * ld + i];
      wi += y.v[j] * Sb[j * ld + i];
    }
    const double ri = wi - theta * xi;
    x[i] = xi;
    w[i] = wi;
    r[i] = ri;
    s += ri * ri;
  }
  s = group_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// t = the flip-symmetric part of (theta - D)^-1 r
__global__ void hbci_precond_kernel(const double* __restrict__ r, const double* __restrict__ diag,
                                    const int32_t* __restrict__ flip, double theta, double* __restrict__ t, int64_t n) {
  auto q = [&](int64_t i) {
    double den = theta - diag[i];
    if (fabs(den) < 1e-10) den = den < 0.0 ? -1e-10 : 1e-10;
    return r[i] / den;
  };
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    t[i] = 0.5 * (q(i) + q(flip[i]));
}

// t -= sum_j d_j V_j; part = partial |t|^2
__global__ void __launch_bounds__(256) hbci_orth_kernel(const double* __restrict__ Vb, int64_t ld, int m, Coef d,
                                                        double* __restrict__ t, int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ti = t[i];
    for (int j = 0; j < m; ++j) ti -= d.v[j] * Vb[j * ld + i];
    t[i] = ti;
    s += ti * ti;
  }
  s = group_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void hbci_scale_kernel(const double* __restrict__ in, double f, double* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = f * in[i];
}

// out_j = sum_l Y[l][j] B_l, j < keep (the kept Ritz vectors of a restart)
__global__ void __launch_bounds__(256) hbci_combo_kernel(const double* __restrict__ B, int64_t ld, int m, CoefKeep Y,
                                                         int keep, double* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double b[kMaxM];
    for (int l = 0; l < m; ++l) b[l] = B[l * ld + i];
    for (int j = 0; j < keep; ++j) {
      double a = 0.0;
      for (int l = 0; l < m; ++l) a += Y.v[l][j] * b[l];
      out[j * ld + i] = a;
    }
  }
}

// N_a += H_ai c_i for every replacement a outside V with |H_ai c_i| > eps.
// With half (flip-symmetric c, flip-closed V) only representatives i are
// walked and N is kept for representatives b only: the term (i, b) of a
// non-representative i equals (flip i, flip b), so a representative i adds
// each term to its target's representative (twice for a flip-invariant
// target, which i and flip(i) both reach); a flip-invariant i (a closed
// shell, whose replacements come in flip pairs) adds only the terms whose
// target is a representative.
__global__ void __launch_bounds__(64 * kWaves) hbci_pt2_kernel(const double* __restrict__ ints, int k, const Space V,
                                                               const double* __restrict__ c, int64_t n, double eps,
                                                               int half, ExtSlot* __restrict__ et,
                                                               int64_t* __restrict__ elist, uint64_t emask,
                                                               int64_t ecap) {
  const Lds s = load_lds(ints, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint8_t* L = s.lists + wave * 64;
  for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < n; i += (int64_t)gridDim.x * kWaves) {
    const double ci = c[i];
    const uint64_t key = V.dets[i];
    if (ci == 0.0 || (half && !canonical(key))) continue;
    const bool self = flip_key(key) == key;
    const Det d = make_det(key, k, L, lane);
    for (int t = lane; t < d.total; t += 64) {
      double v;
      uint64_t a = replacement<true>(d, t, s, k, &v);
      const double hc = v * ci;
      if (!(fabs(hc) > eps)) continue;
      double w = 1.0;
      if (half) {
        if (!canonical(a)) {
          if (self) continue;
          a = flip_key(a);
        } else if (!self && flip_key(a) == a) {
          w = 2.0;  // i and flip(i) reach the flip-invariant a with equal terms
        }
      }
      if (ht_find(V.keys, V.vals, V.mask, a) < 0) ext_add(et, elist, emask, ecap, a, w * hc, V.ctl);
    }
  }
}

// part[block] = partial sum of N_a^2 / (e - H_aa); part[kNB + block] = count
__global__ void __launch_bounds__(64 * kWaves) hbci_e2_kernel(const double* __restrict__ ints, int k,
                                                      const ExtSlot* __restrict__ et,
                                                      const int64_t* __restrict__ elist, int64_t cap,
                                                      const HbciCtl* __restrict__ ctl, double e, int half,
                                                      double* __restrict__ part) {
  const Lds s = load_lds(ints, k);
  double* red = (double*)s.lists;  // no static LDS beside the dynamic block
  const int64_t n_filled = (int64_t)ctl->n_ext < cap ? (int64_t)ctl->n_ext : cap;
  double sum = 0.0, cnt = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_filled;
       t += (int64_t)gridDim.x * blockDim.x) {
    const ExtSlot sl = et[elist[t]];
    const uint64_t key = sl.key;
    const double na = sl.val;
    // a representative stands for itself and its partner
    const double w = (half && flip_key(key) != key) ? 2.0 : 1.0;
    sum += w * (na * na / (e - diag_val(s, k, (uint32_t)key, (uint32_t)(key >> 32))));
    cnt += w;
  }
  sum = group_sum(sum, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
  cnt = group_sum(cnt, red);
  if (threadIdx.x == 0) part[kNB + blockIdx.x] = cnt;
}

// ------------------------------------- Davidson of a small space in one workgroup

// Spaces of up to kSmallDav determinants solve their Davidson in a single
// launch of one 1024-thread workgroup: the same iteration as the host-driven
// form (thick restart, flip-symmetric diagonal preconditioner, classical
// Gram-Schmidt twice), with the small eigenproblem on one wavefront (the
// one-wave parallel Jacobi) and every reduction in LDS, so a step costs one
// launch and one read-back instead of several per iteration.  The
// increments of an expansion run on concurrent streams, one CU each.
constexpr int64_t kSmallDav = 1024;
constexpr int kSmallThreads = 1024;

struct SmallDav {
  const int64_t* ptr;
  const int32_t* col;
  const double* val;
  const double* diag;
  const uint64_t* dets;
  const int32_t* flip;
  double* x;
  double* Vb;
  double* Sb;
  double* r;
  int64_t ld, n;
  int m_max, max_dav, half;
  double r_tol;
  double* out;  // theta, residual norm, converged (0/1), iterations
};

__device__ void small_spmv(const SmallDav& a, const double* __restrict__ xin, double* __restrict__ y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int64_t row = wave; row < a.n; row += nw) {
    if (a.half && !canonical(a.dets[row])) continue;
    double s = 0.0;
    for (int64_t e = a.ptr[row] + lane; e < a.ptr[row + 1]; e += 64) s += a.val[e] * xin[a.col[e]];
    s = wave_sum(s);
    if (lane == 0) {
      const double ya = s + a.diag[row] * xin[row];
      y[row] = ya;
      if (a.half) y[a.flip[row]] = ya;
    }
  }
  __syncthreads();
}

// res[j] = sum over the workgroup of v[j], j < nv (v per thread, nv <= 17)
__device__ __forceinline__ void small_sums(const double (&v)[kMaxM + 1], int nv, double* red, double* res) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < kMaxM + 1; ++j)
    if (j < nv) {
      const double t = wave_sum(v[j]);
      if (lane == 0) red[wave * (kMaxM + 1) + j] = t;
    }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w * (kMaxM + 1) + threadIdx.x];
    res[threadIdx.x] = t;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kSmallThreads) hbci_dav_small_kernel(SmallDav a) {
  __shared__ double Hs[256], A[256], Q[256], ev[16], yv[16], th[1];
  __shared__ double red[(kSmallThreads / 64) * (kMaxM + 1)], res[kMaxM + 1];
  __shared__ int perm[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t n = a.n, ld = a.ld;
  double* Vb = a.Vb;
  double* Sb = a.Sb;
  for (int64_t i = tid; i < n; i += nt) Vb[i] = a.x[i];
  for (int t = tid; t < 256; t += nt) Hs[t] = 0.0;
  __syncthreads();
  small_spmv(a, Vb, Sb);
  {
    double v[kMaxM + 1] = {};
    for (int64_t i = tid; i < n; i += nt) v[0] += Vb[i] * Sb[i];
    small_sums(v, 1, red, res);
  }
  if (tid == 0) Hs[0] = res[0];
  __syncthreads();
  int m = 1, conv = 0, it = 0;
  double theta = res[0], rn = 1e300;
  // Ritz pair of the current basis: x, r = H x - theta x, |r|
  auto ritz = [&]() {
    if (tid < 64) {
      for (int t = tid; t < 256; t += 64) A[t] = Hs[t];
      jacobi_lowest(A, Q, m, th, yv, ev, perm);
    }
    __syncthreads();
    theta = th[0];
    double v[kMaxM + 1] = {};
    for (int64_t i = tid; i < n; i += nt) {
      double xi = 0.0, wi = 0.0;
      for (int j = 0; j < m; ++j) {
        xi += yv[j] * Vb[j * ld + i];
        wi += yv[j] * Sb[j * ld + i];
      }
      const double ri = wi - theta * xi;
      a.x[i] = xi;
      a.r[i] = ri;
      v[0] += ri * ri;
    }
    small_sums(v, 1, red, res);
    rn = sqrt(res[0]);
  };
  for (it = 0; it < a.max_dav; ++it) {
    ritz();
    if (rn <= a.r_tol) {
      conv = 1;
      break;
    }
    if (m == a.m_max) {  // thick restart, in place: each thread owns its entries of every vector
      const int keep = a.m_max / 2 < kKeepRitz ? a.m_max / 2 : kKeepRitz;
      for (int64_t i = tid; i < n; i += nt) {
        double bv[kMaxM], bs[kMaxM];
        for (int l = 0; l < kMaxM; ++l)
          if (l < m) {
            bv[l] = Vb[l * ld + i];
            bs[l] = Sb[l * ld + i];
          }
        for (int j = 0; j < keep; ++j) {
          double cv = 0.0, cs = 0.0;
          for (int l = 0; l < kMaxM; ++l)
            if (l < m) {
              const double q = Q[l * 16 + perm[j]];
              cv += q * bv[l];
              cs += q * bs[l];
            }
          Vb[j * ld + i] = cv;
          Sb[j * ld + i] = cs;
        }
      }
      __syncthreads();
      if (tid < 256) Hs[tid] = ((tid >> 4) == (tid & 15) && (tid & 15) < keep) ? ev[tid & 15] : 0.0;
      __syncthreads();
      m = keep;
    }
    // the correction, flip-symmetrised, into the next basis slot
    double* T = Vb + m * ld;
    for (int64_t i = tid; i < n; i += nt) {
      double d1 = theta - a.diag[i];
      if (fabs(d1) < 1e-10) d1 = d1 < 0.0 ? -1e-10 : 1e-10;
      const int64_t f = a.flip[i];
      double d2 = theta - a.diag[f];
      if (fabs(d2) < 1e-10) d2 = d2 < 0.0 ? -1e-10 : 1e-10;
      T[i] = 0.5 * (a.r[i] / d1 + a.r[f] / d2);
    }
    double t2 = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      double v[kMaxM + 1] = {};
      for (int64_t i = tid; i < n; i += nt) {
        const double ti = T[i];
#pragma unroll
        for (int j = 0; j < kMaxM; ++j)
          if (j < m) v[j] += Vb[j * ld + i] * ti;
      }
      small_sums(v, m, red, res);
      double w[kMaxM + 1] = {};
      for (int64_t i = tid; i < n; i += nt) {
        double ti = T[i];
        for (int j = 0; j < m; ++j) ti -= res[j] * Vb[j * ld + i];
        T[i] = ti;
        w[0] += ti * ti;
      }
      if (pass == 1) {
        small_sums(w, 1, red, res);
        t2 = res[0];
      } else {
        __syncthreads();
      }
    }
    if (!(t2 > 1e-28)) break;  // the space is exhausted
    const double inv = 1.0 / sqrt(t2);
    for (int64_t i = tid; i < n; i += nt) T[i] *= inv;
    __syncthreads();
    small_spmv(a, T, Sb + m * ld);
    {
      double v[kMaxM + 1] = {};
      for (int64_t i = tid; i < n; i += nt) {
        const double si = Sb[m * ld + i];
#pragma unroll
        for (int j = 0; j < kMaxM + 1; ++j)
          if (j <= m) v[j] += Vb[j * ld + i] * si;
      }
      small_sums(v, m + 1, red, res);
    }
    if (tid <= m) {
      Hs[tid * 16 + m] = res[tid];
      Hs[m * 16 + tid] = res[tid];
    }
    __syncthreads();
    ++m;
  }
  if (!conv) {  // ended on the iteration limit or an exhausted space: the Ritz pair of the basis
    ritz();
    conv = rn <= a.r_tol ? 1 : 0;
  }
  if (tid == 0) {
    a.out[0] = theta;
    a.out[1] = rn;
    a.out[2] = conv;
    a.out[3] = it;
  }
}

// ---------------------------------------------------------------- host side

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

uint64_t pow2_at_least(int64_t x) {
  uint64_t p = 1;
  while ((int64_t)p < x) p <<= 1;
  return p;
}

struct Layout {
  int64_t ints, ctl, part, bsum, dets, keys, vals, flip, diag, cnt, addc, pos, ptr[2], col[2], val[2], basis, sig, x, w,
      r, t, keep, ext, elist;
  int64_t bytes;
  uint64_t tcap, ecap;
};

Layout layout(int k, const ifci_hbci_options& o) {
  Layout L{};
  int64_t off = 0;
  auto take = [&](int64_t b) {
    const int64_t at = off;
    off = align256(off + b);
    return at;
  };
  const int64_t D = o.max_det;
  L.tcap = pow2_at_least(2 * D);
  L.ecap = pow2_at_least(2 * o.max_ext);
  L.ints = take((int64_t)(k * k + packed_count(k)) * 8);
  L.ctl = take(sizeof(HbciCtl));
  L.part = take((int64_t)kNB * kParts * 8);
  L.bsum = take(((D + 1023) / 1024 + 1) * 8);
  L.dets = take(D * 8);
  L.keys = take((int64_t)L.tcap * 8);
  L.vals = take((int64_t)L.tcap * 4);
  L.flip = take(D * 4);
  L.diag = take(D * 8);
  L.cnt = take(D * 4);
  L.addc = take(D * 4);
  L.pos = take(D * 4);
  // two CSR buffers: a selection step builds the new H from the old one
  for (int b = 0; b < 2; ++b) {
    L.ptr[b] = take((D + 1) * 8);
    L.col[b] = take(o.max_nnz * 4);
    L.val[b] = take(o.max_nnz * 8);
  }
  L.basis = take((int64_t)o.m_max * D * 8);
  L.sig = take((int64_t)o.m_max * D * 8);
  L.x = take(D * 8);
  L.w = take(D * 8);
  L.r = take(D * 8);
  L.t = take(D * 8);
  L.keep = take((int64_t)2 * kKeepRitz * D * 8);
  L.ext = take((int64_t)L.ecap * (int64_t)sizeof(ExtSlot));
  L.elist = take(o.max_ext * 8);
  L.bytes = off;
  return L;
}

// Eigenpairs of the symmetric m x m matrix A (cyclic Jacobi), ascending:
// evals[j] with the unit eigenvector in column j of Y.
void sym_eigen(const double (&A0)[kMaxM][kMaxM], int m, double* evals, double (&Y)[kMaxM][kMaxM]) {
  double A[kMaxM][kMaxM], Q[kMaxM][kMaxM];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      A[i][j] = A0[i][j];
      Q[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        if (A[p][q] == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < m; ++r) {
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < m; ++r) {
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
        for (int r = 0; r < m; ++r) {
          const double qrp = Q[r][p], qrq = Q[r][q];
          Q[r][p] = c * qrp - s * qrq;
          Q[r][q] = s * qrp + c * qrq;
        }
      }
  }
  int idx[kMaxM];
  for (int i = 0; i < m; ++i) idx[i] = i;
  for (int i = 1; i < m; ++i)  // insertion sort by eigenvalue
    for (int j = i; j > 0 && A[idx[j]][idx[j]] < A[idx[j - 1]][idx[j - 1]]; --j) std::swap(idx[j], idx[j - 1]);
  for (int j = 0; j < m; ++j) {
    const int c = idx[j];
    evals[j] = A[c][c];
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += Q[i][c] * Q[i][c];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) Y[i][j] = Q[i][c] / nrm;
  }
}

void lowest_eigen(const double (&A)[kMaxM][kMaxM], int m, double* theta, double* y) {
  double ev[kMaxM], Y[kMaxM][kMaxM];
  sym_eigen(A, m, ev, Y);
  *theta = ev[0];
  for (int i = 0; i < m; ++i) y[i] = Y[i][0];
}

// Pinned host staging for read-backs, one per host thread.
double* staging() {
  static thread_local double* p = nullptr;
  if (!p && hipHostMalloc((void**)&p, sizeof(double) * (2 * kNB * kParts + 64)) != hipSuccess) p = nullptr;
  return p;
}

struct Run {
  HbciInc I;
  ifci_hbci_options o;
  Layout L;
  char* w;
  hipStream_t st;
  double* pin = nullptr;
  HbciCtl ctl{};
  int lds = 0;
  int half = 0;  // flip-symmetric vectors over a flip-closed space: walk representatives only
  int cur = 0;   // the CSR buffer that holds H

  template <typename T>
  T* at(int64_t off) const {
    return (T*)(w + off);
  }
  Space space() const {
    return Space{at<uint64_t>(L.dets), at<uint64_t>(L.keys), at<int32_t>(L.vals), L.tcap - 1, o.max_det,
                 at<HbciCtl>(L.ctl)};
  }
  static int blocks(int64_t n, int per, int cap) {
    const int64_t b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
  }

  hipError_t read_ctl() {
    hipError_t e = hipMemcpyAsync(pin, at<HbciCtl>(L.ctl), sizeof(HbciCtl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) std::memcpy(&ctl, pin, sizeof(HbciCtl));
    return e;
  }
  // sums of m rows of kNB partials, each in block order
  hipError_t read_parts(int m, double* out) {
    hipError_t e = hipMemcpyAsync(pin, at<double>(L.part), sizeof(double) * kNB * m, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int b = 0; b < kNB; ++b) s += pin[j * kNB + b];
      out[j] = s;
    }
    return hipSuccess;
  }

  hipError_t prepare() {
    pin = staging();
    if (!pin) return hipErrorOutOfMemory;
    lds = lds_bytes_for(I.k);
    hipError_t e = hipSuccess;
    for (const void* fn : {(const void*)hbci_select_kernel, (const void*)hbci_diag_kernel,
                           (const void*)hbci_count_kernel, (const void*)hbci_fill_kernel, (const void*)hbci_pt2_kernel,
                           (const void*)hbci_count_new_kernel, (const void*)hbci_fill_new_kernel,
                           (const void*)hbci_e2_kernel})
      if (e == hipSuccess) e = allow_max_lds(fn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hbci_prep_kernel, dim3(1), dim3(256), 0, st, I.h, I.eri, I.n_orb, I.act, I.k, I.core,
                       I.n_core, I.e_core, at<double>(L.ints), at<HbciCtl>(L.ctl));
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks((int64_t)L.tcap, 256, 4096)), dim3(256), 0, st,
                       at<uint64_t>(L.keys), (int64_t)L.tcap, kEmpty);
    e = hipGetLastError();
    if (e == hipSuccess) e = read_ctl();
    return e;
  }

  hipError_t load(const uint64_t* dets, int64_t n) {
    hipLaunchKernelGGL(hbci_load_kernel, dim3(dets ? blocks(n, 256, 4096) : 1), dim3(256), 0, st, dets, n, I.ref,
                       space());
    return hipGetLastError();
  }

  hipError_t diag(int64_t lo, int64_t n, bool partners) {
    if (n <= lo) return hipSuccess;
    hipLaunchKernelGGL(hbci_diag_kernel, dim3(blocks(n - lo, 64 * kWaves, 2048)), dim3(64 * kWaves), lds, st, at<double>(L.ints), I.k,
                       space(), lo, n, partners ? 1 : 0, at<double>(L.diag), at<int32_t>(L.flip));
    return hipGetLastError();
  }

  // CSR of H over the n keys; IFCI_ERR_OOM past max_nnz
  ifci_status build_h(int64_t n, hipError_t* he) {
    hipLaunchKernelGGL(hbci_count_kernel, dim3(blocks(n, kWaves, 8192)), dim3(64 * kWaves), lds, st,
                       at<double>(L.ints), I.k, space(), n, half, at<int32_t>(L.cnt));
    ifci_status s = scan_rows(n, L.ptr[cur], he);
    if (s != IFCI_OK) return s;
    hipLaunchKernelGGL(hbci_fill_kernel, dim3(blocks(n, kWaves, 8192)), dim3(64 * kWaves), lds, st,
                       at<double>(L.ints), I.k, space(), n, half, at<int64_t>(L.ptr[cur]), at<int32_t>(L.col[cur]),
                       at<double>(L.val[cur]));
    *he = hipGetLastError();
    return *he == hipSuccess ? IFCI_OK : IFCI_ERR_DEVICE;
  }

  // row offsets at ptr_off from cnt[0..n); the total checked against max_nnz
  ifci_status scan_rows(int64_t n, int64_t ptr_off, hipError_t* he) {
    const int64_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(scan_block_kernel, dim3((unsigned)nb), dim3(1024), 0, st, at<int32_t>(L.cnt), n,
                       at<int64_t>(ptr_off), at<int64_t>(L.bsum));
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, st, at<int64_t>(L.bsum), nb, at<HbciCtl>(L.ctl));
    hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(n, 256, 1 << 30)), dim3(256), 0, st, at<int64_t>(ptr_off), n,
                       at<int64_t>(L.bsum));
    *he = hipGetLastError();
    if (*he == hipSuccess) *he = read_ctl();
    if (*he != hipSuccess) return IFCI_ERR_DEVICE;
    if (ctl.nnz > o.max_nnz) {
      set_error("HBCI: H over the selected space has more nonzeros than max_nnz");
      return IFCI_ERR_OOM;
    }
    return IFCI_OK;
  }

  // H over n keys from H over the first lo (representative rows, flip
  // partners known): the new rows from scratch, the old ones copied and
  // extended by the entries the new rows imply; the result in the other
  // buffer, which becomes current.
  ifci_status extend_h(int64_t lo, int64_t n, hipError_t* he) {
    const int nxt = cur ^ 1;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks(lo, 256, 4096)), dim3(256), 0, st, at<int32_t>(L.addc), lo, 0);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks(lo, 256, 4096)), dim3(256), 0, st, at<int32_t>(L.pos), lo, 0);
    hipLaunchKernelGGL(hbci_count_new_kernel, dim3(blocks(n - lo, kWaves, 8192)), dim3(64 * kWaves), lds, st,
                       at<double>(L.ints), I.k, space(), lo, n, at<int32_t>(L.flip), at<int32_t>(L.cnt),
                       at<int32_t>(L.addc));
    hipLaunchKernelGGL(hbci_rowlen_kernel, dim3(blocks(lo, 256, 4096)), dim3(256), 0, st, at<int64_t>(L.ptr[cur]), lo,
                       at<int32_t>(L.addc), at<int32_t>(L.cnt));
    ifci_status s = scan_rows(n, L.ptr[nxt], he);
    if (s != IFCI_OK) return s;
    hipLaunchKernelGGL(hbci_copy_rows_kernel, dim3(blocks(lo, 4, 8192)), dim3(256), 0, st, at<int64_t>(L.ptr[cur]),
                       at<int32_t>(L.col[cur]), at<double>(L.val[cur]), lo, at<int64_t>(L.ptr[nxt]),
                       at<int32_t>(L.col[nxt]), at<double>(L.val[nxt]));
    hipLaunchKernelGGL(hbci_fill_new_kernel, dim3(blocks(n - lo, kWaves, 8192)), dim3(64 * kWaves), lds, st,
                       at<double>(L.ints), I.k, space(), lo, n, at<int32_t>(L.flip), at<int64_t>(L.ptr[cur]),
                       at<int64_t>(L.ptr[nxt]), at<int32_t>(L.pos), at<int32_t>(L.col[nxt]), at<double>(L.val[nxt]));
    *he = hipGetLastError();
    if (*he != hipSuccess) return IFCI_ERR_DEVICE;
    cur = nxt;
    return IFCI_OK;
  }

  hipError_t spmv(const double* x, double* y, int64_t n) {
    hipLaunchKernelGGL(hbci_spmv_kernel, dim3(blocks(n, 4, 8192)), dim3(256), 0, st, at<int64_t>(L.ptr[cur]),
                       at<int32_t>(L.col[cur]), at<double>(L.val[cur]), at<double>(L.diag), at<uint64_t>(L.dets),
                       half ? at<int32_t>(L.flip) : nullptr, x, y, n);
    return hipGetLastError();
  }

  hipError_t dots(const double* B, int m, const double* v, int64_t n, double* out) {
    hipLaunchKernelGGL(hbci_dots_kernel, dim3(kNB), dim3(256), 0, st, B, o.max_det, m, v, n, at<double>(L.part), 0,
                       0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? read_parts(m, out) : e;
  }

  // Davidson for the lowest root over the n keys from the unit,
  // flip-symmetric start vector in x; the Ritz vector is left in x.
  hipError_t davidson(int64_t n, double* theta_out, double* res_out, bool* conv) {
    if (n <= kSmallDav) {
      SmallDav a{at<int64_t>(L.ptr[cur]), at<int32_t>(L.col[cur]), at<double>(L.val[cur]), at<double>(L.diag),
                 at<uint64_t>(L.dets), at<int32_t>(L.flip), at<double>(L.x), at<double>(L.basis),
                 at<double>(L.sig), at<double>(L.r), o.max_det, n, o.m_max, o.max_dav, half, o.r_tol,
                 at<double>(L.part)};
      hipLaunchKernelGGL(hbci_dav_small_kernel, dim3(1), dim3(kSmallThreads), 0, st, a);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(pin, a.out, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      *theta_out = pin[0];
      *res_out = pin[1];
      *conv = pin[2] != 0.0;
      return hipSuccess;
    }
    double* Vb = at<double>(L.basis);
    double* Sb = at<double>(L.sig);
    double* x = at<double>(L.x);
    double* w = at<double>(L.w);
    double* r = at<double>(L.r);
    double* t = at<double>(L.t);
    const int64_t ld = o.max_det;
    const int gb = blocks(n, 256, kNB);
    double Hs[kMaxM][kMaxM] = {};
    double hv[kMaxM];
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(hbci_scale_kernel, dim3(gb), dim3(256), 0, st, x, 1.0, Vb, n);
    if ((e = spmv(Vb, Sb, n)) != hipSuccess) return e;
    if ((e = dots(Vb, 1, Sb, n, hv)) != hipSuccess) return e;
    Hs[0][0] = hv[0];
    int m = 1;
    double theta = hv[0], rn = INFINITY;
    *conv = false;
    // Per iteration three read-backs: the residual norm with the first
    // Gram-Schmidt overlaps (the correction is formed before the
    // convergence test is known, and dropped if it passes), the second
    // overlaps with the correction's norm (|t - V d|^2 = |t|^2 - |d|^2 for an
    // orthonormal V), and the new column of the subspace matrix.
    double* part = at<double>(L.part);
    double rd[kParts];
    for (int it = 0; it < o.max_dav; ++it) {
      Coef y{};
      lowest_eigen(Hs, m, &theta, y.v);
      hipLaunchKernelGGL(hbci_ritz_kernel, dim3(kNB), dim3(256), 0, st, Vb, Sb, ld, m, y, theta, x, w, r, n, part);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (m == o.m_max) {
        double r2;
        if ((e = read_parts(1, &r2)) != hipSuccess) return e;
        rn = std::sqrt(r2);
        if (rn <= o.r_tol) {
          *conv = true;
          break;
        }
        // thick restart: the lowest Ritz vectors and their sigmas
        const int keep = std::min(kKeepRitz, o.m_max / 2);
        double ev[kMaxM], Y[kMaxM][kMaxM];
        sym_eigen(Hs, m, ev, Y);
        CoefKeep K{};
        for (int l = 0; l < m; ++l)
          for (int j = 0; j < keep; ++j) K.v[l][j] = Y[l][j];
        double* kv = at<double>(L.keep);
        double* ks = kv + (int64_t)kKeepRitz * ld;
        hipLaunchKernelGGL(hbci_combo_kernel, dim3(gb), dim3(256), 0, st, Vb, ld, m, K, keep, kv, n);
        hipLaunchKernelGGL(hbci_combo_kernel, dim3(gb), dim3(256), 0, st, Sb, ld, m, K, keep, ks, n);
        for (int j = 0; j < keep; ++j) {
          hipLaunchKernelGGL(hbci_scale_kernel, dim3(gb), dim3(256), 0, st, kv + j * ld, 1.0, Vb + j * ld, n);
          hipLaunchKernelGGL(hbci_scale_kernel, dim3(gb), dim3(256), 0, st, ks + j * ld, 1.0, Sb + j * ld, n);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int i = 0; i < kMaxM; ++i)
          for (int j = 0; j < kMaxM; ++j) Hs[i][j] = 0.0;
        for (int j = 0; j < keep; ++j) Hs[j][j] = ev[j];
        m = keep;
      }
      hipLaunchKernelGGL(hbci_precond_kernel, dim3(gb), dim3(256), 0, st, r, at<double>(L.diag),
                         at<int32_t>(L.flip), theta, t, n);
      hipLaunchKernelGGL(hbci_dots_kernel, dim3(kNB), dim3(256), 0, st, Vb, ld, m, t, n, part, 1, 0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = read_parts(m + 1, rd)) != hipSuccess) return e;  // row 0: |r|^2 of this Ritz pair
      rn = std::sqrt(rd[0]);
      if (rn <= o.r_tol) {
        *conv = true;
        break;
      }
      Coef d{};
      for (int j = 0; j < m; ++j) d.v[j] = rd[j + 1];
      hipLaunchKernelGGL(hbci_orth_kernel, dim3(kNB), dim3(256), 0, st, Vb, ld, m, d, t, n, part);
      hipLaunchKernelGGL(hbci_dots_kernel, dim3(kNB), dim3(256), 0, st, Vb, ld, m, t, n, part, 0, 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = read_parts(m + 1, rd)) != hipSuccess) return e;
      Coef d2{};
      double dd = 0.0;
      for (int j = 0; j < m; ++j) {
        d2.v[j] = rd[j];
        dd += rd[j] * rd[j];
      }
      const double tt = rd[m];
      hipLaunchKernelGGL(hbci_orth_kernel, dim3(kNB), dim3(256), 0, st, Vb, ld, m, d2, t, n, part);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      double t2 = tt - dd;
      if (!(t2 > 1e-6 * tt)) {  // cancellation: the norm as summed by the second pass
        if ((e = read_parts(1, &t2)) != hipSuccess) return e;
      }
      if (!(t2 > 1e-28)) break;  // the space is exhausted
      hipLaunchKernelGGL(hbci_scale_kernel, dim3(gb), dim3(256), 0, st, t, 1.0 / std::sqrt(t2), Vb + m * ld, n);
      if ((e = spmv(Vb + m * ld, Sb + m * ld, n)) != hipSuccess) return e;
      if ((e = dots(Vb, m + 1, Sb + m * ld, n, hv)) != hipSuccess) return e;
      for (int j = 0; j <= m; ++j) Hs[j][m] = Hs[m][j] = hv[j];
      ++m;
    }
    if (!*conv && m >= 1) {
      // the loop ended without a final Ritz step: refresh x from the basis
      Coef y{};
      lowest_eigen(Hs, m, &theta, y.v);
      hipLaunchKernelGGL(hbci_ritz_kernel, dim3(kNB), dim3(256), 0, st, Vb, Sb, ld, m, y, theta, x, w, r, n,
                         at<double>(L.part));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      double r2;
      if ((e = read_parts(1, &r2)) != hipSuccess) return e;
      rn = std::sqrt(r2);
      *conv = rn <= o.r_tol;
    }
    *theta_out = theta;
    *res_out = rn;
    return hipSuccess;
  }

  hipError_t pt2(int64_t n, const double* c, double e_act, double eps2, double* e2, int64_t* n_ext) {
    hipLaunchKernelGGL(fill_slots_kernel, dim3(blocks((int64_t)L.ecap, 256, 4096)), dim3(256), 0, st,
                       at<ExtSlot>(L.ext), (int64_t)L.ecap);
    hipLaunchKernelGGL(hbci_pt2_kernel, dim3(blocks(n, kWaves, 8192)), dim3(64 * kWaves), lds, st,
                       at<double>(L.ints), I.k, space(), c, n, eps2, half, at<ExtSlot>(L.ext),
                       at<int64_t>(L.elist), L.ecap - 1, o.max_ext);
    hipLaunchKernelGGL(hbci_e2_kernel, dim3(kNB), dim3(64 * kWaves), lds, st, at<double>(L.ints), I.k,
                       at<ExtSlot>(L.ext), at<int64_t>(L.elist), o.max_ext, at<HbciCtl>(L.ctl), e_act, half,
                       at<double>(L.part));
    hipError_t e = hipGetLastError();
    double s[2];
    if (e == hipSuccess) e = read_parts(2, s);
    if (e == hipSuccess) e = read_ctl();
    *e2 = s[0];
    *n_ext = (int64_t)std::llround(s[1]);
    return e;
  }
};

ifci_status device_failure(hipError_t e, const char* where) {
  set_error(std::string(where) + ": " + hipGetErrorString(e));
  return IFCI_ERR_DEVICE;
}

ifci_status capacity_failure(unsigned flags) {
  if (flags & kFlagDetCap) set_error("HBCI: the selected space outgrew max_det");
  else if (flags & kFlagExtCap) set_error("HBCI: the PT2 external space outgrew max_ext");
  else if (flags & kFlagDuplicate) set_error("HBCI: the determinant list repeats a key");
  else set_error("HBCI: a determinant's spin-flipped partner is missing from the space");
  return (flags & (kFlagDetCap | kFlagExtCap)) ? IFCI_ERR_OOM : IFCI_ERR_ARG;
}

#define HB_TRY(expr, where)                                   \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return device_failure(e_, where);   \
  } while (0)

}  // namespace

int64_t hbci_work_bytes(int k, const ifci_hbci_options& o) { return layout(k, o).bytes; }

ifci_status hbci_solve(const HbciInc& I, const ifci_hbci_options& o, void* work, double* result, uint64_t* dets_out,
                       double* c_out, hipStream_t st) {
  Run R{I, o, layout(I.k, o), (char*)work, st};
  R.half = 1;
  HB_TRY(R.prepare(), "hbci prepare");
  const double shift = R.ctl.e_core + I.e_const;
  HB_TRY(R.load(nullptr, 0), "hbci load");
  HB_TRY(R.read_ctl(), "hbci load");
  int64_t n = (int64_t)R.ctl.n_det;
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  HB_TRY(R.diag(0, n, true), "hbci diagonal");
  // V = {reference}: c = 1 (over the reference and, for an open shell, the
  // normalised symmetric pair), E = its diagonal
  double* x = R.at<double>(R.L.x);
  hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, st, x, n, 1.0 / std::sqrt((double)n));
  HB_TRY(hipGetLastError(), "hbci start");
  double theta = 0.0, res = 0.0;
  bool all_conv = true;
  {
    hipError_t he;
    ifci_status s = R.build_h(n, &he);
    if (s == IFCI_ERR_DEVICE) return device_failure(he, "hbci H");
    if (s != IFCI_OK) return s;
    bool cv;
    HB_TRY(R.davidson(n, &theta, &res, &cv), "hbci davidson");
    all_conv = all_conv && cv;
  }
  int steps = 0;
  bool fixed = false;
  while (steps < o.max_iter) {
    const int64_t n_old = n;
    hipLaunchKernelGGL(hbci_select_kernel, dim3(Run::blocks(n_old, kWaves, 8192)), dim3(64 * kWaves), R.lds, st,
                       R.at<double>(R.L.ints), I.k, x, n_old, o.eps1, R.space(), R.half);
    HB_TRY(hipGetLastError(), "hbci select");
    HB_TRY(R.read_ctl(), "hbci select");
    ++steps;
    if (R.ctl.flags) return capacity_failure(R.ctl.flags);
    n = (int64_t)R.ctl.n_det;
    if (n == n_old) {
      fixed = true;
      break;
    }
    HB_TRY(R.diag(n_old, n, true), "hbci diagonal");
    hipLaunchKernelGGL(fill_f64_kernel, dim3(Run::blocks(n - n_old, 256, 4096)), dim3(256), 0, st, x + n_old,
                       n - n_old, 0.0);
    HB_TRY(hipGetLastError(), "hbci start");
    hipError_t he;
    ifci_status s = R.extend_h(n_old, n, &he);
    if (s == IFCI_ERR_DEVICE) return device_failure(he, "hbci H");
    if (s != IFCI_OK) return s;
    bool cv;
    HB_TRY(R.davidson(n, &theta, &res, &cv), "hbci davidson");
    all_conv = all_conv && cv;
    HB_TRY(R.read_ctl(), "hbci davidson");
    if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  }
  double e2 = 0.0;
  int64_t n_ext = 0;
  HB_TRY(R.pt2(n, x, theta, o.eps2, &e2, &n_ext), "hbci pt2");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  if (dets_out) HB_TRY(hipMemcpyAsync(dets_out, R.at<uint64_t>(R.L.dets), n * 8, hipMemcpyDeviceToDevice, st), "copy");
  if (c_out) HB_TRY(hipMemcpyAsync(c_out, x, n * 8, hipMemcpyDeviceToDevice, st), "copy");
  HB_TRY(hipStreamSynchronize(st), "hbci");
  result[0] = theta + shift;
  result[1] = e2;
  result[2] = (double)n;
  result[3] = (double)steps;
  result[4] = (fixed && all_conv) ? 1.0 : 0.0;
  result[5] = res;
  result[6] = (double)n_ext;
  result[7] = (double)R.ctl.nnz;
  return IFCI_OK;
}

ifci_status hbci_sigma(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                       const double* c, double* sigma, hipStream_t st) {
  Run R{I, o, layout(I.k, o), (char*)work, st};
  HB_TRY(R.prepare(), "hbci prepare");
  HB_TRY(R.load(dets, n), "hbci load");
  HB_TRY(R.read_ctl(), "hbci load");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  HB_TRY(R.diag(0, n, false), "hbci diagonal");
  hipError_t he;
  ifci_status s = R.build_h(n, &he);
  if (s == IFCI_ERR_DEVICE) return device_failure(he, "hbci H");
  if (s != IFCI_OK) return s;
  HB_TRY(R.spmv(c, sigma, n), "hbci sigma");
  HB_TRY(hipStreamSynchronize(st), "hbci sigma");
  return IFCI_OK;
}

ifci_status hbci_select(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                        const double* c, double eps1, uint64_t* added, int64_t* n_added, hipStream_t st) {
  Run R{I, o, layout(I.k, o), (char*)work, st};
  HB_TRY(R.prepare(), "hbci prepare");
  HB_TRY(R.load(dets, n), "hbci load");
  HB_TRY(R.read_ctl(), "hbci load");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  hipLaunchKernelGGL(hbci_select_kernel, dim3(Run::blocks(n, kWaves, 8192)), dim3(64 * kWaves), R.lds, st,
                     R.at<double>(R.L.ints), I.k, c, n, eps1, R.space(), 0);
  HB_TRY(hipGetLastError(), "hbci select");
  HB_TRY(R.read_ctl(), "hbci select");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  const int64_t m = (int64_t)R.ctl.n_det - n;
  if (m > 0)
    HB_TRY(hipMemcpyAsync(added, R.at<uint64_t>(R.L.dets) + n, m * 8, hipMemcpyDeviceToDevice, st), "copy");
  HB_TRY(hipStreamSynchronize(st), "hbci select");
  *n_added = m;
  return IFCI_OK;
}

ifci_status hbci_pt2(const HbciInc& I, const ifci_hbci_options& o, void* work, const uint64_t* dets, int64_t n,
                     const double* c, double e_var, double eps2, double* e_pt2, int64_t* n_ext, hipStream_t st) {
  Run R{I, o, layout(I.k, o), (char*)work, st};
  HB_TRY(R.prepare(), "hbci prepare");
  HB_TRY(R.load(dets, n), "hbci load");
  HB_TRY(R.read_ctl(), "hbci load");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  const double shift = R.ctl.e_core + I.e_const;
  HB_TRY(R.pt2(n, c, e_var - shift, eps2, e_pt2, n_ext), "hbci pt2");
  if (R.ctl.flags) return capacity_failure(R.ctl.flags);
  return IFCI_OK;
}

}  // namespace ifci
