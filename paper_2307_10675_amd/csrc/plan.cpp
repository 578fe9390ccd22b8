// Host plan of libifci: validation, increment enumeration (eqs. 1-5 of the
// paper's iFCI section), the string and single-replacement tables of each
// active-space shape, expansion weights and the workspace layout.
#include "plan.hpp"

#include "launch.hpp"

#include <algorithm>
#include <cstring>
#include <map>
#include <utility>

namespace ifci {

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

static inline int popc(uint32_t x) { return __builtin_popcount(x); }

// Position of a string among equal-popcount masks in increasing order:
// sum over occupied orbitals o_0 < o_1 < ... of C(o_m, m + 1).
static int32_t address(uint32_t mask) {
  int32_t a = 0;
  int m = 0;
  for (int p = 0; p < 32; ++p)
    if (mask >> p & 1u) a += (int32_t)binom(p, ++m);
  return a;
}

// E_pq = a+_p a_q on one string: returns false if zero, else sign and target.
static bool excite(uint32_t I, int p, int q, uint32_t* J, int* sign) {
  if (!(I >> q & 1u)) return false;
  uint32_t rest = I & ~(1u << q);
  if (rest >> p & 1u) return false;
  int lo = p < q ? p : q, hi = p < q ? q : p;
  uint32_t between = rest & ((1u << hi) - 1u) & ~((2u << lo) - 1u);
  *sign = (popc(between) & 1) ? -1 : 1;
  *J = rest | (1u << p);
  return true;
}

static inline int32_t pair_index(int i, int j) {  // i >= j
  return i * (i + 1) / 2 + j;
}

ShapeTables build_shape(int k, int na, std::vector<int32_t>& blob) {
  ShapeTables t;
  t.k = k;
  t.na = na;
  t.n_str = (int)binom(k, na);
  t.npair = k * (k + 1) / 2;
  t.n_link = na * (k - na + 1);
  std::vector<uint32_t> strs;
  strs.reserve(t.n_str);
  for (uint32_t m = 0; m < (1u << k); ++m)
    if (popc(m) == na) strs.push_back(m);
  t.str_off = (int64_t)blob.size();
  for (uint32_t s : strs) blob.push_back((int32_t)s);
  // pair table: E_ij|I> or E_ji|I> for the unordered pair {i, j}
  t.pair_off = (int64_t)blob.size();
  blob.resize(blob.size() + (size_t)t.n_str * t.npair, -1);
  t.link_off = (int64_t)blob.size();
  blob.resize(blob.size() + (size_t)t.n_str * t.n_link, 0);
  t.ord_off = (int64_t)blob.size();
  blob.resize(blob.size() + (size_t)t.n_str * k * k, -1);
  for (int I = 0; I < t.n_str; ++I) {
    int n = 0;
    for (int q = 0; q < k; ++q) {
      if (!(strs[I] >> q & 1u)) continue;
      for (int p = 0; p < k; ++p) {
        uint32_t Jm;
        int sg;
        if (!excite(strs[I], p, q, &Jm, &sg)) continue;
        int32_t J = address(Jm);
        int32_t code = (J << 1) | (sg < 0 ? 1 : 0);
        int32_t Q = p >= q ? pair_index(p, q) : pair_index(q, p);
        blob[t.pair_off + (int64_t)I * t.npair + Q] = code;
        blob[t.link_off + (int64_t)I * t.n_link + n] = (Q << 17) | code;
        blob[t.ord_off + (int64_t)I * k * k + p * k + q] = code;
        ++n;
      }
    }
  }
  // the same pair table pair-major, [npair][n_str] of int16 (2 n_str + 1
  // <= 25,741 at 16 orbitals), as an index into a column copy stored with
  // its negation: J + neg (n_str + 1), n_str for no link (a zero entry after
  // the last string).  A row of strings for one pair is contiguous
  // (coalesced loads over 16 consecutive strings); int16 keeps the 16-orbital
  // table (3.5 MB) within an L2.
  t.pairT_off = (int64_t)blob.size();
  const int64_t nT = (int64_t)t.n_str * t.npair;
  blob.resize(blob.size() + (size_t)((nT + 1) / 2), 0);
  int16_t* pT = (int16_t*)(blob.data() + t.pairT_off);
  for (int I = 0; I < t.n_str; ++I)
    for (int Q = 0; Q < t.npair; ++Q) {
      const int32_t e = blob[t.pair_off + (int64_t)I * t.npair + Q];
      pT[(int64_t)Q * t.n_str + I] = (int16_t)(e < 0 ? t.n_str : (e >> 1) + (e & 1) * (t.n_str + 1));
    }
  return t;
}

void fill_link_dump(int k, int na, int32_t* strings, int32_t* link) {
  std::vector<int32_t> blob;
  ShapeTables t = build_shape(k, na, blob);
  if (strings)
    for (int I = 0; I < t.n_str; ++I) strings[I] = blob[t.str_off + I];
  if (link) {
    for (int I = 0; I < t.n_str; ++I) {
      uint32_t s = (uint32_t)blob[t.str_off + I];
      int n = 0;
      for (int q = 0; q < k; ++q) {
        if (!(s >> q & 1u)) continue;
        for (int p = 0; p < k; ++p) {
          uint32_t Jm;
          int sg;
          if (!excite(s, p, q, &Jm, &sg)) continue;
          int32_t* e = link + ((int64_t)I * t.n_link + n) * 4;
          e[0] = p;
          e[1] = q;
          e[2] = address(Jm);
          e[3] = sg;
          ++n;
        }
      }
    }
  }
}

}  // namespace ifci

using namespace ifci;

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

namespace ifci {
WideSlot wide_slot(const IncDev& d) {
  WideSlot w;
  w.T = 0;
  w.F = align_up(d.stride, 32);
  w.part = w.F + align_up(d.n_str, 32);
  w.state = w.part + align_up(wide_part_doubles(d), 32);
  w.sc = w.state + 4096;
  return w;
}
int64_t wide_slot_doubles(const IncDev& d) { return wide_slot(d).sc + wide_sigma_scratch_doubles(d); }
int64_t wide_ctl_bytes(int cap) {
  return align_up((int64_t)cap * sizeof(WideItem), 256) + align_up((int64_t)cap * 8, 256) +
         align_up((int64_t)wide_ctl_ints(cap) * 4, 256) + align_up((int64_t)cap * 4, 256);
}
}  // namespace ifci

// Builds everything host-side.  Returns IFCI_OK or an error with message set.
ifci_status plan_build(ifci_plan_s* P, const ifci_problem* pr, const ifci_options* op) {
  if (!pr || !pr->body_ptr || !pr->body_orb || !pr->body_nocc) {
    set_error("null problem pointer");
    return IFCI_ERR_ARG;
  }
  if (pr->n_orb < 1 || pr->n_orb > 64) {
    set_error("n_orb must be in 1..64");
    return IFCI_ERR_ARG;
  }
  if (pr->n_bodies < 1) {
    set_error("n_bodies must be >= 1");
    return IFCI_ERR_ARG;
  }
  if (pr->order < 1 || pr->order > pr->n_bodies) {
    set_error("order must be in 1..n_bodies");
    return IFCI_ERR_ARG;
  }
  P->n_orb = pr->n_orb;
  P->n_bodies = pr->n_bodies;
  P->order = pr->order;
  P->e_const = pr->e_const;
  P->opt = *op;
  std::memset(P->tune.ps_block, -1, sizeof(P->tune.ps_block));
  std::memset(P->tune.e_waves, 0, sizeof(P->tune.e_waves));
  if (op->max_space < 2 || op->max_space > kMaxSpace || op->max_iter < 1 || !(op->r_tol > 0) ||
      (op->precision != IFCI_FP64 && op->precision != IFCI_MIXED) ||
      (op->solver != IFCI_SOLVER_BATCHED && op->solver != IFCI_SOLVER_PLAIN) || op->n_guess < 0 ||
      op->n_guess > kPsMax || (op->flags & ~(uint32_t)IFCI_FLAG_ASYNC_WIDE) != 0) {
    set_error("invalid options (max_space 2..16, max_iter >= 1, r_tol > 0, precision, solver, n_guess 0..64, "
              "flags)");
    return IFCI_ERR_ARG;
  }
  if (pr->body_ptr[0] != 0) {
    set_error("body_ptr[0] must be 0");
    return IFCI_ERR_ARG;
  }
  std::vector<int> seen(pr->n_orb, -1);
  for (int b = 0; b < pr->n_bodies; ++b) {
    int lo = pr->body_ptr[b], hi = pr->body_ptr[b + 1];
    if (hi <= lo) {
      set_error("every body needs at least one orbital");
      return IFCI_ERR_ARG;
    }
    std::vector<int> orbs;
    for (int i = lo; i < hi; ++i) {
      int o = pr->body_orb[i];
      if (o < 0 || o >= pr->n_orb) {
        set_error("orbital index out of range");
        return IFCI_ERR_ARG;
      }
      if (seen[o] >= 0) {
        set_error("bodies overlap");
        return IFCI_ERR_ARG;
      }
      seen[o] = b;
      orbs.push_back(o);
    }
    int no = pr->body_nocc[b];
    if (no < 0 || no > (int)orbs.size()) {
      set_error("body_nocc out of range");
      return IFCI_ERR_ARG;
    }
    P->bodies.push_back(orbs);
    P->nocc.push_back(no);
    for (int i = 0; i < no; ++i) P->ref_occ.push_back(orbs[i]);
  }
  std::sort(P->ref_occ.begin(), P->ref_occ.end());

  // weights w_k = sum_{m=0}^{n-k} (-1)^m C(N_b - k, m)
  for (int k = 1; k <= P->order; ++k) {
    double w = 0;
    for (int m = 0; m <= P->order - k; ++m) w += ((m & 1) ? -1.0 : 1.0) * (double)binom(P->n_bodies - k, m);
    P->weights.push_back(w);
  }

  // increments by size then lexicographic body tuple
  std::map<std::pair<int, int>, ShapeTables> shapes;
  const int mmax = op->max_space;
  for (int sz = 1; sz <= P->order; ++sz) {
    std::vector<int> S(sz);
    for (int i = 0; i < sz; ++i) S[i] = i;
    while (true) {
      std::vector<int> act, core;
      std::vector<char> in(P->n_bodies, 0);
      int na = 0;
      for (int b : S) in[b] = 1, na += P->nocc[b];
      for (int b = 0; b < P->n_bodies; ++b) {
        if (in[b])
          act.insert(act.end(), P->bodies[b].begin(), P->bodies[b].end());
        else
          core.insert(core.end(), P->bodies[b].begin(), P->bodies[b].begin() + P->nocc[b]);
      }
      std::sort(act.begin(), act.end());
      std::sort(core.begin(), core.end());
      int k = (int)act.size();
      if (k > kMaxAct) {
        set_error("an increment has more than 16 active orbitals");
        return IFCI_ERR_UNSUPPORTED;
      }
      if (na > k) {
        set_error("more electrons than orbitals in an increment");
        return IFCI_ERR_ARG;
      }
      auto key = std::make_pair(k, na);
      if (!shapes.count(key)) shapes[key] = build_shape(k, na, P->tables);
      const ShapeTables& t = shapes[key];
      IncDev d{};
      d.k = k;
      d.na = na;
      d.n_str = t.n_str;
      d.npair = t.npair;
      d.n_link = t.n_link;
      d.n_core = (int)core.size();
      d.id = (int)P->inc.size();
      d.n_det = (int64_t)t.n_str * t.n_str;
      d.n_sym = tri(t.n_str);
      d.stride = align_up(d.n_sym, 8);
      d.act_off = (int64_t)P->orbs.size();
      P->orbs.insert(P->orbs.end(), act.begin(), act.end());
      d.core_off = (int64_t)P->orbs.size();
      P->orbs.insert(P->orbs.end(), core.begin(), core.end());
      d.str_off = t.str_off;
      d.pair_off = t.pair_off;
      d.link_off = t.link_off;
      d.ord_off = t.ord_off;
      d.pairT_off = t.pairT_off;
      d.int_off = P->ints_doubles;
      P->ints_doubles += int_block_size(k);
      // increments for the device-wide solver get the default subspace
      // when 3 selects the on-chip three-vector iteration
      const bool on_chip = op->solver != IFCI_SOLVER_PLAIN && k <= 8 &&
                           ifci::batched_lds_bytes(k, t.n_str, t.n_link) <= ifci::kMaxLds;
      d.mspace = (!on_chip && mmax == 3) ? 12 : mmax;
      d.vec_off = P->dav_doubles;
      P->dav_doubles += vec_block_size(d.stride, d.mspace);
      P->max_ndet = std::max(P->max_ndet, d.n_det);
      P->max_npair = std::max<int64_t>(P->max_npair, d.npair);
      P->max_stride = std::max(P->max_stride, d.stride);
      P->rdm_off.push_back(P->rdm_doubles);
      P->rdm_doubles += (int64_t)k * k + (int64_t)k * k * k * k;
      P->inc.push_back(d);
      P->inc_bodies.push_back(S);
      // next combination
      int i = sz - 1;
      while (i >= 0 && S[i] == P->n_bodies - sz + i) --i;
      if (i < 0) break;
      ++S[i];
      for (int j = i + 1; j < sz; ++j) S[j] = S[j - 1] + 1;
    }
  }
  // heaviest first: determinant count, then canonical index
  P->order_all.resize(P->inc.size());
  for (size_t i = 0; i < P->inc.size(); ++i) P->order_all[i] = (int32_t)i;
  std::stable_sort(P->order_all.begin(), P->order_all.end(), [&](int32_t a, int32_t b) {
    return P->inc[a].n_det > P->inc[b].n_det;
  });

  // workspace layout
  const int64_t A = 256;
  int64_t off = 0;
  P->off_ints = off;
  off = align_up(off + P->ints_doubles * 8, A);
  P->off_dav = off;
  off = align_up(off + P->dav_doubles * 8, A);
  // device-wide scratch: the materialised E (npair x n_det) where the
  // general product may run; at 16 orbitals only the column path's (full C,
  // S and fragments: 2.7 GB instead of 180 GB of E)
  {
    int64_t need = 0;
    for (const ifci::IncDev& d : P->inc) {
      int64_t e = d.npair * d.n_det;
      if (ifci::sigma_column_supported(d))
        e = d.k > 14 ? ifci::sigma_column_ws_doubles(d) : std::max(e, ifci::sigma_column_ws_doubles(d));
      need = std::max(need, e);
    }
    P->E_doubles = align_up(need, 32);
  }
  // device-wide solves run several increments at once when their scratch is
  // small: up to 8 slots within 2 GiB of E scratch beyond the first, and no
  // more slots than increments that can take that path
  // (the plain solver's per-increment loops; the batched solver needs one
  // slot, for ifci_sigma and ifci_sigma_sector)
  {
    int64_t n_wide = 0;
    for (const ifci::IncDev& d : P->inc)
      if (op->solver == IFCI_SOLVER_PLAIN) ++n_wide;
    const int64_t by_mem = 1 + ((int64_t)2 << 30) / std::max<int64_t>(1, P->E_doubles * 8);
    P->n_slots = (int)std::max<int64_t>(1, std::min<int64_t>({8, by_mem, n_wide}));
  }
  P->off_E = off;
  off = align_up(off + P->n_slots * P->E_doubles * 8, A);
  P->tmp_doubles = align_up(4 * P->max_stride + 8, 32);
  P->off_tmp = off;
  off = align_up(off + P->n_slots * P->tmp_doubles * 8, A);
  P->part_doubles = 2048 * 40;
  P->off_part = off;
  off = align_up(off + P->n_slots * P->part_doubles * 8, A);
  P->off_state = off;
  off = align_up(off + P->n_slots * 4096 * 8, A);
  // batched device-wide solver: one slot per increment it runs at once
  // (temporaries, partial sums, state, sigma scratch), up to kWideBudget
  // bytes of slots, and the control block (items, their pointers, live
  // lists, output positions)
  {
    int64_t slot = 0, n_wide = 0;
    for (const ifci::IncDev& d : P->inc) {
      const bool on_chip = op->solver != IFCI_SOLVER_PLAIN && d.k <= 8 &&
                           ifci::batched_lds_bytes(d.k, d.n_str, d.n_link) <= ifci::kMaxLds;
      if (on_chip || op->solver == IFCI_SOLVER_PLAIN) continue;
      ++n_wide;
      slot = std::max(slot, wide_slot_doubles(d));
    }
    P->wide_slot_doubles = align_up(slot, 32);
    P->wide_cap = 0;
    if (n_wide > 0) {
      const int64_t by_mem = std::max<int64_t>(1, kWideBudget / (P->wide_slot_doubles * 8));
      P->wide_cap = (int)std::min<int64_t>(n_wide, by_mem);
    }
    P->off_wide = off;
    off = align_up(off + (int64_t)P->wide_cap * P->wide_slot_doubles * 8, A);
    P->off_wide_ctl = off;
    off = align_up(off + wide_ctl_bytes(P->wide_cap), A);
  }
  P->off_rdm = off;
  off = align_up(off + P->rdm_doubles * 8, A);
  P->off_misc = off;
  off = align_up(off + 256 * 8, A);
  P->off_eps = off;
  off = align_up(off + (int64_t)P->inc.size() * 8, A);
  P->ws_bytes = off;
  P->solved.assign(P->inc.size(), 0);
  P->ref_off = (int64_t)P->orbs.size();
  P->orbs.insert(P->orbs.end(), P->ref_occ.begin(), P->ref_occ.end());
  return IFCI_OK;
}
