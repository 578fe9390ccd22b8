/*
 * ifci.h -- C ABI of libifci, the MI355X (gfx950) iFCI increment solver.
 *
 * The problem is stated as in the paper (Methods, "Incremental Full
 * Configuration Interaction"): integrals h_pq and (pq|rs) over a localized
 * orbital basis, a partition of the occupied orbitals into "bodies", and a
 * truncation order n of the many-body expansion (eq. 1).  The library
 * enumerates every increment S (1 <= |S| <= n), solves for the lowest root
 * of the Hamiltonian in the space of S on the GPU, and assembles the
 * incremental energies of eqs. 2-5 and the expansion total.
 *
 * Conventions shared by every call:
 *  - integrals are FP64, row-major; (pq|rs) (chemists' order) sits at
 *    eri[((p*n + q)*n + r)*n + s]; both must be symmetric as real integrals are;
 *  - an increment S correlates every orbital of its bodies; the reference-
 *    occupied orbitals of the other bodies stay doubly occupied (frozen core)
 *    and their virtual orbitals are removed;
 *  - the active orbitals of S, in increasing full-space index, are numbered
 *    0..k-1; a one-spin string is a k-bit mask, strings are ordered by
 *    increasing mask value; a determinant is |A,B> = a+(A, alpha) a+(B, beta)
 *    |core>, and a CI vector is C[A][B] row-major (beta index fastest);
 *  - the root solved for is the lowest one with C symmetric (C = C^T), the
 *    even-spin states, which hold the closed-shell singlet;
 *  - increments are numbered by size, then lexicographically by body tuple.
 *
 * Ownership: the caller owns every device buffer it passes (integrals,
 * vectors, outputs, the workspace); the library never frees them.  A plan
 * owns its host tables and a few small device tables it allocates itself.
 * Buffers are contiguous and live on the plan's device.  A plan is not
 * thread-safe; distinct plans are independent.
 *
 * Errors: every call returns ifci_status.  Invalid arguments return
 * IFCI_ERR_ARG before any device work is queued; shapes the kernels do not
 * handle return IFCI_ERR_UNSUPPORTED; HIP failures return IFCI_ERR_DEVICE.
 * ifci_last_error() gives a human-readable detail (thread-local).  Calls that
 * take a stream only enqueue work on it unless stated otherwise.
 */
#ifndef IFCI_H
#define IFCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IFCI_ABI_VERSION 4

typedef struct ifci_plan_s* ifci_plan_t;
typedef void* ifci_stream_t; /* a hipStream_t; NULL = the null stream */

typedef enum {
  IFCI_OK = 0,
  IFCI_ERR_ARG = 1,
  IFCI_ERR_UNSUPPORTED = 2,
  IFCI_ERR_OOM = 3,
  IFCI_ERR_DEVICE = 4,
  IFCI_ERR_NOT_CONVERGED = 5,
  IFCI_ERR_STATE = 6
} ifci_status;

typedef enum {
  IFCI_FP64 = 0,   /* every step in FP64 */
  IFCI_MIXED = 1   /* sigma in FP32 (MFMA, FP32 accumulation) on the shifted
                      Hamiltonian, FP64 subspace, FP64 residual refinement */
} ifci_precision;

typedef enum {
  IFCI_SOLVER_BATCHED = 0, /* one persistent workgroup per increment, whole
                              eigensolve on chip, increments of at most 8
                              active orbitals (larger ones take the plain
                              path inside the same call) */
  IFCI_SOLVER_PLAIN = 1    /* per increment, device-wide kernels for sigma and
                              vector steps, host-driven loop; any size */
} ifci_solver;

/* Per-increment status words written by ifci_davidson. */
enum {
  IFCI_INC_PENDING = 0,
  IFCI_INC_DONE = 1,
  IFCI_INC_NOT_CONVERGED = 2,
  IFCI_INC_EVICTED = 3,
  IFCI_INC_SCREENED = 4  /* dropped by ifci_screen: not solved, energy NaN */
};

/* The problem (paper, Methods: eqs. 1-5 and the reference determinant). */
typedef struct {
  int32_t n_orb;            /* spatial orbitals of the full system, 1..64 */
  int32_t n_bodies;         /* >= 1 */
  const int32_t* body_ptr;  /* host [n_bodies + 1] CSR offsets, body_ptr[0] = 0 */
  const int32_t* body_orb;  /* host [body_ptr[n_bodies]] disjoint orbital indices */
  const int32_t* body_nocc; /* host [n_bodies]: the first body_nocc[b] orbitals
                               of body b are doubly occupied in the reference */
  int32_t order;            /* truncation order n, 1..n_bodies */
  double e_const;           /* constant added to every energy */
} ifci_problem;

typedef struct {
  int32_t precision;  /* ifci_precision */
  int32_t solver;     /* ifci_solver */
  double r_tol;       /* converged when ||H c - E c|| <= r_tol (unit c, FP64) */
  double r_tol_inner; /* IFCI_MIXED: FP32 stage stops at this residual */
  int32_t max_iter;   /* eigensolver iterations (sigma builds) per increment */
  int32_t max_space;  /* Davidson subspace size before a thick restart,
                         2..16; in the batched solver 3 selects the
                         three-vector {x, w, p} iteration (locally
                         optimal, no restarts) */
  uint32_t flags;     /* IFCI_FLAG_* bits */
  int32_t n_guess;    /* on-chip solvers (increments of up to 8 active
                         orbitals): the n_guess lowest diagonal entries of
                         the symmetric sector (rounded down to even, at most
                         64 and an eighth of the sector) span a block of H
                         (Slater-Condon rules) that is diagonalised once per
                         increment; its lowest eigenvector is the initial
                         guess and its shifted inverse (theta - H_PP)^-1 the
                         preconditioner on those entries, the diagonal one
                         elsewhere (a block Davidson preconditioner).  0 or
                         1: the single lowest determinant and the diagonal
                         preconditioner.  The device-wide solver (above 8
                         orbitals) uses the latter in any case. */
} ifci_options;

/* ifci_davidson returns as soon as the work of every increment is
 * enqueued: the batched device-wide solver (increments above 8 active
 * orbitals) enqueues max_iter iterations' worth of launches, each a no-op
 * once every increment has stopped, instead of the host checking the number
 * of live increments between groups of iterations. */
#define IFCI_FLAG_ASYNC_WIDE 1u

/* Version of this header the library was built from (IFCI_ABI_VERSION). */
int ifci_abi_version(void);

/* Fill *opt with the defaults: FP64, batched, r_tol 1e-7, r_tol_inner 1e-4,
 * max_iter 300, max_space 12, flags 0, n_guess 64. */
void ifci_default_options(ifci_options* opt);

/* Validate the problem, enumerate the increments, build the string and
 * single-replacement tables of every distinct active-space shape, size the
 * workspace, and upload the small tables to `hip_device`.  Synchronous.
 * Returns IFCI_ERR_ARG for overlapping or out-of-range bodies, order outside
 * 1..n_bodies, or a null pointer; IFCI_ERR_UNSUPPORTED when an increment has
 * more than 16 active orbitals. */
ifci_status ifci_plan_create(const ifci_problem* problem, const ifci_options* options,
                             int hip_device, ifci_plan_t* out);
ifci_status ifci_plan_destroy(ifci_plan_t plan);

/* Sizes: number of increments, bytes of device workspace ifci_set_workspace
 * needs, and the largest increment's determinant count. */
ifci_status ifci_plan_info(ifci_plan_t plan, int64_t* n_inc, int64_t* workspace_bytes,
                           int64_t* max_ndet);

/* Description of increment idx: its bodies (host [order], -1 padded), active
 * orbitals k, alpha electrons, and determinant count. */
ifci_status ifci_increment(ifci_plan_t plan, int64_t idx, int32_t* bodies, int32_t* n_act,
                           int32_t* n_alpha, int64_t* n_det);

/* Expansion weights w_k (host [order]): the coefficient with which every
 * E_c(T), |T| = k, enters the truncated sum of eqs. 1-5. */
ifci_status ifci_weights(ifci_plan_t plan, double* w);

/* String and single-replacement tables of a (k, n_alpha) space, for checking
 * bit-exactly.  Host only, no plan or device needed.  These are the
 * occupation strings and the coupling coefficients <J|E_pq|I> of the
 * string-driven determinant CI of Knowles and Handy (Chem. Phys. Lett. 111,
 * 315, 1984) and Olsen et al. (J. Chem. Phys. 89, 2185, 1988); the paper
 * gives the determinant counts of such spaces (Methods, Table 1).
 * strings: host [C(k, n_alpha)] bitmasks, increasing.
 * link:    host [C(k, n_alpha)][n_alpha*(k - n_alpha + 1)][4] entries
 *          (p, q, J, sign) meaning E_pq |I> = sign |J>; for each string,
 *          q runs over its occupied orbitals in increasing order and p over
 *          the orbitals empty once q is removed (p = q included), increasing.
 * Either pointer may be NULL. */
ifci_status ifci_tables(int32_t k, int32_t n_alpha, int32_t* strings, int32_t* link);

/* Hand the plan a caller-owned device workspace of at least
 * workspace_bytes (ifci_plan_info), 256-byte aligned. */
ifci_status ifci_set_workspace(ifci_plan_t plan, void* dev_ptr, int64_t bytes);

/* Load integrals (device h [n*n], eri [n^4]) and embed every increment:
 * frozen-core energy, effective one-electron operator, active two-electron
 * block, and diagonal of H.  Reads h and eri only while the queued work runs. */
ifci_status ifci_set_integrals(ifci_plan_t plan, const double* h, const double* eri,
                               ifci_stream_t stream);

/* sigma = H c for increment `inc`, with H the active-space Hamiltonian
 * (without the frozen-core energy and e_const), the matrix-vector product of
 * determinant FCI in the Knowles-Handy form: D[kl][I] = (E_kl c)_I,
 * E = (1/2) (ij|kl) D (a dense pair-by-pair contraction), sigma gathered
 * back through the single-replacement tables.  The Hamiltonian is the one of
 * the paper's increments (Methods, iFCI: the calculation restricted to the
 * bodies of the increment).  c and sigma: device
 * [n_det] FP64, C[A][B] layout, any c (no symmetry needed); precision is
 * IFCI_FP64 or IFCI_MIXED (FP32 arithmetic, results widened to FP64).
 * Uses the workspace; c and sigma must not alias.  Materialises E
 * (npair x n_det); where the plan's workspace is sized only for the column
 * path (half-filled 16-orbital increments, 180 GB of E otherwise) it returns
 * IFCI_ERR_UNSUPPORTED: use ifci_sigma_sector there. */
ifci_status ifci_sigma(ifci_plan_t plan, int64_t inc, const double* c, double* sigma,
                       int32_t precision, ifci_stream_t stream);

/* ifci_sigma for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same product, arguments, layout and errors as ifci_sigma, but the
 * product's scratch (E, npair x n_det values of the contraction precision)
 * lives in a fixed array of 32 MiB that the library holds on every device
 * it runs on until the process ends, instead of in the plan's workspace.
 * The call allocates nothing (the plan, its workspace and integrals are set
 * up beforehand).  Increments whose E exceeds 32 MiB (in FP64: 10o10e fits,
 * 12o12e does not) return IFCI_ERR_UNSUPPORTED.  Every call on one device
 * shares that device's array, which keeps the last call's contents (each
 * call overwrites all it reads): calls that overlap on one device -- on
 * different streams, or from different threads -- race. */
ifci_status ifci_sigma_noalloc(ifci_plan_t plan, int64_t inc, const double* c, double* sigma,
                               int32_t precision, ifci_stream_t stream);

/* Same product restricted to symmetric c (C = C^T, the sector the solvers
 * search): c and sigma are packed scaled vectors (entry (a <= b) at
 * b (b + 1) / 2 + a, off-diagonal entries times sqrt 2), n_str (n_str + 1) / 2
 * FP64 each.  Increments that fit the batched solver (up to 8 active
 * orbitals) run as that solver computes sigma, in one workgroup; half-filled
 * increments of 10, 12, 14 or 16 orbitals run the fused column kernel (one
 * workgroup per beta string, E never leaves LDS; uses the workspace).
 * Other shapes: IFCI_ERR_UNSUPPORTED.  c and sigma must not alias. */
ifci_status ifci_sigma_sector(ifci_plan_t plan, int64_t inc, const double* c, double* sigma,
                              int32_t precision, ifci_stream_t stream);

/* Lowest even-spin root of increments [first, first + count): E(S) of every
 * increment S of eqs. 1-5 (Methods, iFCI), by Davidson's method (J. Comput.
 * Phys. 17, 87, 1975), thick restart or the three-vector {x, w, p} form
 * (locally optimal, Knyazev) per max_space; on chip started from and
 * preconditioned by the P-space block of n_guess, device-wide from the
 * lowest determinant with the diagonal preconditioner.
 * e_out: device [count] total energies E(S) (frozen core and e_const
 * included); status_out: device [count] IFCI_INC_* words; evict_mask: device
 * [count] or NULL -- increments whose byte is nonzero are abandoned after one
 * iteration and reported EVICTED (failure injection); iters_out/resid_out:
 * device [count] or NULL.  Converged vectors stay in the workspace for
 * ifci_vector and ifci_rdm.  Increments dropped by a screening mask
 * (ifci_screen) are not solved: status IFCI_INC_SCREENED, energy NaN.
 * Increments that fit on chip run in one launch of the batched solver; the
 * others (more than 8 active orbitals) run in the batched device-wide
 * solver, every increment of a shape in the same launches, its iterations
 * replayed from a captured graph with restart, precision switch and stop
 * decided on the device (with IFCI_FLAG_ASYNC_WIDE the host never reads the
 * live count and the call only enqueues).  With the plain solver every
 * increment runs device-wide on its own, up to 8 at a time on streams the
 * plan owns, each driven by a host thread; that work starts after what is
 * already queued on `stream` and `stream` continues after it, so the call
 * keeps stream order. */
ifci_status ifci_davidson(ifci_plan_t plan, int64_t first, int64_t count, double* e_out,
                          int32_t* status_out, const uint8_t* evict_mask, int32_t* iters_out,
                          double* resid_out, ifci_stream_t stream);

/* Lowest even-spin roots of every increment of n_plans plans (for instance
 * independent FCI problems, each a one-increment plan) in one batched solve:
 * each plan's increments that fit on chip run in one launch of the batched
 * solver, and the others of all plans join the same batched device-wide
 * solve (one per active-space shape).  plans: host [n_plans], distinct, on
 * one device, each with workspace and integrals set, all created with the
 * batched solver and identical options.  e_out[j], status_out[j] (and,
 * where given, iters_out[j], resid_out[j]): device arrays of plan j's
 * increment count, as in ifci_davidson; iters_out and resid_out may be NULL.
 * Stream order and return as in ifci_davidson; converged vectors stay in
 * each plan's workspace.  The first plan keeps the solve's control block
 * (device memory it allocates on first use and grows as needed).
 * IFCI_ERR_UNSUPPORTED for a plan with a screening mask (ifci_screen). */
ifci_status ifci_davidson_group(const ifci_plan_t* plans, int32_t n_plans, double* const* e_out,
                                int32_t* const* status_out, int32_t* const* iters_out,
                                double* const* resid_out, ifci_stream_t stream);

/* Connected n-body screening (paper, Methods, iFCI subsection, the CnB
 * paragraph; the criterion's details are in the paper's Supplementary
 * Information, which is not available -- this is the reading taken).  From
 * the total energies of every increment of one and two bodies (e_inc, device
 * [n_inc], increment order; the entries of larger increments are not read):
 * bodies i and j are connected when |eps_ij| >= threshold (eq. 3); an
 * increment of three or more bodies is kept when its bodies form one
 * connected graph under that relation; increments of one or two bodies are
 * always kept.  The mask stays with the plan: ifci_davidson then skips
 * dropped increments (status IFCI_INC_SCREENED, energy NaN, no work),
 * ifci_energy sums the screened expansion, and ifci_rdm (weights NULL)
 * weights each kept increment's densities by its coefficient in that sum
 * (user weights must be zero on dropped increments).  keep (host [n_inc],
 * may be NULL) receives the mask, n_kept (may be NULL) its count.
 * threshold < 0 removes the mask.  Synchronises the stream.  IFCI_ERR_ARG
 * when a one- or two-body energy is not finite (solve those first). */
ifci_status ifci_screen(ifci_plan_t plan, const double* e_inc, double threshold, uint8_t* keep,
                        int64_t* n_kept, ifci_stream_t stream);

/* Grouped contributions (paper, Results, the PFAS bond-breaking analysis and
 * its Fig. 4): each body carries a group label (group_of_body, host
 * [n_bodies], values 0 .. n_groups - 1), and every increment belongs to the
 * combination of its bodies' labels, a multiset written as the sorted label
 * list.  ifci_group_count gives the number of combinations of 1 .. order
 * labels; ifci_group_sums fills sums (host [n_combos]) with the sum of eps_S
 * (device [n_inc], from ifci_energy) over each combination's increments, in
 * increment order with compensated addition, and combos (host
 * [n_combos][order], may be NULL) with the labels, -1 padded; combinations
 * run by size, then lexicographically.  The difference of two calculations
 * with comparable orbitals (two geometries) is the difference of their
 * sums.  Synchronises the stream.  IFCI_ERR_ARG for a label out of range. */
ifci_status ifci_group_count(ifci_plan_t plan, int32_t n_groups, int64_t* n_combos);
ifci_status ifci_group_sums(ifci_plan_t plan, const double* eps, const int32_t* group_of_body, int32_t n_groups,
                            double* sums, int32_t* combos, ifci_stream_t stream);

/* Summation natural orbitals (paper, Methods, iFCI subsection, the SNO
 * paragraph, eq. 6) for a system whose bodies are single occupied orbitals
 * sharing the virtual orbitals vir (device [n_vir], n_vir <= 16).  gamma:
 * device [n_occ][n_orb][n_orb], per occupied orbital the one-particle
 * density of the FCI of its two electrons in itself plus every virtual,
 * the other occupied orbitals frozen (exact CISD for two electrons: solve it
 * as a one-body problem and take ifci_rdm with weight 1 on that increment).
 * inc_occ: device [n_inc][order], the occupied-orbital positions (0 ..
 * n_occ - 1) of each increment, -1 padded.  For each increment rho_S = sum
 * of its members' blocks over vir; its natural orbitals (eigenvectors, one
 * wavefront each, parallel Jacobi) with occupation >= 10^-eta are written as
 * the first n_keep[inc] columns of rot (device [n_inc][n_vir][n_vir], row =
 * virtual, largest occupation first, the other columns zero); n_keep:
 * device [n_inc].  Stream-ordered; allocates nothing. */
ifci_status ifci_sno_orbitals(const double* gamma, int32_t n_orb, const int32_t* vir, int32_t n_vir,
                              const int32_t* inc_occ, int64_t n_inc, int32_t order, double eta, double* rot,
                              int32_t* n_keep, ifci_stream_t stream);

/* The integrals of one SNO increment in its rotated basis: m = n_s + n_keep
 * + n_other orbitals, in order S's occupied orbitals, the first n_keep
 * columns of rot (that increment's [n_vir][n_vir] block from
 * ifci_sno_orbitals) over vir, the other occupied orbitals; col_orb (device
 * [n_s + n_other]) the full-space indices of the occupied ones in that
 * order.  h_out = C^T h C (device [m][m]) and eri_out (device [m^4], chemist
 * order) by four quarter transformations of eri (device [n_orb^4]); work:
 * device [work_doubles], at least n_orb m + 2 n_orb^3 m (IFCI_ERR_ARG
 * otherwise, before any device work).  The increment is then an
 * ordinary problem over these integrals: one body of its first n_s + n_keep
 * orbitals with n_s occupied, and one frozen body per other occupied
 * orbital.  Stream-ordered; allocates nothing. */
ifci_status ifci_sno_transform(const double* h, const double* eri, int32_t n_orb, const int32_t* vir, int32_t n_vir,
                               const int32_t* col_orb, int32_t n_s, int32_t n_other, const double* rot,
                               int32_t n_keep, double* work, int64_t work_doubles, double* h_out, double* eri_out,
                               ifci_stream_t stream);

/* Copy the converged unit vector of increment inc (device [n_det]). */
ifci_status ifci_vector(ifci_plan_t plan, int64_t inc, double* c_out, ifci_stream_t stream);

/* Energy assembly, eqs. 2-5: from device e_inc [n_inc] total energies
 * compute eps [n_inc] (device, may be NULL) and host out[order + 2] =
 * {E_total, E_ref, E_c^(1), ..., E_c^(n)}.  Synchronises the stream.
 * status (device [n_inc] or NULL): IFCI_ERR_NOT_CONVERGED if any word is
 * neither IFCI_INC_DONE nor IFCI_INC_SCREENED (outputs still written).
 * With a screening mask (ifci_screen) a dropped increment has eps = 0 and a
 * kept one eps_S = E_c(S) - sum over proper non-empty subsets of eps_T (the
 * recursion of eqs. 2-5); without one, the same sums in their closed
 * inclusion-exclusion form. */
ifci_status ifci_energy(ifci_plan_t plan, const double* e_inc, const int32_t* status,
                        double* eps, double* out, ifci_stream_t stream);

/* Gradient of E_total (or of sum_S weights[S] E(S) + (1 - sum) E_ref when
 * weights, device [n_inc], is given) with respect to every entry of h and
 * eri taken as independent, by the Hellmann-Feynman theorem (each E(S) is an
 * eigenvalue, so its derivative is the expectation value of the derivative
 * of H: the 1- and 2-particle density matrices of the converged vector),
 * weighted as the expansion of eqs. 1-5 weights each E(S): dE_dh (device [n*n]) = weighted 1-RDM gamma,
 * dE_deri (device [n^4], may be NULL) = weighted Gamma / 2.  Needs the
 * converged vectors of every increment that is not screened out
 * (ifci_davidson first). */
ifci_status ifci_rdm(ifci_plan_t plan, const double* weights, double* dE_dh, double* dE_deri,
                     ifci_stream_t stream);

/* Tracing: when `counters` (device [n_inc][8] int64, or NULL to switch off)
 * is set, the batched solver adds per increment the shader-clock cycles of
 * its phases: 0 set-up and diagonal, 1 sigma, 2 subspace matrix and
 * eigensolve, 3 residual and preconditioning, 4 thick restart, 5
 * orthogonalisation, and writes 6 the sigma count and 7 the total cycles.
 * The caller zeroes the buffer; it must outlive the next ifci_davidson. */
ifci_status ifci_set_phase_counters(ifci_plan_t plan, int64_t* counters, int64_t n);

/* Tuning of the on-chip solvers (increments of up to 8 active orbitals) for
 * increments of k active orbitals.  precision selects the row: IFCI_FP64
 * for FP64 plans and for every FP64 sigma, IFCI_MIXED for mixed plans and
 * their FP32 sigmas.  ps_block caps the P-space block (n_guess) of that
 * shape in plans of that precision (-1: n_guess itself; 0: no block);
 * e_waves sets the number of waves of the 512-thread workgroup that
 * contract the pair matrix in sigmas of that precision, each into its own
 * LDS slice (0: as many as LDS holds; a larger request is lowered to what
 * fits).  Neither changes the converged
 * result beyond rounding: ps_block changes the starting vector and the
 * preconditioner, e_waves the order of the sigma's column work.  Values
 * come from a tuner that times the solver on the caller's workload
 * (paper_2307_10675_amd/tune.py); a plan starts with every entry at its
 * built-in choice.  IFCI_ERR_ARG outside k 1..8, ps_block -1..64,
 * e_waves 0..8. */
ifci_status ifci_set_tuning(ifci_plan_t plan, int32_t k, int32_t precision, int32_t ps_block, int32_t e_waves);

/* ---------------------------------------------------------------------------
 * Heat-bath selected CI with a second-order Epstein-Nesbet correction (HBCI;
 * paper, Methods, iFCI subsection, the HBCI paragraph, where it is the
 * solver of every increment; the method of Holmes, Tubman and Umrigar,
 * J. Chem. Theory Comput. 12, 3674 (2016)), on one increment of a plan whose
 * integrals are set (ifci_set_integrals).
 *
 * Determinant keys (uint64): bit p (0 <= p < k) is the increment's p-th
 * active orbital (ascending orbital index) with spin alpha, bit 32 + p the
 * same orbital with spin beta.  The core's creation operators come first,
 * then the alpha ones, then the beta ones, each group ascending; vectors over
 * keys follow that sign convention.
 *
 * Selection: V starts as the reference determinant (the increment's closed
 * shell) with c = 1; each step adds every determinant a outside V with
 * max over i in V of |H_ai c_i| > eps1, together with its spin-flipped
 * partner (alpha and beta strings exchanged), and re-solves the lowest root
 * of H over V in the flip-symmetric sector (Davidson, restarted from the
 * previous vector); it ends when a step adds nothing (converged) or after
 * max_iter steps.  PT2: for every a outside V,
 * N_a = sum over i in V with |H_ai c_i| > eps2 of H_ai c_i and
 * E_PT2 = sum_a N_a^2 / (E_var - H_aa).  Every step runs in device kernels
 * over hash tables in the caller's work buffer; the host drives the loop.
 * ------------------------------------------------------------------------- */
typedef struct {
  double eps1;       /* variational selection threshold (Eh), >= 0 */
  double eps2;       /* PT2 screening threshold (Eh), >= 0 */
  int32_t max_iter;  /* selection steps, >= 1 */
  int32_t max_dav;   /* Davidson iterations per step, >= 1 */
  int32_t m_max;     /* Davidson subspace before a restart, 2..16 */
  double r_tol;      /* a variational root is taken at ||H c - E c|| <= r_tol */
  int64_t max_det;   /* capacity of V (determinants), >= 2 */
  int64_t max_nnz;   /* capacity of H over V (off-diagonal nonzeros), >= 1 */
  int64_t max_ext;   /* capacity of the PT2 external space, >= 1 */
} ifci_hbci_options;

/* The paper's thresholds (eps1 = 1 mEh, eps2 = 1 uEh) and capacities of
 * 2^20 determinants, 2^28 nonzeros and 2^26 external determinants. */
void ifci_hbci_default_options(ifci_hbci_options* options);

/* Bytes of the device work buffer that the HBCI calls on increment inc need
 * with these capacities (256-byte aligned buffer). */
ifci_status ifci_hbci_work_bytes(ifci_plan_t plan, int64_t inc, const ifci_hbci_options* options,
                                 int64_t* bytes);

/* HBCI of increment inc.  result: host [8] = E_var (total energy, the
 * plan's e_const and the frozen core included), E_PT2, |V|, selection steps
 * taken, converged (1 when a step added nothing and every root met r_tol,
 * else 0), the final residual norm, the number of external determinants
 * with a nonzero N_a, and the nonzeros of H over V.  dets_out (device
 * [max_det] keys, insertion order) and c_out (device [max_det], unit norm)
 * receive V and its vector when non-NULL.  work: device [work_bytes] from
 * ifci_hbci_work_bytes, 256-byte aligned, owned by the caller.  Synchronises
 * the stream.  IFCI_ERR_OOM when V, H or the external space outgrow their
 * capacities (the results are then not written); IFCI_ERR_ARG for bad
 * options or a buffer too small; IFCI_ERR_STATE before ifci_set_integrals. */
ifci_status ifci_hbci_solve(ifci_plan_t plan, int64_t inc, const ifci_hbci_options* options, void* work,
                            int64_t work_bytes, double* result, uint64_t* dets_out, double* c_out,
                            ifci_stream_t stream);

/* ifci_hbci_solve of increments first .. first+count-1 by n_workers host
 * threads (1..64), each with a stream of its own (created and destroyed
 * here) and its own work buffer works[w] (host array of n_workers device
 * pointers, each work_bytes long and at least ifci_hbci_work_bytes of every
 * increment of the range); the largest increments start first.  results:
 * host [count][8], each row as ifci_hbci_solve's result.  Returns when every
 * increment is done; the first failure stops the workers and is returned
 * (the other rows are then undefined).  The increments are independent, so
 * their small host-driven loops overlap on the device. */
ifci_status ifci_hbci_solve_range(ifci_plan_t plan, int64_t first, int64_t count, const ifci_hbci_options* options,
                                  void* const* works, int64_t work_bytes, int32_t n_workers, double* results);

/* The steps of ifci_hbci_solve on a caller's space, for checking them.
 * dets: device [n] distinct keys (n <= max_det); c: device [n].
 * ifci_hbci_sigma: sigma (device [n]) = (H - E_core - e_const) c over the
 * space, the constant energy left out as in ifci_sigma.
 * ifci_hbci_select: the keys added by one selection step from (dets, c) at
 * eps1, flip partners included, into added (device [max_det - n], in no
 * particular order) and their count into *n_added (host).
 * ifci_hbci_pt2: *e_pt2 and *n_ext (host) of the PT2 step at eps2 about the
 * total energy e_var.  All synchronise the stream; IFCI_ERR_OOM as above. */
ifci_status ifci_hbci_sigma(ifci_plan_t plan, int64_t inc, const ifci_hbci_options* options, void* work,
                            int64_t work_bytes, const uint64_t* dets, int64_t n, const double* c, double* sigma,
                            ifci_stream_t stream);
ifci_status ifci_hbci_select(ifci_plan_t plan, int64_t inc, const ifci_hbci_options* options, void* work,
                             int64_t work_bytes, const uint64_t* dets, int64_t n, const double* c, double eps1,
                             uint64_t* added, int64_t* n_added, ifci_stream_t stream);
ifci_status ifci_hbci_pt2(ifci_plan_t plan, int64_t inc, const ifci_hbci_options* options, void* work,
                          int64_t work_bytes, const uint64_t* dets, int64_t n, const double* c, double e_var,
                          double eps2, double* e_pt2, int64_t* n_ext, ifci_stream_t stream);

const char* ifci_status_string(ifci_status s);
const char* ifci_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IFCI_H */
