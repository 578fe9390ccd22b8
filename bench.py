"""Benchmark of the iFCI increment solver on one MI355X.

Workload: 16 bodies of 2 orbitals / 2 electrons (32 orbitals), 4-body
truncation: 16 + 120 + 560 + 1820 increments of 2o2e, 4o4e, 6o6e and 8o8e
(2516 increments, 9,146,384 determinants), seeded synthetic integrals.

One step = embed every increment (frozen-core integrals, H diagonal),
solve every increment (batched persistent solver, one workgroup per
increment, three-vector {x, w, p} iteration, FP32 MFMA sigma with FP64
subspace and FP64 residual refinement) and assemble the expansion
energies (eqs. 2-5).  The metric counts increments whose energy is within
1 uEh of the oracle's exact energy (stored, sha-checked), per second of step
time.  The FP64 batched path and the plain per-increment FP64 path are timed
beside it at the same FP64 residual tolerance, and the CPU oracle on a
bounded, seeded sample of the same workload.

Legs (--legs, comma separated; default all):
  mixed  the headline (batched, mixed precision)
  fp64   batched FP64
  plain  per-increment device-wide FP64
  large  14o14e / 16o16e: symmetric-sector sigma and whole solves
  w3     12 bodies, order 5 (1585 increments incl. 792 x 10o10e) and its gradient
  w4     256 independent 10o10e problems (K = 20, seeds 4000..4255)
  cnb    connected n-body screening at 10^-4.6 Eh on a decaying 10-body chain
  sno    summation natural orbitals: 6 occupied + 12 virtuals, order 3
  hbci   heat-bath selected CI + EN-PT2 on a 16o16e increment against its FCI,
         and whole HBCI expansions of workloads 1 and 2
  cpu    the oracle on the host cores

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs mixed,fp64,...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}
KERNEL_SOURCES = ["batched.hip", "pspace.hpp", "device_common.hpp", "ifci_internal.h", "launch.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_lobpcg_kernel_workload2.traffic.json")
ORACLE_W2 = os.path.join(ROOT, "tests", "golden", "oracle_w2.json")
ALL_LEGS = ("mixed", "fp64", "plain", "large", "w3", "w4", "cnb", "sno", "hbci", "cpu")

TOL_UEH = 1e-6
# One FP64 acceptance test for every leg: converged when the FP64 residual
# of the unit vector is at most R_TOL.  The mixed leg switches from FP32 to
# FP64 sigma at the FP32 residual R_TOL_INNER and keeps iterating in FP64
# until the FP64 residual passes R_TOL.
R_TOL = 1e-5
R_TOL_INNER = 1e-5
SPACE = 3  # batched solver subspace: 3 = {x, w, p} iteration (12 = thick-restart Davidson)
CPU_8O8E_SAMPLE = 64
CPU_SAMPLE_SEED = 2024


def kernel_source_hash() -> str:
    import hashlib
    m = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2307_10675_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the batched kernel (mixed leg) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by the
    same counter's reading for a device copy of known size; None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


def f_sym(k: int, na: int) -> float:
    """Algorithmic flops of one sigma: 2 npair^2 N_det."""
    np_ = k * (k + 1) // 2
    return 2.0 * np_ * np_ * math.comb(k, na) ** 2


def f_exec(k: int, na: int) -> float:
    """Flops the batched kernel performs for one sigma: the pair contraction
    over the off-diagonal pairs plus one dot product per determinant for the
    diagonal pairs, 2 (n_off + 1) npair N_det."""
    np_ = k * (k + 1) // 2
    return 2.0 * (k * (k - 1) // 2 + 1) * np_ * math.comb(k, na) ** 2


# ------------------------------------------------------------------ CPU oracle
def _cpu_task(args):
    """One oracle increment solve, timed in its two parts: the Slater-Condon
    build of H and the symmetric-sector eigensolve (LAPACK)."""
    problem, S, threads = args
    from threadpoolctl import threadpool_limits

    from oracle import fci, hamiltonian
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        dets, n_str, active = fci.increment_dets(problem.n_orb, problem.bodies, problem.nocc, S)
        H = hamiltonian.build(dets, problem.h, problem.eri, active, problem.e_const)
        t1 = time.perf_counter()
        e, _, _ = fci.lowest_symmetric(H, n_str)
        t2 = time.perf_counter()
    return tuple(S), e, t1 - t0, t2 - t1


def host_description() -> dict:
    out = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                "CPU max MHz", "L3 cache", "NUMA node(s)")
        out["lscpu"] = {ln.split(":", 1)[0].strip(): ln.split(":", 1)[1].strip()
                        for ln in txt.splitlines() if ":" in ln and ln.split(":", 1)[0].strip() in keep}
    except (OSError, subprocess.SubprocessError):
        out["lscpu"] = None
    return out


def cpu_baseline(problem, workers: int, n8: int) -> dict:
    """The oracle (dense Slater-Condon FCI + LAPACK, never tuned) on the host
    cores, in two runs:

    * all cores: a process pool of `workers` single-threaded processes over
      every 2o2e, 4o4e and 6o6e increment plus a seeded sample of n8 of the
      1820 8o8e increments;
    * one thread: one process over a seeded sample of 4 increments of each
      size below 8o8e and 2 of 8o8e.

    Each is extrapolated to all 2516 increments from the mean time per size
    (and, for the pool, its measured parallel efficiency)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from oracle import ifci as oifci
    incs = oifci.increments(problem.n_bodies, problem.order)
    by = {k: [S for S in incs if len(S) == k] for k in range(1, problem.order + 1)}
    rng = np.random.default_rng(CPU_SAMPLE_SEED)
    top = problem.order
    pick8 = [by[top][i] for i in sorted(rng.choice(len(by[top]), size=min(n8, len(by[top])), replace=False))]
    pool_set = [S for k in range(1, top) for S in by[k]] + pick8
    one_set = [by[k][i] for k in range(1, top) for i in sorted(rng.choice(len(by[k]), size=4, replace=False))] + \
              [pick8[0], pick8[1]]

    def summarise(rows, wall):
        per = {}
        for S, _, tb, te in rows:
            per.setdefault(len(S), []).append((tb, te))
        sizes = {}
        t_cpu_all = 0.0
        for k in range(1, top + 1):
            tb = float(np.mean([x[0] for x in per[k]]))
            te = float(np.mean([x[1] for x in per[k]]))
            sizes[f"{2 * k}o{2 * k}e"] = {"solved": len(per[k]), "of": len(by[k]), "h_build_s": tb, "eigh_s": te}
            t_cpu_all += (tb + te) * len(by[k])
        t_cpu_sample = sum(tb + te for _, _, tb, te in rows)
        eff = t_cpu_sample / wall
        return sizes, t_cpu_all, t_cpu_sample, eff

    ctx = mp.get_context("spawn")
    t = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        # largest first so the pool drains evenly
        order = sorted(pool_set, key=lambda S: -len(S))
        rows = list(ex.map(_cpu_task, [(problem, S, 1) for S in order], chunksize=1))
    wall = time.perf_counter() - t
    sizes, t_all, t_sample, eff = summarise(rows, wall)
    est_pool = t_all / eff
    t = time.perf_counter()
    rows1 = [_cpu_task((problem, S, 1)) for S in one_set]
    wall1 = time.perf_counter() - t
    sizes1, t_all1, _, _ = summarise(rows1, wall1)
    energies = {S: e for S, e, _, _ in rows}
    return dict(
        value=len(incs) / est_pool, unit="increments/s", cores=workers, kind="oracle",
        sample=(f"extrapolated: all " + ", ".join(f"{len(by[k])} {2 * k}o{2 * k}e" for k in range(1, top)) +
                f" increments plus a seeded sample of {len(pick8)} of the {len(by[top])} {2 * top}o{2 * top}e "
                f"increments, solved by {workers} single-threaded processes in "
                f"{wall:.1f} s (parallel efficiency {eff:.1f} of {workers}); mean time per size x count / "
                f"efficiency = {est_pool:.0f} s for all {len(incs)}"),
        by_size=sizes,
        one_thread={"value": len(incs) / t_all1, "unit": "increments/s", "cores": 1,
                    "sample": f"extrapolated from {len(one_set)} seeded increments ({wall1:.1f} s)",
                    "by_size": sizes1, "est_total_s": t_all1},
        host=host_description(),
        _energies=energies,
    )


# ------------------------------------------------------------------ GPU legs
def oracle_reference(problem):
    """(energies, gaps) of every workload-2 increment from the stored oracle
    run, or None when the file is absent or was made from other integrals."""
    try:
        with open(ORACLE_W2) as fh:
            g = json.load(fh)
    except OSError:
        return None
    if g.get("sha256") != problem.sha256():
        return None
    return (np.array([x["E"] for x in g["increments"]]), np.array([x["gap"] for x in g["increments"]]),
            [tuple(x["bodies"]) for x in g["increments"]])


def run_steps(plan, h, eri, steps, warmup, torch):
    """Time `steps` whole steps (embed + solve + energy assembly) on the
    current stream; returns the last outputs, wall seconds per step, and the
    mean solver-launch time (HIP events around ifci_davidson)."""
    from paper_2307_10675_amd import ifci
    stream = torch.cuda.current_stream()

    def one():
        ifci._check(ifci.lib().ifci_set_integrals(plan._h, ifci._ptr(h), ifci._ptr(eri), ifci._stream(stream)))
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        e, st, it, rs = plan.davidson(stream=stream)
        t1.record(stream)
        en = plan.energy(e, st, stream=stream)
        return (e, st, it, rs, en), (t0, t1)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    kern, out = [], None
    t = time.perf_counter()
    for _ in range(steps):
        out, ev = one()
        kern.append(ev)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    kms = [a.elapsed_time(b) for a, b in kern]
    return out, wall, float(np.mean(kms)), float(np.median(kms))


def large_sigma(torch, ifci, synthetic, n_orb=14, reps=5):
    """Symmetric-sector sigma of one half-filled n_orb-orbital FCI space (the
    single-FCI shape, K = 2 n_orb, seed 4000 + n_orb): the fused column
    kernel, FP32 and FP64, timed with HIP events on the current stream."""
    p = synthetic.single(n_orb, 2 * n_orb, 4000 + n_orb)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(plan.increment(0).n_det ** 0.5))
    rng = np.random.default_rng(5)
    c = torch.tensor(rng.standard_normal(n_str * (n_str + 1) // 2), device="cuda")
    flops = f_sym(n_orb, n_orb // 2)
    out = {"shape": f"{n_orb}o{n_orb}e, {n_str ** 2:,} determinants, sector {n_str * (n_str + 1) // 2:,}",
           "flops_per_sigma": flops, "algorithmic_bytes_fp32": 2 * 4 * n_str ** 2,
           "algorithmic_bytes_fp64": 2 * 8 * n_str ** 2}
    for name, prec, peak in (("fp32", ifci.MIXED, PEAK["fp32_mfma"]), ("fp64", ifci.FP64, PEAK["fp64_mfma"])):
        plan.sigma_sector(0, c, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.sigma_sector(0, c, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # HBM rate on algorithmic bytes (C read once, sigma written once); the
        # counted traffic of the same kernels is in the column-sigma profile
        gbps = out[f"algorithmic_bytes_{name}"] / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "frac_mfma_peak": flops / (ms * 1e-3) / peak,
                     "algorithmic_GBps": gbps, "frac_hbm_peak_algorithmic": gbps * 1e9 / PEAK["hbm"]}
    plan.close()
    del plan
    torch.cuda.empty_cache()
    return out


def large_solve(torch, ifci, synthetic, n_orb, precision):
    """Whole lowest-root solve of the half-filled n_orb-orbital FCI (K = 2 n_orb,
    seed 4000 + n_orb): wall time, iterations, residual, sigma flop rate."""
    p = synthetic.single(n_orb, 2 * n_orb, 4000 + n_orb)
    plan = ifci.Plan(p, precision=precision, r_tol=R_TOL, r_tol_inner=R_TOL_INNER, max_iter=300).attach(p.h, p.eri)
    torch.cuda.synchronize()
    t = time.perf_counter()
    e, st, it, rs = plan.davidson()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    iters = int(it[0])
    flops = iters * f_sym(n_orb, n_orb // 2)
    peak = PEAK["fp32_mfma"] if precision == ifci.MIXED else PEAK["fp64_mfma"]
    out = {"shape": f"{n_orb}o{n_orb}e", "precision": "mixed" if precision == ifci.MIXED else "fp64",
           "seconds": wall, "iterations": iters, "residual": float(rs[0]), "E": float(e[0]),
           "converged": int(st[0]) == ifci.INC_DONE, "sigma_tflops_over_solve": flops / wall / 1e12,
           "frac_mfma_peak_over_solve": flops / wall / peak}
    plan.close()
    del plan
    torch.cuda.empty_cache()
    return out


def workload3_leg(torch, ifci, synthetic):
    """12 bodies, order 5: 12 + 66 + 220 + 495 + 792 increments (up to
    10o10e), mixed and FP64 at the same FP64 residual, and the expansion
    gradient (weighted 1- and 2-particle densities) of the FP64 solve."""
    p = synthetic.workload(3)
    dev = torch.device("cuda", 0)
    h = torch.tensor(p.h, dtype=torch.float64, device=dev)
    eri = torch.tensor(p.eri, dtype=torch.float64, device=dev).contiguous()
    out = {"workload": "12 bodies x (2o, 2e), order 5: 1585 increments (12x2o2e, 66x4o4e, 220x6o6e, "
                       "495x8o8e, 792x10o10e), seed 3000"}
    res = {}
    for name, prec in (("mixed", ifci.MIXED), ("fp64", ifci.FP64)):
        plan = ifci.Plan(p, precision=prec, r_tol=R_TOL, r_tol_inner=R_TOL_INNER, max_iter=500,
                         max_space=SPACE).attach(h, eri)
        (e, st, it, rs, en), wall, kms, _ = run_steps(plan, h, eri, 1, 1, torch)
        e = e.cpu().numpy()
        res[name] = e
        out[name] = {"seconds": wall, "solve_ms": kms, "increments_per_s": len(e) / wall,
                     "all_converged": bool((st.cpu().numpy() == ifci.INC_DONE).all()),
                     "mean_iters_10o10e": float(it.cpu().numpy()[-792:].mean()), "total": en["total"]}
        if prec == ifci.FP64:
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.rdm()
            torch.cuda.synchronize()
            out["gradient_seconds"] = time.perf_counter() - t
        plan.close()
        del plan
    out["max_abs_mixed_minus_fp64"] = float(np.abs(res["mixed"] - res["fp64"]).max())
    torch.cuda.empty_cache()
    return out


def workload4_batch_leg(torch, ifci, synthetic, count=256):
    """256 independent 10o10e FCI problems (K = 20, seeds 4000..4255), one
    plan each, solved together in mixed precision by one batched call
    (ifci_davidson_group) and timed as one job."""
    problems = [synthetic.single(10, 20, 4000 + i) for i in range(count)]
    plans = [ifci.Plan(q, precision=ifci.MIXED, r_tol=R_TOL, r_tol_inner=R_TOL_INNER, max_iter=300).attach(q.h, q.eri)
             for q in problems]
    ifci.davidson_group(plans)  # warm-up (kernel loads, control block)
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = ifci.davidson_group(plans)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    it = np.array([int(o[2][0]) for o in outs])
    ok = all(int(o[1][0]) == ifci.INC_DONE for o in outs)
    flops = float(it.sum()) * f_sym(10, 5)
    for pl in plans:
        pl.close()
    torch.cuda.empty_cache()
    return {"problems": f"{count} x 10o10e (K = 20, seeds 4000..{4000 + count - 1}), 16,257,024 determinants",
            "seconds": wall, "increments_per_s": count / wall, "mean_iters": float(it.mean()), "all_converged": ok,
            "sigma_tflops_over_solve": flops / wall / 1e12}


def screening_leg(torch, ifci, synthetic):
    """Connected n-body screening at the paper's parameter (10^-4.6 Eh) on a
    10-body chain whose pair increments fall off with distance (order 4, 385
    increments), mixed precision: kept increments per order and the time
    against the unscreened expansion of the same problem."""
    p = synthetic.local_chain(10, seed=5100, order=4, rate=1.0)
    C = 10 ** -4.6
    out = {"problem": "10 bodies x (2o, 2e), pair correlation decaying with distance, order 4: 385 increments",
           "threshold_Eh": C}
    kw = dict(precision=ifci.MIXED, r_tol=R_TOL, r_tol_inner=R_TOL_INNER, max_iter=600)
    for name in ("full", "screened"):
        for rep in range(2):  # the second run is timed
            torch.cuda.synchronize()
            t = time.perf_counter()
            if name == "full":
                plan, res = ifci.solve(p, **kw)
            else:
                plan, res = ifci.solve_screened(p, C, **kw)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            plan.close()
        sizes = [len(i) for i in synthetic_increments(p.n_bodies, p.order)]
        entry = {"seconds": wall, "total": res["total"]}
        if name == "screened":
            keep = res["keep"]
            entry["kept_by_order"] = [int(sum(1 for s, k in zip(sizes, keep) if k and s == n)) for n in range(1, 5)]
            entry["increments_by_order"] = [sizes.count(n) for n in range(1, 5)]
        out[name] = entry
    out["total_change_Eh"] = out["screened"]["total"] - out["full"]["total"]
    return out


def synthetic_increments(n_bodies, order):
    import itertools
    return [S for k in range(1, order + 1) for S in itertools.combinations(range(n_bodies), k)]


def sno_leg(torch, ifci, synthetic):
    """SNO expansion: 6 occupied orbitals sharing 12 virtuals, order 3 (41
    increments), natural orbitals kept above 10^-4, mixed precision; seconds
    per step and the kept natural-orbital counts."""
    from paper_2307_10675_amd.sno import solve_sno
    p = synthetic.sno_system(6, 12, seed=8300, order=3)
    for rep in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = solve_sno(p, 4.0, precision=ifci.MIXED, r_tol=R_TOL, r_tol_inner=R_TOL_INNER, max_iter=600)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
    nk = [int(x) for x in res["n_keep"]]
    return {"problem": "6 occupied + 12 virtual orbitals, order 3: 41 increments, eta 4", "seconds": wall,
            "seconds_by_step": res["seconds_by_step"], "all_converged": bool(res["converged"]),
            "kept_virtuals_min_mean_max": [min(nk), sum(nk) / len(nk), max(nk)], "total": res["total"]}


def hbci_leg(torch, ifci, synthetic, increment_only=False):
    """HBCI (eps2 = 1 uEh) of one 16o16e increment (an 8-body decaying chain
    taken as one body, 165,636,900 determinants) at eps1 = 1 mEh (the
    paper's) and 3e-4, against the increment's exact energy from the FCI
    path (mixed precision to residual 1e-5): seconds, |V|, nonzeros of H over
    V, external determinants, errors of E_var and E_var + E_PT2."""
    p = synthetic.merged(synthetic.chain(8, seed=4108, order=1))
    fci_s = e_fci = None
    if not increment_only:
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan, res = ifci.solve(p, precision=ifci.MIXED, r_tol=1e-5, r_tol_inner=1e-5, max_iter=400)
        torch.cuda.synchronize()
        fci_s = time.perf_counter() - t
        e_fci = float(res["E"][0])
        plan.close()
        del plan, res
        torch.cuda.empty_cache()
    pl = ifci.Plan(p, tuning=None).attach(p.h, p.eri)
    runs = []
    for eps1 in (1e-3, 3e-4):
        opts = ifci.hbci_options(eps1=eps1, eps2=1e-6, max_det=1 << 21, max_nnz=1 << 29, max_ext=1 << 26,
                                 r_tol=1e-6)
        work = pl.hbci_work(0, opts)
        pl.hbci(0, opts, work=work)                 # warm-up (kernel attributes, staging)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = pl.hbci(0, opts, work=work)
        secs = time.perf_counter() - t
        runs.append(dict(eps1=eps1, seconds=round(secs, 4), n_det=r["n_det"], steps=r["n_iter"], nnz=r["nnz"],
                         n_ext=r["n_ext"], converged=r["converged"], E_var=r["E_var"], E_pt2=r["E_pt2"]))
        if e_fci is not None:
            runs[-1].update(err_var_Eh=r["E_var"] - e_fci, err_total_Eh=r["E"] - e_fci)
        del work
        torch.cuda.empty_cache()
    pl.close()
    if increment_only:
        return dict(increment="16o16e (merged 8-body chain, seed 4108)", runs=runs)
    # whole expansions with HBCI as the increment solver (eps1 = 1 mEh,
    # eps2 = 1 uEh), increments overlapped by host workers, against the
    # exact expansion's total from the stored oracle energies
    expansions = []
    for wl in (1, 2):
        prob = synthetic.workload(wl)
        path = os.path.join(ROOT, "tests", "golden", f"oracle_w{wl}.json")
        exact = e_inc = None
        if os.path.exists(path):
            with open(path) as f:
                gdoc = json.load(f)
            if gdoc.get("sha256") == prob.sha256():
                exact = gdoc["total"]
                e_inc = np.array([x["E"] for x in gdoc["increments"]])
        plx = ifci.Plan(prob, tuning=None).attach(prob.h, prob.eri)
        opts = ifci.hbci_options(eps1=1e-3, eps2=1e-6, max_det=1 << 13, max_nnz=1 << 22, max_ext=1 << 18,
                                 r_tol=1e-6)
        row = dict(workload=wl, increments=plx.n_inc)
        for workers in ((1, 16) if wl == 1 else (16,)):
            out = plx.hbci_expansion(opts, workers=workers)
            row[f"seconds_{workers}_workers"] = round(out["seconds"], 4)
        row["increments_per_s_16_workers"] = plx.n_inc / row["seconds_16_workers"]
        row["all_converged"] = all(r["converged"] for r in out["results"])
        row["total"] = out["energy"]["total"]
        if exact is not None:
            row["total_minus_exact_Eh"] = out["energy"]["total"] - exact
            # increments whose HBCI energy is more than 1 mEh from the exact
            # one (a selected space grown from the reference cannot reach a
            # ground state that has almost no weight on it)
            d = np.array([r["E"] for r in out["results"]]) - e_inc
            row["increments_off_by_1mEh"] = int((np.abs(d) > 1e-3).sum())
            row["max_increment_error_Eh"] = float(np.abs(d).max())
        plx.close()
        expansions.append(row)
    return dict(increment="16o16e (merged 8-body chain, seed 4108)", fci_seconds_mixed=round(fci_s, 3),
                E_fci=e_fci, runs=runs, expansions=expansions)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default=",".join(ALL_LEGS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 14o14e and 16o16e measurements")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle pool size (default: min(16, cores))")
    ap.add_argument("--cpu-8o8e", type=int, default=CPU_8O8E_SAMPLE)
    ap.add_argument("--hbci-increment-only", action="store_true",
                    help="hbci leg: only the 16o16e increment's HBCI runs (profile runs)")
    ap.add_argument("--no-untuned", action="store_true",
                    help="skip the leg with the built-in settings beside the tuned ones (profile runs)")
    ap.add_argument("--max-space", type=int, default=SPACE,
                    help="batched solver subspace (3: three-vector iteration, 4..16: thick-restart Davidson)")
    ap.add_argument("--n-guess", type=int, default=None,
                    help="P-space block of the three-vector solver (default: the library's)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known "
                         "traffic, to scale HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the increments are independent and would be "
              "sharded across GPUs by increment (see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in a.legs.split(",") if x)
    bad = legs - set(ALL_LEGS)
    if bad:
        ap.error(f"unknown legs {sorted(bad)}")
    if a.no_cpu:
        legs.discard("cpu")
    if a.no_plain:
        legs.discard("plain")
    if a.no_large:
        legs.discard("large")

    from paper_2307_10675_amd import synthetic
    problem = synthetic.workload(2)

    # the oracle runs first, in child processes, before anything touches the GPU
    cpu = None
    if "cpu" in legs:
        workers = a.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        cpu = cpu_baseline(problem, workers, a.cpu_8o8e)

    import torch

    from paper_2307_10675_amd import ifci

    dev = torch.device("cuda", 0)
    if a.copy_calibration > 0:
        src = torch.ones(a.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = torch.tensor(problem.h, dtype=torch.float64, device=dev)
    eri = torch.tensor(problem.eri, dtype=torch.float64, device=dev).contiguous()

    ref = oracle_reference(problem)
    probe = ifci.Plan(problem)
    incs = probe.increments()
    probe.close()
    if ref is not None:
        e_ref, gap_ref, bodies = ref
        assert bodies == [i.bodies for i in incs], "increment order differs from the oracle file"
        gate = "oracle (tests/golden/oracle_w2.json, sha256-checked)"
    else:
        # the stored oracle energies are missing: gate on an FP64 solve to 1e-8
        rp = ifci.Plan(problem, precision=ifci.FP64, r_tol=1e-8, max_iter=600).attach(h, eri)
        e_ref = rp.davidson()[0].cpu().numpy()
        gap_ref = None
        rp.close()
        gate = "GPU FP64 batched solve to residual 1e-8 (oracle file missing)"
    flops = np.array([f_sym(i.n_act, i.n_alpha) for i in incs])
    flops_exec = np.array([f_exec(i.n_act, i.n_alpha) for i in incs])

    def measure(precision, solver, steps, warmup, **kw):
        plan = ifci.Plan(problem, precision=precision, solver=solver, max_iter=600, r_tol=R_TOL,
                         r_tol_inner=R_TOL_INNER, **kw).attach(h, eri)
        (e, st, it, rs, en), wall, kms, kmed = run_steps(plan, h, eri, steps, warmup, torch)
        e = e.cpu().numpy()
        it = it.cpu().numpy()
        rs = rs.cpu().numpy()
        err = np.abs(e - e_ref)
        ok = (err <= TOL_UEH) & (st.cpu().numpy() == ifci.INC_DONE)
        r = dict(wall_ms=wall * 1e3, kernel_ms=kms, kernel_ms_median=kmed, n_ok=int(ok.sum()),
                 inc_per_s=float(ok.sum()) / wall, max_err=float(err.max()), sigmas=int(it.sum()),
                 sigma_flops=float((it * flops).sum()), sigma_flops_executed=float((it * flops_exec).sum()),
                 mean_iters=float(it.mean()), max_iters=int(it.max()), total=en["total"],
                 max_residual=float(rs.max()))
        if gap_ref is not None:
            # every result with its error bound: |E - lambda| <= ||r||^2 / gap
            # (Kato-Temple, gap to the next root of the sector from the oracle)
            kt = rs ** 2 / gap_ref
            r.update(max_error_bound=float(kt.max()), n_bound_within_gate=int((kt <= TOL_UEH).sum()))
        plan.close()
        return r

    out_detail = {}
    n_guess = a.n_guess if a.n_guess is not None else ifci.default_options().n_guess
    mixed = measure(ifci.MIXED, ifci.BATCHED, a.steps, a.warmup, max_space=a.max_space,
                    n_guess=n_guess) if "mixed" in legs else None
    fp64 = measure(ifci.FP64, ifci.BATCHED, max(1, a.steps // 2), 1, max_space=a.max_space,
                   n_guess=n_guess) if "fp64" in legs else None
    plain = measure(ifci.FP64, ifci.PLAIN, 1, 0) if "plain" in legs else None
    # the tuner's per-shape settings (tuning.json, applied by Plan) against
    # the built-in choices
    tuning = ifci.load_tuning()
    if tuning and "mixed" in legs and not a.no_untuned:
        untuned = measure(ifci.MIXED, ifci.BATCHED, max(1, a.steps // 2), 1, max_space=a.max_space,
                          n_guess=n_guess, tuning=None)
        out_detail["tuning"] = {
            "cache": "paper_2307_10675_amd/tuning.json",
            "entries": {f"k{k}_{'mixed' if p == ifci.MIXED else 'fp64'}": {"ps_block": v[0], "e_waves": v[1]}
                        for (k, p), v in sorted(tuning.items())},
            "tuned_kernel_ms": mixed["kernel_ms"], "default_kernel_ms": untuned["kernel_ms"],
            "tuned_inc_per_s": mixed["inc_per_s"], "default_inc_per_s": untuned["inc_per_s"],
            "default_n_ok": untuned["n_ok"],
        }
    if "large" in legs:
        out_detail["large_sigma"] = large_sigma(torch, ifci, synthetic)
        out_detail["large_sigma_16o"] = large_sigma(torch, ifci, synthetic, n_orb=16, reps=3)
        out_detail["large_solves"] = [large_solve(torch, ifci, synthetic, 14, ifci.MIXED),
                                      large_solve(torch, ifci, synthetic, 14, ifci.FP64),
                                      large_solve(torch, ifci, synthetic, 16, ifci.MIXED)]
    if "w3" in legs:
        out_detail["workload3_order5"] = workload3_leg(torch, ifci, synthetic)
    if "w4" in legs:
        out_detail["workload4_batch_10o10e"] = workload4_batch_leg(torch, ifci, synthetic)
    if "cnb" in legs:
        out_detail["cnb_screening"] = screening_leg(torch, ifci, synthetic)
    if "sno" in legs:
        out_detail["sno"] = sno_leg(torch, ifci, synthetic)
    if "hbci" in legs:
        out_detail["hbci_16o16e"] = hbci_leg(torch, ifci, synthetic, a.hbci_increment_only)

    head = mixed or fp64 or plain
    out = {
        "metric": "iFCI increments/sec at 1 uEh (batched mixed-precision solver)",
        "value": mixed["inc_per_s"] if mixed else None,
        "unit": "increments/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["wall_ms"] if mixed else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sigma + f64 subspace/refinement",
        "data": "synthetic",
        "config": {
            "workload": "16 bodies x (2 orbitals, 2 electrons), 4-body iFCI: 16x2o2e + 120x4o4e + "
                        "560x6o6e + 1820x8o8e = 2516 increments, 9,146,384 determinants, seed 2000",
            "precision": "mixed", "solver": "batched", "max_space": a.max_space, "n_guess": n_guess, "r_tol": R_TOL,
            "r_tol_inner": R_TOL_INNER, "accuracy_gate_Eh": TOL_UEH, "gate_reference": gate,
        },
    }
    if mixed:
        kern_s = mixed["kernel_ms"] * 1e-3
        achieved = mixed["sigma_flops"] / kern_s
        out["roofline"] = {
            "bound": "mfma",
            "kernel": "batched_lobpcg_kernel (one workgroup per increment, sigma on FP32/FP64 MFMA)",
            "achieved": achieved / 1e12,
            "peak": PEAK["fp32_mfma"] / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK["fp32_mfma"],
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        }
    detail = {"mixed_batched": mixed, "fp64_batched": fp64, "fp64_plain": plain}
    if mixed and fp64:
        detail["speedup_mixed_vs_fp64_batched"] = mixed["inc_per_s"] / max(fp64["inc_per_s"], 1e-30)
        detail["fp64_batched_sigma_tflops"] = fp64["sigma_flops"] / (fp64["kernel_ms"] * 1e-3) / 1e12
        detail["fp64_batched_frac_fp64_mfma"] = fp64["sigma_flops"] / (fp64["kernel_ms"] * 1e-3) / PEAK["fp64_mfma"]
    if mixed and plain:
        detail["speedup_mixed_vs_fp64_plain"] = mixed["inc_per_s"] / max(plain["inc_per_s"], 1e-30)
    if mixed:
        kern_s = mixed["kernel_ms"] * 1e-3
        detail["flops_per_launch"] = mixed["sigma_flops"]
        # arithmetic the kernel actually performs (the diagonal pairs as a
        # dot product per determinant), and its fraction of the FP32 peak
        detail["executed_flops_per_launch"] = mixed["sigma_flops_executed"]
        detail["executed_frac_fp32_mfma"] = mixed["sigma_flops_executed"] / kern_s / PEAK["fp32_mfma"]
        detail["kernel_ms_per_launch"] = mixed["kernel_ms"]
    detail.update(out_detail)
    out["detail"] = detail
    if cpu is not None:
        # the sampled oracle energies against the headline leg's reference
        en = cpu.pop("_energies")
        idx = {S: i for i, S in enumerate(i.bodies for i in incs)}
        cpu["max_abs_vs_gate_reference"] = float(max(abs(e - e_ref[idx[S]]) for S, e in en.items()))
        out["cpu_baseline"] = cpu
    if head is None and not out_detail and cpu is None:
        print("no legs selected", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
