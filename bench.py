"""Benchmark of the iFCI increment solver on one MI355X.

Workload: 16 bodies of 2 orbitals / 2 electrons (32 orbitals), 4-body
truncation: 16 + 120 + 560 + 1820 increments of 2o2e, 4o4e, 6o6e and 8o8e
(2516 increments, 9,146,384 determinants), seeded synthetic integrals.

One step = embed every increment (frozen-core integrals, H diagonal),
solve every increment (batched persistent solver, one workgroup per
increment, three-vector {x, w, p} iteration, FP32 MFMA sigma with FP64
subspace and FP64 residual refinement) and assemble the expansion
energies (eqs. 2-5).  The metric counts increments whose energy is within
1 uEh of the FP64 solution, per second of step time.  The FP64 batched path
and the plain per-increment FP64 path are timed beside it, and the CPU
oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}
KERNEL_SOURCES = ["batched.hip", "device_common.hpp", "ifci_internal.h", "launch.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_lobpcg_kernel_workload2.traffic.json")


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
TOL_UEH = 1e-6
SPACE = 3  # batched solver subspace: 3 = {x, w, p} iteration (12 = thick-restart Davidson)


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


def timed_solve(plan, h, eri, torch, stream):
    """One step on `plan`; returns (E, status, iters, total, kernel_ms)."""
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    from paper_2307_10675_amd import ifci
    ifci._check(ifci.lib().ifci_set_integrals(plan._h, ifci._ptr(h), ifci._ptr(eri), ifci._stream(stream)))
    t0.record(stream)
    e, st, it, rs = plan.davidson(stream=stream)
    t1.record(stream)
    en = plan.energy(e, st, stream=stream)
    return e, st, it, en, (t0, t1)


def run_steps(plan, h, eri, steps, warmup, torch):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        timed_solve(plan, h, eri, torch, stream)
    torch.cuda.synchronize()
    kern = []
    t = time.perf_counter()
    out = None
    for _ in range(steps):
        out = timed_solve(plan, h, eri, torch, stream)
        kern.append(out[4])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in kern]))
    return out, wall, kms


def cpu_baseline(problem, budget_s: float = 20.0):
    """The oracle (dense Slater-Condon FCI + LAPACK) on a bounded sample of
    the same workload: increments of each size, extrapolated to all 2516."""
    from oracle import fci, ifci as oifci
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    incs = oifci.increments(problem.n_bodies, problem.order)
    by = {k: [S for S in incs if len(S) == k] for k in range(1, problem.order + 1)}
    per = {}
    used = 0.0
    sample = []
    for k in range(1, problem.order + 1):
        times = []
        for S in by[k][:: max(1, len(by[k]) // 8)]:
            t = time.perf_counter()
            fci.solve_increment(problem, S)
            times.append(time.perf_counter() - t)
            used += times[-1]
            if used > budget_s or len(times) >= 8:
                break
        per[k] = float(np.mean(times))
        sample.append(f"{len(times)}x{2 * k}o{2 * k}e")
    total = sum(per[k] * len(by[k]) for k in per)
    return dict(value=len(incs) / total, unit="increments/s", cores=int(cores), kind="oracle",
                sample=f"{', '.join(sample)} solved ({used:.1f} s); per-size mean time x count, "
                       f"extrapolated to all {len(incs)} increments (est. {total:.0f} s)")


def large_sigma(torch, ifci, synthetic, n_orb=14, reps=5):
    """Symmetric-sector sigma of one half-filled n_orb-orbital FCI space (the
    single-FCI shape, seed 4000 + n_orb): the fused column kernel, FP32 and
    FP64, timed with HIP events on the current stream."""
    p = synthetic.single(n_orb, 2 * n_orb, 4000 + n_orb)
    plan = ifci.Plan(p, solver=ifci.PLAIN).attach(p.h, p.eri)
    n_str = int(round(plan.increment(0).n_det ** 0.5))
    rng = np.random.default_rng(5)
    c = torch.tensor(rng.standard_normal(n_str * (n_str + 1) // 2), device="cuda")
    flops = f_sym(n_orb, n_orb // 2)
    out = {"shape": f"{n_orb}o{n_orb}e, {n_str ** 2:,} determinants, sector {n_str * (n_str + 1) // 2:,}",
           "flops_per_sigma": flops}
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
        out[name] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "frac_mfma_peak": flops / (ms * 1e-3) / peak}
    del plan
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 14o14e and 16o16e sigma measurements")
    ap.add_argument("--only-large", action="store_true",
                    help="measure only the 14o14e sigma (fused column kernel) and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known "
                         "traffic, to scale HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the increments are independent and would be "
              "sharded across GPUs by increment (see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2307_10675_amd import ifci, synthetic

    dev = torch.device("cuda", 0)
    if a.copy_calibration > 0:
        src = torch.ones(a.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.only_large:
        print(json.dumps({"large_sigma": large_sigma(torch, ifci, synthetic),
                          "large_sigma_16o": large_sigma(torch, ifci, synthetic, n_orb=16, reps=3)}), flush=True)
        return
    problem = synthetic.workload(2)
    h = torch.tensor(problem.h, dtype=torch.float64, device=dev)
    eri = torch.tensor(problem.eri, dtype=torch.float64, device=dev).contiguous()

    # FP64 reference energies (batched FP64, residual 1e-7)
    ref_plan = ifci.Plan(problem, precision=ifci.FP64, r_tol=1e-7, max_iter=400).attach(h, eri)
    e_ref, st_ref, _, _ = ref_plan.davidson()
    e_ref = e_ref.cpu().numpy()
    assert (st_ref.cpu().numpy() == ifci.INC_DONE).all()
    incs = ref_plan.increments()
    flops = np.array([f_sym(i.n_act, i.n_alpha) for i in incs])
    flops_exec = np.array([f_exec(i.n_act, i.n_alpha) for i in incs])

    def measure(precision, solver, steps, warmup, **kw):
        plan = ifci.Plan(problem, precision=precision, solver=solver, max_iter=500, **kw).attach(h, eri)
        (e, st, it, en, _), wall, kms = run_steps(plan, h, eri, steps, warmup, torch)
        e = e.cpu().numpy()
        it = it.cpu().numpy()
        ok = (np.abs(e - e_ref) <= TOL_UEH) & (st.cpu().numpy() == ifci.INC_DONE)
        return dict(wall_ms=wall * 1e3, kernel_ms=kms, n_ok=int(ok.sum()), inc_per_s=float(ok.sum()) / wall,
                    max_err=float(np.abs(e - e_ref).max()), sigmas=int(it.sum()),
                    sigma_flops=float((it * flops).sum()), sigma_flops_executed=float((it * flops_exec).sum()),
                    mean_iters=float(it.mean()), total=en["total"])

    # headline: batched mixed precision at 1 uEh
    mixed = measure(ifci.MIXED, ifci.BATCHED, a.steps, a.warmup, r_tol=3e-5, r_tol_inner=1e-5,
                    max_space=SPACE)
    fp64 = measure(ifci.FP64, ifci.BATCHED, max(1, a.steps // 2), 1, r_tol=3e-5, max_space=SPACE)
    plain = None if a.no_plain else measure(ifci.FP64, ifci.PLAIN, 1, 0, r_tol=3e-5)

    kern_s = mixed["kernel_ms"] * 1e-3
    traffic = measured_traffic()
    achieved = mixed["sigma_flops"] / kern_s
    out = {
        "metric": "iFCI increments/sec at 1 uEh (batched mixed-precision solver)",
        "value": mixed["inc_per_s"],
        "unit": "increments/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sigma + f64 subspace/refinement",
        "data": "synthetic",
        "config": {
            "workload": "16 bodies x (2 orbitals, 2 electrons), 4-body iFCI: 16x2o2e + 120x4o4e + "
                        "560x6o6e + 1820x8o8e = 2516 increments, 9,146,384 determinants, seed 2000",
            "precision": "mixed", "solver": "batched", "max_space": SPACE, "r_tol": 3e-5, "r_tol_inner": 1e-5,
            "accuracy_gate_Eh": TOL_UEH,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "batched_lobpcg_kernel (one workgroup per increment, sigma on FP32/FP64 MFMA)",
            "achieved": achieved / 1e12,
            "peak": PEAK["fp32_mfma"] / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK["fp32_mfma"],
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "detail": {
            "mixed_batched": mixed,
            "fp64_batched": fp64,
            "fp64_plain": plain,
            "speedup_mixed_vs_fp64_batched": mixed["inc_per_s"] / fp64["inc_per_s"],
            "speedup_mixed_vs_fp64_plain": (mixed["inc_per_s"] / plain["inc_per_s"]) if plain else None,
            "fp64_batched_sigma_tflops": fp64["sigma_flops"] / (fp64["kernel_ms"] * 1e-3) / 1e12,
            "fp64_batched_frac_fp64_mfma": fp64["sigma_flops"] / (fp64["kernel_ms"] * 1e-3) / PEAK["fp64_mfma"],
            "flops_per_launch": mixed["sigma_flops"],
            # arithmetic the kernel actually performs (the diagonal pairs as a
            # dot product per determinant), and its fraction of the FP32 peak
            "executed_flops_per_launch": mixed["sigma_flops_executed"],
            "executed_frac_fp32_mfma": mixed["sigma_flops_executed"] / kern_s / PEAK["fp32_mfma"],
            "kernel_ms_per_launch": mixed["kernel_ms"],
        },
    }
    if not a.no_large:
        out["detail"]["large_sigma"] = large_sigma(torch, ifci, synthetic)
        out["detail"]["large_sigma_16o"] = large_sigma(torch, ifci, synthetic, n_orb=16, reps=3)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
