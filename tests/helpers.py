"""Test helpers: the oracle's full-space Hamiltonian re-expressed in the
library's active-space determinant convention, golden-file loading, and
GPU availability."""
import json
import os

import numpy as np

from oracle import fci, hamiltonian, ifci

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def string_phase(mask: int, core) -> int:
    """(-1)^(sum over occupied p of #core orbitals above p): the sign between
    an ascending full-space string and (core operators first, then active)."""
    n = 0
    for p in range(mask.bit_length()):
        if mask >> p & 1 and p not in core:
            n += sum(1 for c in core if c > p)
    return -1 if n & 1 else 1


def active_hamiltonian(problem, S):
    """H of increment S in the library's convention: the oracle's full-space
    Slater-Condon matrix minus (e_const + closed-shell core energy), with the
    determinant signs of core-first operator ordering.  Returns (H, n_str)."""
    dets, n_str, active = fci.increment_dets(problem.n_orb, problem.bodies, problem.nocc, S)
    _, core, _ = fci.increment_orbitals(problem.bodies, problem.nocc, S)
    H = hamiltonian.build(dets, problem.h, problem.eri, active, problem.e_const)
    n = problem.n_orb
    mask = (1 << n) - 1
    s = np.array([string_phase(d & mask, set(core)) * string_phase(d >> n, set(core)) for d in dets], float)
    shift = ifci.closed_shell_energy(problem.h, problem.eri, core, problem.e_const)
    Ha = s[:, None] * (H - shift * np.eye(len(dets))) * s[None, :]
    return Ha, n_str, s


def load_golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        import pytest
        pytest.skip(f"{path} not written yet (tests/golden/make_oracle_refs.py --only {name})")
    with open(path) as f:
        return json.load(f)
