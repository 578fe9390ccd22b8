"""Python binding of libifci (ctypes).  Argument marshalling only: every step
of the computation runs in the HIP library; PyTorch supplies device memory
and the stream.  The names follow include/ifci.h."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libifci.so")

FP64, MIXED = 0, 1
BATCHED, PLAIN = 0, 1
INC_PENDING, INC_DONE, INC_NOT_CONVERGED, INC_EVICTED, INC_SCREENED = 0, 1, 2, 3, 4
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory", 4: "device error",
          5: "not converged", 6: "invalid state"}


class IfciError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libifci: {STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("n_bodies", ctypes.c_int32),
                ("body_ptr", ctypes.POINTER(ctypes.c_int32)), ("body_orb", ctypes.POINTER(ctypes.c_int32)),
                ("body_nocc", ctypes.POINTER(ctypes.c_int32)), ("order", ctypes.c_int32),
                ("e_const", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("solver", ctypes.c_int32), ("r_tol", ctypes.c_double),
                ("r_tol_inner", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_space", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("n_guess", ctypes.c_int32)]


class HbciOptions(ctypes.Structure):
    _fields_ = [("eps1", ctypes.c_double), ("eps2", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_dav", ctypes.c_int32), ("m_max", ctypes.c_int32), ("r_tol", ctypes.c_double),
                ("max_det", ctypes.c_int64), ("max_nnz", ctypes.c_int64), ("max_ext", ctypes.c_int64)]


_lib = None

_SIGNATURES = {
    "ifci_abi_version": (ctypes.c_int, []),
    "ifci_default_options": (None, [ctypes.POINTER(Options)]),
    "ifci_plan_create": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "ifci_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ifci_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ifci_increment": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "ifci_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "ifci_tables": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]),
    "ifci_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "ifci_set_integrals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_sigma": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_void_p]),
    "ifci_sigma_sector": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p]),
    "ifci_sigma_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_void_p]),
    "ifci_davidson": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "ifci_davidson_group": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_void_p]),
    "ifci_vector": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "ifci_rdm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p]),
    "ifci_set_phase_counters": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "ifci_screen": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "ifci_group_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "ifci_group_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_sno_orbitals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_sno_transform": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32]),
    "ifci_hbci_default_options": (None, [ctypes.POINTER(HbciOptions)]),
    "ifci_hbci_work_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(HbciOptions),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "ifci_hbci_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(HbciOptions),
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_hbci_solve_range": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(HbciOptions), ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "ifci_hbci_sigma": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(HbciOptions),
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ifci_hbci_select": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(HbciOptions),
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "ifci_hbci_pt2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(HbciOptions),
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_void_p]),
    "ifci_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ifci_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded libifci.  Raises if the library has not been built."""
    global _lib
    if _lib is None:
        # torch first: it carries its own HIP runtime, and the library must
        # bind to that one (loaded first, the library would bring up a second
        # runtime beside torch's, which then sees no device for torch's
        # memory: hipSetDevice fails with an invalid ordinal)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libifci.so not found at {LIB_PATH}; build it with "
                               "`python -m paper_2307_10675_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise IfciError(code, lib().ifci_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_options(**kw) -> Options:
    o = Options()
    lib().ifci_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def hbci_options(**kw) -> HbciOptions:
    """ifci_hbci_default_options with fields overridden by keyword."""
    o = HbciOptions()
    lib().ifci_hbci_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def load_tuning(path: str = TUNING_PATH):
    """{(k, precision): (ps_block, e_waves)} from the tuner's cache
    (paper_2307_10675_amd/tune.py), or {} when there is none."""
    import json
    try:
        with open(path) as fh:
            d = json.load(fh)
    except OSError:
        return {}
    out = {}
    for e in d.get("entries", []):
        out[(int(e["k"]), int(e["precision"]))] = (int(e["ps_block"]), int(e["e_waves"]))
    return out


def tables(k: int, n_alpha: int):
    """(strings, link[n_str][n_link][4]) of a (k, n_alpha) space, host only."""
    from math import comb
    n_str = comb(k, n_alpha)
    n_link = n_alpha * (k - n_alpha + 1)
    s = (ctypes.c_int32 * n_str)()
    lk = (ctypes.c_int32 * (n_str * n_link * 4))()
    _check(lib().ifci_tables(k, n_alpha, s, lk))
    return np.array(s, dtype=np.int64), np.array(lk, dtype=np.int64).reshape(n_str, n_link, 4)


@dataclass
class IncrementInfo:
    bodies: tuple
    n_act: int
    n_alpha: int
    n_det: int


class Plan:
    """ifci_plan_t with its workspace.  `problem` needs n_orb, bodies, nocc
    and order (and optionally e_const) -- e.g. synthetic.Problem; the
    integrals come with attach()."""

    def __init__(self, problem, precision=FP64, solver=BATCHED, device: int = 0, tuning="cache", **opts):
        """tuning: "cache" applies the committed tuner results (tuning.json,
        when present), None keeps the built-in choices, or a dict
        {(k, precision): (ps_block, e_waves)}."""
        self._keep = []
        bodies = [list(b) for b in problem.bodies]
        ptr = np.cumsum([0] + [len(b) for b in bodies]).astype(np.int32)
        orb = np.array([o for b in bodies for o in b], dtype=np.int32)
        nocc = np.array(problem.nocc, dtype=np.int32)
        self._keep += [ptr, orb, nocc]
        n_orb = int(problem.n_orb)
        pr = Problem(n_orb=n_orb, n_bodies=len(bodies),
                     body_ptr=ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     body_orb=orb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     body_nocc=nocc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     order=problem.order, e_const=float(getattr(problem, "e_const", 0.0)))
        self.options = default_options(precision=precision, solver=solver, **opts)
        h = ctypes.c_void_p()
        _check(lib().ifci_plan_create(ctypes.byref(pr), ctypes.byref(self.options), device, ctypes.byref(h)))
        self._h = h
        self.device = device
        if tuning == "cache":
            tuning = load_tuning()
        for (k, prec), (ps, ew) in (tuning or {}).items():
            self.set_tuning(k, prec, ps, ew)
        self.order = problem.order
        self.n_orb = n_orb
        self.workspace = None
        self._ints = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ifci_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- host queries
    def info(self):
        n, ws, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ifci_plan_info(self._h, ctypes.byref(n), ctypes.byref(ws), ctypes.byref(nd)))
        return dict(n_inc=n.value, workspace_bytes=ws.value, max_ndet=nd.value)

    @property
    def n_inc(self) -> int:
        return self.info()["n_inc"]

    def increment(self, idx: int) -> IncrementInfo:
        b = (ctypes.c_int32 * self.order)()
        k, na, nd = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().ifci_increment(self._h, idx, b, ctypes.byref(k), ctypes.byref(na), ctypes.byref(nd)))
        return IncrementInfo(tuple(x for x in b if x >= 0), k.value, na.value, nd.value)

    def increments(self):
        return [self.increment(i) for i in range(self.n_inc)]

    def weights(self):
        w = (ctypes.c_double * self.order)()
        _check(lib().ifci_weights(self._h, w))
        return list(w)

    # ---------------------------------------------------------------- device
    def attach(self, h, eri, stream=None):
        """Allocate the workspace (torch) and load integrals (torch CUDA FP64)."""
        import torch
        dev = torch.device("cuda", self.device)
        ws_bytes = self.info()["workspace_bytes"]
        self.workspace = torch.empty(max(ws_bytes, 256) // 8 + 64, dtype=torch.float64, device=dev)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        _check(lib().ifci_set_workspace(self._h, ctypes.c_void_p(base + off), ws_bytes))
        h = torch.as_tensor(h, dtype=torch.float64, device=dev).contiguous()
        eri = torch.as_tensor(eri, dtype=torch.float64, device=dev).contiguous()
        self._ints = (h, eri)
        _check(lib().ifci_set_integrals(self._h, _ptr(h), _ptr(eri), _stream(stream)))
        return self

    def sigma(self, inc: int, c, precision=FP64, stream=None):
        import torch
        c = c.contiguous()
        out = torch.empty_like(c)
        _check(lib().ifci_sigma(self._h, inc, _ptr(c), _ptr(out), precision, _stream(stream)))
        return out

    def sigma_noalloc(self, inc: int, out, c, precision=FP64, stream=None):
        """ifci_sigma_noalloc into the caller's `out` (nothing is allocated)."""
        _check(lib().ifci_sigma_noalloc(self._h, inc, _ptr(c), _ptr(out), precision, _stream(stream)))
        return out

    def sigma_sector(self, inc: int, c, precision=FP64, stream=None):
        import torch
        c = c.contiguous()
        out = torch.empty_like(c)
        _check(lib().ifci_sigma_sector(self._h, inc, _ptr(c), _ptr(out), precision, _stream(stream)))
        return out

    def davidson(self, first: int = 0, count: int | None = None, evict=None, stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        if count is None:
            count = self.n_inc - first
        e = torch.empty(count, dtype=torch.float64, device=dev)
        st = torch.empty(count, dtype=torch.int32, device=dev)
        it = torch.empty(count, dtype=torch.int32, device=dev)
        rs = torch.empty(count, dtype=torch.float64, device=dev)
        ev = None
        if evict is not None:
            ev = torch.as_tensor(evict, dtype=torch.uint8, device=dev).contiguous()
        _check(lib().ifci_davidson(self._h, first, count, _ptr(e), _ptr(st), _ptr(ev), _ptr(it), _ptr(rs),
                                   _stream(stream)))
        return e, st, it, rs

    def screen(self, e_inc, threshold: float, stream=None):
        """Connected n-body screening (ifci_screen) from the one- and
        two-body energies in e_inc (device [n_inc]); threshold < 0 removes it.
        Returns the keep mask (numpy bool [n_inc])."""
        keep = np.zeros(self.n_inc, dtype=np.uint8)
        n = ctypes.c_int64()
        _check(lib().ifci_screen(self._h, _ptr(e_inc), float(threshold), keep.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(n), _stream(stream)))
        return keep.astype(bool)

    def group_sums(self, eps, group_of_body, n_groups: int | None = None, stream=None):
        """{combination (sorted label tuple): sum of eps_S} (ifci_group_sums)."""
        lab = np.ascontiguousarray(group_of_body, dtype=np.int32)
        ng = int(n_groups if n_groups is not None else lab.max() + 1)
        n = ctypes.c_int64()
        _check(lib().ifci_group_count(self._h, ng, ctypes.byref(n)))
        sums = np.zeros(n.value)
        combos = np.zeros((n.value, self.order), dtype=np.int32)
        _check(lib().ifci_group_sums(self._h, _ptr(eps), lab.ctypes.data_as(ctypes.c_void_p), ng,
                                     sums.ctypes.data_as(ctypes.c_void_p), combos.ctypes.data_as(ctypes.c_void_p),
                                     _stream(stream)))
        return {tuple(int(x) for x in c if x >= 0): float(v) for c, v in zip(combos, sums)}

    def set_tuning(self, k: int, precision: int, ps_block: int = -1, e_waves: int = 0):
        """Per-shape settings of the on-chip solvers (ifci_set_tuning)."""
        _check(lib().ifci_set_tuning(self._h, int(k), int(precision), int(ps_block), int(e_waves)))

    def trace_phases(self, enable: bool = True):
        """Per-increment phase clock counters of the batched solver (int64
        [n_inc][8]: set-up, sigma, subspace, residual, restart, orthogonalise,
        sigma count, total); returns the torch buffer the next davidson fills."""
        import torch
        if not enable:
            _check(lib().ifci_set_phase_counters(self._h, None, 0))
            self._phase = None
            return None
        self._phase = torch.zeros((self.n_inc, 8), dtype=torch.int64, device=torch.device("cuda", self.device))
        _check(lib().ifci_set_phase_counters(self._h, _ptr(self._phase), self._phase.numel()))
        return self._phase

    def vector(self, inc: int, stream=None):
        import torch
        nd = self.increment(inc).n_det
        out = torch.empty(nd, dtype=torch.float64, device=torch.device("cuda", self.device))
        _check(lib().ifci_vector(self._h, inc, _ptr(out), _stream(stream)))
        return out

    def energy(self, e_inc, status=None, stream=None):
        """{'total', 'e_ref', 'by_order', 'eps'} from total increment energies."""
        import torch
        eps = torch.empty_like(e_inc)
        out = (ctypes.c_double * (self.order + 2))()
        code = lib().ifci_energy(self._h, _ptr(e_inc), _ptr(status), _ptr(eps), out, _stream(stream))
        if code not in (0, 5):
            _check(code)
        return dict(total=out[0], e_ref=out[1], by_order=list(out[2:]), eps=eps, converged=(code == 0))

    def rdm(self, weights=None, with_eri=True, stream=None):
        """(dE/dh, dE/d(pq|rs)) of the expansion (or of the given weights)."""
        import torch
        dev = torch.device("cuda", self.device)
        n = self.n_orb
        dh = torch.empty((n, n), dtype=torch.float64, device=dev)
        dg = torch.empty((n, n, n, n), dtype=torch.float64, device=dev) if with_eri else None
        w = None
        if weights is not None:
            w = torch.as_tensor(weights, dtype=torch.float64, device=dev).contiguous()
        _check(lib().ifci_rdm(self._h, _ptr(w), _ptr(dh), _ptr(dg), _stream(stream)))
        return dh, dg


    # ---------------------------------------------------------------- HBCI
    def hbci_work(self, inc: int, opts: HbciOptions):
        """A device work buffer for the HBCI calls on increment inc (torch,
        256-byte aligned view): (tensor, pointer, bytes)."""
        import torch
        nb = ctypes.c_int64()
        _check(lib().ifci_hbci_work_bytes(self._h, inc, ctypes.byref(opts), ctypes.byref(nb)))
        buf = torch.empty(nb.value // 8 + 64, dtype=torch.float64, device=torch.device("cuda", self.device))
        base = buf.data_ptr()
        return buf, ctypes.c_void_p(base + (-base) % 256), nb.value

    def hbci(self, inc: int, opts: HbciOptions | None = None, work=None, with_space: bool = False, stream=None):
        """ifci_hbci_solve: dict(E_var, E_pt2, E, n_det, n_iter, converged,
        residual, n_ext, nnz[, dets, c])."""
        import torch
        opts = opts or hbci_options()
        work = work or self.hbci_work(inc, opts)
        res = (ctypes.c_double * 8)()
        dets = c = None
        if with_space:
            dev = torch.device("cuda", self.device)
            dets = torch.empty(opts.max_det, dtype=torch.int64, device=dev)
            c = torch.empty(opts.max_det, dtype=torch.float64, device=dev)
        _check(lib().ifci_hbci_solve(self._h, inc, ctypes.byref(opts), work[1], work[2], res, _ptr(dets), _ptr(c),
                                     _stream(stream)))
        out = dict(E_var=res[0], E_pt2=res[1], E=res[0] + res[1], n_det=int(res[2]), n_iter=int(res[3]),
                   converged=bool(res[4]), residual=res[5], n_ext=int(res[6]), nnz=int(res[7]))
        if with_space:
            out["dets"] = dets[: out["n_det"]]
            out["c"] = c[: out["n_det"]]
        return out

    def hbci_sigma(self, inc: int, dets, c, opts: HbciOptions | None = None, work=None, stream=None):
        import torch
        opts = opts or hbci_options(max_det=max(2, len(dets)))
        work = work or self.hbci_work(inc, opts)
        dets, c = dets.contiguous(), c.contiguous()
        out = torch.empty_like(c)
        _check(lib().ifci_hbci_sigma(self._h, inc, ctypes.byref(opts), work[1], work[2], _ptr(dets), len(dets),
                                     _ptr(c), _ptr(out), _stream(stream)))
        return out

    def hbci_select(self, inc: int, dets, c, eps1: float, opts: HbciOptions, work=None, stream=None):
        import torch
        work = work or self.hbci_work(inc, opts)
        dets, c = dets.contiguous(), c.contiguous()
        added = torch.empty(max(1, opts.max_det - len(dets)), dtype=torch.int64, device=dets.device)
        n = ctypes.c_int64()
        _check(lib().ifci_hbci_select(self._h, inc, ctypes.byref(opts), work[1], work[2], _ptr(dets), len(dets),
                                      _ptr(c), eps1, _ptr(added), ctypes.byref(n), _stream(stream)))
        return added[: n.value]

    def hbci_pt2(self, inc: int, dets, c, e_var: float, eps2: float, opts: HbciOptions, work=None, stream=None):
        work = work or self.hbci_work(inc, opts)
        dets, c = dets.contiguous(), c.contiguous()
        e2, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().ifci_hbci_pt2(self._h, inc, ctypes.byref(opts), work[1], work[2], _ptr(dets), len(dets),
                                   _ptr(c), e_var, eps2, ctypes.byref(e2), ctypes.byref(n), _stream(stream)))
        return e2.value, n.value

    def hbci_expansion(self, opts: HbciOptions | None = None, workers: int = 16, stream=None):
        """Every increment by HBCI (E = E_var + E_PT2; ifci_hbci_solve_range
        with `workers` host threads), then the energy sums of eqs. 1-5:
        dict(results, energy, seconds)."""
        import time

        import torch
        opts = opts or hbci_options()
        dev = torch.device("cuda", self.device)
        n = self.n_inc
        nb = 0
        for i in range(n):
            b = ctypes.c_int64()
            _check(lib().ifci_hbci_work_bytes(self._h, i, ctypes.byref(opts), ctypes.byref(b)))
            nb = max(nb, b.value)
        bufs = [torch.empty(nb // 8 + 64, dtype=torch.float64, device=dev) for _ in range(workers)]
        ptrs = (ctypes.c_void_p * workers)(*[b.data_ptr() + (-b.data_ptr()) % 256 for b in bufs])
        res = (ctypes.c_double * (8 * n))()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        _check(lib().ifci_hbci_solve_range(self._h, 0, n, ctypes.byref(opts), ptrs, nb, workers, res))
        secs = time.perf_counter() - t0
        results = [dict(E_var=res[8 * i], E_pt2=res[8 * i + 1], E=res[8 * i] + res[8 * i + 1],
                        n_det=int(res[8 * i + 2]), n_iter=int(res[8 * i + 3]), converged=bool(res[8 * i + 4]),
                        residual=res[8 * i + 5], n_ext=int(res[8 * i + 6]), nnz=int(res[8 * i + 7]))
                   for i in range(n)]
        E = torch.tensor([r["E"] for r in results], dtype=torch.float64, device=dev)
        st = torch.tensor([1 if r["converged"] else 2 for r in results], dtype=torch.int32, device=dev)
        en = self.energy(E, st, stream=stream)
        return dict(results=results, energy=en, seconds=secs)

def davidson_group(plans, stream=None):
    """ifci_davidson_group over attached plans: one batched solve of every
    increment of every plan.  Returns [(E, status, iters, resid)] per plan."""
    import torch
    outs = []
    for pl in plans:
        dev = torch.device("cuda", pl.device)
        n = pl.n_inc
        outs.append((torch.empty(n, dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.float64, device=dev)))
    arr = lambda xs: (ctypes.c_void_p * len(xs))(*[ctypes.c_void_p(x.data_ptr()) for x in xs])
    handles = (ctypes.c_void_p * len(plans))(*[pl._h.value for pl in plans])
    _check(lib().ifci_davidson_group(handles, len(plans), arr([o[0] for o in outs]), arr([o[1] for o in outs]),
                                     arr([o[2] for o in outs]), arr([o[3] for o in outs]), _stream(stream)))
    return outs


def group_differences(sums_a: dict, sums_b: dict):
    """Per combination the change from calculation a to calculation b (two
    geometries with comparable orbitals): sums_b - sums_a."""
    return {c: sums_b.get(c, 0.0) - sums_a.get(c, 0.0) for c in sorted(set(sums_a) | set(sums_b),
                                                                      key=lambda c: (len(c), c))}


def solve_screened(problem, threshold: float, precision=FP64, solver=BATCHED, device: int = 0, **opts):
    """The expansion with connected n-body screening: the one- and two-body
    increments first, then ifci_screen on their energies, then the kept
    increments of three or more bodies, and the screened energy sums."""
    import torch
    plan = Plan(problem, precision=precision, solver=solver, device=device, **opts)
    plan.attach(problem.h, problem.eri)
    sizes = [len(i.bodies) for i in plan.increments()]
    n12 = sum(1 for s in sizes if s <= 2)
    dev = torch.device("cuda", device)
    e = torch.full((plan.n_inc,), float("nan"), dtype=torch.float64, device=dev)
    st = torch.zeros(plan.n_inc, dtype=torch.int32, device=dev)
    it = torch.zeros(plan.n_inc, dtype=torch.int32, device=dev)
    rs = torch.zeros(plan.n_inc, dtype=torch.float64, device=dev)
    e1, s1, i1, r1 = plan.davidson(0, n12)
    e[:n12], st[:n12], it[:n12], rs[:n12] = e1, s1, i1, r1
    keep = plan.screen(e, threshold)
    if plan.n_inc > n12:
        e2, s2, i2, r2 = plan.davidson(n12, plan.n_inc - n12)
        e[n12:], st[n12:], it[n12:], rs[n12:] = e2, s2, i2, r2
    en = plan.energy(e, st)
    return plan, dict(E=e, status=st, iters=it, resid=rs, keep=keep, **en)


def solve(problem, precision=FP64, solver=BATCHED, device: int = 0, **opts):
    """Whole expansion on the GPU: plan, embed, Davidson over every increment,
    energy assembly.  Returns the plan (kept for vectors and RDMs) and results."""
    plan = Plan(problem, precision=precision, solver=solver, device=device, **opts)
    plan.attach(problem.h, problem.eri)
    e, st, it, rs = plan.davidson()
    en = plan.energy(e, st)
    return plan, dict(E=e, status=st, iters=it, resid=rs, **en)
