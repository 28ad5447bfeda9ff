"""FP64 CPU oracle for the two-stage (fast/slow) k-means (arXiv 1108.1351).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the GPU library; the C source (``kmeans_oracle.c``) states, step by step,
which passage of the paper each part follows.

Parity unpinned: nothing.  Every function is pinned by the CPU tests against
published SplitMix64 outputs, brute-force enumeration of partitions, closed
forms (k = 1, k = n, 1-D two-means), invariants of Lloyd's method, and (for
the per-pass trace and the empty-cluster variant) hand-built cases whose
answers follow from the definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkmeans_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, FP64, no FMA contraction, OpenMP)."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-o", tmp, os.path.join(_HERE, "kmeans_oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * 2), ("converged", ctypes.c_int32 * 2),
                ("empty", ctypes.c_int32 * 2), ("m", ctypes.c_int64), ("J", ctypes.c_double),
                ("J_stage1", ctypes.c_double), ("dist_evals", ctypes.c_int64),
                ("shift", ctypes.c_double * 2)]

    def as_dict(self):
        return {"iters": list(self.iters), "converged": list(self.converged),
                "empty": list(self.empty), "m": self.m, "J": self.J,
                "J_stage1": self.J_stage1, "dist_evals": self.dist_evals,
                "shift": list(self.shift)}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
        lib.oracle_key.argtypes = [u64, i64]
        lib.oracle_key.restype = u64
        lib.oracle_subset_size.argtypes = [i64, i32, f64]
        lib.oracle_subset_size.restype = i64
        lib.oracle_select.argtypes = [i64, i64, i32, u64, vp, vp]
        lib.oracle_assign.argtypes = [vp, i32, i64, i32, vp, i32, vp, vp, vp]
        lib.oracle_step.argtypes = [vp, i32, i64, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_fit.argtypes = [vp, i32, i64, i32, i32, f64, u64, vp, vp, vp, i32, vp, vp,
                                   ctypes.POINTER(Info), vp, vp, vp, vp]
        lib.oracle_step_ex.argtypes = [vp, i32, i64, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp,
                                       vp]
        lib.oracle_fit_ex.argtypes = [vp, i32, i64, i32, i32, f64, u64, vp, vp, vp, i32, i32, vp,
                                      vp, ctypes.POINTER(Info), vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_get_threads.restype = i32
        _lib = lib
    return _lib


def _xcode(X: np.ndarray) -> int:
    if X.dtype == np.float32:
        return 0
    if X.dtype == np.uint16:  # BF16 bit patterns
        return 1
    if X.dtype == np.float64:
        return 2
    raise TypeError(f"unsupported X dtype {X.dtype}")


def _c(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data


def key(seed: int, i: int) -> int:
    return int(_load().oracle_key(seed, i))


def subset_size(n: int, k: int, f: float) -> int:
    return int(_load().oracle_subset_size(n, k, f))


def select(n: int, m: int, k: int, seed: int):
    """(subset indices ascending [m], initial-center indices in key order [k])."""
    sub = np.empty(m, np.int64)
    ini = np.empty(k, np.int64)
    rc = _load().oracle_select(n, m, k, seed, _c(sub), _c(ini))
    if rc:
        raise ValueError(f"oracle_select failed ({rc})")
    return sub, ini


def assign(X: np.ndarray, C: np.ndarray):
    """(labels, best squared distance, second-best squared distance) per row."""
    X = np.ascontiguousarray(X)
    C = np.ascontiguousarray(C, dtype=np.float64)
    n, d = X.shape
    k = C.shape[0]
    lab = np.empty(n, np.int32)
    D1 = np.empty(n, np.float64)
    D2 = np.empty(n, np.float64)
    rc = _load().oracle_assign(_c(X), _xcode(X), n, d, _c(C), k, _c(lab), _c(D1), _c(D2))
    if rc:
        raise ValueError("oracle_assign failed")
    return lab, D1, D2


@dataclass
class Step:
    labels: np.ndarray
    S: np.ndarray
    N: np.ndarray
    J: float
    C_new: np.ndarray
    shift: float
    empty: int


def step(Y: np.ndarray, C: np.ndarray, reseed: bool = False) -> Step:
    """One Lloyd pass (assignment, J, update) from centers C; with ``reseed`` the
    lowest empty cluster moves to the farthest point (see the C source)."""
    Y = np.ascontiguousarray(Y)
    C = np.ascontiguousarray(C, dtype=np.float64)
    n, d = Y.shape
    k = C.shape[0]
    lab = np.empty(n, np.int32)
    S = np.empty((k, d), np.float64)
    N = np.empty(k, np.int64)
    Cn = np.empty((k, d), np.float64)
    J = ctypes.c_double()
    sh = ctypes.c_double()
    ne = ctypes.c_int32()
    rc = _load().oracle_step_ex(_c(Y), _xcode(Y), n, d, _c(C), k, int(bool(reseed)), _c(lab),
                                _c(S), _c(N), ctypes.addressof(J), _c(Cn), ctypes.addressof(sh),
                                ctypes.addressof(ne))
    if rc:
        raise ValueError("oracle_step failed")
    return Step(lab, S, N, J.value, Cn, sh.value, ne.value)


@dataclass
class Fit:
    centers: np.ndarray
    labels: np.ndarray
    info: dict
    J_hist: tuple
    shift_hist: tuple
    trace_centers: tuple = None   # per stage: (passes, k, d) centers each pass starts from
    trace_counts: tuple = None    # per stage: (passes, k) cluster sizes each pass finds


def fit(X: np.ndarray, k: int, subset_frac: float, seed: int, max_iter, tol,
        init_centers: np.ndarray | None = None, skip_stage1: bool = False,
        reseed: bool = False, trace: bool = False) -> Fit:
    """The two-stage method.  ``max_iter`` / ``tol``: a number or a (fast, slow) pair;
    ``reseed``: the empty-cluster variant; ``trace``: per-pass centers and sizes."""
    X = np.ascontiguousarray(X)
    n, d = X.shape
    mi = np.array(max_iter if np.ndim(max_iter) else (max_iter, max_iter), np.int32)
    tl = np.array(tol if np.ndim(tol) else (tol, tol), np.float64)
    C = np.empty((k, d), np.float64)
    lab = np.empty(n, np.int32)
    info = Info()
    jh = [np.zeros(max(1, int(mi[s])), np.float64) for s in range(2)]
    sh = [np.zeros(max(1, int(mi[s])), np.float64) for s in range(2)]
    ic = None
    if init_centers is not None:
        ic = np.ascontiguousarray(init_centers, dtype=np.float64)
        assert ic.shape == (k, d)
    tc = [np.zeros((max(1, int(mi[s])), k, d), np.float64) if trace else None for s in range(2)]
    tn = [np.zeros((max(1, int(mi[s])), k), np.int64) if trace else None for s in range(2)]
    opt = lambda a: _c(a) if a is not None else None  # noqa: E731
    rc = _load().oracle_fit_ex(_c(X), _xcode(X), n, d, k, subset_frac, seed, _c(mi), _c(tl),
                               opt(ic), int(skip_stage1), int(bool(reseed)), _c(C), _c(lab),
                               ctypes.byref(info), _c(jh[0]), _c(sh[0]), _c(jh[1]), _c(sh[1]),
                               opt(tc[0]), opt(tn[0]), opt(tc[1]), opt(tn[1]))
    if rc:
        raise ValueError(f"oracle_fit failed ({rc})")
    it = info.iters
    out = Fit(C, lab, info.as_dict(), (jh[0][:it[0]], jh[1][:it[1]]),
              (sh[0][:it[0]], sh[1][:it[1]]))
    if trace:
        out.trace_centers = (tc[0][:it[0]], tc[1][:it[1]])
        out.trace_counts = (tn[0][:it[0]], tn[1][:it[1]])
    return out


def set_threads(n: int) -> None:
    _load().oracle_set_threads(n)


def get_threads() -> int:
    return int(_load().oracle_get_threads())
