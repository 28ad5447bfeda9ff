"""Seeded synthetic Gaussian-mixture inputs (a test and benchmark fixture).

This module produces input data only: it holds no clustering arithmetic and is
shared by the CPU oracle and by the GPU library's tests and benchmark.  The
generator itself is C (``synth.c``, counter-based SplitMix64 + Box-Muller),
so any row range of any workload can be regenerated bit-identically.

The workloads stand in for the paper's data, which is not available: the paper
validates on randomly generated clusters (section 4), on a 100,000 x 10
"Synthetic" set (section 6) and on 1M-10M x 12 points (section 6.1), and
motivates the method with datasets of more than 500 million points (abstract).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` (gcc, OpenMP)."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-o", tmp, os.path.join(_HERE, "synth.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


class _Spec(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("mean_kind", ctypes.c_int32), ("weight_kind", ctypes.c_int32),
                ("mean_lo", ctypes.c_double), ("mean_hi", ctypes.c_double),
                ("mean_sd", ctypes.c_double),
                ("sigma_lo", ctypes.c_double), ("sigma_hi", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.synth_params.argtypes = [P(_Spec), ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_params.restype = ctypes.c_int
        lib.synth_points.argtypes = [P(_Spec), ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p]
        lib.synth_points.restype = ctypes.c_int
        for name, rt in (("synth_u64", ctypes.c_uint64), ("synth_uniform", ctypes.c_double),
                         ("synth_normal", ctypes.c_double)):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
            fn.restype = rt
        _lib = lib
    return _lib


@dataclass(frozen=True)
class MixtureSpec:
    """Gaussian mixture: component means, per-component isotropic sigma, weights."""
    d: int
    ncomp: int
    mean_kind: str = "uniform"      # "uniform": U[mean_lo, mean_hi]^d ; "normal": N(0, mean_sd^2 I)
    mean_lo: float = -1.0
    mean_hi: float = 1.0
    mean_sd: float = 1.0
    sigma_lo: float = 1.0
    sigma_hi: float = 1.0
    weights: str = "equal"          # "equal" or "dirichlet1"

    def _c(self) -> _Spec:
        return _Spec(self.d, self.ncomp, 0 if self.mean_kind == "uniform" else 1,
                     0 if self.weights == "equal" else 1, self.mean_lo, self.mean_hi,
                     self.mean_sd, self.sigma_lo, self.sigma_hi)


DTYPES = {"f32": (0, np.float32), "bf16": (1, np.uint16), "f64": (2, np.float64)}


def params(spec: MixtureSpec, seed: int):
    """(means [ncomp, d], sigmas [ncomp], cumulative weights [ncomp]) for a seed."""
    lib = _load()
    means = np.empty((spec.ncomp, spec.d), np.float64)
    sig = np.empty(spec.ncomp, np.float64)
    cumw = np.empty(spec.ncomp, np.float64)
    cs = spec._c()
    rc = lib.synth_params(ctypes.byref(cs), seed, means.ctypes.data, sig.ctypes.data,
                          cumw.ctypes.data)
    if rc:
        raise ValueError("synth_params rejected the spec")
    return means, sig, cumw


def generate(spec: MixtureSpec, seed: int, n: int, dtype: str = "f32", row0: int = 0,
             out: np.ndarray | None = None, with_comp: bool = False, prm=None):
    """Rows [row0, row0+n) of the mixture sample.

    dtype "f32" -> float32, "bf16" -> uint16 holding BF16 bits, "f64" -> float64.
    ``out`` may be a preallocated C-contiguous array of shape (n, d) (for example
    the numpy view of a pinned host tensor).  Returns X, or (X, comp) with the
    drawn component of every row when ``with_comp``.
    """
    lib = _load()
    code, npdt = DTYPES[dtype]
    if out is None:
        out = np.empty((n, spec.d), npdt)
    assert out.dtype == npdt and out.flags.c_contiguous and out.size == n * spec.d
    means, sig, cumw = prm if prm is not None else params(spec, seed)
    comp = np.empty(n, np.int32) if with_comp else None
    cs = spec._c()
    rc = lib.synth_points(ctypes.byref(cs), seed, means.ctypes.data, sig.ctypes.data,
                          cumw.ctypes.data, row0, n, code, out.ctypes.data,
                          comp.ctypes.data if with_comp else None)
    if rc:
        raise ValueError("synth_points rejected the arguments")
    return (out, comp) if with_comp else out


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    """Widen BF16 bit patterns (uint16) to float32, exactly."""
    return (bits.astype(np.uint32) << 16).view(np.float32)


def u64(seed: int, stream: int, ctr: int) -> int:
    return int(_load().synth_u64(seed, stream, ctr))


def uniform(seed: int, stream: int, ctr: int) -> float:
    return float(_load().synth_uniform(seed, stream, ctr))


def normal(seed: int, stream: int, ctr: int) -> float:
    return float(_load().synth_normal(seed, stream, ctr))


@dataclass(frozen=True)
class Workload:
    """One clustering job: data shape and distribution plus the fit parameters."""
    name: str
    n: int
    k: int
    spec: MixtureSpec
    dtype: str
    subset_frac: float
    max_iter: int
    tol: float
    data_seed: int
    fit_seed: int

    @property
    def d(self) -> int:
        return self.spec.d

    def data(self, n: int | None = None, row0: int = 0, out=None):
        return generate(self.spec, self.data_seed, self.n if n is None else n, self.dtype,
                        row0=row0, out=out)

    def scaled(self, n: int, name: str | None = None) -> "Workload":
        """Same distribution and fit parameters at a different n (parity sizes)."""
        return Workload(name or f"{self.name}@n{n}", n, self.k, self.spec, self.dtype,
                        self.subset_frac, self.max_iter, self.tol, self.data_seed,
                        self.fit_seed)


WORKLOADS = {w.name: w for w in [
    # 8 isotropic Gaussians in 2-D, means U[-10,10]^2, sigma 1, equal weights;
    # 1% subset; at most 100 passes per stage; stop at max center shift < 1e-4.
    Workload("gmm2d_n1e5_k8", 100_000, 8,
             MixtureSpec(2, 8, "uniform", -10.0, 10.0, sigma_lo=1.0, sigma_hi=1.0),
             "f32", 0.01, 100, 1e-4, 1001, 1),
    # 64 components in 16-D, means U[-50,50]^16, sigma_c U[0.5,2], Dirichlet(1)
    # weights; 1% subset; 50 passes per stage; tol 1e-4.
    Workload("gmm16d_n1e7_k64", 10_000_000, 64,
             MixtureSpec(16, 64, "uniform", -50.0, 50.0, sigma_lo=0.5, sigma_hi=2.0,
                         weights="dirichlet1"),
             "f32", 0.01, 50, 1e-4, 1002, 2),
    # 1024 components in 128-D stored as BF16, means N(0, 25 I), sigma_c U[0.5,1.5],
    # equal weights; 0.5% subset; 20 passes per stage at tol 0 (fixed work).
    Workload("gmm128d_n1e8_k1024_bf16", 100_000_000, 1024,
             MixtureSpec(128, 1024, "normal", mean_sd=5.0, sigma_lo=0.5, sigma_hi=1.5),
             "bf16", 0.005, 20, 0.0, 1003, 3),
    # 32 components in 4-D, means U[-100,100]^4, sigma 3, equal weights (8 GB of
    # FP32 points); 0.1% subset; 30 passes per stage; tol 1e-3.
    Workload("gmm4d_n5e8_k32", 500_000_000, 32,
             MixtureSpec(4, 32, "uniform", -100.0, 100.0, sigma_lo=3.0, sigma_hi=3.0),
             "f32", 0.001, 30, 1e-3, 1004, 4),
]}


@dataclass(frozen=True)
class Request:
    """One request of the serving stream."""
    rid: int
    arrival_s: float
    workload: Workload


def serving_stream(count: int, rate_per_s: float, seed: int = 5):
    """A stream of independent clustering requests with Poisson arrivals.

    Per request: n log-uniform in [1e3, 1e6], d uniform in {2, 8, 32, 128},
    k log-uniform in [4, 256] (clamped to n), a k-component mixture with means
    U[-50,50]^d, sigma_c U[0.5,2] and Dirichlet(1) weights drawn from the
    request's own seed; FP32 storage for d < 32 and BF16 for d >= 32; 1% subset;
    50 passes per stage; tol 1e-4.
    """
    reqs, t = [], 0.0
    for r in range(count):
        u = [uniform(seed, 100, 8 * r + j) for j in range(5)]
        t += -math.log(u[0]) / rate_per_s
        n = int(round(10 ** (3 + 3 * u[1])))
        d = (2, 8, 32, 128)[min(3, int(u[2] * 4))]
        k = int(round(math.exp(math.log(4) + (math.log(256) - math.log(4)) * u[3])))
        k = max(1, min(k, n))
        spec = MixtureSpec(d, k, "uniform", -50.0, 50.0, sigma_lo=0.5, sigma_hi=2.0,
                           weights="dirichlet1")
        w = Workload(f"req{r}", n, k, spec, "f32" if d < 32 else "bf16", 0.01, 50, 1e-4,
                     seed * 1_000_003 + r, r)
        reqs.append(Request(r, t, w))
    return reqs
