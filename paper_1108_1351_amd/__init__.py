"""Python binding of the MI355X two-stage k-means library (``libkmeans_mi355x.so``).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory and the stream.  The functions carry the names
of the C entry points declared in ``include/kmeans.h``.

The method is the two-stage (fast/slow) k-means of Salman et al., "Fast
k-means algorithm clustering" (arXiv 1108.1351), section 2 (Algorithm).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmeans_mi355x.so")

KM_OK, KM_EINVAL, KM_ENOMEM, KM_EDEVICE, KM_EBUSY, KM_ECANCELLED, KM_ETIMEOUT, KM_ENOTFOUND = \
    range(8)
KM_F32, KM_BF16 = 0, 1
PRECISION = {"auto": 0, "fp32": 1, "bf16_rerank": 2}
EXPORTS = ("kmeans_fit", "kmeans_fit_ex", "kmeans_default_options", "kmeans_workspace_bytes",
           "km_sample", "km_step", "km_assign", "kmeans_last_error", "kmeans_profile_begin",
           "kmeans_profile_end", "kmeans_release_memory", "kmeans_fit_batch", "km_tune_query",
           "km_server_create", "km_server_submit", "km_server_wait", "km_server_stats",
           "km_server_destroy", "km_probe_stream_read", "km_probe_mfma_bf16",
           "kmeans_fit_static")


class KMeansError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status


class km_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * 2), ("converged", ctypes.c_int32 * 2),
                ("empty", ctypes.c_int32 * 2), ("m", ctypes.c_int64), ("J", ctypes.c_double),
                ("J_stage1", ctypes.c_double), ("dist_evals", ctypes.c_int64),
                ("shift", ctypes.c_double * 2), ("uncertain", ctypes.c_int64),
                ("seconds", ctypes.c_double * 3), ("fp64_pairs", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"iters": list(self.iters), "converged": list(self.converged),
                "empty": list(self.empty), "m": self.m, "J": self.J,
                "J_stage1": self.J_stage1, "dist_evals": self.dist_evals,
                "shift": list(self.shift), "uncertain": self.uncertain,
                "fp64_pairs": self.fp64_pairs, "seconds": list(self.seconds)}


class km_options(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_iter", ctypes.c_int32 * 2), ("tol", ctypes.c_double * 2),
                ("init_centers", ctypes.c_void_p), ("skip_stage1", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("centers64_out", ctypes.c_void_p),
                ("J_hist", ctypes.c_void_p), ("shift_hist", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("check_finite", ctypes.c_int32), ("reseed", ctypes.c_int32),
                ("trace_centers", ctypes.c_void_p), ("trace_counts", ctypes.c_void_p)]


class km_prof(ctypes.Structure):
    _fields_ = [("fits", ctypes.c_int64), ("passes", ctypes.c_int64 * 2),
                ("rows", ctypes.c_int64 * 2), ("assign_ms", ctypes.c_double * 2),
                ("pass_ms", ctypes.c_double * 2)]

    def as_dict(self) -> dict:
        return {"fits": self.fits, "passes": list(self.passes), "rows": list(self.rows),
                "assign_ms": list(self.assign_ms), "pass_ms": list(self.pass_ms)}


class km_request(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("x_on_host", ctypes.c_int32), ("dtype", ctypes.c_int),
                ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32),
                ("subset_frac", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("max_iter", ctypes.c_int32 * 2), ("tol", ctypes.c_double * 2),
                ("centers_out", ctypes.c_void_p), ("labels_out", ctypes.c_void_p)]


class km_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("info", km_info), ("queue_seconds", ctypes.c_double),
                ("run_seconds", ctypes.c_double)]


class km_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("passes_per_sync", ctypes.c_int32)]


class km_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("active", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("peak_active", ctypes.c_int64),
                ("syncs", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load the HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: run "
                           "`python -c 'import __graft_entry__ as g; g.build()'` first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    P = ctypes.POINTER
    lib.kmeans_fit.argtypes = [vp, i64, i32, i32, f64, u64, i32, f64, vp, vp, P(km_info)]
    lib.kmeans_fit_ex.argtypes = [vp, i64, i32, i32, f64, u64, P(km_options), vp, vp,
                                  P(km_info)]
    lib.kmeans_fit_static.argtypes = lib.kmeans_fit_ex.argtypes
    lib.kmeans_fit_static.restype = ctypes.c_int
    lib.kmeans_default_options.argtypes = [P(km_options), i32, f64]
    lib.kmeans_default_options.restype = None
    lib.kmeans_workspace_bytes.argtypes = [i64, i32, i32, f64, P(km_options)]
    lib.kmeans_workspace_bytes.restype = ctypes.c_size_t
    lib.km_sample.argtypes = [i64, i64, i32, u64, vp, vp, vp]
    lib.km_step.argtypes = [vp, ctypes.c_int, i64, i32, vp, i32, ctypes.c_int, vp, vp, vp, vp,
                            P(f64), P(f64), P(i32), P(i64), vp]
    lib.km_assign.argtypes = [vp, ctypes.c_int, i64, i32, vp, i32, ctypes.c_int, vp, P(f64),
                              P(i64), vp]
    lib.kmeans_profile_begin.argtypes = []
    lib.kmeans_profile_end.argtypes = [P(km_prof)]
    lib.kmeans_release_memory.argtypes = []
    lib.kmeans_last_error.argtypes = []
    lib.kmeans_last_error.restype = ctypes.c_char_p
    lib.kmeans_fit_batch.argtypes = [P(km_request), i32, P(km_result), vp]
    lib.km_tune_query.argtypes = [ctypes.c_int, i32, i32, P(i32), P(i32)]
    lib.km_server_create.argtypes = [P(km_server_cfg), P(vp)]
    lib.km_server_submit.argtypes = [vp, P(km_request), P(u64)]
    lib.km_server_wait.argtypes = [vp, u64, P(km_result), i64]
    lib.km_server_stats.argtypes = [vp, P(km_server_counters)]
    lib.km_server_destroy.argtypes = [vp]
    lib.km_probe_stream_read.argtypes = [vp, ctypes.c_size_t, i32, P(f64), vp]
    lib.km_probe_mfma_bf16.argtypes = [i32, P(f64), vp]
    for name in ("kmeans_fit", "kmeans_fit_ex", "km_sample", "km_step", "km_assign",
                 "kmeans_profile_begin", "kmeans_profile_end", "kmeans_release_memory",
                 "kmeans_fit_batch", "km_tune_query", "km_server_create", "km_server_submit",
                 "km_server_wait", "km_server_stats", "km_server_destroy",
                 "km_probe_stream_read", "km_probe_mfma_bf16"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def kmeans_last_error() -> str:
    return load().kmeans_last_error().decode()


def _check(rc: int) -> None:
    if rc != KM_OK:
        raise KMeansError(rc, kmeans_last_error())


def _dtype_code(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return KM_F32
    if X.dtype == torch.bfloat16:
        return KM_BF16
    raise TypeError(f"X must be float32 or bfloat16, got {X.dtype}")


def _dev(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _pair(v):
    return (v[0], v[1]) if isinstance(v, (tuple, list)) else (v, v)


def kmeans_fit(X: torch.Tensor, k: int, subset_frac: float, seed: int, max_iter: int,
               tol: float, labels: bool = True):
    """The two-stage method on FP32 data (C: kmeans_fit).  Returns (centers, labels, info)."""
    lib = load()
    if X.dtype != torch.float32:
        raise TypeError("kmeans_fit takes FP32 data; use kmeans_fit_ex for BF16")
    n, d = X.shape
    C = torch.empty((k, d), dtype=torch.float32, device=X.device)
    L = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
    info = km_info()
    rc = lib.kmeans_fit(_dev(X, "X"), n, d, k, subset_frac, seed, max_iter, tol,
                        C.data_ptr(), L.data_ptr() if L is not None else None,
                        ctypes.byref(info))
    _check(rc)
    return C, L, info.as_dict()


def _options(X, k, max_iter, tol, precision, init_centers, skip_stage1, stream, workspace,
             check_finite, reseed):
    """A km_options for kmeans_fit_ex and its no-allocation variant (plus the host
    arrays that must outlive the call)."""
    n, d = X.shape
    opt = km_options()
    mi, tl = _pair(max_iter), _pair(tol)
    opt.dtype = _dtype_code(X)
    opt.precision = PRECISION[precision]
    opt.max_iter[0], opt.max_iter[1] = int(mi[0]), int(mi[1])
    opt.tol[0], opt.tol[1] = float(tl[0]), float(tl[1])
    opt.skip_stage1 = int(bool(skip_stage1))
    opt.stream = _stream(stream)
    opt.check_finite = int(bool(check_finite))
    opt.reseed = int(bool(reseed))
    keep = []
    if init_centers is not None:
        import numpy as np
        ic = np.ascontiguousarray(init_centers, dtype=np.float64)
        if ic.shape != (k, d):
            raise ValueError("init_centers must have shape (k, d)")
        opt.init_centers = ic.ctypes.data
        keep.append(ic)
    if workspace is not None:
        opt.workspace = _dev(workspace, "workspace")
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    return opt, keep


def kmeans_fit_ex(X: torch.Tensor, k: int, subset_frac: float, seed: int, max_iter=50,
                  tol=1e-4, *, precision: str = "auto", init_centers=None,
                  skip_stage1: bool = False, labels: bool = True, centers64: bool = False,
                  history: bool = False, stream=None, workspace: torch.Tensor | None = None,
                  check_finite: bool = False, reseed: bool = False, trace: bool = False):
    """Per-stage limits, FP32 or BF16 data, resume point (C: kmeans_fit_ex).

    Returns (centers FP32, labels or None, info dict); the dict also carries
    ``centers64`` (device FP64), ``J_hist`` / ``shift_hist`` and (``trace``) the
    per-pass ``trace_centers`` / ``trace_counts`` of each stage when requested.
    ``workspace``: a device tensor the call takes its scratch from
    (kmeans_workspace_bytes); ``reseed``: empty-cluster re-seeding.
    """
    lib = load()
    opt, keep = _options(X, k, max_iter, tol, precision, init_centers, skip_stage1, stream,
                         workspace, check_finite, reseed)
    return _fit_call(lib.kmeans_fit_ex, X, k, subset_frac, seed, opt, labels, centers64,
                     history, trace)


def _fit_call(entry, X, k, subset_frac, seed, opt, labels, centers64, history, trace):
    n, d = X.shape
    mi = (opt.max_iter[0], opt.max_iter[1])
    C = torch.empty((k, d), dtype=torch.float32, device=X.device)
    L = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
    C64 = torch.empty((k, d), dtype=torch.float64, device=X.device) if centers64 else None
    opt.centers64_out = C64.data_ptr() if C64 is not None else None
    if history:
        import numpy as np
        jh = np.zeros(int(mi[0]) + int(mi[1]), np.float64)
        sh = np.zeros_like(jh)
        opt.J_hist, opt.shift_hist = jh.ctypes.data, sh.ctypes.data
    if trace:
        import numpy as np
        tc = np.zeros((int(mi[0]) + int(mi[1]), k, d), np.float64)
        tn = np.zeros((int(mi[0]) + int(mi[1]), k), np.int64)
        opt.trace_centers, opt.trace_counts = tc.ctypes.data, tn.ctypes.data
    info = km_info()
    rc = entry(_dev(X, "X"), n, d, k, subset_frac, seed, ctypes.byref(opt), C.data_ptr(),
               L.data_ptr() if L is not None else None, ctypes.byref(info))
    _check(rc)
    out = info.as_dict()
    if C64 is not None:
        out["centers64"] = C64
    it = out["iters"]
    if history:
        out["J_hist"] = (jh[:it[0]].copy(), jh[int(mi[0]):int(mi[0]) + it[1]].copy())
        out["shift_hist"] = (sh[:it[0]].copy(), sh[int(mi[0]):int(mi[0]) + it[1]].copy())
    if trace:
        out["trace_centers"] = (tc[:it[0]].copy(), tc[int(mi[0]):int(mi[0]) + it[1]].copy())
        out["trace_counts"] = (tn[:it[0]].copy(), tn[int(mi[0]):int(mi[0]) + it[1]].copy())
    return C, L, out


def kmeans_fit_static(X: torch.Tensor, k: int, subset_frac: float, seed: int, max_iter=50,
                      tol=1e-4, *, precision: str = "auto", init_centers=None,
                      skip_stage1: bool = False, labels: bool = True, centers64: bool = False,
                      history: bool = False, stream=None, check_finite: bool = False,
                      reseed: bool = False, trace: bool = False):
    """kmeans_fit_ex with the library's fixed scratch array: no device memory is
    allocated by the call (C: kmeans_fit_static; the tensors this binding
    creates for the outputs are the caller's side)."""
    lib = load()
    opt, keep = _options(X, k, max_iter, tol, precision, init_centers, skip_stage1, stream,
                         None, check_finite, reseed)
    return _fit_call(lib.kmeans_fit_static, X, k, subset_frac, seed, opt, labels, centers64,
                     history, trace)


def kmeans_workspace_bytes(n: int, d: int, k: int, subset_frac: float, max_iter=50,
                           dtype=torch.float32, skip_stage1: bool = False,
                           precision: str = "auto", reseed: bool = False,
                           trace: bool = False) -> int:
    """Device bytes a fit with these sizes and options takes (C: kmeans_workspace_bytes)."""
    opt = km_options()
    load().kmeans_default_options(ctypes.byref(opt), 1, 0.0)
    mi = _pair(max_iter)
    opt.max_iter[0], opt.max_iter[1] = int(mi[0]), int(mi[1])
    opt.dtype = KM_F32 if dtype == torch.float32 else KM_BF16
    opt.precision = PRECISION[precision]
    opt.skip_stage1 = int(skip_stage1)
    opt.reseed = int(bool(reseed))
    if trace:  # only whether a trace is asked for matters to the size
        opt.trace_counts = 1
    return int(load().kmeans_workspace_bytes(n, d, k, subset_frac, ctypes.byref(opt)))


def km_sample(n: int, m: int, k: int, seed: int, device="cuda", stream=None):
    """(subset indices ascending [m], initial-center indices in key order [k]) on the device."""
    sub = torch.empty(m, dtype=torch.int64, device=device)
    ini = torch.empty(k, dtype=torch.int64, device=device)
    _check(load().km_sample(n, m, k, seed, sub.data_ptr(), ini.data_ptr(), _stream(stream)))
    return sub, ini


def km_step(X: torch.Tensor, C: torch.Tensor, precision: str = "auto", stream=None) -> dict:
    """One Lloyd pass at centers C (device FP64 k x d)."""
    n, d = X.shape
    k = C.shape[0]
    if C.dtype != torch.float64 or C.shape[1] != d:
        raise ValueError("C must be FP64 with shape (k, d)")
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    S = torch.empty((k, d), dtype=torch.float64, device=X.device)
    N = torch.empty(k, dtype=torch.int64, device=X.device)
    Cn = torch.empty((k, d), dtype=torch.float64, device=X.device)
    J, sh = ctypes.c_double(), ctypes.c_double()
    em, un = ctypes.c_int32(), ctypes.c_int64()
    rc = load().km_step(_dev(X, "X"), _dtype_code(X), n, d, _dev(C, "C"), k,
                        PRECISION[precision], lab.data_ptr(), S.data_ptr(), N.data_ptr(),
                        Cn.data_ptr(), ctypes.byref(J), ctypes.byref(sh), ctypes.byref(em),
                        ctypes.byref(un), _stream(stream))
    _check(rc)
    return {"labels": lab, "S": S, "N": N, "C_new": Cn, "J": J.value, "shift": sh.value,
            "empty": em.value, "uncertain": un.value}


def km_assign(X: torch.Tensor, C: torch.Tensor, precision: str = "auto", stream=None):
    """Nearest centers at fixed centers C (device FP64): (labels, J, uncertain)."""
    n, d = X.shape
    k = C.shape[0]
    if C.dtype != torch.float64 or C.shape[1] != d:
        raise ValueError("C must be FP64 with shape (k, d)")
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    J, un = ctypes.c_double(), ctypes.c_int64()
    rc = load().km_assign(_dev(X, "X"), _dtype_code(X), n, d, _dev(C, "C"), k,
                          PRECISION[precision], lab.data_ptr(), ctypes.byref(J),
                          ctypes.byref(un), _stream(stream))
    _check(rc)
    return lab, J.value, un.value


def kmeans_profile_begin() -> None:
    _check(load().kmeans_profile_begin())


def kmeans_profile_end() -> dict:
    out = km_prof()
    _check(load().kmeans_profile_end(ctypes.byref(out)))
    return out.as_dict()


def kmeans_release_memory() -> None:
    _check(load().kmeans_release_memory())


def km_probe_stream_read(buf: torch.Tensor, reps: int = 5, stream=None) -> float:
    """Measured device-memory read bandwidth (GB/s) over the bytes of ``buf``."""
    v = ctypes.c_double()
    _check(load().km_probe_stream_read(_dev(buf, "buf"), buf.numel() * buf.element_size(),
                                       reps, ctypes.byref(v), _stream(stream)))
    return v.value


def km_probe_mfma_bf16(iters: int = 20000, stream=None) -> float:
    """Measured dense BF16 MFMA rate (TFLOP/s) of a loop with no memory traffic."""
    v = ctypes.c_double()
    _check(load().km_probe_mfma_bf16(iters, ctypes.byref(v), _stream(stream)))
    return v.value


def _request(X: torch.Tensor, k: int, subset_frac: float, seed: int, max_iter, tol,
             C: torch.Tensor, L, on_host: bool) -> km_request:
    n, d = X.shape
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    if not on_host and not X.is_cuda:
        raise ValueError("X must be a device tensor")
    r = km_request()
    r.X = X.data_ptr()
    r.x_on_host = int(on_host)
    r.dtype = _dtype_code(X)
    r.n, r.d, r.k = n, d, k
    r.subset_frac, r.seed = subset_frac, seed
    mi, tl = _pair(max_iter), _pair(tol)
    r.max_iter[0], r.max_iter[1] = int(mi[0]), int(mi[1])
    r.tol[0], r.tol[1] = float(tl[0]), float(tl[1])
    r.centers_out = C.data_ptr()
    r.labels_out = L.data_ptr() if L is not None else None
    return r


def _result_dict(res: km_result) -> dict:
    out = res.info.as_dict()
    out.update(status=res.status, queue_seconds=res.queue_seconds, run_seconds=res.run_seconds)
    return out


def kmeans_fit_batch(problems, labels: bool = True, stream=None):
    """Many independent two-stage fits advanced together (C: kmeans_fit_batch).

    problems: sequence of (X, k, subset_frac, seed, max_iter, tol) with X a device
    tensor (FP32 or BF16, d <= 128).  Returns a list of (centers, labels, info)
    per problem; info["status"] is the problem's own status (0 = ok).
    """
    lib = load()
    reqs = (km_request * max(1, len(problems)))()
    res = (km_result * max(1, len(problems)))()
    outs = []
    for i, (X, k, f, seed, mi, tl) in enumerate(problems):
        n, d = X.shape
        C = torch.empty((k, d), dtype=torch.float32, device=X.device)
        L = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
        reqs[i] = _request(X, k, f, seed, mi, tl, C, L, False)
        outs.append((C, L))
    _check(lib.kmeans_fit_batch(reqs, len(problems), res, _stream(stream)))
    return [(C, L, _result_dict(res[i])) for i, (C, L) in enumerate(outs)]


def km_tune_query(dtype, d: int, k: int):
    """(points per thread, centers per LDS tile) the autotuner picks for a shape."""
    code = KM_F32 if dtype in (torch.float32, KM_F32, "f32") else KM_BF16
    ppt, kt = ctypes.c_int32(), ctypes.c_int32()
    _check(load().km_tune_query(code, d, k, ctypes.byref(ppt), ctypes.byref(kt)))
    return ppt.value, kt.value


class Server:
    """A serving loop (C: km_server_*): problems are admitted by device-memory
    footprint and advance together in batched passes; submit returns a ticket."""

    def __init__(self, hbm_budget_bytes: int = 0, max_active: int = 0, max_pending: int = 0,
                 use_graphs: bool = True, passes_per_sync: int = 0):
        cfg = km_server_cfg()
        cfg.hbm_budget_bytes, cfg.max_active = hbm_budget_bytes, max_active
        cfg.max_pending, cfg.use_graphs = max_pending, int(use_graphs)
        cfg.passes_per_sync = passes_per_sync
        self._h = ctypes.c_void_p()
        _check(load().km_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._outs = {}

    def submit(self, X: torch.Tensor, k: int, subset_frac: float, seed: int, max_iter=50,
               tol=1e-4, labels: bool = True, device="cuda") -> int:
        n, d = X.shape
        C = torch.empty((k, d), dtype=torch.float32, device=device)
        L = torch.empty(n, dtype=torch.int32, device=device) if labels else None
        if X.is_cuda:
            torch.cuda.current_stream().synchronize()  # X is complete before the server copies it
        r = _request(X, k, subset_frac, seed, max_iter, tol, C, L, not X.is_cuda)
        t = ctypes.c_uint64()
        _check(load().km_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._outs[t.value] = (C, L, X)  # X stays alive until the result is collected
        return t.value

    def wait(self, ticket: int, timeout: float | None = None):
        res = km_result()
        us = -1 if timeout is None else int(timeout * 1e6)
        rc = load().km_server_wait(self._h, ticket, ctypes.byref(res), us)
        if rc == KM_ETIMEOUT:
            raise TimeoutError(kmeans_last_error())
        C, L, _ = self._outs.pop(ticket, (None, None, None))
        _check(rc)
        return C, L, _result_dict(res)

    def stats(self) -> dict:
        c = km_server_counters()
        _check(load().km_server_stats(self._h, ctypes.byref(c)))
        return c.as_dict()

    def close(self) -> None:
        if self._h:
            _check(load().km_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
