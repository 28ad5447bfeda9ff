"""kmeans_fit_static (the entry point that allocates nothing; its scratch is a
fixed device array of the library) against kmeans_fit_ex, through the C ABI:
the same bits on two calls in a row, the second on a smaller problem, and
KM_ENOMEM beyond the array's size."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

km = pytest.importorskip("paper_1108_1351_amd")


def _static(X, k, f, seed, max_iter, tol, precision="auto"):
    lib = km.load()
    fn = lib.kmeans_fit_static
    fn.argtypes = lib.kmeans_fit_ex.argtypes
    fn.restype = ctypes.c_int
    opt, keep = km._options(X, k, max_iter, tol, precision, None, False, None, None, False,
                            False)
    return km._fit_call(fn, X, k, f, seed, opt, True, True, True, False)


def _compare(X, k, f, seed, max_iter, tol):
    a = km.kmeans_fit_ex(X, k, f, seed, max_iter, tol, centers64=True, history=True)
    b = _static(X, k, f, seed, max_iter, tol)
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1], b[1])
    assert torch.equal(a[2]["centers64"], b[2]["centers64"])
    for key in ("iters", "converged", "empty", "m", "J", "J_stage1", "dist_evals", "uncertain"):
        assert a[2][key] == b[2][key], key
    for s in range(2):
        assert np.array_equal(a[2]["J_hist"][s], b[2]["J_hist"][s])


def test_static_fit_matches_fit_ex_twice_shrinking():
    w = synth.WORKLOADS["gmm16d_n1e7_k64"]
    big = torch.from_numpy(w.data(n=400_000)).cuda()
    small = torch.from_numpy(w.data(n=30_011)).cuda()
    print("[static] 400000 x 16, k = 64", flush=True)
    _compare(big, 64, 0.01, 2, 30, 1e-4)
    print("[static] 30011 x 16, k = 64", flush=True)
    _compare(small, 64, 0.01, 2, 30, 1e-4)
    # another path family (sorted update) on the same array
    w2 = synth.WORKLOADS["gmm2d_n1e5_k8"]
    X2 = torch.from_numpy(w2.data(n=20_000)).cuda()
    print("[static] 20000 x 2, k = 2000", flush=True)
    _compare(X2, 2000, 0.2, 5, 5, 0.0)


def test_static_fit_rejects_problems_beyond_its_array():
    X = torch.empty((100_000_000, 2), dtype=torch.float32, device="cuda")
    lib = km.load()
    fn = lib.kmeans_fit_static
    fn.argtypes = lib.kmeans_fit_ex.argtypes
    fn.restype = ctypes.c_int
    opt, _ = km._options(X, 8, 10, 1e-4, "auto", None, False, None, None, False, False)
    C = torch.empty((8, 2), dtype=torch.float32, device="cuda")
    info = km.km_info()
    rc = fn(X.data_ptr(), X.shape[0], 2, 8, 0.5, 0, ctypes.byref(opt), C.data_ptr(), None,
            ctypes.byref(info))
    assert rc == km.KM_ENOMEM
    assert "scratch" in km.kmeans_last_error()
