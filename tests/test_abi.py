"""The C-ABI library on the host: it loads, exports every symbol the header
declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kmeans.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(k(?:m|means)_\w+)\s*\(", src,
                       flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1108_1351_amd as km
    return km.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("kmeans_fit", "kmeans_fit_ex", "km_sample", "km_step", "km_assign",
              "kmeans_last_error", "kmeans_workspace_bytes", "kmeans_default_options"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    import paper_1108_1351_amd as km
    assert set(km.EXPORTS) == set(_declared())


def test_invalid_arguments_rejected_on_host(lib):
    import paper_1108_1351_amd as km
    info = km.km_info()
    X = ctypes.c_void_p(0x1000)  # never dereferenced: validation comes first
    C = ctypes.c_void_p(0x2000)
    cases = [
        (0, 2, 1, 0.5, 10, 0.0, "n must be"),
        (10, 0, 1, 0.5, 10, 0.0, "d must be"),
        (10, 2, 0, 0.5, 10, 0.0, "k must be"),
        (10, 2, 11, 0.5, 10, 0.0, "must not exceed"),
        (10, 2, 3, 0.0, 10, 0.0, "subset_frac"),
        (10, 2, 3, 1.5, 10, 0.0, "subset_frac"),
        (10, 2, 3, 0.5, 0, 0.0, "max_iter"),
        (10, 2, 3, 0.5, 10, -1.0, "tol"),
        (10, 2, 3, 0.5, 10, float("nan"), "tol"),
    ]
    for n, d, k, f, mi, tol, msg in cases:
        rc = lib.kmeans_fit(X, n, d, k, f, 0, mi, tol, C, None, ctypes.byref(info))
        assert rc == km.KM_EINVAL
        assert msg in km.kmeans_last_error()
    assert lib.kmeans_fit(None, 10, 2, 3, 0.5, 0, 10, 0.0, C, None, ctypes.byref(info)) == \
        km.KM_EINVAL
    assert lib.km_sample(10, 11, 3, 0, X, X, None) == km.KM_EINVAL
    assert lib.km_sample(10, 2, 3, 0, X, X, None) == km.KM_EINVAL
    opt = km.km_options()
    lib.kmeans_default_options(ctypes.byref(opt), 5, 1e-3)
    assert list(opt.max_iter) == [5, 5] and list(opt.tol) == [1e-3, 1e-3]
    nan = (ctypes.c_double * 4)(float("nan"), 0, 0, 0)
    opt.init_centers = ctypes.cast(nan, ctypes.c_void_p)
    rc = lib.kmeans_fit_ex(X, 10, 2, 2, 0.5, 0, ctypes.byref(opt), C, None, ctypes.byref(info))
    assert rc == km.KM_EINVAL and "init_centers" in km.kmeans_last_error()


def test_workspace_bytes_grows_with_n():
    import paper_1108_1351_amd as km
    a = km.kmeans_workspace_bytes(10_000, 16, 64, 0.01)
    b = km.kmeans_workspace_bytes(10_000_000, 16, 64, 0.01)
    assert 0 < a < b
    assert km.kmeans_workspace_bytes(10, 2, 11, 0.5) == 0
