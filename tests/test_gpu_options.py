"""Options of kmeans_fit_ex against the FP64 oracle, through the C ABI: the
per-pass trace (Table 1's old/new centers and memberships), the opt-in
empty-cluster re-seeding, a caller workspace, and the up-front finiteness
check."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import JTOL, assert_centers, assert_labels, j_atol, to_device

pytestmark = pytest.mark.gpu

km = pytest.importorskip("paper_1108_1351_amd")


def _mixture(n, d, k, seed, dtype="f32", spread=20.0):
    spec = synth.MixtureSpec(d, k, "uniform", -spread, spread, sigma_lo=0.5, sigma_hi=2.0,
                             weights="dirichlet1")
    return synth.generate(spec, seed, n, dtype)


# (name, n, d, k, dtype, precision): one case per pass family
TRACE_CASES = [
    ("split screen", 40_000, 8, 20, "f32", "auto"),
    ("fp32 mfma", 30_000, 24, 40, "f32", "auto"),
    ("point per lane", 20_000, 40, 20, "f32", "fp32"),
    ("bf16 screen", 30_000, 64, 300, "bf16", "auto"),
    ("sorted update", 30_000, 3, 5000, "f32", "auto"),
]


@pytest.mark.parametrize("name,n,d,k,dtype,precision", TRACE_CASES)
def test_trace_matches_oracle(name, n, d, k, dtype, precision):
    Xh = _mixture(n, d, max(2, min(k, 40)), seed=n + d + k, dtype=dtype)
    # tol 0: exactly max_iter passes per stage (a tolerance below the sums'
    # fixed-point quantum would let that quantum decide the pass counts)
    mi, tol = (8, 6), 0.0
    print(f"[trace] {name} n={n} d={d} k={k}", flush=True)
    C, L, info = km.kmeans_fit_ex(to_device(Xh), k, 0.1, 3, mi, tol, precision=precision,
                                  centers64=True, trace=True)
    ref = oracle.fit(Xh, k, 0.1, 3, mi, tol, trace=True)
    assert info["iters"] == ref.info["iters"]
    for s in range(2):
        tc, tn = info["trace_centers"][s], info["trace_counts"][s]
        assert tc.shape == ref.trace_centers[s].shape
        for t in range(len(tc)):
            assert_centers(tc[t], ref.trace_centers[s][t], Xh, name=f"{name} stage {s} pass {t}")
        # sizes: equal, up to points at near-ties of the pass's centers
        slack = np.abs(tn - ref.trace_counts[s]).sum(1)
        assert slack.max() <= 4, (name, s, slack)
        assert (tn.sum(1) == (info["m"] if s == 0 else n)).all()
    # the first fast row holds the sampled initial centers exactly
    sub, ini = oracle.select(n, info["m"], k, 3)
    Xw = Xh.astype(np.float64) if dtype == "f32" else synth.bf16_to_f32(Xh).astype(np.float64)
    assert np.array_equal(info["trace_centers"][0][0], Xw[ini])
    # the slow stage's last row's new centers are the returned ones: one pass
    # from the last row reproduces them within the parity tolerance
    last = info["trace_centers"][1][-1]
    st = oracle.step(Xh, last)
    assert_centers(info["centers64"].cpu().numpy(), st.C_new, Xh, name=f"{name} last pass")


RESEED_CASES = [
    ("split screen", 20_000, 4, 12, "f32", "auto"),
    ("fp32 mfma", 20_000, 24, 12, "f32", "auto"),
    ("bf16 screen", 20_000, 64, 12, "bf16", "auto"),
    ("sorted update", 20_000, 3, 3000, "f32", "auto"),
    ("point per lane", 20_000, 40, 12, "f32", "fp32"),
]


@pytest.mark.parametrize("name,n,d,k,dtype,precision", RESEED_CASES)
def test_reseed_matches_oracle(name, n, d, k, dtype, precision):
    """Starting centers that include copies far outside the data: under the keep
    rule they stay empty; re-seeding moves one per pass to the farthest point.
    The GPU must take the oracle's passes, centers and J."""
    Xh = _mixture(n, d, 6, seed=d * 13 + k, dtype=dtype)
    Xw = Xh.astype(np.float64) if dtype == "f32" else synth.bf16_to_f32(Xh).astype(np.float64)
    rng = np.random.default_rng(k)
    C0 = Xw[rng.choice(n, size=k, replace=False)].copy()
    far = max(3, k // 4)
    C0[-far:] = 1e4 + rng.normal(0, 1.0, size=(far, d))  # never win a point
    mi, tol = (1, 40), 1e-7
    print(f"[reseed] {name} n={n} d={d} k={k}", flush=True)
    C, L, info = km.kmeans_fit_ex(to_device(Xh), k, 1.0, 0, mi, tol, precision=precision,
                                  init_centers=C0, skip_stage1=True, reseed=True,
                                  centers64=True, history=True)
    ref = oracle.fit(Xh, k, 1.0, 0, mi, tol, init_centers=C0, skip_stage1=True, reseed=True)
    keep = oracle.fit(Xh, k, 1.0, 0, mi, tol, init_centers=C0, skip_stage1=True)
    assert keep.info["empty"][1] >= far and ref.info["empty"][1] < keep.info["empty"][1]
    assert info["iters"] == ref.info["iters"], (info["iters"], ref.info["iters"])
    assert info["empty"] == ref.info["empty"]
    assert_centers(info["centers64"].cpu().numpy(), ref.centers, Xh, name=name)
    assert abs(info["J"] - ref.info["J"]) <= JTOL * ref.info["J"] + j_atol(Xh)
    amax = float(np.abs(Xw).max())
    assert np.allclose(info["shift_hist"][1], ref.shift_hist[1], rtol=1e-5, atol=1e-6 * amax)
    assert_labels(L, Xh, ref.centers, ref_labels=ref.labels, name=name)


def test_reseed_two_stage_fit_default_keeps_results():
    """reseed = 0 (the default) gives the same bits as before; a two-stage fit
    with re-seeding matches the oracle's two-stage fit with re-seeding."""
    w = synth.WORKLOADS["gmm16d_n1e7_k64"].scaled(60_000)
    Xh = w.data()
    X = to_device(Xh)
    a = km.kmeans_fit_ex(X, w.k, 0.01, w.fit_seed, w.max_iter, w.tol, centers64=True)
    b = km.kmeans_fit_ex(X, w.k, 0.01, w.fit_seed, w.max_iter, w.tol, centers64=True,
                         reseed=False)
    assert torch.equal(a[2]["centers64"], b[2]["centers64"])
    C, L, info = km.kmeans_fit_ex(X, w.k, 0.01, w.fit_seed, w.max_iter, w.tol, centers64=True,
                                  reseed=True)
    ref = oracle.fit(Xh, w.k, 0.01, w.fit_seed, w.max_iter, w.tol, reseed=True)
    assert info["iters"] == ref.info["iters"]
    assert_centers(info["centers64"].cpu().numpy(), ref.centers, Xh)
    assert abs(info["J"] - ref.info["J"]) <= JTOL * ref.info["J"]


@pytest.mark.parametrize("d,k,dtype", [(16, 64, "f32"), (128, 300, "bf16"), (3, 5000, "f32")])
def test_caller_workspace(d, k, dtype):
    """A workspace of kmeans_workspace_bytes gives the bits of an allocating
    call; one byte less is KM_ENOMEM (the size asked for covers every option,
    labels given or not)."""
    n = 30_011
    Xh = _mixture(n, d, min(k, 40), seed=d + k, dtype=dtype)
    X = to_device(Xh)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    need = km.kmeans_workspace_bytes(n, d, k, 0.05, max_iter=10, dtype=tdt)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    a = km.kmeans_fit_ex(X, k, 0.05, 1, 10, 1e-6, centers64=True)
    b = km.kmeans_fit_ex(X, k, 0.05, 1, 10, 1e-6, centers64=True, workspace=ws)
    assert torch.equal(a[2]["centers64"], b[2]["centers64"]) and torch.equal(a[1], b[1])
    assert a[2]["J"] == b[2]["J"] and a[2]["iters"] == b[2]["iters"]
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_fit_ex(X, k, 0.05, 1, 10, 1e-6, workspace=ws[:need - 1])
    assert e.value.status == km.KM_ENOMEM


def test_check_finite_rejects_before_any_pass():
    """A NaN outside the fast-stage subset: both modes return KM_EINVAL (with
    check_finite the scan runs before the fast stage)."""
    n = 50_000
    Xh = _mixture(n, 4, 5, seed=9)
    sub, _ = oracle.select(n, oracle.subset_size(n, 5, 0.01), 5, 3)
    bad = int(np.setdiff1d(np.arange(n), sub)[7])
    Xh[bad, 1] = np.nan
    for cf in (True, False):
        with pytest.raises(km.KMeansError) as e:
            km.kmeans_fit_ex(to_device(Xh), 5, 0.01, 3, 10, 1e-4, check_finite=cf)
        assert e.value.status == km.KM_EINVAL
    Xh[bad, 1] = np.inf
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_fit_ex(to_device(Xh), 5, 0.01, 3, 10, 1e-4, check_finite=True)
    assert e.value.status == km.KM_EINVAL
